"""Adaptive time stepping of the mechanical problem (paper Sec. 3.4) on
the GPU against the CPU FP64 oracle, step by step.

The same driver runs both sides: each step is an implicit Newton step
(library: hm_newton_step on the H-matrix at ACA 1e-12; oracle: dense E,
its own interface law, dense LU), a step that does not converge is
halved and retried, the quasi-dynamic term's previous increment is
rescaled to the current step, and the truncation-error estimate and the
controller (library: hm_lte_estimate and hm_timestep_next; oracle:
oracle.timestep) give the next step.  Bars: the same accepted and rejected
steps, step sizes within 1e-9, Newton counts within one, the total DD
within 1e-8 and the same mode counts in the last step.
"""
import numpy as np
import pytest

import oracle
from oracle import interface as law
from oracle import newton
from oracle import timestep as ts
from workloads import square_fault

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25
EP = YOUNG / (1 - NU * NU)
CTRL = dict(eps_tol=1e-2, n_target=6, growth_max=1.2, dt_min=1e-3)
N_STEPS = 6


def _case():
    """16 x 16 slip-weakening dilatant fault shear-loaded below its peak
    strength; the pore pressure on a central patch rises linearly by 2 MPa
    per second, so the patch starts slipping during the run."""
    n = 16
    m = square_fault(n)
    cent, _, _ = oracle.frames(m)
    r = np.hypot(cent[:, 0] - n / 2, cent[:, 1] - n / 2)
    mats = law.material(EP / 3, EP, 0.6, 0.45, 0.05, 0.05, 0.0, 0.0, 0.0)[None]
    t0 = np.zeros((m.ne, 3))
    t0[:, 0] = 5.5e6
    t0[:, 2] = -10e6
    pressure = lambda t: np.where(r < 5.0, 2e6 * t, 0.0)
    return m, mats, t0, pressure, 2.5e7        # eta in Pa s / m on every component


def _adaptive(step, lte, nxt, m, t0, pressure, eta):
    """Shared driver.  step(state, dpress, eta_dt, dd_prev) -> (dd, state, its, converged, mode counts);
    lte(dd, dt, dd_prev, dt_prev, total) -> e; nxt(dt, dt_prev, e, e_prev, its) -> next dt."""
    state = (t0, np.zeros((m.ne, 3)), np.zeros((m.ne, 3)))
    total = np.zeros((m.ne, 3))
    t, dt, dt_prev, e_prev, dd_prev = 0.0, 0.25, 0.0, 0.0, None
    log = []
    while sum(1 for s in log if s[0] == "ok") < N_STEPS:
        dpress = pressure(t + dt) - pressure(t)
        prev = np.zeros((m.ne, 3)) if dd_prev is None else dd_prev * (dt / dt_prev)
        dd, new_state, its, conv, modes = step(state, dpress, np.full((m.ne, 3), eta / dt), prev)
        if not conv:
            log.append(("rejected", dt, its, 0.0))
            dt *= 0.5
            assert len(log) < 20
            continue
        total = total + dd
        # the first step has no previous rate: taken as on target
        e = CTRL["eps_tol"] if dd_prev is None else lte(dd, dt, dd_prev, dt_prev, total)
        log.append(("ok", dt, its, e))
        t += dt
        state, dd_prev = new_state, dd
        dt, dt_prev, e_prev = nxt(dt, dt_prev, e, e_prev, max(its, 1)), dt, e
    return log, total, modes


def test_adaptive_steps_match_the_oracle():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available(), "GPU tests need a device"
    m, mats, t0, pressure, eta = _case()
    E = oracle.dense(m, YOUNG, NU)
    mat_id = np.zeros(m.ne, np.int32)

    def o_step(state, dpress, eta_dt, prev):
        z = np.zeros((m.ne, 3))
        dd, st, hist = newton.newton_step(E, mats, mat_id, *state, z, dpress=dpress, eta_dt=eta_dt, dd_prev=prev,
                                          rtol=1e-12)
        return dd, st[:3], len(hist) - 1, hist[-1] <= 1e-12 * hist[0], np.bincount(st[4], minlength=5).tolist()

    o_log, o_total, o_modes = _adaptive(o_step, ts.truncation_error,
                                        lambda *a: ts.next_step(*a, **CTRL), m, t0, pressure, eta)

    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=16, aca_tol=1e-12)
    cu = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    def g_step(state, dpress, eta_dt, prev):
        dd, t_new, dp_new, chi_new, rep = op.newton_step(mats, *(cu(s) for s in state), dpress=cu(dpress),
                                                         eta_dt=cu(eta_dt), dd_prev=cu(prev), rtol=1e-12,
                                                         lin_rtol=1e-12, raise_on_notconv=False)
        return (dd.cpu().numpy(), tuple(a.cpu().numpy() for a in (t_new, dp_new, chi_new)), rep["iterations"],
                bool(rep["converged"]), rep["modes"])

    def g_lte(dd, dt, dd_prev, dt_prev, total):
        return hm.lte_estimate(cu(dd).reshape(-1), dt, cu(dd_prev).reshape(-1), dt_prev, cu(total).reshape(-1))

    g_log, g_total, g_modes = _adaptive(g_step, g_lte, lambda *a: hm.timestep_next(*a, **CTRL), m, t0, pressure,
                                        eta)
    print("oracle", [(s[0], round(s[1], 6), s[2], f"{s[3]:.3e}") for s in o_log], flush=True)
    print("gpu   ", [(s[0], round(s[1], 6), s[2], f"{s[3]:.3e}") for s in g_log], flush=True)
    assert [s[0] for s in g_log] == [s[0] for s in o_log]
    np.testing.assert_allclose([s[1] for s in g_log], [s[1] for s in o_log], rtol=1e-9)
    assert all(abs(a[2] - b[2]) <= 1 for a, b in zip(g_log, o_log))
    err = np.linalg.norm(g_total - o_total) / np.linalg.norm(o_total)
    print("total DD difference", err, flush=True)
    assert err <= 1e-8
    print("modes of the last step", o_modes, g_modes, flush=True)
    assert g_modes == o_modes and o_modes[law.SHEAR] > 0
