"""GPU flow assembly and coupled hydro-mechanical step against the CPU oracle
(oracle/flow.py: dense P1 matrices, dense exact Jacobian, dense LU).

  * S and L assembled on the GPU equal the oracle's entry by entry (cubic
    law and constant permeability, jittered two-part mesh; bar 1e-13 of the
    largest entry: both are sums of the same few FP64 products);
  * the coupled Newton step (interface law, flow, P_up-preconditioned
    FGMRES with inner A11 GMRES) returns the oracle's increments within 1e-8
    (relative, per block) on a shear-loaded fault with a pressure source,
    with the same Newton iteration count within one, and conserves the
    fluid volume like the oracle;
  * the solution does not depend on the block scaling (Sec. 3.3.2), and
    P_up keeps the outer iterations per Jacobian solve to a few tens at 1e-9.
"""
import numpy as np
import pytest

import oracle
from oracle import flow as OF
from oracle import interface as law
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25
EP = YOUNG / (1 - NU * NU)


def _hm():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available()
    return hm


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _two_part_tri(seed=5):
    rng = np.random.default_rng(seed)
    a = W.rect_tri_mesh(8.0, 6.0, 8, 6, (0.0, 0.0, 0.0), np.eye(3), "a")
    ax = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(1.0), np.sin(1.0)], [0.0, -np.sin(1.0), np.cos(1.0)]])
    b = W.rect_tri_mesh(6.0, 5.0, 6, 5, (1.0, 0.5, 3.5), ax, "b")
    xyz = np.concatenate([a.xyz, b.xyz])
    xyz = xyz + rng.normal(0.0, 0.07, xyz.shape)
    conn = np.concatenate([a.conn, b.conn + a.nv])
    return W.Mesh(xyz, conn, "two_parts")


def _dense_csr(rowptr, col, v, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rowptr[i]:rowptr[i + 1]]] = v[rowptr[i]:rowptr[i + 1]]
    return A


@pytest.mark.parametrize("law_", ["cubic", "constant"])
def test_flow_matrices_match_the_oracle(law_):
    hm = _hm()
    m = _two_part_tri()
    M, mu, k0 = 2e9, 1e-3, 3e-12
    perm = hm.HM_PERM_CUBIC if law_ == "cubic" else hm.HM_PERM_CONSTANT
    fl = hm.Flow(hm.Mesh.from_workload(m), M, mu, perm, k0)
    w = np.random.default_rng(6).uniform(1e-4, 5e-4, m.ne)
    rowptr, col, S, L = fl.matrices(cuda(w))
    s, _, t, _ = OF.coefficients(w, np.zeros(m.ne), M, mu, OF.PERM_CUBIC if law_ == "cubic" else OF.PERM_CONSTANT, k0)
    _, So, Lo, _ = OF.assemble(m, (s, t))
    Sg, Lg = _dense_csr(rowptr, col, S, m.nv), _dense_csr(rowptr, col, L, m.nv)
    assert np.array_equal(Sg != 0, So != 0)
    assert np.abs(Sg - So).max() <= 1e-13 * np.abs(So).max()
    assert np.abs(Lg - Lo).max() <= 1e-13 * np.abs(Lo).max()
    # every row lists each node at most once, the diagonal included
    for i in range(m.nv):
        r = col[rowptr[i]:rowptr[i + 1]]
        assert len(set(r.tolist())) == r.size and i in r


def _case(n=8):
    m = W.rect_tri_mesh(8.0, 8.0, n, n)
    N, nn = m.ne, m.nv
    h = np.sqrt(64.0 / N * 2)
    # a slip-weakening fault under shear, close to failure: the pressure
    # source lowers the effective normal stress and the centre slips
    mats = law.material(EP / h / 3, EP / h, 0.6, 0.45, 0.05, 0.05, 0.0, 0.0, 0.0)[None]
    t_n = np.tile([5.8e6, 0.0, -10e6], (N, 1))
    f = np.zeros(nn)
    f[np.argmin(np.sum(m.xyz ** 2, axis=1))] = 3e-4
    mech = dict(mats=mats, mat_id=np.zeros(N, np.int32), t_n=t_n, dp_n=np.zeros((N, 3)), chi_n=np.zeros((N, 3)),
                dT0=np.zeros((N, 3)), eta_dt=np.full((N, 3), 5e7), dd_prev=np.zeros((N, 3)))
    flow = dict(p_n=np.zeros(nn), p_o=np.zeros(nn), f=f, dt=2.0, dn_start=np.zeros(N), w0=np.full(N, 2e-4),
                M=1e9, mu=1e-3, perm_law=OF.PERM_CUBIC)
    return m, mech, flow


def _gpu_step(hm, m, mech, flow, scales=(1.0, 1.0, 1e-6, 1.0), **opts):
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, aca_tol=1e-12)
    fl = hm.Flow(hm.Mesh.from_workload(m), flow["M"], flow["mu"], hm.HM_PERM_CUBIC)
    N = m.ne
    z3 = cuda(np.zeros((N, 3)))
    return hm.coupled_step(op, fl, mech["mats"], cuda(mech["t_n"]), z3, z3, cuda(flow["p_n"]), cuda(flow["w0"]),
                           flow["dt"], eta_dt=cuda(mech["eta_dt"]), dd_prev=z3, p_o=cuda(flow["p_o"]),
                           source=cuda(flow["f"]), dn_start=cuda(flow["dn_start"]), scales=scales, **opts)


def test_coupled_step_matches_the_oracle():
    hm = _hm()
    m, mech, flow = _case()
    E = oracle.dense(m, YOUNG, NU)
    injected = flow["dt"] * flow["f"].sum()
    dd_o, dp_o, st_o, hist_o = OF.coupled_newton_step(E, m, mech, flow, (1e6, injected), rtol=1e-12)
    sR = (1.0, 1.0, 1e-6, 1.0 / injected)
    dd, dpn, t_new, _, _, rep = _gpu_step(hm, m, mech, flow, scales=sR, rtol=1e-12, outer_rtol=1e-10,
                                          inner_rtol=1e-10, inner_max_iter=2000, max_newton=30)
    dd, dpn = dd.cpu().numpy(), dpn.cpu().numpy()
    e_dd = np.linalg.norm(dd - dd_o) / np.linalg.norm(dd_o)
    e_dp = np.linalg.norm(dpn - dp_o) / np.linalg.norm(dp_o)
    modes_o = np.bincount(st_o[4], minlength=5)
    print(f"coupled step: Newton {rep['iterations']} (oracle {len(hist_o) - 1}), outer {rep['outer_iterations']}, "
          f"inner {rep['inner_iterations']}; errors dd {e_dd:.2e} dp {e_dp:.2e}; modes {rep['modes']}", flush=True)
    assert rep["converged"] and e_dd <= 1e-8 and e_dp <= 1e-8
    assert abs(rep["iterations"] - (len(hist_o) - 1)) <= 1
    assert list(rep["modes"]) == modes_o.tolist()
    assert modes_o[0] > 0 and modes_o[1] > 0          # elastic and slipping elements both present
    # volume balance at the GPU solution
    s_new, _, _, _ = OF.coefficients(flow["dn_start"] + dd[:, 2], flow["w0"], flow["M"], flow["mu"])
    _, S, _, _ = OF.assemble(m, (s_new, np.zeros(m.ne)))
    area, _, _ = OF.geometry(m)
    assert np.sum(area * dd[:, 2]) + np.ones(m.nv) @ S @ dpn == pytest.approx(injected, rel=1e-8)


def test_scaling_leaves_the_solution_and_p_up_keeps_outer_iterations_low():
    hm = _hm()
    m, mech, flow = _case(6)
    injected = flow["dt"] * flow["f"].sum()
    res = []
    for sc in ((1.0, 1.0, 1e-6, 1.0 / injected), (1e4, 1e-6, 1e-7, 1e2 / injected)):
        dd, dpn, _, _, _, rep = _gpu_step(hm, m, mech, flow, scales=sc, rtol=1e-11, outer_rtol=1e-9,
                                          inner_rtol=1e-10, inner_max_iter=2000)
        assert rep["converged"]
        # P_up with a tight inner A11 solve: each Jacobian solve to 1e-9 in a
        # few tens of iterations (measured 14: the Schur complement from
        # diag(A11) and its ILU(0) leave a contraction of about 0.2 per step)
        assert max(rep["outer_iterations"]) <= 20, rep["outer_iterations"]
        res.append((dd.cpu().numpy(), dpn.cpu().numpy()))
    assert np.linalg.norm(res[0][0] - res[1][0]) <= 1e-7 * np.linalg.norm(res[0][0])
    assert np.linalg.norm(res[0][1] - res[1][1]) <= 1e-7 * np.linalg.norm(res[0][1])


def test_second_schur_choice_gives_the_same_step():
    """The paper's second approximation of the Schur complement (A~11 the ILU
    of C^ep plus the largest near-field entries, S~ applied matrix-free and
    inverted by GMRES preconditioned with the first choice): the same
    converged step, with no more outer iterations than the first choice."""
    hm = _hm()
    m, mech, flow = _case(6)
    injected = flow["dt"] * flow["f"].sum()
    sc = (1.0, 1.0, 1e-6, 1.0 / injected)
    out = {}
    for schur in (0, 1):
        dd, dpn, _, _, _, rep = _gpu_step(hm, m, mech, flow, scales=sc, rtol=1e-11, outer_rtol=1e-9,
                                          inner_rtol=1e-10, inner_max_iter=2000, inner_precond=hm.HM_PC_ILU,
                                          inner_ilu_fraction=0.05, schur=schur, schur_rtol=1e-6, schur_max_iter=60)
        assert rep["converged"]
        out[schur] = (dd.cpu().numpy(), dpn.cpu().numpy(), rep)
    print("outer iterations: first choice", out[0][2]["outer_iterations"], "second", out[1][2]["outer_iterations"],
          "schur GMRES", out[1][2]["schur_iterations"], flush=True)
    assert np.linalg.norm(out[0][0] - out[1][0]) <= 1e-7 * np.linalg.norm(out[0][0])
    assert np.linalg.norm(out[0][1] - out[1][1]) <= 1e-7 * np.linalg.norm(out[0][1])
    assert sum(out[1][2]["outer_iterations"]) <= sum(out[0][2]["outer_iterations"])
    assert all(k > 0 for k in out[1][2]["schur_iterations"])


def test_adaptive_coupled_steps_match_the_oracle():
    """Adaptive time stepping of the coupled problem (Sec. 3.4): each step's
    truncation error is the larger of the DD estimate and the pressure
    estimate (each the rate change over the step, relative to the current
    solution); the controller sets the next step.  Library (coupled step,
    GPU estimates, host controller) against the oracle's driver (dense
    coupled Newton, its own estimate and controller) over four steps: the
    same step sizes, Newton counts and states."""
    from oracle import timestep as OT

    hm = _hm()
    m, mech, flow = _case(6)
    N, nn = m.ne, m.nv
    E = oracle.dense(m, YOUNG, NU)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, aca_tol=1e-12)
    fl = hm.Flow(hm.Mesh.from_workload(m), flow["M"], flow["mu"], hm.HM_PERM_CUBIC)
    ctl = dict(eps_tol=1e-2, n_target=4, growth_max=1.5)
    q = float(flow["f"].sum())
    # oracle state
    o = dict(t=mech["t_n"].copy(), dpl=np.zeros((N, 3)), chi=np.zeros((N, 3)), p=np.zeros(nn), dn=np.zeros(N),
             d=np.zeros((N, 3)), dd_prev=None, dp_prev=None)
    g = dict(t=cuda(mech["t_n"]), dpl=cuda(np.zeros((N, 3))), chi=cuda(np.zeros((N, 3))),
             p=cuda(np.zeros(nn)), dn=cuda(np.zeros(N)), d=cuda(np.zeros((N, 3))), dd_prev=None, dp_prev=None)
    dt, dt_prev, e_prev = 0.5, 0.0, 0.0
    for k in range(4):
        eta = mech["eta_dt"] * (2.0 / dt)       # eta / dt for this step (eta_dt was given for dt = 2 s)
        prev_o = np.zeros((N, 3)) if o["dd_prev"] is None else o["dd_prev"] * dt / dt_prev
        mo = dict(mech, t_n=o["t"], dp_n=o["dpl"], chi_n=o["chi"], eta_dt=eta, dd_prev=prev_o)
        fo = dict(flow, p_n=o["p"], dt=dt, dn_start=o["dn"])
        dd_o, dp_o, st_o, hist_o = OF.coupled_newton_step(E, m, mo, fo, (1e6, q * dt), rtol=1e-12)
        prev_g = cuda(prev_o) if g["dd_prev"] is None else g["dd_prev"] * (dt / dt_prev)
        dd, dpn, t_new, dpl_new, chi_new, rep = hm.coupled_step(
            op, fl, mech["mats"], g["t"], g["dpl"], g["chi"], g["p"], cuda(flow["w0"]), dt, eta_dt=cuda(eta),
            dd_prev=prev_g, p_o=cuda(flow["p_o"]), source=cuda(flow["f"]), dn_start=g["dn"],
            scales=(1.0, 1.0, 1e-6, 1.0 / (q * dt)), rtol=1e-12, outer_rtol=1e-10, inner_rtol=1e-10,
            inner_max_iter=2000, max_newton=30)
        assert rep["converged"] and abs(rep["iterations"] - (len(hist_o) - 1)) <= 1
        assert np.linalg.norm(dd.cpu().numpy() - dd_o) <= 1e-8 * np.linalg.norm(dd_o)
        assert np.linalg.norm(dpn.cpu().numpy() - dp_o) <= 1e-8 * np.linalg.norm(dp_o)
        # truncation errors: DD and pressure, the larger one drives the controller
        e_o = max(OT.truncation_error(dd_o, dt, o["dd_prev"], dt_prev, o["d"] + dd_o),
                  OT.truncation_error(dp_o, dt, o["dp_prev"], dt_prev, o["p"] + dp_o))
        e_g = max(hm.lte_estimate(dd.reshape(-1), dt, None if g["dd_prev"] is None else g["dd_prev"].reshape(-1),
                                  dt_prev, (g["d"] + dd).reshape(-1)),
                  hm.lte_estimate(dpn, dt, g["dp_prev"], dt_prev, g["p"] + dpn))
        assert e_g == pytest.approx(e_o, rel=1e-6), (k, e_g, e_o)
        n_it = max(1, len(hist_o) - 1)
        dt_next_o = OT.next_step(dt, dt_prev, e_o, e_prev, n_it, **ctl)
        dt_next_g = hm.timestep_next(dt, dt_prev, e_g, e_prev, max(1, rep["iterations"]), **ctl)
        assert dt_next_g == pytest.approx(dt_next_o, rel=1e-6)
        print(f"step {k}: dt {dt:.4f} s, Newton {rep['iterations']}, e {e_g:.3e}, next {dt_next_g:.4f} s", flush=True)
        # advance both
        o.update(t=st_o[0], dpl=st_o[1], chi=st_o[2], p=o["p"] + dp_o, dn=o["dn"] + dd_o[:, 2], d=o["d"] + dd_o,
                 dd_prev=dd_o, dp_prev=dp_o)
        g.update(t=t_new, dpl=dpl_new, chi=chi_new, p=g["p"] + dpn, dn=g["dn"] + dd[:, 2], d=g["d"] + dd,
                 dd_prev=dd, dp_prev=dpn)
        dt_prev, e_prev, dt = dt, e_g, dt_next_g
    assert np.linalg.norm(g["p"].cpu().numpy() - o["p"]) <= 1e-8 * np.linalg.norm(o["p"])
