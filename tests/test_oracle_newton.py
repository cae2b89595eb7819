"""Pins of the oracle's Newton step of the mechanical problem (CPU only).

The residual's sign conventions are pinned by closed forms: a pressurised
open penny crack (Sneddon) and a frictionless penny under a uniform shear
stress drop (Eshelby); the consistency of the residual with the tangent by
quadratic convergence (and the slower convergence of the same iteration
with the elastic stiffness in place of C^ep).
"""
import numpy as np
import pytest

import oracle
from oracle import interface as law
from oracle import newton
from workloads import penny_active_mask, square_fault

YOUNG, NU = 30e9, 0.25
EP = YOUNG / (1 - NU * NU)
LOCKED = law.material(1e16, 1e16, 0.6, 0.6, 0.0, float("inf"), 1e12, 1e11, float("inf"))


def _penny_setup(n):
    m = square_fault(n)
    act = penny_active_mask(m).astype(bool)
    cent, _, _ = oracle.frames(m)
    r = np.hypot(cent[:, 0] - n / 2, cent[:, 1] - n / 2)
    return m, act, r


def test_pressurised_penny_opens_as_sneddon(oracle_lib):
    """Pre-existing crack closed under 1 MPa; a pore-pressure rise of 3 MPa
    opens it (traction-free faces), net opening pressure 2 MPa; the outside
    is locked by a stiff unbreakable interface."""
    n = 32
    m, act, r = _penny_setup(n)
    crack = law.material(EP, EP, 0.6, 0.6, 0.0, 0.0, 0.0, 0.0, 0.0)
    mats = np.stack([crack, LOCKED])
    mat_id = np.where(act, 0, 1).astype(np.int32)
    t_n = np.zeros((m.ne, 3))
    t_n[act, 2] = -1e6
    dpress = np.where(act, 3e6, 0.0)
    E = oracle.dense(m, YOUNG, NU)
    dd, state, hist = newton.newton_step(E, mats, mat_id, t_n, np.zeros((m.ne, 3)), np.zeros((m.ne, 3)),
                                         np.zeros((m.ne, 3)), dpress=dpress)
    assert hist[-1] <= 1e-12 * hist[0] and len(hist) <= 4
    assert (state[4][act] == law.OPEN).all() and (state[4][~act] == law.ELASTIC).all()
    w = oracle.penny_opening(r, 0.45 * n, 2e6, YOUNG, NU)
    assert abs(dd[act, 2].max() / w.max() - 1) < 0.02
    assert np.linalg.norm(dd[act, 2] - w[act]) / np.linalg.norm(w[act]) < 0.06
    assert np.abs(dd[~act]).max() < 1e-5 * dd[act, 2].max()


def test_frictionless_penny_slips_as_eshelby(oracle_lib):
    """Frictionless pre-existing crack under 1 MPa shear and 10 MPa
    compression: the shear traction drops to zero and the slip is the
    uniform-stress-drop penny solution."""
    n, tau = 32, 1e6
    m, act, r = _penny_setup(n)
    crack = law.material(EP / 2, EP, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    mats = np.stack([crack, LOCKED])
    mat_id = np.where(act, 0, 1).astype(np.int32)
    t_n = np.zeros((m.ne, 3))
    t_n[act, 0] = tau
    t_n[act, 2] = -10e6
    E = oracle.dense(m, YOUNG, NU)
    dd, state, hist = newton.newton_step(E, mats, mat_id, t_n, np.zeros((m.ne, 3)), np.zeros((m.ne, 3)),
                                         np.zeros((m.ne, 3)))
    assert hist[-1] <= 1e-12 * hist[0]
    assert (state[4][act] == law.SHEAR).all()
    np.testing.assert_allclose(state[0][act, 0], 0.0, atol=1e-6)
    s = oracle.penny_slip(r, 0.45 * n, tau, YOUNG, NU)
    assert abs(dd[act, 0].max() / s.max() - 1) < 0.02
    assert np.abs(dd[act, 1]).max() < 0.03 * dd[act, 0].max()


def _weakening_case():
    """16 x 16 fault, slip-weakening and dilatant, shear-loaded near its peak
    strength; a pore-pressure rise of 2 MPa on a central patch sets it
    slipping."""
    n = 16
    m = square_fault(n)
    cent, _, _ = oracle.frames(m)
    r = np.hypot(cent[:, 0] - n / 2, cent[:, 1] - n / 2)
    k = EP / 1.0
    mats = law.material(k / 3, k, 0.6, 0.45, 0.05, 0.05, 0.0, 0.0, 0.0)[None]
    mat_id = np.zeros(m.ne, np.int32)
    t_n = np.zeros((m.ne, 3))
    t_n[:, 0] = 5.5e6
    t_n[:, 2] = -10e6
    dpress = np.where(r < 5.0, 2e6, 0.0)
    eta_dt = np.full((m.ne, 3), 1e8)
    return m, mats, mat_id, t_n, dpress, eta_dt


def test_newton_converges_quadratically_with_the_consistent_tangent(oracle_lib):
    m, mats, mat_id, t_n, dpress, eta_dt = _weakening_case()
    E = oracle.dense(m, YOUNG, NU)
    z = np.zeros((m.ne, 3))
    dd, state, hist = newton.newton_step(E, mats, mat_id, t_n, z, z, z, dpress=dpress, eta_dt=eta_dt, dd_prev=z,
                                         rtol=1e-13)
    assert hist[-1] <= 1e-13 * hist[0]
    assert (state[4] == law.SHEAR).sum() >= 20
    rho = [h / hist[0] for h in hist]
    # once in the quadratic regime each step squares the relative residual (constant 10),
    # above the rounding floor
    quad = [(a, b) for a, b in zip(rho, rho[1:]) if a < 1e-2 and b > 1e-13]
    assert quad and all(b <= 10 * a * a for a, b in quad), rho
    assert len(hist) <= 8, rho


def test_elastic_stiffness_jacobian_converges_only_linearly(oracle_lib, monkeypatch):
    """Planted mistake, on the CPU: with C (the elastic stiffness) in place
    of C^ep the same iteration needs many more steps to the same residual."""
    m, mats, mat_id, t_n, dpress, eta_dt = _weakening_case()
    E = oracle.dense(m, YOUNG, NU)
    z = np.zeros((m.ne, 3))
    _, _, hist_exact = newton.newton_step(E, mats, mat_id, t_n, z, z, z, dpress=dpress, eta_dt=eta_dt,
                                          dd_prev=z, rtol=1e-10)
    real_update = law.update

    def elastic_tangent(mats_, mat_id_, *a):
        T, dp, chi, cep, mode = real_update(mats_, mat_id_, *a)
        C = np.zeros_like(cep)
        ids = np.zeros(len(cep), np.int32) if mat_id_ is None else mat_id_
        C[:, 0, 0] = mats_[ids, law.KS]
        C[:, 1, 1] = mats_[ids, law.KS]
        C[:, 2, 2] = mats_[ids, law.KN]
        return T, dp, chi, C, mode

    monkeypatch.setattr(law, "update", elastic_tangent)
    _, _, hist_elastic = newton.newton_step(E, mats, mat_id, t_n, z, z, z, dpress=dpress, eta_dt=eta_dt,
                                            dd_prev=z, rtol=1e-10, max_newton=60)
    assert len(hist_elastic) >= 2 * len(hist_exact), (hist_exact, hist_elastic)
