"""Pins of the interface-law oracle (CPU only).

Each pin uses something other than the oracle's own code: closed forms
derived by hand for the returns without weakening, the closest-point
projection of associated plasticity, energy integrals of the weakening
laws, central finite differences of the whole algorithm, and symmetry.
"""
import math

import numpy as np
import pytest

from oracle import interface as I

INF = float("inf")


def _mat(ks=3.2e10, kn=3.2e10, fp=0.6, fr=0.6, psi=0.0, dc=INF, c=2e6, st=1e6, wc=INF):
    return I.material(ks, kn, fp, fr, psi, dc, c, st, wc)


def _upd(m, dd, T0, dp0=(0.0, 0.0, 0.0), chi0=(0.0, 0.0, 0.0)):
    return I.update_element(m, np.asarray(dd, float), np.asarray(T0, float), np.asarray(dp0, float),
                            np.asarray(chi0, float))


def test_elastic_step_is_the_stiffness():
    m = _mat()
    r = _upd(m, [1e-5, -2e-5, -1e-5], [0.3e6, 0.1e6, -10e6])
    C = np.diag([m[I.KS], m[I.KS], m[I.KN]])
    assert r["mode"] == I.ELASTIC
    np.testing.assert_allclose(r["T"], [0.3e6, 0.1e6, -10e6] + C @ [1e-5, -2e-5, -1e-5], rtol=1e-15)
    np.testing.assert_array_equal(r["cep"], C)
    np.testing.assert_array_equal(r["dp"], 0.0)


@pytest.mark.parametrize("psi", [0.0, 0.15])
def test_coulomb_return_without_weakening_matches_closed_form(psi):
    """Perfectly plastic Coulomb with constant dilatancy: lam = Fc_tr/(Ks + f psi Kn),
    T = T_tr - lam C N, and the tangent derived by hand,
    C^ep = C - C N g^T C / (g^T C N) - (Ks^2 lam / q) (I - s s^T) on the shear plane,
    N = s + psi n, g = s + f n."""
    ks, kn, f, c = 2.0e10, 5.0e10, 0.55, 1.5e6
    m = _mat(ks=ks, kn=kn, fp=f, fr=f, psi=psi, c=c, st=0.0)
    T0, dd = np.array([7e6, -1e6, -12e6]), np.array([2e-4, 1e-4, -3e-5])
    C = np.diag([ks, ks, kn])
    Ttr = T0 + C @ dd
    q = math.hypot(Ttr[0], Ttr[1])
    s = np.array([Ttr[0] / q, Ttr[1] / q, 0.0])
    n = np.array([0.0, 0.0, 1.0])
    F = q + f * Ttr[2] - c
    assert F > 0
    lam = F / (ks + f * psi * kn)
    N, g = s + psi * n, s + f * n
    T = Ttr - lam * C @ N
    P = np.diag([1.0, 1.0, 0.0]) - np.outer(s, s)
    cep = C - np.outer(C @ N, g @ C) / (g @ C @ N) - (ks * ks * lam / q) * P
    r = _upd(m, dd, T0)
    assert r["mode"] == I.SHEAR
    np.testing.assert_allclose(r["T"], T, rtol=1e-13, atol=1e-7)
    np.testing.assert_allclose(r["dp"], lam * N, rtol=1e-13, atol=1e-20)
    np.testing.assert_allclose(r["cep"], cep, rtol=1e-10, atol=1e-10 * ks)
    assert r["chi"][0] == pytest.approx(lam, rel=1e-14)
    assert r["chi"][2] == pytest.approx(lam * psi, rel=1e-14, abs=1e-30)


def test_tension_cutoff_without_weakening_matches_closed_form():
    ks, kn, st = 2.0e10, 4.0e10, 1.2e6
    m = _mat(ks=ks, kn=kn, c=5e6, st=st)
    T0, dd = np.array([0.1e6, 0.05e6, 0.5e6]), np.array([1e-6, 0.0, 4e-5])
    Ttr = T0 + np.array([ks, ks, kn]) * dd
    r = _upd(m, dd, T0)
    assert r["mode"] == I.TENSILE
    np.testing.assert_allclose(r["T"], [Ttr[0], Ttr[1], st], rtol=1e-14)
    np.testing.assert_allclose(r["dp"], [0, 0, (Ttr[2] - st) / kn], rtol=1e-13, atol=1e-20)
    np.testing.assert_allclose(r["cep"], np.diag([ks, ks, 0.0]), atol=1e-6)


def _closest_point(Ttr, f, c, st):
    """Euclidean projection of a traction onto {|tau| + f Tn <= c, Tn <= st}
    (cut-off below the cone apex), by enumerating the candidate faces."""
    q, tn = math.hypot(Ttr[0], Ttr[1]), Ttr[2]
    cands = []

    def feasible(qq, tt):
        return qq >= -1e-9 and qq + f * tt <= c * (1 + 1e-12) + 1e-6 and tt <= st + 1e-6

    if feasible(q, tn):
        cands.append((q, tn))
    # cone face: project (tn, q) onto the line q = c - f tn in the (tn, q) half-plane
    d = (q + f * tn - c) / (1 + f * f)
    cands.append((q - d, tn - f * d))
    cands.append((q, st))                               # cut-off plane
    cands.append((c - f * st, st))                      # corner circle
    best = min((v for v in cands if feasible(*v)), key=lambda v: (v[0] - q) ** 2 + (v[1] - tn) ** 2)
    qq, tt = best
    return np.array([Ttr[0] * qq / q, Ttr[1] * qq / q, tt])


@pytest.mark.parametrize("f", [0.25, 0.6, 1.2])
def test_associated_return_is_the_closest_point_projection(f):
    """With psi = f, Ks = Kn and no weakening the backward-Euler return is the
    Euclidean closest point of the elastic domain to the trial traction
    (independent check of the mode selection, the corner and the returns)."""
    c, st, k = 2e6, 1e6, 3e10
    m = _mat(ks=k, kn=k, fp=f, fr=f, psi=f, c=c, st=st)
    rng = np.random.default_rng(71)
    modes = set()
    for _ in range(400):
        Ttr = np.array([*rng.normal(0, 3e6, 2), rng.uniform(-6e6, 5e6)])
        r = _upd(m, np.zeros(3), Ttr)
        modes.add(r["mode"])
        np.testing.assert_allclose(r["T"], _closest_point(Ttr, f, c, st), rtol=1e-12, atol=1e-6)
    assert {I.ELASTIC, I.SHEAR, I.TENSILE, I.CORNER} <= modes


def test_mode_one_cohesive_law_and_fracture_energy():
    """Monotonic opening: T'n = sigma_p (1 - d^p_n / w_c) while weakening,
    zero once fully weakened, and the work of T'n on d^p_n is sigma_p w_c / 2."""
    sp, wc, kn = 1.0e6, 1.0e-3, 1.0e11
    m = _mat(kn=kn, c=3e6, st=sp, wc=wc)
    T, dp, chi = np.zeros(3), np.zeros(3), np.zeros(3)
    work, steps = 0.0, 4000
    for _ in range(steps):
        r = _upd(m, [0.0, 0.0, 1.5 * wc / steps], T, dp, chi)
        work += 0.5 * (T[2] + r["T"][2]) * (r["dp"][2] - dp[2])
        T, dp, chi = r["T"], r["dp"], r["chi"]
        if r["mode"] == I.TENSILE:
            assert T[2] == pytest.approx(sp * max(0.0, 1 - dp[2] / wc), rel=1e-12, abs=1e-6)
    assert T[2] == 0.0 and r["mode"] == I.OPEN
    assert work == pytest.approx(0.5 * sp * wc, rel=1e-3)


def test_slip_weakening_friction_and_energy():
    """Monotonic slip under a constant normal traction: |tau| =
    (f_r + (f_p - f_r) W(slip/d_c)) sigma_n, and the breakdown work is
    (f_p - f_r) sigma_n d_c / 2."""
    fp, fr, dc, sn, ks = 0.6, 0.35, 2e-3, -10e6, 1e11
    m = _mat(ks=ks, kn=1e11, fp=fp, fr=fr, dc=dc, c=0.0, st=0.0)
    T, dp, chi = np.array([0.0, 0.0, sn]), np.zeros(3), np.zeros(3)
    work, steps = 0.0, 4000
    for _ in range(steps):
        r = _upd(m, [1.6 * dc / steps, 0.0, 0.0], T, dp, chi)
        work += 0.5 * (T[0] + r["T"][0] + 2 * fr * sn) * (r["dp"][0] - dp[0])
        T, dp, chi = r["T"], r["dp"], r["chi"]
        if r["mode"] == I.SHEAR:
            f = fr + (fp - fr) * max(0.0, 1 - dp[0] / dc)
            assert T[0] == pytest.approx(-f * sn, rel=1e-12)
            assert T[2] == sn
    assert T[0] == pytest.approx(-fr * sn, rel=1e-12)
    assert work == pytest.approx(0.5 * (fp - fr) * (-sn) * dc, rel=1e-3)


def test_dilatant_opening_of_a_weakening_slip():
    """Monotonic slip past d_c: the dilatant inelastic opening is
    int psi = psi_p d_c / 2, it is added to the residual width, and the
    shear traction stays on the Coulomb line of the current normal traction."""
    fp, fr, psi, dc, sn = 0.6, 0.35, 0.2, 2e-3, -10e6
    m = _mat(ks=1e11, kn=1e11, fp=fp, fr=fr, psi=psi, dc=dc, c=0.0, st=0.0)
    T, dp, chi = np.array([0.0, 0.0, sn]), np.zeros(3), np.zeros(3)
    steps = 4000
    for _ in range(steps):
        r = _upd(m, [0.0, 1.5 * dc / steps, 0.0], T, dp, chi)
        T, dp, chi = r["T"], r["dp"], r["chi"]
        if r["mode"] == I.SHEAR:
            f = fr + (fp - fr) * max(0.0, 1 - chi[0] / dc)
            assert T[1] == pytest.approx(-f * T[2], rel=1e-12)
            assert T[2] == pytest.approx(sn - m[I.KN] * dp[2], rel=1e-12)
    assert dp[2] == pytest.approx(0.5 * psi * dc, rel=1e-3)
    assert chi[2] == pytest.approx(dp[2], rel=1e-12)


def test_open_fracture_stays_traction_free_until_the_gap_closes():
    """A pre-existing fracture (no strength, w_R = 0): opening carries no
    traction; closing carries none until the inelastic opening is used up,
    after which the overclosure is elastic."""
    kn, ks = 4e10, 2e10
    m = _mat(ks=ks, kn=kn, fp=0.6, fr=0.6, c=0.0, st=0.0, wc=0.0)
    r = _upd(m, [1e-4, 0.0, 3e-4], [0.0, 0.0, -2e6])
    assert r["mode"] == I.OPEN
    np.testing.assert_array_equal(r["T"], 0.0)
    np.testing.assert_array_equal(r["cep"], 0.0)
    gap = r["dp"][2]
    assert gap == pytest.approx(3e-4 - 2e6 / kn, rel=1e-14)
    r2 = _upd(m, [0.0, 0.0, -0.5 * gap], r["T"], r["dp"], r["chi"])
    assert r2["mode"] == I.OPEN and r2["dp"][2] == pytest.approx(0.5 * gap, rel=1e-13)
    r3 = _upd(m, [0.0, 0.0, -0.5 * gap - 1e-5], r2["T"], r2["dp"], r2["chi"])
    assert r3["mode"] == I.ELASTIC
    assert r3["T"][2] == pytest.approx(-kn * 1e-5, rel=1e-9)
    assert r3["dp"][2] == pytest.approx(0.0, abs=1e-18)


def test_damage_not_strength_decides_the_open_state():
    """An interface with cohesion but no tensile strength keeps its shear
    stiffness when it opens below full damage (tensile return, T'n = 0);
    once chi_t >= w_c it opens traction-free with zero tangent."""
    ks, kn, wc = 2e10, 4e10, 1e-3
    m = _mat(ks=ks, kn=kn, fp=0.6, fr=0.6, c=2e6, st=0.0, wc=wc)
    r = _upd(m, [1e-6, 0.0, 1e-4], [0.0, 0.0, -1e6])
    assert r["mode"] == I.TENSILE
    assert r["T"][2] == pytest.approx(0.0, abs=1e-6) and r["T"][0] == pytest.approx(ks * 1e-6, rel=1e-14)
    np.testing.assert_allclose(r["cep"], np.diag([ks, ks, 0.0]), atol=1e-6)
    r = _upd(m, [1e-6, 0.0, 1e-4], [0.0, 0.0, -1e6], dp0=[0, 0, 1.2 * wc], chi0=[0, 1.2 * wc, 0])
    assert r["mode"] == I.OPEN
    np.testing.assert_array_equal(r["T"], 0.0)


def test_vanishing_return_gives_the_continuum_tangent():
    """A trial just past the Coulomb surface: the consistent tangent tends to
    C - C N g^T C / (g^T C N) (the continuum elasto-plastic tangent)."""
    ks, kn, f, psi = 2e10, 3e10, 0.6, 0.1
    m = _mat(ks=ks, kn=kn, fp=f, fr=f, psi=psi, c=0.0, st=0.0)
    T0 = np.array([6e6 * (1 - 1e-9), 0.0, -10e6])
    r = _upd(m, [1e-12, 0.0, 0.0], T0)
    assert r["mode"] == I.SHEAR
    C = np.diag([ks, ks, kn])
    s, n = np.array([1.0, 0, 0]), np.array([0, 0, 1.0])
    N, g = s + psi * n, s + f * n
    cont = C - np.outer(C @ N, g @ C) / (g @ C @ N)
    np.testing.assert_allclose(r["cep"], cont, atol=1e-6 * ks)


def _random_state(rng, m, kind):
    if kind == 0:
        return np.array([*rng.normal(0, 3e6, 2), rng.uniform(-20e6, 0)]), np.zeros(3), np.array([0, 0, 0.3 * m[I.WC]])
    if kind == 1:
        return (np.array([*rng.normal(0, 0.2e6, 2), rng.uniform(-0.5e6, 0.8e6)]), np.zeros(3),
                np.array([0, 0, 0.3 * m[I.WC]]))
    dp0 = np.array([*rng.normal(0, 2e-4, 2), rng.uniform(0, 3e-4)])
    chi0 = np.array([np.hypot(*dp0[:2]) * rng.uniform(1, 1.5), np.linalg.norm(dp0) * rng.uniform(1, 1.3),
                     0.3 * m[I.WC]])
    return np.array([*rng.normal(0, 1e6, 2), rng.uniform(-5e6, 0.3e6)]), dp0, chi0


def test_consistent_tangent_matches_finite_differences():
    """Central differences of the whole algorithm (weakening, dilatancy,
    every mode) against the complex-step tangent."""
    mats = [I.material(3.2e10, 3.2e10, 0.6, 0.4, 0.1, 5e-3, 2e6, 1e6, 1e-3),
            I.material(1.0e10, 5.0e10, 0.7, 0.3, 0.2, 2e-3, 0.5e6, 0.4e6, 5e-4)]
    rng = np.random.default_rng(72)
    seen = set()
    for k in range(240):
        m = mats[k % 2]
        T0, dp0, chi0 = _random_state(rng, m, int(rng.integers(0, 3)))
        dd = rng.normal(0, 3e-4, 3) * rng.choice([0.01, 0.1, 1.0])
        r = I.update_element(m, dd, T0, dp0, chi0)
        seen.add(r["mode"])
        h = 1e-10
        fd = np.zeros((3, 3))
        for j in range(3):
            a, b = dd.copy(), dd.copy()
            a[j] += h
            b[j] -= h
            fd[:, j] = (I.update_element(m, a, T0, dp0, chi0)["T"] - I.update_element(m, b, T0, dp0, chi0)["T"]) / (2 * h)
        np.testing.assert_allclose(r["cep"], fd, atol=1e-4 * max(m[I.KS], m[I.KN]))
    assert {I.ELASTIC, I.SHEAR, I.TENSILE, I.CORNER} <= seen


def test_in_plane_rotation_invariance():
    m = I.material(3.2e10, 3.2e10, 0.6, 0.4, 0.1, 5e-3, 2e6, 1e6, 1e-3)
    rng = np.random.default_rng(73)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    for k in range(60):
        T0, dp0, chi0 = _random_state(rng, m, k % 3)
        dd = rng.normal(0, 2e-4, 3)
        a = I.update_element(m, dd, T0, dp0, chi0)
        b = I.update_element(m, R @ dd, R @ T0, R @ dp0, chi0)
        assert a["mode"] == b["mode"]
        np.testing.assert_allclose(b["T"], R @ a["T"], rtol=1e-11, atol=1e-4)
        np.testing.assert_allclose(b["dp"], R @ a["dp"], rtol=1e-10, atol=1e-16)
        np.testing.assert_allclose(b["cep"], R @ a["cep"] @ R.T, atol=1e-6 * m[I.KS])


def test_yield_consistency_and_flow_direction():
    m = I.material(3.2e10, 3.2e10, 0.6, 0.4, 0.1, 5e-3, 2e6, 1e6, 1e-3)
    rng = np.random.default_rng(74)
    for k in range(200):
        T0, dp0, chi0 = _random_state(rng, m, k % 3)
        dd = rng.normal(0, 3e-4, 3)
        r = I.update_element(m, dd, T0, dp0, chi0)
        T, chi = r["T"], r["chi"]
        fc = math.hypot(T[0], T[1]) + I.friction(m, chi[0]) * T[2] - I.cohesion(m, chi[1])
        ft = T[2] - I.tensile_strength(m, chi[1])
        tol = 1e-9 * 1e7
        assert fc <= tol and ft <= tol
        if r["mode"] == I.SHEAR:
            assert abs(fc) <= tol
            ddp = r["dp"] - dp0
            Ttr = T0 + np.array([m[I.KS], m[I.KS], m[I.KN]]) * dd
            s = Ttr[:2] / math.hypot(*Ttr[:2])
            lam = math.hypot(*ddp[:2])
            np.testing.assert_allclose(ddp[:2], lam * s, rtol=1e-9, atol=1e-18)
            assert ddp[2] == pytest.approx(lam * I.dilatancy(m, chi[0]), rel=1e-9, abs=1e-18)
        if r["mode"] in (I.TENSILE, I.CORNER):
            assert abs(ft) <= tol
        if r["mode"] == I.CORNER:
            assert abs(fc) <= tol
        assert chi[0] >= math.hypot(*r["dp"][:2]) * (1 - 1e-14)
        assert chi[1] >= np.linalg.norm(r["dp"]) * (1 - 1e-14)
