"""Pins of the flow and coupled-step oracle (oracle/flow.py, paper Sec. 3.2
and Sec. 3.3) against what the mathematics fixes:
  * P1 gradients: they sum to zero and reproduce in-plane linear fields;
  * storage integrates a constant (1^T S 1 = sum of (w/M) A) and is
    symmetric positive definite; transmissibility annihilates constants, is
    symmetric positive semi-definite, and passes the patch test (a linear
    pressure gives zero flux at interior nodes of a jittered mesh);
  * V's columns integrate the normal DD over each element; N_p averages;
  * pressure diffusion along a strip: the backward-Euler P1 solution of the
    cos(pi x / L) mode converges to exp(-(k M / mu) (pi / L)^2 t) under
    refinement (constant permeability, width and storage);
  * the coupled Jacobian equals central finite differences of the coupled
    residual (cubic law: the width derivatives of S and L included);
  * Newton on the coupled step converges quadratically and, at the
    solution, conserves the fluid volume: the volume change of the
    fractures plus the stored volume equals the injected volume.
"""
import numpy as np
import pytest

import oracle
from oracle import flow as OF
from oracle import interface as law
import workloads as W

YOUNG, NU = 30e9, 0.25
EP = YOUNG / (1 - NU * NU)


def _jittered(nx=6, ny=5, seed=1):
    m = W.rect_tri_mesh(6.0, 5.0, nx, ny)
    rng = np.random.default_rng(seed)
    inner = np.all(np.abs(m.xyz[:, :2]) < np.array([2.999, 2.499]), axis=1)
    m.xyz[inner, :2] += rng.uniform(-0.2, 0.2, (inner.sum(), 2))
    return m, inner


def test_gradients_sum_to_zero_and_reproduce_linear_fields():
    m, _ = _jittered()
    area, n, g = OF.geometry(m)
    assert np.abs(g.sum(axis=1)).max() < 1e-12
    c = np.array([0.7, -1.3, 0.0])
    vals = m.xyz[m.conn] @ c                         # [N, 3]
    grad = np.einsum("ea,eak->ek", vals, g)
    assert np.abs(grad - c[None, :]).max() < 1e-12
    assert np.allclose(area.sum(), 30.0) and np.allclose(np.abs(n[:, 2]), 1.0)


def test_storage_and_transmissibility_properties_and_patch_test():
    m, inner = _jittered()
    rng = np.random.default_rng(2)
    s = rng.uniform(1e-12, 3e-12, m.ne)
    t = np.full(m.ne, 4e-9)
    V, S, L, Np = OF.assemble(m, (s, t))
    area, _, _ = OF.geometry(m)
    one = np.ones(m.nv)
    assert one @ S @ one == pytest.approx(np.sum(s * area), rel=1e-13)
    assert np.allclose(S, S.T, rtol=0, atol=1e-28) and np.linalg.eigvalsh(S).min() > 0
    assert np.abs(L @ one).max() <= 1e-12 * np.abs(L).max()
    assert np.allclose(L, L.T, rtol=0, atol=1e-24) and np.linalg.eigvalsh(L).min() > -1e-12 * np.abs(L).max()
    p = m.xyz @ np.array([2.0e6, -0.5e6, 0.0])
    flux = L @ p
    assert np.abs(flux[inner]).max() <= 1e-10 * np.abs(flux).max()
    assert np.abs(flux[~inner]).max() > 1e-3 * np.abs(L).max() * 1e6
    assert np.allclose(V.reshape(m.nv, m.ne, 3)[:, :, 2].sum(axis=0), area, rtol=1e-14)
    assert np.abs(V.reshape(m.nv, m.ne, 3)[:, :, :2]).max() == 0.0
    assert np.allclose(Np[2::3].sum(axis=1), 1.0) and np.abs(Np[0::3]).max() == 0.0


def test_strip_diffusion_converges_to_the_decaying_cosine():
    # a strip of length Lx: with zero-flux ends the mode cos(pi x / Lx) decays
    # at rate D (pi / Lx)^2, D = (w k / mu) / (w / M) = k M / mu
    Lx, Ly = 10.0, 1.0
    k0, M, mu, w = 1e-12, 1e9, 1e-3, 1e-3
    D = k0 * M / mu
    T = 0.1 * Lx ** 2 / (D * np.pi ** 2)
    errs = []
    for nx, steps in ((10, 10), (20, 40), (40, 160)):
        m = W.rect_tri_mesh(Lx, Ly, nx, 2)
        s, _, t, _ = OF.coefficients(np.zeros(m.ne), np.full(m.ne, w), M, mu, OF.PERM_CONSTANT, k0)
        _, S, L, _ = OF.assemble(m, (s, t))
        dt = T / steps
        p = np.cos(np.pi * (m.xyz[:, 0] + Lx / 2) / Lx)
        A = S + dt * L
        for _ in range(steps):
            p = np.linalg.solve(A, S @ p)
        exact = np.exp(-D * (np.pi / Lx) ** 2 * T) * np.cos(np.pi * (m.xyz[:, 0] + Lx / 2) / Lx)
        errs.append(np.abs(p - exact).max() / np.abs(exact).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 5e-3, errs


def _coupled_case(n=4, seed=3):
    m = W.rect_tri_mesh(4.0, 4.0, n, n)
    N, nn = m.ne, m.nv
    E = oracle.dense(m, YOUNG, NU)
    h = np.sqrt(16.0 / N * 2)
    mats = law.material(EP / h, EP / h, 0.6, 0.6, 0.0, float("inf"), 1e12, 1e11, float("inf"))[None]
    rng = np.random.default_rng(seed)
    mech = dict(mats=mats, mat_id=np.zeros(N, np.int32), t_n=np.tile([0.0, 0.0, -5e6], (N, 1)),
                dp_n=np.zeros((N, 3)), chi_n=np.zeros((N, 3)), dT0=np.zeros((N, 3)),
                eta_dt=np.full((N, 3), 1e8), dd_prev=np.zeros((N, 3)))
    f = np.zeros(nn)
    f[np.argmin(np.sum(m.xyz ** 2, axis=1))] = 1e-4            # injection at the centre node (m^3/s)
    flow = dict(p_n=np.full(nn, 1e6), p_o=np.zeros(nn), f=f, dt=0.5, dn_start=rng.uniform(0, 1e-4, N),
                w0=np.full(N, 1e-4), M=1e9, mu=1e-3, perm_law=OF.PERM_CUBIC)
    return m, E, mech, flow


def test_coupled_jacobian_equals_finite_differences():
    m, E, mech, flow = _coupled_case()
    N, nn = m.ne, m.nv
    rng = np.random.default_rng(4)
    dd = rng.normal(0, 2e-5, (N, 3))
    dp = rng.normal(0, 3e5, nn)
    r_m, r_f, st = OF.coupled_residual(E, m, mech, flow, dd, dp)
    A11, A12, A21, A22 = OF.jacobian_blocks(E, m, mech, flow, dd, dp, st[3])
    J = np.block([[A11, A12], [A21, A22]])
    x0 = np.concatenate([dd.reshape(-1), dp])
    scale = np.concatenate([np.full(3 * N, 1e-7), np.full(nn, 1e2)])
    Jfd = np.empty_like(J)
    for j in range(x0.size):
        xp, xm = x0.copy(), x0.copy()
        xp[j] += scale[j]
        xm[j] -= scale[j]
        rp = OF.coupled_residual(E, m, mech, flow, xp[:3 * N].reshape(N, 3), xp[3 * N:])
        rn = OF.coupled_residual(E, m, mech, flow, xm[:3 * N].reshape(N, 3), xm[3 * N:])
        Jfd[:, j] = (np.concatenate([rp[0].reshape(-1), rp[1]]) - np.concatenate([rn[0].reshape(-1), rn[1]])) / (2 * scale[j])
    for rows, cols in ((slice(0, 3 * N), slice(0, 3 * N)), (slice(0, 3 * N), slice(3 * N, None)),
                       (slice(3 * N, None), slice(0, 3 * N)), (slice(3 * N, None), slice(3 * N, None))):
        blk, fd = J[rows, cols], Jfd[rows, cols]
        assert np.abs(blk - fd).max() <= 1e-6 * np.abs(fd).max() + 1e-300
    # the width derivatives matter: dropping them from A21 fails the check
    V, _, _, _ = OF.assemble(m, (np.zeros(N), np.zeros(N)))
    assert np.abs(V - Jfd[3 * N:, :3 * N]).max() > 1e-3 * np.abs(Jfd[3 * N:, :3 * N]).max()


def test_coupled_newton_converges_and_conserves_fluid_volume():
    m, E, mech, flow = _coupled_case()
    injected = flow["dt"] * flow["f"].sum()
    dd, dp, st, hist = OF.coupled_newton_step(E, m, mech, flow, (1e6, injected), rtol=1e-13)
    assert hist[-1] <= 1e-13 * hist[0] and len(hist) <= 8
    # quadratic: each contraction factor at most a constant times the previous residual
    rel = np.array(hist) / hist[0]
    assert rel[2] <= 10 * rel[1] ** 2 and rel[3] <= max(10 * rel[2] ** 2, 1e-14)
    dn_new = flow["dn_start"] + dd[:, 2]
    s_new, _, t_new, _ = OF.coefficients(dn_new, flow["w0"], flow["M"], flow["mu"])
    V, S, L, _ = OF.assemble(m, (s_new, t_new))
    area, _, _ = OF.geometry(m)
    one = np.ones(m.nv)
    balance = np.sum(area * dd[:, 2]) + one @ S @ dp
    assert balance == pytest.approx(injected, rel=1e-9)
    assert np.sum(area * dd[:, 2]) > 0      # the injection opens the fracture
