"""CPU FP64 oracle of the fluid flow in the discontinuities and of the fully
coupled hydro-mechanical step (paper Sec. 3.2 "Fluid-flow in the
discontinuities" and Sec. 3.3 "A fully-coupled hydro-mechanical solver").

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the library.
It shares no code with the GPU path.

Galerkin P1 finite elements on the triangles of the mesh, pressure at the
vertices (nodes).  Per element e (area A_e, unit normal n_e, vertices
x_0, x_1, x_2, shape-function gradients grad N_a = n_e x (x_{a+2} - x_{a+1})
/ (2 A_e)):
  V_e[a]      = A_e / 3                      (volume of the normal DD, column 3e+2)
  S_e[a][b]   = (w_e / M) A_e (1 + [a = b]) / 12       (storage)
  L_e[a][b]   = (w_e k(w_e) / mu) A_e grad N_a . grad N_b   (transmissibility)
  N_p[3e+2][a] = 1 / 3                       (pressure at the collocation point)
with w_e = w0_e + delta_n,e the hydraulic width (delta_n the total normal
DD) and k(w) = w^2 / 12 (cubic law) or a constant k0.  A vertex that no
element uses carries a decoupled unit storage row (its pressure increment
stays zero).  Residuals of a
backward-Euler step with unknowns (dd, dp):
  r_m = dT'o - dT'(dd) + E dd + N_p dp - eta (dd - dd_prev) / dt
  r_f = V dd + (S + dt L)(dd) dp + dt L(dd) (p_n - p_o) - dt f
and the Jacobian is their exact derivative:
  A11 = E - eta/dt - C^ep, A12 = N_p,
  A21 = V + [dS/dd] dp + dt [dL/dd] (dp + p_n - p_o),   A22 = S + dt L.
(The paper prints A21 with dp alone; with p_n = p_o the two agree.)
The upper block-triangular preconditioner P_up = [[A11, A12], [0, S~]],
S~ = A22 - A21 diag(A11)^-1 A12, is applied by z2 = S~^-1 y2, then
A11 z1 = y1 - A12 z2.
"""
from __future__ import annotations

import numpy as np

from . import interface as law

PERM_CUBIC, PERM_CONSTANT = 0, 1


def geometry(mesh):
    """Per-element area [N], unit normal [N, 3] and P1 gradients [N, 3, 3]
    (gradient of the shape function of local vertex a in row a)."""
    if mesh.conn.shape[1] != 3:
        raise ValueError("the flow elements are triangles")
    x = mesh.xyz[mesh.conn]                      # [N, 3 vertices, 3]
    c = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    two_a = np.linalg.norm(c, axis=1)
    n = c / two_a[:, None]
    grads = np.empty_like(x)
    for a in range(3):
        edge = x[:, (a + 2) % 3] - x[:, (a + 1) % 3]
        grads[:, a] = np.cross(n, edge) / two_a[:, None]
    return 0.5 * two_a, n, grads


def coefficients(dn, w0, M, mu, perm_law=PERM_CUBIC, k0=0.0):
    """Per element: storage w/M, transmissibility w k(w)/mu and their
    derivatives with respect to the normal DD."""
    w = w0 + dn
    s, ds = w / M, np.full_like(w, 1.0 / M)
    if perm_law == PERM_CUBIC:
        t, dt_ = w ** 3 / (12.0 * mu), w ** 2 / (4.0 * mu)
    else:
        t, dt_ = w * k0 / mu, np.full_like(w, k0 / mu)
    return s, ds, t, dt_


def local_matrices(area, grads):
    """Unit-coefficient element mass [N, 3, 3] and stiffness [N, 3, 3]."""
    mass = area[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None] / 12.0
    stiff = area[:, None, None] * np.einsum("eak,ebk->eab", grads, grads)
    return mass, stiff


def assemble(mesh, coef):
    """Global V [n, 3N], S [n, n], L [n, n], N_p [3N, n] for per-element
    coefficients coef = (s, t) (storage, transmissibility)."""
    nn, ne = mesh.xyz.shape[0], mesh.conn.shape[0]
    area, _, grads = geometry(mesh)
    mass, stiff = local_matrices(area, grads)
    s, t = coef
    V = np.zeros((nn, 3 * ne))
    S = np.zeros((nn, nn))
    L = np.zeros((nn, nn))
    Np = np.zeros((3 * ne, nn))
    for e in range(ne):
        nodes = mesh.conn[e]
        V[nodes, 3 * e + 2] += area[e] / 3.0
        S[np.ix_(nodes, nodes)] += s[e] * mass[e]
        L[np.ix_(nodes, nodes)] += t[e] * stiff[e]
        Np[3 * e + 2, nodes] += 1.0 / 3.0
    # a vertex no element uses: a decoupled unit storage row
    unused = np.setdiff1d(np.arange(nn), mesh.conn.ravel())
    S[unused, unused] = 1.0
    return V, S, L, Np


def flow_residual(mesh, dd, dp, p_n, p_o, f, dt, total_dn_start, w0, M, mu, perm_law=PERM_CUBIC, k0=0.0):
    """r_f at the end-of-step normal DD (start value + increment)."""
    dn = total_dn_start + dd[:, 2]
    s, _, t, _ = coefficients(dn, w0, M, mu, perm_law, k0)
    V, S, L, _ = assemble(mesh, (s, t))
    return V @ dd.reshape(-1) + (S + dt * L) @ dp + dt * L @ (p_n - p_o) - dt * f


def coupled_residual(E, mesh, mech, flow, dd, dp):
    """(r_m [N, 3], r_f [n], interface state) at the unknowns (dd, dp).
    mech: dict(mats, mat_id, t_n, dp_n, chi_n, dT0, eta_dt, dd_prev);
    flow: dict(p_n, p_o, f, dt, dn_start, w0, M, mu, perm_law, k0)."""
    N = dd.shape[0]
    _, _, _, Np = assemble(mesh, (np.zeros(N), np.zeros(N)))
    dpress = (Np @ dp)[2::3]
    T, dpl, chi, cep, mode = law.update(mech["mats"], mech["mat_id"], dd, mech["t_n"], mech["dp_n"], mech["chi_n"])
    r_m = mech["dT0"] - (T - mech["t_n"]) + (E @ dd.reshape(-1)).reshape(N, 3)
    r_m[:, 2] += dpress
    r_m -= mech["eta_dt"] * (dd - mech["dd_prev"])
    r_f = flow_residual(mesh, dd, dp, flow["p_n"], flow["p_o"], flow["f"], flow["dt"], flow["dn_start"],
                        flow["w0"], flow["M"], flow["mu"], flow.get("perm_law", PERM_CUBIC), flow.get("k0", 0.0))
    return r_m, r_f, (T, dpl, chi, cep, mode)


def jacobian_blocks(E, mesh, mech, flow, dd, dp, cep):
    """Dense A11, A12, A21, A22 at (dd, dp) with the interface tangent cep."""
    N = dd.shape[0]
    dt = flow["dt"]
    A11 = E.copy()
    for e in range(N):
        A11[3 * e:3 * e + 3, 3 * e:3 * e + 3] -= cep[e] + np.diag(mech["eta_dt"][e])
    dn = flow["dn_start"] + dd[:, 2]
    s, ds, t, dtr = coefficients(dn, flow["w0"], flow["M"], flow["mu"], flow.get("perm_law", PERM_CUBIC),
                                 flow.get("k0", 0.0))
    V, S, L, Np = assemble(mesh, (s, t))
    area, _, grads = geometry(mesh)
    mass, stiff = local_matrices(area, grads)
    A21 = V.copy()
    q = dp + flow["p_n"] - flow["p_o"]
    for e in range(N):
        nodes = mesh.conn[e]
        A21[nodes, 3 * e + 2] += ds[e] * mass[e] @ dp[nodes] + dt * dtr[e] * stiff[e] @ q[nodes]
    return A11, Np, A21, S + dt * L


def schur_approx(A11, A12, A21, A22):
    """S~ = A22 - A21 diag(A11)^-1 A12."""
    return A22 - A21 @ (A12 / np.diag(A11)[:, None])


def p_up_apply(A11, A12, S_tilde, y1, y2):
    """z = P_up^-1 y with exact dense solves: z2 = S~^-1 y2, A11 z1 = y1 - A12 z2."""
    z2 = np.linalg.solve(S_tilde, y2)
    z1 = np.linalg.solve(A11, y1 - A12 @ z2)
    return z1, z2


def coupled_newton_step(E, mesh, mech, flow, scales, dd0=None, dp0=None, max_newton=25, rtol=1e-12):
    """Newton on (dd, dp) with the exact Jacobian and dense LU.  The history
    holds sqrt(||r_m / scales[0]||^2 + ||r_f / scales[1]||^2) (a traction
    scale in Pa and a volume scale in m^3); stop at rtol times the first.
    Returns (dd, dp, interface state, history)."""
    N, nn = E.shape[0] // 3, mesh.xyz.shape[0]
    dd = np.zeros((N, 3)) if dd0 is None else np.array(dd0, dtype=np.float64)
    dp = np.zeros(nn) if dp0 is None else np.array(dp0, dtype=np.float64)
    hist = []
    sm, sf = 1.0 / scales[0], 1.0 / scales[1]
    for k in range(max_newton + 1):
        r_m, r_f, state = coupled_residual(E, mesh, mech, flow, dd, dp)
        hist.append(float(np.sqrt(np.sum((sm * r_m) ** 2) + np.sum((sf * r_f) ** 2))))
        if hist[-1] <= rtol * hist[0] or k == max_newton:
            break
        A11, A12, A21, A22 = jacobian_blocks(E, mesh, mech, flow, dd, dp, state[3])
        J = np.block([[A11, A12], [A21, A22]])
        step = np.linalg.solve(J, -np.concatenate([r_m.reshape(-1), r_f]))
        dd = dd + step[:3 * N].reshape(N, 3)
        dp = dp + step[3 * N:]
    return dd, dp, state, hist
