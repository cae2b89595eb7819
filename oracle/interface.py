"""CPU FP64 oracle of the interface elasto-plastic law and its consistent tangent.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
CPU-baseline leg, never by the library.  It shares no code with the GPU
path: plain Python per element, scipy's bracketing root finder for the
scalar consistency equations, complex-step partial derivatives.

The law (paper Sec. 2.2.2-2.2.3), in each element's local frame (s1, s2, n),
tension and opening positive:
  * T' - T'o = C (d - d^p), C = diag(Ks, Ks, Kn), constant stiffnesses;
  * Coulomb surface Fc = |tau| + f(chi_s) T'n - c(chi_t) with the
    non-associated flow d(d^p) = dlam (s_hat + psi(chi_s) n);
  * tension cut-off Ft = T'n - sigma_t(chi_t) with associated flow along n;
  * linear weakening W(x) = max(0, 1 - x): f = f_r + (f_p - f_r) W(chi_s/d_c),
    psi = psi_p W(chi_s/d_c), c = c_p W(chi_t/w_c), sigma_t = sigma_p W(chi_t/w_c);
    a zero critical distance means the residual value from the start;
  * chi_s = max over time of |d^p_s|, chi_t = max over time of |d^p|;
  * the mode selector h = |tau| - (c - f sigma_t) - alpha (T'n - sigma_t),
    alpha = sqrt(1 + f^2) - f: h > 0 selects Coulomb failure, else tension;
  * a fully damaged interface (damage min(chi_t / w_c, 1) = 1; w_c = 0 for
    a pre-existing fracture) that opens carries zero effective traction
    (both stiffnesses vanish); it closes back into contact once its inelastic
    opening has returned to the residual width w_R, which grows with the
    dilatant part psi dlam of shear flow; its initial value (the paper's
    alpha w_c for an intact interface, 0 for a pre-existing fracture) is
    part of the initial state.

Integration over a step (backward Euler, elastic predictor - plastic
corrector): given the increment dd of the total DD and the state at the
start of the step (T'n, d^p, chi = (chi_s, chi_t, w_R)), return the state at
the end and the consistent tangent C^ep = d T' / d dd (Sec. 3.1.1, the
mechanical Jacobian J = E - eta/dt - C^ep).  The steps, in order:

  1. trial T_tr = T'n + C dd;
  2. fully damaged at the start: gap g = max(0, d^p_n - w_R); if
     T_tr,n + Kn g >= 0 the element is OPEN (T' = 0, C^ep = 0, all of the
     increment inelastic); otherwise the gap closes first (d^p_n -= g,
     T_tr,n += Kn g);
  3. Fc and Ft at the trial state and chi at the start: both <= 0 gives
     ELASTIC (C^ep = C) (every surface test here and below allows 1e-12 of
     the trial traction scale, so that ties created by the algorithm itself
     are not decided by rounding);
  4. h at the trial selects SHEAR or TENSILE;
  5. SHEAR: solve Fc(T'(lam), chi(lam)) = 0 for lam in [0, |tau_tr|/Ks],
     T'(lam) = T_tr - lam C (s_hat + psi n), s_hat = tau_tr/|tau_tr|, with
     f, psi, c at the end-of-step chi; if no root lies in the bracket or
     the result violates the cut-off, go to CORNER;
  6. TENSILE: solve Ft = 0 for mu in [0, T_tr,n/Kn], T'n = T_tr,n - Kn mu,
     tau unchanged; if the result violates Coulomb, go to CORNER;
  7. CORNER: both surfaces active; unknowns lam (shear slip) and nu (total
     normal inelastic DD): Ft(nu; lam) = 0 is solved inside, for nu in
     [0, T_tr,n/Kn] (nu = 0 when the cut-off is not reached at lam), and
     Fc(lam) = 0 outside, for lam in [0, |tau_tr|/Ks] (lam = 0 when
     Coulomb holds at lam = 0).

The local problems are taken to be well posed: every stiffness exceeds the
softening rate of the strength it controls, so each scalar consistency
function decreases across its bracket and has one root there.

The tangent is the derivative of this algorithm: with unknowns y solving
R(dd, y) = 0 and end-of-step traction T(dd, y),
C^ep = dT/ddd - dT/dy (dR/dy)^-1 dR/ddd (implicit function theorem), every
partial derivative taken by the complex-step method (Squire & Trapp 1998)
on the explicit functions R and T.  Pins: central finite differences of the
whole algorithm, closed forms of the non-softening returns, the elastic
stiffness, and path checks (tests/test_oracle_interface.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

# material record fields
KS, KN, FP, FR, PSIP, DC, CP, SP, WC = range(9)
N_MAT_FIELDS = 9

ELASTIC, SHEAR, TENSILE, CORNER, OPEN = 0, 1, 2, 3, 4
MODE_NAMES = {ELASTIC: "elastic", SHEAR: "shear", TENSILE: "tensile", CORNER: "corner", OPEN: "open"}

_H = 1e-30  # complex step


def material(ks, kn, f_peak, f_res, psi_peak, d_c, c_peak, sigma_peak, w_c):
    """Material record as a float array (field order KS ... WC); an infinite
    critical distance means no weakening."""
    return np.array([ks, kn, f_peak, f_res, psi_peak, d_c, c_peak, sigma_peak, w_c], dtype=np.float64)


# ------------------------------------------------------------------ weakening laws

def _w(x, L):
    """Linear weakening W(x/L) = max(0, 1 - x/L); a zero length means fully weakened."""
    if L <= 0.0:
        return 0.0 * x
    r = 1.0 - x / L
    return r if r.real > 0.0 else 0.0 * x


def friction(m, chi_s):
    return m[FR] + (m[FP] - m[FR]) * _w(chi_s, m[DC])


def dilatancy(m, chi_s):
    return m[PSIP] * _w(chi_s, m[DC])


def cohesion(m, chi_t):
    return m[CP] * _w(chi_t, m[WC])


def tensile_strength(m, chi_t):
    return m[SP] * _w(chi_t, m[WC])


def _norm(*xs):
    return (sum(x * x for x in xs)) ** 0.5


def _grow(old, new):
    """Running maximum of a magnitude (the new value wins only when strictly larger)."""
    return new if new.real > old else old + 0.0 * new


# ------------------------------------------------------------------ explicit maps

def _end_state(m, Ttr, dp0, chi0, lam, nu, dilatant):
    """End-of-step traction, inelastic DD and internal variables for given
    multipliers.  lam: shear slip along s_hat; the normal inelastic DD
    increment is lam * psi(chi_s) when `dilatant` (Coulomb flow alone), else nu.
    Returns (T[3], dp[3], chi[3], |tau|)."""
    q = _norm(Ttr[0], Ttr[1])
    if lam == 0.0 and getattr(lam, "imag", 0.0) == 0.0:
        ps1, ps2 = dp0[0] + 0.0 * q, dp0[1] + 0.0 * q
        t1, t2, tau = Ttr[0], Ttr[1], q
    else:
        s1, s2 = Ttr[0] / q, Ttr[1] / q
        ps1, ps2 = dp0[0] + lam * s1, dp0[1] + lam * s2
        tau = q - m[KS] * lam
        t1, t2 = tau * s1, tau * s2
    chi_s = _grow(chi0[0], _norm(ps1, ps2))
    psi = dilatancy(m, chi_s)
    dn = lam * psi if dilatant else nu
    pn = dp0[2] + dn
    chi_t = _grow(chi0[1], _norm(ps1, ps2, pn))
    w_r = chi0[2] + lam * psi
    Tn = Ttr[2] - m[KN] * dn
    return [t1, t2, Tn], [ps1, ps2, pn], [chi_s, chi_t, w_r], tau


def _fc(m, tau, Tn, chi):
    return tau + friction(m, chi[0]) * Tn - cohesion(m, chi[1])


def _ft(m, Tn, chi):
    return Tn - tensile_strength(m, chi[1])


def _trial(m, dd, T0, dp0, chi0):
    """Steps 1-2: trial traction, gap closure, OPEN detection.
    Returns (open, Ttr, dp_start)."""
    Ttr = [T0[0] + m[KS] * dd[0], T0[1] + m[KS] * dd[1], T0[2] + m[KN] * dd[2]]
    dps = list(dp0)
    if _w(chi0[1], m[WC]) == 0.0:  # damage min(chi_t / w_c, 1) = 1
        g = max(0.0, dp0[2] - chi0[2])
        if (Ttr[2] + m[KN] * g).real >= 0.0:
            return True, Ttr, dps
        Ttr[2] = Ttr[2] + m[KN] * g
        dps[2] = dp0[2] - g
    return False, Ttr, dps


# ------------------------------------------------------------------ one element

def yield_tolerance(m, Ttr):
    """Tolerance of every surface test: 1e-12 of the trial traction scale.
    States that the algorithm puts exactly on a surface (a return that ends
    at zero strength, an element left on its surface with no increment)
    would otherwise be decided by the sign of a rounding error."""
    return 1e-12 * (abs(Ttr[0]) + abs(Ttr[1]) + abs(Ttr[2]) + m[CP] + m[SP])


def _root(fun, hi, tol):
    """Root of a function decreasing on [0, hi] (0 if fun(0) <= tol, hi if fun(hi) >= -tol)."""
    if hi <= 0.0 or fun(0.0) <= tol:
        return 0.0
    if fun(hi) >= -tol:
        return hi
    return brentq(fun, 0.0, hi, xtol=1e-300, rtol=8.9e-16, maxiter=400)


def _corner(m, Ttr, dps, chi0, tol):
    """Nested scalar solves of the corner: returns (lam, nu)."""
    q = math.hypot(Ttr[0], Ttr[1])
    nu_hi = max(Ttr[2], 0.0) / m[KN]

    def nu_of(lam):
        def r1(nu):
            T, _, chi, _ = _end_state(m, Ttr, dps, chi0, lam, nu, False)
            return _ft(m, T[2], chi)
        return _root(r1, nu_hi, tol)

    def r2(lam):
        nu = nu_of(lam)
        T, _, chi, tau = _end_state(m, Ttr, dps, chi0, lam, nu, False)
        return _fc(m, tau, T[2], chi)

    lam = _root(r2, q / m[KS], tol)
    return lam, nu_of(lam)


def update_element(m, dd, T0, dp0, chi0):
    """Integrate one element over one step.

    m: material record; dd[3]: increment of the total DD; T0[3], dp0[3]:
    effective traction and inelastic DD at the start; chi0[3] = (chi_s,
    chi_t, w_R) at the start.  Returns dict(T, dp, chi, cep[3,3], mode)."""
    dd = [float(v) for v in dd]
    T0 = [float(v) for v in T0]
    dp0 = [float(v) for v in dp0]
    chi0 = [float(v) for v in chi0]
    is_open, Ttr, dps = _trial(m, dd, T0, dp0, chi0)
    if is_open:
        dp = [dp0[0] + Ttr[0] / m[KS], dp0[1] + Ttr[1] / m[KS], dp0[2] + Ttr[2] / m[KN]]
        chi_s = max(chi0[0], math.hypot(dp[0], dp[1]))
        chi_t = max(chi0[1], math.sqrt(dp[0] ** 2 + dp[1] ** 2 + dp[2] ** 2))
        return dict(T=np.zeros(3), dp=np.array(dp), chi=np.array([chi_s, chi_t, chi0[2]]),
                    cep=np.zeros((3, 3)), mode=OPEN)
    q = math.hypot(Ttr[0], Ttr[1])
    lam, nu = 0.0, 0.0
    ytol = yield_tolerance(m, Ttr)
    if _fc(m, q, Ttr[2], chi0) <= ytol and _ft(m, Ttr[2], chi0) <= ytol:
        mode = ELASTIC
    else:
        f0, c0, st0 = friction(m, chi0[0]), cohesion(m, chi0[1]), tensile_strength(m, chi0[1])
        alpha = math.sqrt(1.0 + f0 * f0) - f0
        h = q - (c0 - f0 * st0) - alpha * (Ttr[2] - st0)
        mode = SHEAR if h > 0.0 else TENSILE
        if mode == SHEAR:
            def rs(x):
                T, _, chi, tau = _end_state(m, Ttr, dps, chi0, x, 0.0, True)
                return _fc(m, tau, T[2], chi)
            lam_hi = q / m[KS]
            if rs(lam_hi) > ytol:
                mode = CORNER
            else:
                lam = _root(rs, lam_hi, ytol)
                T, _, chi, _ = _end_state(m, Ttr, dps, chi0, lam, 0.0, True)
                if _ft(m, T[2], chi) > ytol:
                    mode, lam = CORNER, 0.0
        if mode == TENSILE:
            def rt(x):
                T, _, chi, _ = _end_state(m, Ttr, dps, chi0, 0.0, x, False)
                return _ft(m, T[2], chi)
            nu = _root(rt, Ttr[2] / m[KN], ytol)
            T, _, chi, tau = _end_state(m, Ttr, dps, chi0, 0.0, nu, False)
            if _fc(m, tau, T[2], chi) > ytol:
                mode, nu = CORNER, 0.0
        if mode == CORNER:
            lam, nu = _corner(m, Ttr, dps, chi0, ytol)
    unknowns = active_unknowns(m, Ttr, dps, chi0, mode, lam, nu)
    T, dp, chi, _ = _end_state(m, Ttr, dps, chi0, lam, nu, mode == SHEAR)
    cep = tangent(m, dd, T0, dp0, chi0, mode, lam, nu, unknowns)
    return dict(T=np.array([float(v) for v in T]), dp=np.array([float(v) for v in dp]),
                chi=np.array([float(v) for v in chi]), cep=cep, mode=mode)


def active_unknowns(m, Ttr, dps, chi0, mode, lam, nu):
    """Multipliers that solve a consistency equation (as opposed to sitting
    at the lower end 0 of their bracket, where they are constants)."""
    if mode == SHEAR:
        return ("lam",) if lam > 0.0 else ()
    if mode == TENSILE:
        return ("nu",) if nu > 0.0 else ()
    if mode == CORNER:
        return tuple(u for u, v in (("lam", lam), ("nu", nu)) if v > 0.0)
    return ()


# ------------------------------------------------------------------ consistent tangent

def _residuals(m, dd, T0, dp0, chi0, mode, lam, nu, unknowns):
    """Explicit end-of-step traction and the residuals of the active unknowns."""
    _, Ttr, dps = _trial(m, dd, T0, dp0, chi0)
    T, _, chi, tau = _end_state(m, Ttr, dps, chi0, lam, nu, mode == SHEAR)
    R = [_fc(m, tau, T[2], chi) if u == "lam" else _ft(m, T[2], chi) for u in unknowns]
    return T, R


def tangent(m, dd, T0, dp0, chi0, mode, lam, nu, unknowns):
    """C^ep = dT/ddd - dT/dy (dR/dy)^-1 dR/ddd, partials by complex step."""
    if mode == OPEN:
        return np.zeros((3, 3))
    k = len(unknowns)
    dT_dd = np.zeros((3, 3))
    dR_dd = np.zeros((k, 3))
    for j in range(3):
        ddc = [complex(v) for v in dd]
        ddc[j] += 1j * _H
        T, R = _residuals(m, ddc, T0, dp0, chi0, mode, complex(lam), complex(nu), unknowns)
        dT_dd[:, j] = [t.imag / _H for t in T]
        dR_dd[:, j] = [r.imag / _H for r in R]
    if k == 0:
        return dT_dd
    dT_dy = np.zeros((3, k))
    dR_dy = np.zeros((k, k))
    for a, u in enumerate(unknowns):
        lam_c = complex(lam) + (1j * _H if u == "lam" else 0.0)
        nu_c = complex(nu) + (1j * _H if u == "nu" else 0.0)
        T, R = _residuals(m, [complex(v) for v in dd], T0, dp0, chi0, mode, lam_c, nu_c, unknowns)
        dT_dy[:, a] = [t.imag / _H for t in T]
        dR_dy[:, a] = [r.imag / _H for r in R]
    return dT_dd - dT_dy @ np.linalg.solve(dR_dy, dR_dd)


# ------------------------------------------------------------------ arrays

def update(mats, mat_id, dd, T0, dp0, chi0):
    """Element loop over arrays: mats [n_mat, 10], mat_id [N] (or None),
    dd/T0/dp0/chi0 [N, 3].  Returns (T, dp, chi, cep [N,3,3], mode [N])."""
    N = dd.shape[0]
    T = np.zeros((N, 3))
    dp = np.zeros((N, 3))
    chi = np.zeros((N, 3))
    cep = np.zeros((N, 3, 3))
    mode = np.zeros(N, dtype=np.int32)
    for e in range(N):
        m = mats[0 if mat_id is None else int(mat_id[e])]
        r = update_element(m, dd[e], T0[e], dp0[e], chi0[e])
        T[e], dp[e], chi[e], cep[e], mode[e] = r["T"], r["dp"], r["chi"], r["cep"], r["mode"]
    return T, dp, chi, cep, mode
