"""Seeded interface materials and states for the interface-law tests and
benchmark: parameter tables and random draws only (no part of the law).

Field order of a material row (shared with the C struct
hm_interface_material): k_s, k_n, f_peak, f_res, psi_peak, d_c, c_peak,
sigma_peak, w_c.  States are element-major float64 arrays [n, 3] in each
element's local frame (s1, s2, n): traction t, inelastic DD dp, internal
variables chi = (chi_s, chi_t, w_R), and the DD increment dd of the step.
"""
from __future__ import annotations

import numpy as np

MATERIAL_FIELDS = ("k_s", "k_n", "f_peak", "f_res", "psi_peak", "d_c", "c_peak", "sigma_peak", "w_c")


def interface_materials(young: float = 30e9, nu: float = 0.25, h: float = 1.0) -> np.ndarray:
    """Three interfaces with stiffness E'/h (E' = E / (1 - nu^2)):
    0 an intact rock joint on a new fracture path (cohesion 2 MPa, tensile
      strength 1 MPa weakening over 1 mm, friction 0.6 -> 0.4 over 5 mm,
      dilatancy 0.1);
    1 a pre-existing fault without strength (w_c = 0), constant friction 0.6;
    2 a weakening, dilatant fault (0.7 -> 0.3 over 2 mm, dilatancy 0.2,
      cohesion 0.5 MPa, tensile strength 0.4 MPa over 0.5 mm), shear
      stiffness a third of the normal one."""
    k = young / (1.0 - nu * nu) / h
    return np.array([
        [k, k, 0.6, 0.4, 0.1, 5e-3, 2.0e6, 1.0e6, 1e-3],
        [0.6 * k, k, 0.6, 0.6, 0.0, 0.0, 0.0, 0.0, 0.0],
        [k / 3.0, k, 0.7, 0.3, 0.2, 2e-3, 0.5e6, 0.4e6, 5e-4],
    ])


def interface_states(n: int, seed: int, mats: np.ndarray, mat_id: np.ndarray | None = None) -> dict:
    """n seeded element states covering every regime of the law: compressed
    and shear-loaded, near the tension cut-off, partly weakened, and fully
    damaged (open or in contact).  Increments are N(0, 0.3 mm) scaled by
    0.01, 0.1 or 1.  chi_s and chi_t are drawn at or above |dp_s| and |dp|
    (they are maxima over the history)."""
    rng = np.random.default_rng(seed)
    if mat_id is None:
        mat_id = rng.integers(0, mats.shape[0], n).astype(np.int32)
    kind = rng.integers(0, 4, n)
    wc = mats[mat_id, 8]
    t = np.zeros((n, 3))
    dp = np.zeros((n, 3))
    chi = np.zeros((n, 3))
    # compressed, shear-loaded
    k0 = kind == 0
    t[k0, :2] = rng.normal(0.0, 3e6, (k0.sum(), 2))
    t[k0, 2] = rng.uniform(-20e6, 0.0, k0.sum())
    chi[k0, 2] = 0.3 * wc[k0]
    # near the tension cut-off
    k1 = kind == 1
    t[k1, :2] = rng.normal(0.0, 0.2e6, (k1.sum(), 2))
    t[k1, 2] = rng.uniform(-0.5e6, 0.8e6, k1.sum())
    chi[k1, 2] = 0.3 * wc[k1]
    # partly weakened
    k2 = kind == 2
    m2 = int(k2.sum())
    dp[k2, :2] = rng.normal(0.0, 2e-4, (m2, 2))
    dp[k2, 2] = rng.uniform(0.0, 3e-4, m2)
    chi[k2, 0] = np.hypot(dp[k2, 0], dp[k2, 1]) * rng.uniform(1.0, 1.5, m2)
    chi[k2, 1] = np.linalg.norm(dp[k2], axis=1) * rng.uniform(1.0, 1.3, m2)
    chi[k2, 2] = 0.3 * wc[k2]
    t[k2, :2] = rng.normal(0.0, 1e6, (m2, 2))
    t[k2, 2] = rng.uniform(-5e6, 0.3e6, m2)
    # fully damaged: open (zero traction) or in contact
    k3 = kind == 3
    m3 = int(k3.sum())
    dp[k3, :2] = rng.normal(0.0, 1e-3, (m3, 2))
    dp[k3, 2] = rng.uniform(0.0, 2e-3, m3)
    chi[k3, 0] = np.hypot(dp[k3, 0], dp[k3, 1])
    chi[k3, 1] = np.maximum(np.linalg.norm(dp[k3], axis=1), 1.01 * wc[k3])
    chi[k3, 2] = rng.uniform(0.0, 1.0, m3) * dp[k3, 2]
    contact = rng.uniform(0.0, 1.0, m3) < 0.5
    tk = np.zeros((m3, 3))
    tk[contact, :2] = rng.normal(0.0, 1e6, (int(contact.sum()), 2))
    tk[contact, 2] = rng.uniform(-5e6, 0.0, int(contact.sum()))
    t[k3] = tk
    dd = rng.normal(0.0, 3e-4, (n, 3)) * rng.choice([0.01, 0.1, 1.0], n)[:, None]
    return dict(mat_id=np.ascontiguousarray(mat_id, dtype=np.int32), dd=dd, t=t, dp=dp, chi=chi)


def injection_path(mesh, n_states: int = 20, young: float = 30e9, nu: float = 0.25, rho: float = 2700.0,
                   injection=(20.0, 0.0, 0.0), rmax: float = 60.0, step_dd: float = 0.5e-3,
                   weakening_scale: float = 1.0, seed: int = 5001) -> dict:
    """Seeded loading path of an injection on a two-part mesh (first part the
    hydraulic fracture, the rest the fault), to drive the interface law.

    Materials (interface_materials with h = sqrt of the mean element area,
    weakening lengths d_c and w_c times weakening_scale, which keeps the
    local problems well posed on coarse test meshes whose stiffness E'/h is
    small): fracture elements intact joints (0), fault elements a
    pre-existing fault without strength (1).
    Initial effective tractions: fracture (0, 0, -5 MPa), fault (4, 0, -10)
    MPa; inelastic DD and chi_s, chi_t zero; residual width 0.3 w_c.  Step k
    reaches the elements within rmax sqrt((k + 1) / n_states) of the
    injection point; there the fracture opens by step_dd and the fault slips
    by step_dd along s1 (both times U(0.5, 1.5)) and closes by up to a tenth
    of it; elsewhere the increment is zero.  eta/dt_k: eta = (1/2) diag(G/cs,
    G/cs, G/cp) with the seeded time step of the synthetic tangent states
    (10^U(-1, 2) s from default_rng(seed + k))."""
    v = mesh.xyz[mesh.conn]
    if mesh.nvpe == 3:
        area = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
    else:
        area = np.linalg.norm(v[:, 1] - v[:, 0], axis=1) * np.linalg.norm(v[:, 3] - v[:, 0], axis=1)
    mats = interface_materials(young, nu, float(np.sqrt(area.mean())))
    mats[:, [5, 8]] *= weakening_scale
    ne = mesh.ne
    parts = mesh.meta.get("parts", [(0, ne)])
    first = np.zeros(ne, dtype=bool)
    first[parts[0][0]:parts[0][0] + parts[0][1]] = True
    mat_id = np.where(first, 0, 1).astype(np.int32)
    t0 = np.zeros((ne, 3))
    t0[first, 2] = -5e6
    t0[~first, 0] = 4e6
    t0[~first, 2] = -10e6
    chi0 = np.zeros((ne, 3))
    chi0[:, 2] = 0.3 * mats[mat_id, 8]
    G = young / (2.0 * (1.0 + nu))
    K = young / (3.0 * (1.0 - 2.0 * nu))
    cs, cp = np.sqrt(G / rho), np.sqrt((K + 4.0 * G / 3.0) / rho)
    eta = 0.5 * np.array([G / cs, G / cs, G / cp])
    dist = np.linalg.norm(mesh.vertex_means() - np.asarray(injection), axis=1)
    rng = np.random.default_rng(seed + 1000)
    dd, eta_dt = [], []
    for k in range(n_states):
        dt = 10.0 ** np.random.default_rng(seed + k).uniform(-1.0, 2.0)
        inside = dist <= rmax * np.sqrt((k + 1.0) / n_states)
        d = np.zeros((ne, 3))
        amp = step_dd * rng.uniform(0.5, 1.5, ne)
        d[inside & first, 2] = amp[inside & first]
        d[inside & ~first, 0] = amp[inside & ~first]
        d[inside & ~first, 2] = -0.1 * step_dd * rng.uniform(0.0, 1.0, int((inside & ~first).sum()))
        dd.append(d)
        eta_dt.append(np.tile(eta / dt, (ne, 1)))
    return dict(mats=mats, mat_id=mat_id, t=t0, dp=np.zeros((ne, 3)), chi=chi0, dd=dd, eta_dt=eta_dt)


def injection_pressure_time(mesh, t: float, duration: float = 20.0, peak: float = 8e6, sigma0: float = 6.0,
                            sigma1: float = 20.0, injection=(20.0, 0.0, 0.0)) -> np.ndarray:
    """Pore pressure above its initial value at the element vertex means at
    time t of a growing injection: amplitude peak t / duration, Gaussian of
    width sigma0 + (sigma1 - sigma0) t / duration (m) around the injection
    point; zero for t <= 0."""
    if t <= 0.0:
        return np.zeros(mesh.ne)
    f = t / duration
    r2 = ((mesh.vertex_means() - np.asarray(injection)) ** 2).sum(axis=1)
    s = sigma0 + (sigma1 - sigma0) * f
    return peak * f * np.exp(-r2 / (2.0 * s * s))


def injection_pressure(mesh, k: int, n_states: int = 20, **kw) -> np.ndarray:
    """The pressure of injection_pressure_time after step k of n_states unit
    steps (t = k + 1, duration n_states); k = -1 gives zero."""
    return injection_pressure_time(mesh, k + 1.0, float(n_states), **kw)
