"""CPU FP64 oracle of one implicit step of the mechanical problem.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the library.
It shares no code with the GPU path: the dense collocation matrix of the
oracle, its interface law (oracle.interface) and dense LU.

The mechanical residual of a step (paper Sec. 3.1.1, "Elasto-plastic
solver"), with the increment of the total DD as unknown:

    r(dd) = dT'o - dT'(dd) + E dd + I_n dp - eta (dd - dd_prev) / dt,

dT'o the increment of the in-situ effective traction, dT'(dd) the increment
of the interface effective traction given by the interface law from the
state at the start of the step, I_n dp the pore-pressure increment at the
collocation points acting along each element normal, eta/dt the
quasi-dynamic term and dd_prev the previous step's increment rescaled to
this step (times dt / dt_prev), so that eta (dd - dd_prev) / dt is eta
times the backward-Euler change of rate.  Newton's
method with the mechanical Jacobian J = E - eta/dt - C^ep:

    dd <- dd - J^-1 r(dd),

until ||r|| <= rtol ||r_0|| (2-norms over all elements).  Vectors are
element-major [N, 3] in local frames (s1, s2, n).
"""
from __future__ import annotations

import numpy as np

from . import interface as law


def residual(E, mats, mat_id, dd, t_n, dp_n, chi_n, dT0, dpress=None, eta_dt=None, dd_prev=None):
    """r(dd) and the interface law's outputs (T, dp, chi, cep, mode) at dd."""
    N = dd.shape[0]
    T, dp, chi, cep, mode = law.update(mats, mat_id, dd, t_n, dp_n, chi_n)
    r = dT0 - (T - t_n) + (E @ dd.reshape(-1)).reshape(N, 3)
    if dpress is not None:
        r[:, 2] += dpress
    if eta_dt is not None:
        r -= eta_dt * (dd - (dd_prev if dd_prev is not None else 0.0))
    return r, (T, dp, chi, cep, mode)


def newton_step(E, mats, mat_id, t_n, dp_n, chi_n, dT0, dpress=None, eta_dt=None, dd_prev=None, dd0=None,
                max_newton=25, rtol=1e-12):
    """Newton iteration of one step.  Returns (dd, state, history) with state =
    (T, dp, chi, cep, mode) at the returned dd and history the residual
    2-norms, one per residual evaluation."""
    N = t_n.shape[0]
    dd = np.zeros((N, 3)) if dd0 is None else np.array(dd0, dtype=np.float64)
    hist = []
    for k in range(max_newton + 1):
        r, state = residual(E, mats, mat_id, dd, t_n, dp_n, chi_n, dT0, dpress, eta_dt, dd_prev)
        hist.append(float(np.linalg.norm(r)))
        if hist[-1] <= rtol * hist[0] or k == max_newton:
            break
        D = state[3].copy()
        if eta_dt is not None:
            D[:, [0, 1, 2], [0, 1, 2]] += eta_dt
        J = E.copy()
        for i in range(N):
            J[3 * i:3 * i + 3, 3 * i:3 * i + 3] -= D[i]
        dd = dd - np.linalg.solve(J, r.reshape(-1)).reshape(N, 3)
    return dd, state, hist
