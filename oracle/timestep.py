"""CPU FP64 oracle of the adaptive time stepping of the mechanical problem.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the library.
It shares no code with the library's step-size controller or its GPU
truncation-error reduction.

Paper Sec. 3.4.  The implicit step solves for the increment dd over a step
of length dt, so dd / dt is the rate at the end of the step.  The local
truncation error is estimated from the change of that rate between two
consecutive steps, half a step times the rate difference, measured
relative to the current total displacement discontinuity d:

    e_{n+1} = (dt_n / 2) || dd_n / dt_n - dd_{n-1} / dt_{n-1} || / || d ||.

The next step size is the current one times four factors: the ratio of
the last two step sizes to the power -1/4, the ratio of the tolerance to
the new error to the power 1/4, the ratio of the previous error to the
tolerance to the power -1/4, and the ratio of the last step's Newton
iterations to a target count to the power -1/3.  The square root of the
FP64 unit roundoff is added to every error estimate (it keeps e_{n+1}
away from zero), the step may grow by at most a factor M, and it is kept
inside [dt_min, dt_max].  With no previous step (the first step) the
step-ratio and previous-error factors are left out.
"""
from __future__ import annotations

import numpy as np

FLOOR = float(np.sqrt(np.finfo(np.float64).eps))


def truncation_error(dd, dt, dd_prev, dt_prev, total) -> float:
    """e_{n+1} of a step; dd_prev None: no previous rate (taken as zero)."""
    dd = np.asarray(dd, dtype=np.float64).ravel()
    rate_prev = 0.0 if dd_prev is None else np.asarray(dd_prev, dtype=np.float64).ravel() / dt_prev
    return 0.5 * dt * float(np.linalg.norm(dd / dt - rate_prev)) / float(np.linalg.norm(np.ravel(total)))


def next_step(dt_n, dt_prev, e_next, e_n, n_its, eps_tol=1e-3, n_target=6, growth_max=1.2, dt_min=0.0,
              dt_max=np.inf) -> float:
    """Delta t_{n+1}; dt_prev <= 0 and e_n <= 0 mean "no previous step"."""
    dt = dt_n
    if dt_prev > 0.0:
        dt *= (dt_n / dt_prev) ** -0.25
    dt *= (eps_tol / (max(e_next, 0.0) + FLOOR)) ** 0.25
    if e_n > 0.0:
        dt *= ((e_n + FLOOR) / eps_tol) ** -0.25
    dt *= (n_its / n_target) ** (-1.0 / 3.0)
    dt = min(dt, growth_max * dt_n)
    return min(max(dt, dt_min), dt_max)


def scale_update(L_old, L_new, alpha=0.62, rho_min=0.84, rho_max=1.16):
    """Scaling of unknowns and residuals (paper Sec. 3.3.2): smooth the new
    scale with the old one, L = alpha L_old + (1 - alpha) L_new, then keep
    its ratio to the old one within [rho_min, rho_max].  (The paper names
    the upper bound rho_min a second time; read as rho_max.)"""
    smooth = alpha * L_old + (1.0 - alpha) * L_new
    return L_old * min(max(smooth / L_old, rho_min), rho_max)
