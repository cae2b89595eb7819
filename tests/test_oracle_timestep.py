"""Pins of the time-stepping oracle (CPU only; paper Sec. 3.4).

The truncation-error estimate is pinned by trajectories whose rates are
known in closed form: along a linear path the rate does not change (zero
estimate); along a quadratic path X(t) = a t^2 + b the increments' rates
differ by a (dt_n + dt_{n-1}), so with equal steps the estimate is the
second-order Taylor term (dt^2 / 2) |X''| relative to |X|.  The controller
is pinned by its fixed point and the exponent of each factor.  The
library's host-side controller is then compared with the oracle's.
"""
import numpy as np
import pytest

from oracle import timestep as ts


def _increments(X, times):
    return [X(times[i + 1]) - X(times[i]) for i in range(len(times) - 1)]


def test_linear_path_has_zero_estimate():
    X = lambda t: np.array([3.0, -1.0, 0.5]) * t + 2.0
    times = [0.0, 0.4, 1.0, 1.25]
    inc = _increments(X, times)
    for k in (1, 2):
        e = ts.truncation_error(inc[k], times[k + 1] - times[k], inc[k - 1], times[k] - times[k - 1], X(times[k + 1]))
        assert abs(e) < 1e-15


@pytest.mark.parametrize("steps", [(0.5, 0.5), (0.3, 0.7), (1.1, 0.2)])
def test_quadratic_path_estimate_is_the_taylor_term(steps):
    a, b = np.array([2.0, -0.5, 1.5]), np.array([1.0, 4.0, -2.0])
    X = lambda t: a * t * t + b
    dt_prev, dt = steps
    t0 = 0.8
    times = [t0, t0 + dt_prev, t0 + dt_prev + dt]
    prev, cur = _increments(X, times)
    e = ts.truncation_error(cur, dt, prev, dt_prev, X(times[-1]))
    # rates a (2 t - dt): their change over the two steps is a (dt + dt_prev)
    assert e == pytest.approx(0.5 * dt * np.linalg.norm(a * (dt + dt_prev)) / np.linalg.norm(X(times[-1])), rel=1e-13)
    if dt == dt_prev:
        assert e == pytest.approx(0.5 * dt * dt * np.linalg.norm(2 * a) / np.linalg.norm(X(times[-1])), rel=1e-13)


def test_first_step_estimate_uses_a_zero_previous_rate():
    dd, tot = np.array([1.0, 2.0, 2.0]), np.array([0.0, 0.0, 6.0])
    assert ts.truncation_error(dd, 0.5, None, 0.0, tot) == pytest.approx(0.5 * 3.0 / 6.0)


def test_controller_fixed_point_and_exponents():
    eps = 1e-3
    nxt = lambda *a, **k: ts.next_step(*a, eps_tol=eps, n_target=6, growth_max=10.0, **k)
    e_fix = eps - ts.FLOOR                # the estimate plus the floor equals the tolerance
    e_half = 0.5 * eps - ts.FLOOR
    assert nxt(2.0, 2.0, e_fix, e_fix, 6) == pytest.approx(2.0, rel=1e-14)
    assert nxt(2.0, 2.0, e_half, e_fix, 6) == pytest.approx(2.0 * 2 ** 0.25, rel=1e-13)   # new error halved
    assert nxt(2.0, 2.0, e_fix, e_half, 6) == pytest.approx(2.0 * 2 ** 0.25, rel=1e-13)   # previous error halved
    assert nxt(2.0, 1.0, e_fix, e_fix, 6) == pytest.approx(2.0 * 2 ** -0.25, rel=1e-13)   # step just doubled
    assert nxt(2.0, 2.0, e_fix, e_fix, 12) == pytest.approx(2.0 * 2 ** (-1 / 3), rel=1e-13)  # twice the iterations
    assert nxt(2.0, 0.0, e_fix, 0.0, 6) == pytest.approx(2.0, rel=1e-14)                   # first step
    assert ts.next_step(1.0, 1.0, 0.0, 0.0, 1, eps_tol=eps, growth_max=1.2) == pytest.approx(1.2)
    assert ts.next_step(1.0, 1.0, 10.0, 0.0, 50, dt_min=0.5) == 0.5
    assert ts.next_step(1.0, 1.0, 0.0, 0.0, 1, growth_max=100.0, dt_max=3.0) == 3.0


def test_library_controller_matches_the_oracle():
    """Host logic: hm_timestep_next against the oracle on seeded inputs
    spanning first steps, growth caps and both bounds."""
    hm = pytest.importorskip("paper_2605_14397_amd")
    rng = np.random.default_rng(3401)
    for _ in range(300):
        dt_n = 10 ** rng.uniform(-3, 1)
        dt_prev = 0.0 if rng.random() < 0.2 else 10 ** rng.uniform(-3, 1)
        e_next, e_n = 10 ** rng.uniform(-6, 0), (0.0 if rng.random() < 0.2 else 10 ** rng.uniform(-6, 0))
        n_its = int(rng.integers(1, 20))
        kw = dict(eps_tol=10 ** rng.uniform(-4, -1), n_target=int(rng.integers(2, 10)),
                  growth_max=float(rng.uniform(1.05, 2.0)), dt_min=1e-3, dt_max=5.0)
        assert hm.timestep_next(dt_n, dt_prev, e_next, e_n, n_its, **kw) == pytest.approx(
            ts.next_step(dt_n, dt_prev, e_next, e_n, n_its, **kw), rel=1e-13)


def test_scale_update_fixed_point_clipping_and_smoothing():
    """The scale update of Sec. 3.3.2: an unchanged scale stays, the ratio
    to the old scale never leaves [rho_min, rho_max], and inside the clips it
    is the alpha-weighted mean."""
    from oracle.timestep import scale_update

    assert scale_update(3.0, 3.0) == 3.0
    assert scale_update(1.0, 100.0) == pytest.approx(1.16)
    assert scale_update(1.0, 0.0) == pytest.approx(0.84)
    assert scale_update(2.0, 2.2, alpha=0.62) == pytest.approx(0.62 * 2.0 + 0.38 * 2.2)
    assert scale_update(2.0, 2.2, alpha=1.0) == 2.0
