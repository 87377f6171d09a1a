"""Pins of the oracle's integrator against mathematics that does not come from
the oracle itself.

eq. (SIRD) of Sec. 2.2 has linear invariants, exact discrete solutions of RK4
in special cases, a first integral, and a continuous solution that an
independent library integrator (scipy's DOP853) approximates to 1e-13.  A
dropped term, a wrong sign, a transposed stage weight or a wrong segment
index breaks at least one of the checks below.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

N = 3.8e7


def poly4(x):
    """Stability polynomial of classical RK4, R(z) = sum_{k<=4} z^k/k!."""
    return 1 + x + x * x / 2 + x ** 3 / 6 + x ** 4 / 24


def test_conservation_random(orc):
    rng = np.random.default_rng(11)
    for _ in range(20):
        K = int(rng.integers(1, 6))
        prob = orc.Problem(W=int(rng.integers(5, 80)), spd=int(rng.integers(1, 12)),
                           seg_days=int(rng.integers(1, 20)), K=K, N=N,
                           R0=float(rng.uniform(0, 1e4)), D0=float(rng.uniform(0, 1e3)))
        th = np.concatenate([rng.uniform(0, 1, K), [rng.uniform(0, .5), rng.uniform(0, .05),
                                                    rng.uniform(1e2, 1e5)]])
        days = orc.integrate(prob, th)
        total = days.sum(axis=0)
        assert np.max(np.abs(total - N)) <= 64 * np.finfo(float).eps * N


@pytest.mark.parametrize("spd", [1, 4, 10, 20])
def test_beta_zero_exact_discrete(orc, spd):
    # beta = 0: I' = -lam I is linear, so RK4 multiplies I by R(-lam h) each
    # step exactly; D and R follow from the invariants lam D - mu (I0 - I) ...
    gamma, mu, I0, R0, D0, W = 0.13, 0.007, 2500.0, 40.0, 3.0, 50
    lam = gamma + mu
    prob = orc.Problem(W=W, spd=spd, seg_days=7, K=3, N=N, R0=R0, D0=D0)
    days, steps = orc.integrate(prob, [0.0, 0.0, 0.0, gamma, mu, I0], steps=True)
    n = np.arange(prob.T + 1)
    h = 1.0 / spd
    I_exact = I0 * poly4(-lam * h) ** n
    np.testing.assert_allclose(steps[1], I_exact, rtol=2e-13)
    np.testing.assert_allclose(steps[3], D0 + mu / lam * (I0 - I_exact), rtol=2e-13)
    np.testing.assert_allclose(steps[2], R0 + gamma / lam * (I0 - I_exact), rtol=2e-13)
    assert np.all(steps[0] == N - I0 - R0 - D0)
    # and it approximates the continuous exponential decay to O(h^4)
    t = n * h
    cont = I0 * np.exp(-lam * t)
    assert np.max(np.abs(steps[1] - cont) / cont) < 1e-3 * h ** 4 * 60 + 1e-14


def test_logistic_special_case(orc):
    # gamma = mu = 0, R0 = D0 = 0: S + I = N, I' = beta I (N - I)/N
    beta, I0, W = 0.3, 1000.0, 60
    errs = []
    for spd in (5, 10, 20):
        prob = orc.Problem(W=W, spd=spd, seg_days=W, K=1, N=N)
        days = orc.integrate(prob, [beta, 0.0, 0.0, I0])
        t = np.arange(W + 1.0)
        e = np.exp(beta * t)
        exact = N * I0 * e / (N - I0 + I0 * e)
        errs.append(np.max(np.abs(days[1] - exact) / exact))
    assert errs[-1] < 1e-8
    # fourth order: halving h divides the error by ~16
    assert 12 < errs[0] / errs[1] < 20
    assert 12 < errs[1] / errs[2] < 20


def test_first_integral_constant_beta(orc):
    # constant beta: dS/d(R+D) = -beta S/(N lam), so
    # S = S0 exp(-beta (R + D - R0 - D0)/(N lam)) along the exact solution
    beta, gamma, mu, I0, R0, D0 = 0.35, 0.1, 0.004, 5e3, 1e4, 2e2
    lam = gamma + mu
    prob = orc.Problem(W=200, spd=20, seg_days=14, K=1, N=N, R0=R0, D0=D0)
    days = orc.integrate(prob, [beta, gamma, mu, I0])
    S0 = N - I0 - R0 - D0
    S_pred = S0 * np.exp(-beta * (days[2] + days[3] - R0 - D0) / (N * lam))
    assert np.max(np.abs(days[0] - S_pred) / days[0]) < 1e-9
    # the epidemic really moved: S fell by more than a third
    assert days[0][-1] < 0.66 * S0


def _scipy_reference(theta, W, seg_days, K, R0, D0):
    """Continuous solution of eq. (SIRD) by DOP853, restarted at every
    beta-segment boundary; returns S, I, R, D at every day."""
    beta = theta[:K]
    gamma, mu, I0 = theta[K:]
    y = np.array([N - I0 - R0 - D0, I0, R0, D0])
    out = np.zeros((4, W + 1))
    out[:, 0] = y
    bounds = [k * seg_days for k in range(K)] + [W]
    bounds = [min(b, W) for b in bounds]
    for k in range(K):
        a, b = bounds[k], bounds[k + 1] if k < K - 1 else W
        if b <= a:
            continue
        bk = beta[k]

        def f(t, z, bk=bk):
            S, I = z[0], z[1]
            inf = bk / N * S * I
            return [-inf, inf - (gamma + mu) * I, gamma * I, mu * I]

        teval = np.arange(a, b + 1, dtype=float)
        sol = solve_ivp(f, (a, b), y, method="DOP853", t_eval=teval, rtol=1e-13,
                        atol=1e-16 * N)
        out[:, a:b + 1] = sol.y
        y = sol.y[:, -1]
    return out


def test_against_scipy_piecewise_and_order(orc):
    rng = np.random.default_rng(5)
    K, seg = 5, 14
    W = 70
    theta = np.concatenate([rng.uniform(0.05, 0.4, K), [0.1, 0.002, 1000.0]])
    ref = _scipy_reference(theta, W, seg, K, 0.0, 0.0)
    errs = []
    for spd in (5, 10, 20, 40):
        prob = orc.Problem(W=W, spd=spd, seg_days=seg, K=K, N=N)
        days = orc.integrate(prob, theta)
        rel = np.abs(days[1:] - ref[1:]) / np.maximum(np.abs(ref[1:]), 1e-300)
        errs.append(np.max(rel[:, 1:]))
    # spd = 10 (dt = 0.1 day) is already within 1e-6 of the continuous solution
    assert errs[1] < 1e-6
    for a, b in zip(errs, errs[1:]):
        assert 13 < a / b < 19, errs


def test_segment_index_uses_step_boundary(orc):
    # beta switches exactly at day seg_days: integrating K=2 over W days must
    # equal integrating the first seg_days with beta1 and restarting with beta2
    seg, W, spd = 6, 15, 10
    th = [0.5, 0.05, 0.12, 0.003, 4000.0]
    full = orc.integrate(orc.Problem(W=W, spd=spd, seg_days=seg, K=2, N=N), th)
    first = orc.integrate(orc.Problem(W=seg, spd=spd, seg_days=seg, K=1, N=N),
                          [0.5, 0.12, 0.003, 4000.0])
    np.testing.assert_array_equal(full[:, :seg + 1], first)
    S, I, R, D = first[:, -1]
    second = orc.integrate(orc.Problem(W=W - seg, spd=spd, seg_days=W, K=1, N=N, R0=R, D0=D),
                           [0.05, 0.12, 0.003, I])
    # restarted run rebuilds S = N - I - R - D, so agreement is to rounding
    np.testing.assert_allclose(full[:, seg:], second, rtol=1e-13, atol=1e-9)


def test_last_segment_extends_to_window_end(orc):
    # K segments cover K*seg days; later days keep beta_K
    th = [0.2, 0.3, 0.1, 0.002, 1000.0]
    a = orc.integrate(orc.Problem(W=40, spd=5, seg_days=7, K=2, N=N), th)
    b = orc.integrate(orc.Problem(W=40, spd=5, seg_days=7, K=3, N=N),
                      [0.2, 0.3, 0.3, 0.1, 0.002, 1000.0])
    np.testing.assert_array_equal(a, b)


def test_euler_beta_zero_exact_and_ramp(orc):
    gamma, mu, I0, spd, W = 0.1, 0.01, 1e4, 4, 30
    lam = gamma + mu
    y0 = [N - I0, I0, 0.0, 0.0]
    days = orc.integrate_euler_ramp(W, spd, [0, 0, 3, 9, gamma, mu], y0, N)
    i = np.arange(W + 1)
    np.testing.assert_allclose(days[1], I0 * (1 - lam / spd) ** (i * spd), rtol=1e-13)
    # the ramp of eq. (beta) at hand-picked points
    assert orc.beta_ramp(0.0, 0.4, 0.1, 5, 15) == 0.4
    assert orc.beta_ramp(4.999, 0.4, 0.1, 5, 15) == 0.4
    assert orc.beta_ramp(10.0, 0.4, 0.1, 5, 15) == pytest.approx(0.25, rel=1e-15)
    assert orc.beta_ramp(15.0, 0.4, 0.1, 5, 15) == 0.1
    assert orc.beta_ramp(100.0, 0.4, 0.1, 5, 15) == 0.1
    # Euler is first order: error vs the scipy solution halves with h
    errs = []
    for s in (10, 20, 40):
        d = orc.integrate_euler_ramp(W, s, [0.3, 0.3, 0, 0, gamma, mu], y0, N)
        ref = _scipy_reference(np.array([0.3, gamma, mu, I0]), W, W, 1, 0.0, 0.0)
        errs.append(np.max(np.abs(d[1] - ref[1]) / ref[1]))
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2
