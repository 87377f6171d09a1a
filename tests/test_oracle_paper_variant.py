"""Pins of the oracle's paper-exact variant: forward Euler with the ramp of
eq. (beta) (Sec. 2.2, 3.1, 3.3) and the F_IRD costs of Sec. 3.1."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

N = 3.8e7


def test_ird_costs_hand_toy(orc):
    # I: range 20, errors (0, -5, 0)/20; R: range 5, errors (0, 0, -4)/5;
    # D: flat series, normalised by 1, errors (0, -0.5, 0)
    yI, hI = [10.0, 20.0, 30.0], [10.0, 25.0, 30.0]
    yR, hR = [0.0, 5.0, 5.0], [0.0, 5.0, 9.0]
    yD, hD = [1.0, 1.0, 1.0], [1.0, 1.5, 1.0]
    args = (hI, hR, hD, yI, yR, yD)
    assert orc.loss_ird("mxse", *args) == pytest.approx(0.64, rel=1e-14)
    assert orc.loss_ird("mse", *args) == pytest.approx(0.64 / 3, rel=1e-14)
    assert orc.loss_ird("mae", *args) == pytest.approx(0.8 / 3, rel=1e-14)
    # MAPE is not normalised: I 100/3*(5/20), R 100/3*(4/5), D 100/3*(0.5/1)
    assert orc.loss_ird("mape", *args) == pytest.approx(100 / 3 * 0.8, rel=1e-14)


def test_ird_is_invariant_to_shifting_a_series(orc):
    rng = np.random.default_rng(0)
    W = 20
    y = [np.cumsum(rng.uniform(0, 5, W + 1)) for _ in range(3)]
    h = [a + rng.normal(0, 1, W + 1) for a in y]
    for kind in ("mxse", "mse", "mae"):
        base = orc.loss_ird(kind, *h, *y)
        shifted = orc.loss_ird(kind, h[0] + 1e4, h[1], h[2], y[0] + 1e4, y[1], y[2])
        assert shifted == pytest.approx(base, rel=1e-9)


def _ramp_reference(theta, W, R0, D0):
    b1, b2, t1, t2, gamma, mu, I0 = theta

    def beta(t):
        if t < t1:
            return b1
        if t < t2:
            return b1 + (b2 - b1) / (t2 - t1) * (t - t1)
        return b2

    def f(t, z):
        S, I = z[0], z[1]
        inf = beta(t) / N * S * I
        return [-inf, inf - (gamma + mu) * I, gamma * I, mu * I]

    y0 = [N - I0 - R0 - D0, I0, R0, D0]
    sol = solve_ivp(f, (0, W), y0, method="DOP853", t_eval=np.arange(W + 1.0), rtol=1e-12,
                    atol=1e-10, max_step=0.05)
    return sol.y


def test_euler_ramp_converges_first_order(orc):
    theta = [0.35, 0.12, 6.0, 17.0, 0.1, 0.004, 3000.0]
    W = 30
    ref = _ramp_reference(theta, W, 200.0, 20.0)
    errs = []
    for spd in (20, 40, 80):
        prob = orc.Problem(W, spd, 1, 4, N, R0=200.0, D0=20.0, model=1)
        d = orc.integrate_model(prob, theta)
        errs.append(np.max(np.abs(d[1] - ref[1]) / ref[1]))
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3
    # S + I + R + D is conserved by Euler exactly up to rounding
    prob = orc.Problem(W, 1, 1, 4, N, R0=200.0, D0=20.0, model=1)
    d = orc.integrate_model(prob, theta)
    assert np.max(np.abs(d.sum(axis=0) - N)) < 1e-6


def test_model_zero_matches_plain_rk4(orc):
    prob = orc.Problem(25, 4, 7, 3, N, R0=5.0, D0=1.0)
    th = [0.3, 0.2, 0.1, 0.1, 0.003, 800.0]
    np.testing.assert_array_equal(orc.integrate_model(prob, th), orc.integrate(prob, th))
    y = orc.integrate(prob, th)[3] * 1.01
    assert orc.loss_batch_model(prob, np.array([th]), y, "ssre")[0] == \
        orc.loss_batch(prob, np.array([th]), y, "ssre")[0]


def test_swarm_keeps_ramp_times_ordered_and_fits(orc):
    W = 40
    R0, D0, I0 = 1e4, 300.0, 5e3
    prob = orc.Problem(W, 1, 1, 4, N, R0=R0, D0=D0, model=1)
    truth = np.array([0.3, 0.08, 8.0, 20.0, 0.1, 0.003, I0])
    tr = orc.integrate_model(prob, truth)
    obs = np.concatenate([tr[1], tr[2], tr[3]])
    lo = np.array([0, 0, 0, 0, 0, 0, I0])
    hi = np.array([2, 2, W - 7, W - 7, 1, 0.1, I0])
    hf, hidx, hm, s = orc.pso_run_model(prob, obs, "ird_mxse", 512, lo, hi, 0.5, 0.5, 0.5,
                                        1, 0, 60, nthreads=4)
    assert np.all(s.x[:, 2] <= s.x[:, 3]) and np.all(s.pbest_x[:, 2] <= s.pbest_x[:, 3])
    assert np.all(s.x >= lo) and np.all(s.x <= hi)
    assert np.all(np.diff(hf) <= 0) and hf[-1] < 0.7 * hf[0]
    assert orc.loss_batch_model(prob, truth[None, :], obs, "ird_mxse")[0] == 0.0


@pytest.mark.parametrize("spd", [1, 3])
def test_euler_without_transmission_is_the_discrete_geometric_decay(orc, spd):
    # beta1 = beta2 = 0: I_n = I0 (1 - lam h)^n exactly, R and D collect the
    # partial geometric sums, S stays put
    gamma, mu, I0, R0, D0, W = 0.13, 0.011, 2500.0, 40.0, 7.0, 30
    theta = [0.0, 0.0, 5.0, 20.0, gamma, mu, I0]
    prob = orc.Problem(W, spd, 1, 4, N, R0=R0, D0=D0, model=1)
    d = orc.integrate_model(prob, theta)
    lam, h = gamma + mu, 1.0 / spd
    n = np.arange(W + 1) * spd
    q = (1 - lam * h) ** n
    np.testing.assert_allclose(d[1], I0 * q, rtol=1e-13)
    np.testing.assert_allclose(d[2], R0 + gamma / lam * I0 * (1 - q), rtol=1e-13)
    np.testing.assert_allclose(d[3], D0 + mu / lam * I0 * (1 - q), rtol=1e-13)
    assert np.all(d[0] == N - I0 - R0 - D0)


def test_ramp_values_at_its_breakpoints(orc):
    b1, b2, t1, t2 = 0.4, 0.1, 5.0, 11.0
    assert orc.beta_ramp(0.0, b1, b2, t1, t2) == b1
    assert orc.beta_ramp(4.999, b1, b2, t1, t2) == b1
    assert orc.beta_ramp(t1, b1, b2, t1, t2) == b1
    assert orc.beta_ramp(8.0, b1, b2, t1, t2) == pytest.approx(0.25, rel=1e-15)
    assert orc.beta_ramp(t2, b1, b2, t1, t2) == b2
    assert orc.beta_ramp(100.0, b1, b2, t1, t2) == b2
    # a degenerate ramp is a step at t1
    assert orc.beta_ramp(6.0, b1, b2, 6.0, 6.0) == b2


def test_euler_ramp_one_step_by_hand(orc):
    # one day at one step per day: y1 = y0 + f(0, y0) with beta = beta1
    theta = [0.3, 0.1, 2.0, 4.0, 0.1, 0.01, 1000.0]
    prob = orc.Problem(1, 1, 1, 4, 1e6, R0=50.0, D0=5.0, model=1)
    d = orc.integrate_model(prob, theta)
    S0, I0 = 1e6 - 1000 - 50 - 5, 1000.0
    inf = 0.3 / 1e6 * S0 * I0
    assert d[0, 1] == pytest.approx(S0 - inf, rel=1e-15)
    assert d[1, 1] == pytest.approx(I0 + inf - 0.11 * I0, rel=1e-15)
    assert d[2, 1] == pytest.approx(50 + 0.1 * I0, rel=1e-15)
    assert d[3, 1] == pytest.approx(5 + 0.01 * I0, rel=1e-15)
