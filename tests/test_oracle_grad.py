"""Pins of the oracle's forward-mode gradient of the discrete loss and of its
projected Adam step.

The gradient is checked against (a) a closed form: with beta = 0 the RK4
solution is I_n = I0 R(-lam h)^n exactly, so dD/dgamma, dD/dmu and dD/dI0
are explicit; (b) Richardson-extrapolated central differences of the
oracle's own loss, which share no code with the tangent recursion; and (c)
the complex step (Squire & Trapp 1998): the discrete RK4 loss evaluated
here in complex arithmetic with theta_j + i 1e-30, whose imaginary part
over 1e-30 is the derivative to rounding, with no cancellation.
"""
import numpy as np
import pytest

N = 3.8e7


def R(x):
    return 1 + x + x * x / 2 + x ** 3 / 6 + x ** 4 / 24


def dR(x):
    return 1 + x + x * x / 2 + x ** 3 / 6


def test_beta_zero_closed_form_gradient(orc):
    W, spd, K = 40, 10, 2
    gamma, mu, I0, D0 = 0.12, 0.004, 3000.0, 5.0
    lam, h = gamma + mu, 1.0 / spd
    prob = orc.Problem(W=W, spd=spd, seg_days=20, K=K, N=N, D0=D0)
    rng = np.random.default_rng(2)
    y = D0 + np.cumsum(rng.uniform(0, 5, W + 1))
    y[0] = D0
    L, g = orc.loss_grad_fwd(prob, [0.0, 0.0, gamma, mu, I0], y, "mse")
    n = np.arange(W + 1) * spd
    x = -lam * h
    P = R(x) ** n
    D = D0 + mu / lam * I0 * (1 - P)
    dP_dlam = n * R(x) ** (n - 1) * dR(x) * (-h)
    dD_dgamma = I0 * (-mu / lam ** 2 * (1 - P) - mu / lam * dP_dlam)
    dD_dmu = I0 * ((1 / lam - mu / lam ** 2) * (1 - P) - mu / lam * dP_dlam)
    dD_dI0 = mu / lam * (1 - P)
    e = y - D
    dL_dD = -2 * e / (W + 1)
    assert L == pytest.approx(np.mean(e ** 2), rel=1e-12)
    assert g[K] == pytest.approx(np.sum(dL_dD * dD_dgamma), rel=1e-10)
    assert g[K + 1] == pytest.approx(np.sum(dL_dD * dD_dmu), rel=1e-10)
    assert g[K + 2] == pytest.approx(np.sum(dL_dD * dD_dI0), rel=1e-10)


def fd_richardson(f, x, j, h):
    def cd(hh):
        xp, xm = x.copy(), x.copy()
        xp[j] += hh
        xm[j] -= hh
        return (f(xp) - f(xm)) / (2 * hh)
    return (4 * cd(h / 2) - cd(h)) / 3


@pytest.mark.parametrize("kind", ["ssre", "mse", "mae", "mape", "mxse"])
def test_forward_mode_matches_finite_differences(orc, kind):
    K, W, spd = 4, 50, 10
    prob = orc.Problem(W=W, spd=spd, seg_days=14, K=K, N=N, R0=50.0, D0=2.0)
    truth = orc.integrate(prob, [0.3, 0.22, 0.15, 0.12, 0.1, 0.003, 2000.0])[3]
    rng = np.random.default_rng(9)
    y = truth * (1 + rng.normal(0, 0.05, W + 1))
    y[0] = 2.0
    th = np.array([0.27, 0.24, 0.13, 0.14, 0.11, 0.0028, 1800.0])
    L, g = orc.loss_grad_fwd(prob, th, y, kind)

    def f(t):
        return orc.loss(kind, orc.integrate(prob, t)[3], y)

    assert L == f(th)
    for j in range(prob.d):
        h = 1e-4 * abs(th[j])
        fd = fd_richardson(f, th, j, h)
        assert g[j] == pytest.approx(fd, rel=2e-6, abs=1e-9 * np.max(np.abs(g))), (kind, j)


def test_gradient_zero_at_noise_free_truth(orc):
    prob = orc.Problem(W=60, spd=10, seg_days=60, K=1, N=N)
    th = [0.25, 0.1, 0.002, 1000.0]
    y = orc.integrate(prob, th)[3]
    L, g = orc.loss_grad_fwd(prob, th, y, "ssre")
    assert L == 0.0 and np.all(g == 0.0)


def test_adam_first_step_and_projection(orc):
    lo = np.array([0.0, 0.0, 5.0])
    hi = np.array([1.0, 2.0, 5.0])
    th = np.array([[0.5, 1.0, 5.0], [0.0005, 1.0, 5.0]])
    grad = np.array([[2.0, -3.0, 7.0], [1.0, 0.0, 1.0]])
    m, v = np.zeros_like(th), np.zeros_like(th)
    orc.adam_step(th, grad, m, v, lo, hi, t=1, lr=1e-3)
    # first step: mhat = g_u, vhat = g_u^2, so u moves by -lr g_u/(|g_u| + eps)
    gu = 2.0 * 1.0
    assert th[0, 0] == pytest.approx(0.5 - 1e-3 * gu / (abs(gu) + 1e-8), rel=1e-14)
    gu = -3.0 * 2.0
    assert th[0, 1] == pytest.approx(2.0 * (0.5 + 1e-3 * 6.0 / (6.0 + 1e-8)), rel=1e-14)
    assert th[0, 2] == 5.0 and th[1, 2] == 5.0          # fixed dimension untouched
    assert th[1, 0] == 0.0                               # projected onto the box
    assert th[1, 1] == 1.0                               # zero gradient: no move


def test_adam_descends_a_quadratic(orc):
    lo, hi = np.zeros(3), np.ones(3)
    a = np.array([0.2, 0.7, 0.4])
    th = np.array([[0.9, 0.1, 0.5]])
    m, v = np.zeros_like(th), np.zeros_like(th)
    for t in range(1, 3001):
        orc.adam_step(th, 2 * (th - a), m, v, lo, hi, t, lr=1e-2)
    np.testing.assert_allclose(th[0], a, atol=1e-3)


def rk4_loss_complex(theta, W, spd, seg_days, K, N_, R0, D0, y, kind):
    """The discrete loss in complex arithmetic, one column per direction:
    theta is (d, m) complex.  Classical RK4 on (S, I, R, D) with f =
    (-b S I, b S I - (gamma + mu) I, gamma I, mu I), b = beta_k / N, the
    segment of step n min(n // (seg_days spd), K - 1) for all four stages,
    h = 1/spd; Dhat_i = D after i spd steps."""
    beta, gamma, mu, I0 = theta[:K], theta[K], theta[K + 1], theta[K + 2]
    h = 1.0 / spd
    S = N_ - I0 - R0 - D0
    I = I0 + 0j
    Rr = np.zeros_like(I) + R0
    D = np.zeros_like(I) + D0

    def f(S, I, b):
        p = b * S * I
        return -p, p - (gamma + mu) * I, gamma * I, mu * I

    Dhat = [D]
    for n in range(W * spd):
        b = beta[min(n // (seg_days * spd), K - 1)] / N_
        k1 = f(S, I, b)
        k2 = f(S + h / 2 * k1[0], I + h / 2 * k1[1], b)
        k3 = f(S + h / 2 * k2[0], I + h / 2 * k2[1], b)
        k4 = f(S + h * k3[0], I + h * k3[1], b)
        S, I, Rr, D = [v + h / 6 * (a + 2 * bb + 2 * c + e) for v, a, bb, c, e in
                       zip((S, I, Rr, D), k1, k2, k3, k4)]
        if (n + 1) % spd == 0:
            Dhat.append(D)
    Dhat = np.array(Dhat)  # (W+1, m)
    yy = np.asarray(y)[:, None]
    if kind == "ssre":
        r = (Dhat[1:] - yy[1:]) / np.maximum(yy[1:], 1.0)
        return np.sum(r * r, axis=0)
    e = yy - Dhat
    return np.sum(e * e, axis=0) / (W + 1)


@pytest.mark.parametrize("kind", ["ssre", "mse"])
def test_forward_mode_matches_complex_step(orc, kind):
    K, W, spd, seg = 5, 45, 4, 10
    R0, D0 = 30.0, 4.0
    prob = orc.Problem(W=W, spd=spd, seg_days=seg, K=K, N=N, R0=R0, D0=D0)
    truth = orc.integrate(prob, [0.3, 0.25, 0.2, 0.15, 0.12, 0.1, 0.004, 2500.0])[3]
    rng = np.random.default_rng(12)
    y = truth * (1 + rng.normal(0, 0.05, W + 1))
    y[0] = D0
    th = np.array([0.28, 0.26, 0.18, 0.16, 0.13, 0.11, 0.0035, 2200.0])
    d = th.size
    hc = 1e-30
    cols = np.tile(th[:, None], (1, d)).astype(np.complex128)
    cols[np.arange(d), np.arange(d)] += 1j * hc
    cs = np.imag(rk4_loss_complex(cols, W, spd, seg, K, N, R0, D0, y, kind)) / hc
    L0 = np.real(rk4_loss_complex(th[:, None].astype(np.complex128), W, spd, seg, K, N, R0,
                                  D0, y, kind))[0]
    L, g = orc.loss_grad_fwd(prob, th, y, kind)
    assert L == pytest.approx(L0, rel=1e-12)
    np.testing.assert_allclose(g, cs, rtol=1e-9, atol=1e-12 * np.max(np.abs(cs)))
