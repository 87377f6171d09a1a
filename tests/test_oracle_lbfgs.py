"""Pins of the oracle's projected L-BFGS: exact convergence on quadratics
(interior and bound-constrained minimisers), Rosenbrock's valley, and
recovery of the noise-free constant-beta truth with forward-mode gradients;
with several trial steps per round, the trials' geometry and the selection
among them checked by brute force."""
import numpy as np

import synth


def drive(orc, fg, theta0, lo, hi, rounds, m=8, n_trials=1, until=None):
    """rounds rounds (or, with until, the rounds until f <= until: returns
    (state, rounds used))."""
    st = orc.Lbfgs(np.atleast_2d(theta0), m=m, n_trials=n_trials)
    for q in range(st.theta.shape[0]):
        st.f[q], st.grad[q] = fg(st.theta[q])
    for r in range(1, rounds + 1):
        st.propose(lo, hi)
        for i in range(st.theta_t.shape[0]):
            st.f_t[i], st.grad_t[i] = fg(st.theta_t[i])
        st.accept(lo, hi)
        if until is not None and st.f.min() <= until:
            return st, r
    return (st, None) if until is not None else st


def test_quadratic_interior_minimum(orc):
    rng = np.random.default_rng(0)
    d = 8
    M = rng.normal(size=(d, d))
    A = M @ M.T + 0.05 * np.eye(d)   # condition number ~1e3
    lo, hi = np.full(d, -1.0), np.full(d, 3.0)
    c = rng.uniform(0.1, 0.9, d)

    def fg(th):
        u = (th - lo) / (hi - lo)
        r = u - c
        return 0.5 * r @ A @ r, (A @ r) / (hi - lo)

    st = drive(orc, fg, np.zeros(d), lo, hi, 200)
    np.testing.assert_allclose((st.theta[0] - lo) / (hi - lo), c, atol=1e-9)
    assert st.f[0] < 1e-18


def test_bound_constrained_separable_quadratic():
    import oracle as orc
    d = 5
    lo, hi = np.zeros(d), np.ones(d)
    c = np.array([0.3, -0.5, 1.7, 0.9, 2.0])     # three coordinates outside the box
    w = np.array([1.0, 10.0, 0.1, 5.0, 1.0])

    def fg(th):
        r = th - c
        return 0.5 * np.sum(w * r * r), w * r

    st = drive(orc, fg, np.full(d, 0.5), lo, hi, 300)
    np.testing.assert_allclose(st.theta[0], np.clip(c, 0, 1), atol=1e-9)


def test_fixed_dimension_untouched(orc):
    lo = np.array([0.0, 5.0, 0.0])
    hi = np.array([1.0, 5.0, 1.0])

    def fg(th):
        return (th[0] - 0.2) ** 2 + (th[2] - 0.7) ** 2, np.array([2 * (th[0] - 0.2), 99.0,
                                                                     2 * (th[2] - 0.7)])

    st = drive(orc, fg, np.array([0.9, 5.0, 0.1]), lo, hi, 100)
    assert st.theta[0, 1] == 5.0
    np.testing.assert_allclose(st.theta[0, [0, 2]], [0.2, 0.7], atol=1e-9)


def test_rosenbrock_valley(orc):
    lo, hi = np.full(2, -2.0), np.full(2, 2.0)

    def fg(th):
        x, y = th
        f = (1 - x) ** 2 + 100 * (y - x * x) ** 2
        return f, np.array([-2 * (1 - x) - 400 * x * (y - x * x), 200 * (y - x * x)])

    st = drive(orc, fg, np.array([-1.2, 1.0]), lo, hi, 400)
    np.testing.assert_allclose(st.theta[0], [1.0, 1.0], atol=1e-6)


def test_recovers_noise_free_truth_with_forward_mode_gradients(orc):
    wl = synth.c1()
    f = wl.fits[0]
    prob = orc.Problem(f.W, f.spd, f.seg_days, f.K, f.N)
    y = orc.integrate(prob, f.truth)[3]
    start = f.truth * np.array([1.1, 1.15, 0.9, 1.0])

    def fg(th):
        return orc.loss_grad_fwd(prob, th, y, "ssre")

    st = drive(orc, fg, start, f.lo, f.hi, 300)
    np.testing.assert_allclose(st.theta[0], f.truth, rtol=1e-6)
    assert st.f[0] < 1e-12


def test_log_scaled_last_dimension(orc):
    # minimiser of a quadratic in (u0, log I) sits at I = 3e3 in [1e2, 1e5]
    lo, hi = np.array([0.0, 1e2]), np.array([1.0, 1e5])
    c = np.array([0.4, np.log(3e3)])

    def fg(th):
        z = np.array([th[0], np.log(th[1])])
        r = z - c
        A = np.array([[2.0, 0.3], [0.3, 1.0]])
        gz = A @ r
        return 0.5 * r @ A @ r, np.array([gz[0], gz[1] / th[1]])

    st = orc.Lbfgs(np.array([[0.9, 150.0]]), log_last=True)
    st.f[0], st.grad[0] = fg(st.theta[0])
    for _ in range(100):
        st.propose(lo, hi)
        st.f_t[0], st.grad_t[0] = fg(st.theta_t[0])
        st.accept(lo, hi)
    np.testing.assert_allclose(st.theta[0], [0.4, 3e3], rtol=1e-9)


def _quadratic(d, seed, cond_shift=0.05):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(d, d))
    A = M @ M.T + cond_shift * np.eye(d)
    lo, hi = np.full(d, -1.0), np.full(d, 3.0)
    c = rng.uniform(0.1, 0.9, d)

    def fg(th):
        u = (th - lo) / (hi - lo)
        r = u - c
        return 0.5 * r @ A @ r, (A @ r) / (hi - lo)

    return fg, lo, hi, c


def test_trials_lie_at_doubling_steps_and_the_best_armijo_trial_is_kept(orc):
    """Every round: trial t is theta + 2^t (trial 0 - theta) while no
    coordinate is clamped; the kept point is the trial of lowest f among
    those passing f_t <= f + c1 alpha 2^t g.p (the test's own Armijo test),
    or none (theta unchanged, alpha halved)."""
    d, T, n = 6, 4, 3
    fg, lo, hi, _ = _quadratic(d, 7)
    rng = np.random.default_rng(8)
    st = orc.Lbfgs(rng.uniform(0.0, 2.0, (n, d)), m=5, n_trials=T)
    for q in range(n):
        st.f[q], st.grad[q] = fg(st.theta[q])
    kept_trial = set()
    for _ in range(25):
        th0, f0 = st.theta.copy(), st.f.copy()
        st.propose(lo, hi)
        gp = st.gp.copy()
        for i in range(T * n):
            st.f_t[i], st.grad_t[i] = fg(st.theta_t[i])
        trials = st.theta_t.reshape(T, n, d)
        ft = st.f_t.reshape(T, n)
        a1 = st.alpha.copy()   # after the cap on a first step
        st.accept(lo, hi)
        for q in range(n):
            step0 = trials[0, q] - th0[q]
            for t in range(T):
                inside = (trials[t, q] > lo).all() and (trials[t, q] < hi).all()
                if inside:
                    np.testing.assert_allclose(trials[t, q] - th0[q], 2.0 ** t * step0,
                                               rtol=1e-12, atol=1e-13)
            ok = [t for t in range(T)
                  if np.isfinite(ft[t, q]) and ft[t, q] <= f0[q] + 1e-4 * (a1[q] * 2 ** t) * gp[q]]
            if ok:
                best = min(ok, key=lambda t: (ft[t, q], t))
                kept_trial.add(best)
                np.testing.assert_array_equal(st.theta[q], trials[best, q])
                assert st.f[q] == ft[best, q] and st.alpha[q] == 1.0
            else:
                np.testing.assert_array_equal(st.theta[q], th0[q])
                assert st.alpha[q] == 0.5 * a1[q] or (st.alpha[q] == 1.0 and a1[q] < 2e-20)
    assert len(kept_trial) > 1   # the rounds kept more than the first trial


def test_trials_converge_on_quadratic_and_rosenbrock(orc):
    fg, lo, hi, c = _quadratic(8, 0)
    st = drive(orc, fg, np.zeros(8), lo, hi, 200, n_trials=4)
    np.testing.assert_allclose((st.theta[0] - lo) / (hi - lo), c, atol=1e-9)
    assert st.f[0] < 1e-18

    def rosen(th):
        x, y = th
        f = (1 - x) ** 2 + 100 * (y - x * x) ** 2
        return f, np.array([-2 * (1 - x) - 400 * x * (y - x * x), 200 * (y - x * x)])

    lo2, hi2 = np.array([-2.0, -1.0]), np.array([2.0, 3.0])
    r1 = drive(orc, rosen, np.array([-1.2, 1.0]), lo2, hi2, 3000, until=1e-14)[1]
    r4 = drive(orc, rosen, np.array([-1.2, 1.0]), lo2, hi2, 3000, n_trials=4, until=1e-14)[1]
    assert r1 is not None and r4 is not None
    assert r4 <= r1
