"""End-to-end pins of the oracle's calibration on noise-free data: the loss
is exactly zero at the truth, and the swarm (Sec. 3.3) recovers the three
parameters of the constant-beta workload."""
import numpy as np

import synth


def test_noise_free_truth_has_zero_loss(orc):
    for wl in (synth.c1(), synth.c2()):
        f = wl.fits[0]
        prob = orc.Problem(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0)
        y = orc.integrate(prob, f.truth)[3]
        for kind in ("ssre", "mse", "mxse", "mae", "mape"):
            assert orc.loss(kind, y, y) == 0.0
            assert orc.loss_batch(prob, f.truth[None, :], y, kind)[0] == 0.0


def test_pso_recovers_constant_beta_truth(orc):
    # 400 iterations: from every seed tried (1..5) the swarm then ends below
    # 1e-8 with the parameters within 4e-4 of the truth
    wl = synth.c1(iters=400)
    f = wl.fits[0]
    prob = orc.Problem(f.W, f.spd, f.seg_days, f.K, f.N)
    y = orc.integrate(prob, f.truth)[3]
    hf, hidx, hm, s = orc.pso_run(prob, y, "ssre", f.n_part, f.lo, f.hi, wl.w, wl.c1,
                                  wl.c2, wl.seed, f.stream, wl.iters, nthreads=4)
    assert hf[-1] < 1e-6 and hf[0] > 1.0
    np.testing.assert_allclose(s.gbest_x, f.truth, rtol=2e-3)


def test_pso_then_adam_refines(orc):
    wl = synth.c1(n_part=64, iters=40)
    f = wl.fits[0]
    prob = orc.Problem(f.W, f.spd, f.seg_days, f.K, f.N)
    y = orc.integrate(prob, f.truth)[3]
    hf, hidx, hm, s = orc.pso_run(prob, y, "ssre", f.n_part, f.lo, f.hi, wl.w, wl.c1,
                                  wl.c2, wl.seed, f.stream, wl.iters)
    th = s.gbest_x[None, :].copy()
    m, v = np.zeros_like(th), np.zeros_like(th)
    L0 = orc.loss_grad_fwd(prob, th[0], y)[0]
    Ls = []
    for t in range(1, 501):
        L, g = orc.loss_grad_fwd(prob, th[0], y)
        Ls.append(L)
        orc.adam_step(th, g[None, :].copy(), m, v, f.lo, f.hi, t, lr=1e-3)
    L1 = orc.loss_grad_fwd(prob, th[0], y)[0]
    # the valley between beta and gamma is narrow: Adam descends it steadily
    assert L1 < 0.8 * L0
    assert all(b <= a * (1 + 1e-3) for a, b in zip(Ls[::50], Ls[50::50]))
