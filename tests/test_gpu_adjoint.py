"""GPU parity of the discrete-adjoint gradient (sird_loss_backward) against
the oracle's forward-mode gradient and against central differences of the
GPU's own loss; bitwise independence of the checkpoint interval."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2204_12346_amd as S
from gpu_helpers import (assert_loss_close, kappa, make_batch, need_gpu, oracle_problem,
                         random_theta)

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def assert_grad_close(got, ref, what=""):
    """|g - g_ref| <= 1e-6 |g_ref| + 1e-9 max|g_ref| per component."""
    got, ref = np.asarray(got), np.asarray(ref)
    tol = GRAD_RTOL * np.abs(ref) + 1e-9 * np.max(np.abs(ref))
    bad = ~(np.abs(got - ref) <= tol)
    if bad.any():
        j = int(np.argmax(bad))
        raise AssertionError(f"{what}: component {j}: gpu={got[j]!r} ref={ref[j]!r}")


@pytest.mark.parametrize("shape", ["c1", "c2"])
@pytest.mark.parametrize("kind", ["ssre", "mse", "mxse", "mae", "mape"])
def test_adjoint_matches_forward_mode(shape, kind):
    f = (synth.c1() if shape == "c1" else synth.c2()).fits[0]
    P = 70
    th = random_theta(f, P, seed=3)
    th[:, :f.K] *= 0.5  # keep most trajectories away from total burn-out
    b = make_batch([f], [P])
    g, L = S.sird_loss_backward(b, b.pack_theta([th]), b.pack_obs([f.y]), kind,
                                loss_out=b.empty_particles())
    gg = b.unpack_theta(g)[0]
    LL = L.cpu().numpy()
    lf = S.sird_loss(b, b.pack_theta([th]), b.pack_obs([f.y]), kind).cpu().numpy()
    # the backward's own forward (which carries S) is the loss kernel's
    # (which carries s = b S alone) up to rounding
    prob = oracle_problem(f)
    kap = [kappa(kind, oracle.integrate(prob, t)[3], f.y) for t in th]
    assert_loss_close(LL[:P], lf[:P], kap, 1e-13, f"{shape}/{kind} backward loss")
    for p in range(0, P, 3):
        Lr, gr = oracle.loss_grad_fwd(prob, th[p], f.y, kind)
        assert_grad_close(gg[p], gr, f"{shape}/{kind}/particle {p}")


def test_checkpoint_interval_is_bitwise_irrelevant():
    f = synth.c2().fits[0]
    th = random_theta(f, 100, seed=4)
    b = make_batch([f], [100])
    theta, obs = b.pack_theta([th]), b.pack_obs([f.y])
    ref = None
    for s in (0, 1, 7, 43, 1800, 5000):
        g, _ = S.sird_loss_backward(b, theta, obs, "ssre", ckpt_interval=s)
        h = g.cpu().numpy()
        if ref is None:
            ref = h
        assert np.array_equal(h, ref), s


def test_grad_loss_scales_and_batched_uneven():
    wl = synth.c3(regions=list(range(10)))
    n_parts = [33, 64, 1, 90, 0, 128, 65, 5, 40, 70]
    ths = [random_theta(f, n, seed=r) for r, (f, n) in enumerate(zip(wl.fits, n_parts))]
    b = make_batch(wl.fits, n_parts)
    theta, obs = b.pack_theta(ths), b.pack_obs([f.y for f in wl.fits])
    scale = torch.linspace(-2, 3, b.total_particles, dtype=torch.float64, device=theta.device)
    g1, _ = S.sird_loss_backward(b, theta, obs, "mse")
    g2, _ = S.sird_loss_backward(b, theta, obs, "mse", grad_loss=scale)
    G1, G2 = b.unpack_theta(g1), b.unpack_theta(g2)
    sc = b.split_particles(scale)
    for r, f in enumerate(wl.fits):
        if n_parts[r] == 0:
            continue
        np.testing.assert_array_equal(G2[r], G1[r] * sc[r][:, None])
        prob = oracle_problem(f)
        for p in {0, n_parts[r] - 1}:
            assert_grad_close(G1[r][p], oracle.loss_grad_fwd(prob, ths[r][p], f.y, "mse")[1],
                              f"region {r} particle {p}")


def test_adjoint_matches_central_differences_of_gpu_loss():
    f = synth.c2().fits[0]
    th0 = random_theta(f, 1, seed=8)[0]
    th0[:f.K] *= 0.6
    d = f.d
    # rows: theta, then theta +- h e_j
    h = np.where(th0 != 0, 1e-6 * np.abs(th0), 1e-6 * (f.hi - f.lo))
    rows = [th0]
    for j in range(d):
        for sgn in (1, -1):
            t = th0.copy()
            t[j] += sgn * h[j]
            rows.append(t)
    rows = np.array(rows)
    b = make_batch([f], [len(rows)])
    theta, obs = b.pack_theta([rows]), b.pack_obs([f.y])
    L = S.sird_loss(b, theta, obs, "ssre").cpu().numpy()
    g, _ = S.sird_loss_backward(b, theta, obs, "ssre")
    g0 = b.unpack_theta(g)[0][0]
    fd = np.array([(L[1 + 2 * j] - L[2 + 2 * j]) / (2 * h[j]) for j in range(d)])
    np.testing.assert_allclose(g0, fd, rtol=1e-5, atol=1e-7 * np.abs(fd).max())


def test_full_size_gradient_workload_sampled():
    """65536 parameter vectors on a 365-day window at dt = 0.05 (7300 steps),
    sqrt(T) checkpoints; a sample checked against the oracle."""
    wl, thetas = synth.c4()
    f = wl.fits[0]
    b = make_batch([f])
    theta, obs = b.pack_theta([thetas]), b.pack_obs([f.y])
    g, L = S.sird_loss_backward(b, theta, obs, "ssre", loss_out=b.empty_particles())
    gg = b.unpack_theta(g)[0]
    prob = oracle_problem(f)
    for p in (0, 12345, 65535):
        Lr, gr = oracle.loss_grad_fwd(prob, thetas[p], f.y, "ssre")
        assert_grad_close(gg[p], gr, f"particle {p}")


@pytest.mark.parametrize("spd", [1, 3, 8, 10, 20])
def test_adjoint_few_steps_per_day_and_zero_beta(spd):
    """Steps per day below and at the 8-step replay chunk (several day starts
    in a chunk, or exactly one at its start), a segment with beta = 0, and
    segments shorter than a chunk; with 10 or 20 steps per day, one-day
    segments and intervals that are multiples of 10 (the aligned 10-step
    sweep) next to intervals that are not (the general one): against the
    oracle's forward-mode gradient, and bitwise the same for every
    checkpoint interval."""
    f = synth.c2().fits[0]
    f.spd = spd
    # segments of 2 steps when spd = 1, of one day when spd >= 10
    f.seg_days = 2 if spd == 1 else (1 if spd >= 10 else f.seg_days)
    f.K = min(f.K, (f.W + f.seg_days - 1) // f.seg_days)
    f.lo, f.hi = np.concatenate([f.lo[:f.K], f.lo[-3:]]), np.concatenate([f.hi[:f.K], f.hi[-3:]])
    th = random_theta(f, 40, seed=11)
    th[:, :f.K] *= 0.5
    th[:, 1] = 0.0  # no transmission in the second segment
    b = make_batch([f], [40])
    theta, obs = b.pack_theta([th]), b.pack_obs([f.y])
    prob = oracle_problem(f)
    ref = None
    for s in (0, 1, 5, 13, 10, 30):
        print(f"case spd={spd} interval={s}", flush=True)
        g, _ = S.sird_loss_backward(b, theta, obs, "ssre", ckpt_interval=s)
        h = b.unpack_theta(g)[0]
        if ref is None:
            ref = h
            for p in range(0, 40, 7):
                assert_grad_close(h[p], oracle.loss_grad_fwd(prob, th[p], f.y, "ssre")[1],
                                  f"spd {spd} particle {p}")
        assert np.array_equal(h, ref), s


def test_mixed_sweeps_in_one_batch_equal_single_launches():
    """Problems with 10 and 20 steps per day take the aligned 10-step sweep,
    one with 3 the general sweep; in one batch each gradient is bitwise
    its single-problem launch's, and within the oracle's tolerance."""
    base = synth.c2().fits[0]
    fits = []
    for spd, W, K in ((10, 60, 5), (3, 45, 4), (20, 30, 3)):
        f = synth.c2().fits[0]
        f.spd, f.W, f.K, f.seg_days = spd, W, K, 14
        f.y = base.y[:W + 1]
        f.lo = np.concatenate([base.lo[:K], base.lo[-3:]])
        f.hi = np.concatenate([base.hi[:K], base.hi[-3:]])
        fits.append(f)
    n_parts = [70, 33, 64]
    ths = [random_theta(f, n, seed=20 + r) for r, (f, n) in enumerate(zip(fits, n_parts))]
    for th, f in zip(ths, fits):
        th[:, :f.K] *= 0.5
    b = make_batch(fits, n_parts)
    print("case mixed sweeps batch", flush=True)
    g, _ = S.sird_loss_backward(b, b.pack_theta(ths), b.pack_obs([f.y for f in fits]), "ssre",
                                ckpt_interval=30)
    G = b.unpack_theta(g)
    for r, f in enumerate(fits):
        b1 = make_batch([f], [n_parts[r]])
        g1, _ = S.sird_loss_backward(b1, b1.pack_theta([ths[r]]), b1.pack_obs([f.y]), "ssre",
                                     ckpt_interval=30)
        assert np.array_equal(G[r], b1.unpack_theta(g1)[0]), f"problem {r}"
        prob = oracle_problem(f)
        for p in (0, n_parts[r] - 1):
            assert_grad_close(G[r][p], oracle.loss_grad_fwd(prob, ths[r][p], f.y, "ssre")[1],
                              f"problem {r} particle {p}")
