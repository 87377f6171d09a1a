"""GPU parity of the forward path (sird_loss, sird_integrate) against the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2204_12346_amd as S
from gpu_helpers import (TOL32, TOL64, assert_loss_close, assert_traj_close,
                         assert_traj_close_f32, format_worst, kappa, make_batch, need_gpu,
                         oracle_problem, random_theta)

pytestmark = pytest.mark.gpu

KINDS = ["ssre", "mse", "mxse", "mae", "mape"]


def _shapes():
    c1 = synth.c1().fits[0]
    c2 = synth.c2().fits[0]
    return {"c1": c1, "c2": c2}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("shape", ["c1", "c2"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_loss_all_kinds(shape, dtype):
    f = _shapes()[shape]
    P = 200  # three full tiles and a ragged one
    th = random_theta(f, P, seed=1)
    b = make_batch([f], [P], dtype=dtype)
    theta = b.pack_theta([th])
    obs = b.pack_obs([f.y])
    prob = oracle_problem(f)
    days = [oracle.integrate(prob, t)[3] for t in th]
    eps = TOL64 if dtype == "f64" else TOL32
    for kind in KINDS:
        print(f"case loss {shape} {dtype} {kind}", flush=True)
        got = S.sird_loss(b, theta, obs, kind).cpu().numpy()[:P]
        ref = oracle.loss_batch(prob, th, f.y, kind)
        kap = [kappa(kind, d, f.y) for d in days]
        assert_loss_close(got, ref, kap, eps, f"{shape}/{dtype}/{kind}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_integrate_trajectories(dtype):
    f = _shapes()["c2"]
    P = 130
    th = random_theta(f, P, seed=2)
    th[-5:] = np.asarray(f.truth)  # the synthetic truth: the epidemic the data shows
    b = make_batch([f], [P], dtype=dtype, with_traj=True)
    tr = b.unpack_traj(S.sird_integrate(b, b.pack_theta([th])))[0]
    prob = oracle_problem(f)
    worst = {}
    for p in range(P):
        ref = oracle.integrate(prob, th[p])
        if dtype == "f64":
            assert_traj_close(tr[p], ref, TOL64, f"particle {p}")
        else:
            assert_traj_close_f32(tr[p], ref, TOL32, f"particle {p}", worst, f"particle {p}")
    if worst:
        print("segmented workload, FP32 state: worst per-value relative error "
              + format_worst(worst))


def test_uneven_batch_equals_single_launches_and_oracle():
    wl = synth.c3(regions=list(range(24)))
    n_parts = [(7 * r + 1) % 150 for r in range(24)]
    n_parts[5] = 0  # a problem with no particles
    fits = wl.fits
    ths = [random_theta(f, n, seed=10 + r) for r, (f, n) in enumerate(zip(fits, n_parts))]
    b = make_batch(fits, n_parts)
    loss = S.sird_loss(b, b.pack_theta(ths), b.pack_obs([f.y for f in fits]), "ssre")
    per = b.split_particles(loss)
    for r, f in enumerate(fits):
        if n_parts[r] == 0:
            continue
        single = make_batch([f], [n_parts[r]])
        one = S.sird_loss(single, single.pack_theta([ths[r]]), single.pack_obs([f.y]), "ssre")
        assert np.array_equal(one.cpu().numpy()[:n_parts[r]], per[r]), f"region {r}"
        prob = oracle_problem(f)
        ref = oracle.loss_batch(prob, ths[r], f.y, "ssre")
        kap = [kappa("ssre", oracle.integrate(prob, t)[3], f.y) for t in ths[r]]
        assert_loss_close(per[r], ref, kap, TOL64, f"region {r}")


def test_launch_shapes_are_bitwise_equivalent():
    wl = synth.c3(regions=list(range(40)))
    n_parts = [100 + 3 * r for r in range(40)]
    ths = [random_theta(f, n, seed=r) for r, (f, n) in enumerate(zip(wl.fits, n_parts))]
    b = make_batch(wl.fits, n_parts)
    theta = b.pack_theta(ths)
    obs = b.pack_obs([f.y for f in wl.fits])
    ref = S.sird_loss(b, theta, obs, "ssre").cpu().numpy()
    for block, pers, cap in [(64, 0, 0), (128, 0, 0), (512, 0, 0), (640, 0, 0), (64, 37, 0),
                             (256, 256, 0), (256, 1, 0), (128, 4096, 0), (256, 0, 2),
                             (256, 0, 4), (64, 0, 1), (64, 0, 5), (512, 0, 4), (64, 37, 3)]:
        print(f"case launch block={block} persistent={pers} waves_per_simd={cap}", flush=True)
        b.configure(block=block, persistent=pers, waves_per_simd=cap)
        for rep in range(2):  # the persistent counters must reset between launches
            got = S.sird_loss(b, theta, obs, "ssre").cpu().numpy()
            assert np.array_equal(got, ref), (block, pers, cap, rep)
    # a cap that no LDS reservation within one block's 64 KiB can enforce
    b.configure(block=256, persistent=0, waves_per_simd=1)
    with pytest.raises(S.SirdError, match="waves_per_simd"):
        S.sird_loss(b, theta, obs, "ssre")
    b.configure(block=0, persistent=0, waves_per_simd=0)


def test_edge_cases():
    N = 1e5
    specs = [
        S.ProblemSpec(1, 1, 1, 1, N, n_part=3),               # one day, one step
        S.ProblemSpec(20, 3, 5, 9, N, n_part=65),             # segments past the end
        S.ProblemSpec(10, 7, 30, 2, N, R0=500.0, D0=40.0, n_part=64),  # seg > W
        S.ProblemSpec(8, 2, 1, 8, N, n_part=1),               # one-day segments
    ]
    b = S.Batch(specs, with_traj=True)
    rng = np.random.default_rng(4)
    ths, ys = [], []
    for s in specs:
        th = np.column_stack([rng.uniform(0, 1, (s.n_part, s.K)), rng.uniform(0, .5, s.n_part),
                              rng.uniform(0, .05, s.n_part), rng.uniform(10, 1000, s.n_part)])
        ths.append(th)
        ys.append(np.concatenate([[s.D0], s.D0 + np.cumsum(rng.integers(0, 20, s.W))]).astype(float))
    theta = b.pack_theta(ths)
    obs = b.pack_obs(ys)
    traj = b.unpack_traj(S.sird_integrate(b, theta))
    for kind in KINDS:
        loss = b.split_particles(S.sird_loss(b, theta, obs, kind))
        for s, th, y, l, tr in zip(specs, ths, ys, loss, traj):
            prob = oracle.Problem(s.W, s.spd, s.seg_days, s.K, s.N, s.R0, s.D0)
            ref = oracle.loss_batch(prob, th, y, kind)
            kap = [kappa(kind, oracle.integrate(prob, t)[3], y) for t in th]
            assert_loss_close(l, ref, kap, TOL64, f"edge {s.W}/{s.spd}/{s.K} {kind}")
            for p in range(s.n_part):
                assert_traj_close(tr[p], oracle.integrate(prob, th[p]), TOL64)


def test_nan_and_extreme_parameters():
    f = _shapes()["c1"]
    th = random_theta(f, 64, seed=5)
    th[0, 0] = np.nan          # NaN beta -> NaN loss
    th[1, :3] = [1.0, 0.0, 0.0]  # fastest growth, no removal
    th[2, :3] = [0.0, 0.5, 0.05]
    b = make_batch([f], [64])
    got = S.sird_loss(b, b.pack_theta([th]), b.pack_obs([f.y]), "ssre").cpu().numpy()
    ref = oracle.loss_batch(oracle_problem(f), th, f.y, "ssre")
    assert np.isnan(got[0]) and np.isnan(ref[0])
    kap = [kappa("ssre", oracle.integrate(oracle_problem(f), t)[3], f.y) for t in th[1:]]
    assert_loss_close(got[1:], ref[1:], kap, TOL64)


def test_full_size_batched_workload_sampled():
    """All 512 regions x 1024 particles in the launch shape the benchmark
    uses; two particles per region checked against the oracle."""
    wl = synth.c3()
    fits = wl.fits
    b = make_batch(fits)
    rng = np.random.default_rng(3)
    ths = [f.lo + rng.uniform(0, 1, (f.n_part, f.d)) * (f.hi - f.lo) for f in fits]
    theta = b.pack_theta(ths)
    obs = b.pack_obs([f.y for f in fits])
    from bench import C3_LAUNCH
    b.configure(**C3_LAUNCH)
    per = b.split_particles(S.sird_loss(b, theta, obs, "ssre"))
    for r, f in enumerate(fits):
        prob = oracle_problem(f)
        for p in (r % f.n_part, f.n_part - 1):
            ref = oracle.loss_batch(prob, ths[r][p:p + 1], f.y, "ssre")
            kap = [kappa("ssre", oracle.integrate(prob, ths[r][p])[3], f.y)]
            assert_loss_close(per[r][p:p + 1], ref, kap, TOL64, f"region {r} particle {p}")


@pytest.mark.parametrize("dtype,launch", [("f64", dict(block=256)),
                                          ("f64", dict(block=64, waves_per_simd=4)),
                                          ("f32", dict(block=128))])
def test_two_particles_per_lane_bitwise(dtype, launch):
    """Two particles per lane (tile pairs) gives bitwise the losses of one
    particle per lane, for every deceased-count cost, on an uneven batch
    whose problems have odd and even tile counts (a lone last tile, a
    problem with one particle, one with none)."""
    wl = synth.c3(regions=list(range(7)))
    n_parts = [300, 1, 128, 0, 200, 64, 65]
    ths = [random_theta(f, n, seed=60 + r) for r, (f, n) in enumerate(zip(wl.fits, n_parts))]
    obs_list = [f.y for f in wl.fits]
    out = {}
    for ppl in (1, 2):
        b = make_batch(wl.fits, n_parts, dtype=dtype, ppl=ppl, **launch)
        theta, obs = b.pack_theta(ths), b.pack_obs(obs_list)
        for kind in KINDS:
            print(f"case ppl={ppl} {dtype} {launch} {kind}", flush=True)
            out[(ppl, kind)] = S.sird_loss(b, theta, obs, kind).cpu().numpy()
    for kind in KINDS:
        assert np.array_equal(out[(1, kind)], out[(2, kind)], equal_nan=True), kind
    # and the oracle on the lone-tile and one-particle problems
    b = make_batch(wl.fits, n_parts, dtype=dtype, ppl=2, **launch)
    per = b.split_particles(S.sird_loss(b, b.pack_theta(ths), b.pack_obs(obs_list), "ssre"))
    eps = TOL64 if dtype == "f64" else TOL32
    for r in (1, 6):
        f = wl.fits[r]
        prob = oracle_problem(f)
        ref = oracle.loss_batch(prob, ths[r], f.y, "ssre")
        kap = [kappa("ssre", oracle.integrate(prob, t)[3], f.y) for t in ths[r]]
        assert_loss_close(per[r], ref, kap, eps, f"region {r}")
