"""GPU parity of the swarm (pso_init, pso_step, sird_pso_iterate, graphs)
against the oracle: bitwise in lockstep, and the global-best sequence of
whole runs up to the first near-tie the oracle reports."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2204_12346_amd as S
from gpu_helpers import (TOL64, assert_loss_close, compared_iterations, kappa,
                         loss_discrepancy, make_batch, need_gpu, oracle_problem)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _swarm_to_oracle(b, sw, r=0):
    """Copy problem r of a device swarm into an oracle Swarm."""
    s = b.specs[r]
    o = oracle.Swarm(s.n_part, s.d)
    o.x[:] = b.unpack_theta(sw.x)[r]
    o.v[:] = b.unpack_theta(sw.v)[r]
    o.pbest_x[:] = b.unpack_theta(sw.pbest_x)[r]
    o.pbest_f[:] = b.split_particles(sw.pbest_f)[r]
    o.gbest_x[:] = b.unpack_box(sw.gbest_x)[r]
    o.gbest_f[0] = sw.gbest_f[r].item()
    o.gbest_idx[0] = sw.gbest_idx[r].item()
    return o


def test_init_bitwise():
    wl = synth.c3(regions=[0, 1, 2])
    n_parts = [70, 1, 130]
    b = make_batch(wl.fits, n_parts)
    params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], seed=wl.seed)
    sw = S.Swarm(b)
    S.pso_init(b, params, sw)
    torch.cuda.synchronize()
    for r, f in enumerate(wl.fits):
        ref = oracle.pso_init(n_parts[r], f.lo, f.hi, wl.seed, f.stream)
        got = _swarm_to_oracle(b, sw, r)
        assert np.array_equal(got.x, ref.x) and np.array_equal(got.pbest_x, ref.x)
        assert np.all(got.v == 0) and np.all(np.isinf(got.pbest_f))
        assert np.array_equal(got.gbest_x, f.lo) and got.gbest_idx[0] == -1
    assert sw.iter.cpu().tolist() == [0, 0]


@pytest.mark.parametrize("regions,n_parts", [
    ([3, 4], [200, 77]),                     # global best: one wavefront per problem, one block
    ([3, 4], [5000, 77]),                    # one block per problem (a problem above 4096)
    (list(range(9)), [64, 1, 130, 200, 77, 5, 300, 64, 90]),  # wavefronts, three blocks
])
def test_step_lockstep_bitwise(regions, n_parts):
    """Same f and state on both sides -> bitwise equal bests and moves."""
    wl = synth.c3(regions=regions)
    b = make_batch(wl.fits, n_parts)
    params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], w=0.7, c1=1.5,
                         c2=1.5, seed=wl.seed)
    sw = S.Swarm(b, hist_len=8)
    S.pso_init(b, params, sw)
    rng = np.random.default_rng(0)
    refs = [oracle.pso_init(n, f.lo, f.hi, wl.seed, f.stream) for f, n in zip(wl.fits, n_parts)]
    for it in range(6):
        fs = [rng.uniform(0, 10, n) for n in n_parts]
        for r in range(len(n_parts)):
            if n_parts[r] > 5:
                fs[r][rng.integers(0, n_parts[r], 5)] = np.nan
                fs[r][:3] = fs[r][3]  # exact ties
        f_all = np.concatenate(fs)
        sw.f.copy_(torch.from_numpy(f_all).to(sw.f.device))
        S.pso_step(b, params, sw)
        torch.cuda.synchronize()
        for r, f in enumerate(wl.fits):
            oracle.pso_bests(refs[r], fs[r])
            oracle.pso_move(refs[r], it, 0.7, 1.5, 1.5, f.lo, f.hi, wl.seed, f.stream)
            got = _swarm_to_oracle(b, sw, r)
            assert np.array_equal(got.pbest_f, refs[r].pbest_f), (it, r)
            assert np.array_equal(got.pbest_x, refs[r].pbest_x), (it, r)
            assert got.gbest_idx[0] == refs[r].gbest_idx[0] and got.gbest_f[0] == refs[r].gbest_f[0]
            assert np.array_equal(got.gbest_x, refs[r].gbest_x)
            assert np.array_equal(got.v, refs[r].v), (it, r)
            assert np.array_equal(got.x, refs[r].x), (it, r)
        assert sw.iter[0].item() == it + 1 and sw.iter[1].item() == 0
    hf = sw.hist_f.cpu().numpy()
    assert np.all(np.isfinite(hf[:6])) and np.all(np.isnan(hf[6:]))


def _run_compare(wl, fits, n_parts, iters, kind="ssre", launch=None, min_compared=None,
                 pool=False):
    """The whole swarm run on the GPU (fused iterations) against the
    oracle's, problem by problem: gbest indices equal and gbest losses
    within 1e-11 up to the first near-tie of the oracle's run.  pool: run
    the problems' oracles side by side on one thread each."""
    from concurrent.futures import ThreadPoolExecutor
    b = make_batch(fits, n_parts, **(launch or {}))
    params = S.PsoParams(b, [f.lo for f in fits], [f.hi for f in fits], wl.w, wl.c1, wl.c2,
                         wl.seed)
    sw = S.Swarm(b, hist_len=iters)
    obs = b.pack_obs([f.y for f in fits])
    S.pso_init(b, params, sw)
    S.sird_pso_iterate(b, params, sw, obs, kind, iters)
    torch.cuda.synchronize()
    gh_f = sw.hist_f.cpu().numpy()
    gh_i = sw.hist_idx.cpu().numpy()
    pbx = b.unpack_theta(sw.pbest_x)
    pbf = b.split_particles(sw.pbest_f)
    nt = 1 if pool else 0

    def oracle_side(r):
        f = fits[r]
        prob = oracle_problem(f)
        run = oracle.pso_run(prob, f.y, kind, n_parts[r], f.lo, f.hi, wl.w, wl.c1, wl.c2,
                             wl.seed, f.stream, iters, nthreads=nt)
        at_pbest = oracle.loss_batch(prob, pbx[r], f.y, kind, nthreads=nt)
        return run, at_pbest

    if pool:
        with ThreadPoolExecutor(16) as ex:
            res = list(ex.map(oracle_side, range(len(fits))))
    else:
        res = [oracle_side(r) for r in range(len(fits))]
    delta = max(loss_discrepancy(pbf[r], res[r][1]) for r in range(len(fits)))
    assert delta < 1e-11, f"personal-best losses off the oracle's by {delta:.2e}"
    need = min(iters, 20) if min_compared is None else min_compared
    shortest = iters
    for r, f in enumerate(fits):
        hf, hidx, hm, _ = res[r][0]
        upto, thr = compared_iterations(hm, delta, iters)
        shortest = min(shortest, upto)
        assert upto >= need, f"problem {r}: oracle near-tie too early ({upto})"
        np.testing.assert_array_equal(gh_i[:upto, r], hidx[:upto], err_msg=f"problem {r}")
        np.testing.assert_allclose(gh_f[:upto, r], hf[:upto], rtol=1e-11, atol=0,
                                   err_msg=f"problem {r}")
    print(f"{len(fits)} problems: loss discrepancy {delta:.2e}, near-tie threshold {thr:.1e}, "
          f"at least {shortest} of {iters} iterations compared", flush=True)
    return b, sw


def test_full_run_constant_beta_workload():
    wl = synth.c1()  # 256 particles x 200 iterations
    _run_compare(wl, wl.fits, [256], wl.iters)


def test_run_segmented_beta_workload_full_population():
    """8192 particles, 13 segments, 180 days: 150 iterations."""
    wl = synth.c2()
    _run_compare(wl, wl.fits, [wl.fits[0].n_part], 150, min_compared=100)


def test_run_batched_uneven_workload_ragged_populations():
    wl = synth.c3(regions=list(range(12)))
    _run_compare(wl, wl.fits, [64 + 37 * r for r in range(12)], 15)


def test_run_batched_uneven_workload_full():
    """All 512 regions x 1024 particles in the benchmark's launch shape,
    10 iterations, every region against its own oracle run."""
    from bench import C3_LAUNCH
    wl = synth.c3()
    _run_compare(wl, wl.fits, [f.n_part for f in wl.fits], 10, launch=C3_LAUNCH,
                 min_compared=10, pool=True)


@pytest.mark.parametrize("launch", [dict(), dict(block=256, persistent=0, waves_per_simd=4)])
def test_graph_replay_equals_eager(launch):
    """HIP-graph replays (with host work between them) leave bitwise the
    eager sequence's state, also in the batched workload's launch shape."""
    wl = synth.c3(regions=list(range(8)))
    n_parts = [128] * 8
    results = []
    for mode in ("eager", "graph"):
        print(f"case graph {launch} {mode}", flush=True)
        b = make_batch(wl.fits, n_parts, **launch)
        params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                             wl.c2, wl.seed)
        sw = S.Swarm(b, hist_len=12)
        obs = b.pack_obs([f.y for f in wl.fits])
        S.pso_init(b, params, sw)
        if mode == "eager":
            S.sird_pso_iterate(b, params, sw, obs, "ssre", 12)
        else:
            g = S.Graph(b, params, sw, obs, "ssre", iters_per_launch=3)
            for _ in range(4):  # replays with host work and syncs between them
                g.launch(1)
                torch.cuda.synchronize()
                _ = sw.gbest_f.cpu()
            g.close()
        torch.cuda.synchronize()
        results.append([t.cpu().numpy().copy() for t in
                        (sw.x, sw.v, sw.pbest_f, sw.gbest_f, sw.hist_f, sw.hist_idx, sw.iter)])
    for a, c in zip(*results):
        assert np.array_equal(a, c, equal_nan=True)


def test_resume_is_bitwise():
    wl = synth.c1(n_part=128)
    f = wl.fits[0]
    outs = []
    for split in (None, 7):
        b = make_batch([f], [128])
        params = S.PsoParams(b, [f.lo], [f.hi], wl.w, wl.c1, wl.c2, wl.seed)
        sw = S.Swarm(b)
        obs = b.pack_obs([f.y])
        S.pso_init(b, params, sw)
        if split is None:
            S.sird_pso_iterate(b, params, sw, obs, "ssre", 14)
        else:
            S.sird_pso_iterate(b, params, sw, obs, "ssre", split)
            torch.cuda.synchronize()
            saved = {k: getattr(sw, k).clone() for k in
                     ("x", "v", "pbest_x", "pbest_f", "gbest_x", "gbest_f", "gbest_idx", "iter")}
            sw2 = S.Swarm(b)
            for k, v in saved.items():
                getattr(sw2, k).copy_(v)
            S.sird_pso_iterate(b, params, sw2, obs, "ssre", 14 - split)
            sw = sw2
        torch.cuda.synchronize()
        outs.append((sw.x.cpu().numpy(), sw.pbest_f.cpu().numpy(), sw.gbest_idx.cpu().numpy()))
    for a, c in zip(*outs):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("dtype,launch", [("f64", dict(block=256, persistent=0)),
                                          ("f64", dict(block=256, persistent=0, waves_per_simd=4)),
                                          ("f64", dict(block=64, persistent=300)),
                                          ("f32", dict(block=128, persistent=0))])
def test_fused_iterate_equals_loss_plus_step(dtype, launch):
    """sird_pso_iterate (swarm fused into the integration) leaves bitwise the
    state of n x [sird_loss; pso_step]."""
    wl = synth.c3(regions=list(range(6)))
    n_parts = [100, 64, 1, 150, 33, 70]
    states = []
    for mode in ("unfused", "fused", "halves"):
        b = make_batch(wl.fits, n_parts, dtype=dtype, **launch)
        params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                             wl.c2, wl.seed)
        sw = S.Swarm(b, hist_len=9)
        obs = b.pack_obs([f.y for f in wl.fits])
        S.pso_init(b, params, sw)
        if mode == "unfused":
            for _ in range(9):
                S.sird_loss(b, sw.x, obs, "ssre", sw.f)
                S.pso_step(b, params, sw)
        elif mode == "fused":
            S.sird_pso_iterate(b, params, sw, obs, "ssre", 4)
            S.sird_pso_iterate(b, params, sw, obs, "ssre", 5)
        else:
            for i in range(9):
                S.pso_evaluate(b, params, sw, obs, "ssre", move_first=i > 0)
                S.pso_gbest(b, params, sw)
            S.pso_complete_move(b, params, sw)
        torch.cuda.synchronize()
        states.append([t.cpu().numpy().copy() for t in
                       (sw.x, sw.v, sw.pbest_x, sw.pbest_f, sw.gbest_x, sw.gbest_f,
                        sw.gbest_idx, sw.iter, sw.hist_f, sw.hist_idx, sw.f)])
    for other in states[1:]:
        for a, c in zip(states[0], other):
            assert np.array_equal(a, c, equal_nan=True)


def test_full_size_fused_evaluate_sampled():
    """The benchmark's step at full size (512 regions x 1024 particles, the
    benchmark's launch): after two iterations, one pso_evaluate with the
    move.  For every 16th region the whole move is checked bitwise against
    the oracle's swarm update of the state before it, and two particles'
    losses against the oracle's loss of the moved positions."""
    from bench import C3_LAUNCH
    wl = synth.c3()
    b = make_batch(wl.fits, **C3_LAUNCH)
    params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                         wl.c2, wl.seed)
    sw = S.Swarm(b)
    obs = b.pack_obs([f.y for f in wl.fits])
    S.pso_init(b, params, sw)
    S.pso_evaluate(b, params, sw, obs, "ssre", move_first=False)
    S.pso_gbest(b, params, sw)
    S.pso_evaluate(b, params, sw, obs, "ssre", move_first=True)
    S.pso_gbest(b, params, sw)
    torch.cuda.synchronize()
    regions = list(range(0, len(wl.fits), 16))
    before = {r: _swarm_to_oracle(b, sw, r) for r in regions}
    it = int(sw.iter[0].item())
    print(f"case full-size fused evaluate, iteration {it}", flush=True)
    S.pso_evaluate(b, params, sw, obs, "ssre", move_first=True)
    torch.cuda.synchronize()
    f_all = b.split_particles(sw.f)
    for r in regions:
        f = wl.fits[r]
        ref = before[r]
        oracle.pso_move(ref, it - 1, wl.w, wl.c1, wl.c2, f.lo, f.hi, wl.seed, f.stream)
        got = _swarm_to_oracle(b, sw, r)
        assert np.array_equal(got.x, ref.x), f"region {r}: positions"
        assert np.array_equal(got.v, ref.v), f"region {r}: velocities"
        prob = oracle_problem(f)
        for p in (r % f.n_part, f.n_part - 1):
            L = oracle.loss_batch(prob, ref.x[p:p + 1], f.y, "ssre")
            kap = [kappa("ssre", oracle.integrate(prob, ref.x[p])[3], f.y)]
            assert_loss_close(f_all[r][p:p + 1], L, kap, TOL64, f"region {r} particle {p}")


@pytest.mark.parametrize("launch", [dict(block=256, persistent=0),
                                    dict(block=256, persistent=0, waves_per_simd=4),
                                    dict(block=64, persistent=300)])
def test_fused_move_every_block_layout(launch):
    """The fused kernel moves Philox block 0 (gamma, mu, I0, beta_1) before
    integrating and each later block of betas as the segment loop reaches
    it: for 1 to 13 segments, segments past the window end (never
    integrated, still moved) and ragged tiles, the fused sequence leaves
    bitwise the state of n x [sird_loss; pso_step]."""
    shapes = [(30, 3, 30, 1, 70), (30, 2, 10, 2, 64), (40, 1, 10, 4, 65), (50, 2, 10, 5, 1),
              (20, 5, 5, 9, 100), (60, 2, 5, 12, 33), (45, 4, 3, 13, 128), (7, 10, 1, 8, 64)]
    specs = [S.ProblemSpec(W, spd, seg, K, 1e6, n_part=n, stream=r)
             for r, (W, spd, seg, K, n) in enumerate(shapes)]
    los = [np.concatenate([np.full(s.K, 0.05), [0.05, 0.001, 100.0]]) for s in specs]
    his = [np.concatenate([np.full(s.K, 0.5), [0.2, 0.01, 1000.0]]) for s in specs]
    ys = [np.array([2.0 * i + 0.05 * i * i for i in range(s.W + 1)]) for s in specs]
    states = []
    for mode in ("unfused", "fused"):
        print(f"case fused move layout {launch} {mode}", flush=True)
        b = S.Batch(specs, **launch)
        params = S.PsoParams(b, los, his, 0.7, 1.5, 1.5, 21)
        sw = S.Swarm(b, hist_len=6)
        obs = b.pack_obs(ys)
        S.pso_init(b, params, sw)
        if mode == "unfused":
            for _ in range(6):
                S.sird_loss(b, sw.x, obs, "ssre", sw.f)
                S.pso_step(b, params, sw)
        else:
            S.sird_pso_iterate(b, params, sw, obs, "ssre", 6)
        torch.cuda.synchronize()
        states.append([t.cpu().numpy().copy() for t in
                       (sw.x, sw.v, sw.pbest_x, sw.pbest_f, sw.gbest_x, sw.gbest_f,
                        sw.gbest_idx, sw.iter, sw.hist_f, sw.hist_idx, sw.f)])
    for a, c in zip(*states):
        assert np.array_equal(a, c, equal_nan=True)


@pytest.mark.parametrize("dtype,launch", [("f64", dict(block=256, waves_per_simd=4)),
                                          ("f64", dict(block=64)),
                                          ("f32", dict(block=256))])
def test_two_particles_per_lane_swarm_bitwise(dtype, launch):
    """The fused swarm iteration with two particles per lane leaves bitwise
    the swarm state of one particle per lane (moves, losses, bests,
    history), on an uneven batch with lone last tiles."""
    wl = synth.c3(regions=list(range(6)))
    n_parts = [100, 64, 1, 150, 33, 257]
    states = []
    for ppl in (1, 2):
        print(f"case swarm ppl={ppl} {dtype} {launch}", flush=True)
        b = make_batch(wl.fits, n_parts, dtype=dtype, ppl=ppl, **launch)
        params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                             wl.c2, wl.seed)
        sw = S.Swarm(b, hist_len=8)
        obs = b.pack_obs([f.y for f in wl.fits])
        S.pso_init(b, params, sw)
        S.sird_pso_iterate(b, params, sw, obs, "ssre", 8)
        torch.cuda.synchronize()
        states.append([t.cpu().numpy().copy() for t in
                       (sw.x, sw.v, sw.pbest_x, sw.pbest_f, sw.gbest_x, sw.gbest_f,
                        sw.gbest_idx, sw.iter, sw.hist_f, sw.hist_idx, sw.f)])
    for a, c in zip(*states):
        assert np.array_equal(a, c, equal_nan=True)
