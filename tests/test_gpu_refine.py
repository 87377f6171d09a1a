"""GPU checks of the refinement pieces: top-k selection, gather, projected
Adam, the autograd Function, the refinement driver, the forecast, and the
autotuner's bitwise invariance."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2204_12346_amd as S
from paper_2204_12346_amd import autotune, fit
from paper_2204_12346_amd.autograd import SirdLoss
from gpu_helpers import (TOL64, assert_grad_close, assert_traj_close, make_batch, near_truth,
                         need_gpu, oracle_grad, oracle_problem, random_theta)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_topk_order_ties_and_nan():
    specs = [S.ProblemSpec(10, 2, 5, 2, 1e5, n_part=n) for n in (300, 5, 1000, 0)]
    b = S.Batch(specs)
    rng = np.random.default_rng(0)
    fs = [np.round(rng.uniform(0, 5, s.n_part), 1) for s in specs]  # many exact ties
    fs[0][[3, 7]] = np.nan
    fs[2][[10, 20, 30]] = np.inf
    f_all = torch.from_numpy(np.concatenate(fs)).cuda()
    k = 8
    idx = S.pso_topk(b, f_all, k).cpu().numpy()
    for r, f in enumerate(fs):
        key = np.where(np.isnan(f), np.inf, f)
        order = np.lexsort((np.arange(len(f)), key))[:k]
        exp = list(order) + [-1] * (k - len(order))
        assert list(idx[r]) == exp, r


def test_topk_by_rank_for_large_k():
    """Above 32 the selection counts ranks; same order, ties and padding."""
    specs = [S.ProblemSpec(10, 2, 5, 2, 1e5, n_part=n) for n in (3000, 70, 0, 500)]
    b = S.Batch(specs)
    rng = np.random.default_rng(4)
    fs = [np.round(rng.uniform(0, 5, s.n_part), 2) for s in specs]
    fs[0][[3, 7, 2999]] = np.nan
    fs[3][[10, 20]] = np.inf
    f_all = torch.from_numpy(np.concatenate(fs)).cuda()
    for k in (33, 300, 3000, 4096):
        idx = S.pso_topk(b, f_all, k).cpu().numpy()
        for r, f in enumerate(fs):
            key = np.where(np.isnan(f), np.inf, f)
            order = np.lexsort((np.arange(len(f)), key))[:k]
            exp = list(order) + [-1] * (k - len(order))
            assert list(idx[r]) == exp, (k, r)


def test_gather_and_adam_match_oracle():
    wl = synth.c3(regions=[0, 1, 2])
    n_parts = [100, 40, 64]
    b = make_batch(wl.fits, n_parts)
    ths = [random_theta(f, n, seed=r) for r, (f, n) in enumerate(zip(wl.fits, n_parts))]
    src = b.pack_theta(ths)
    lo = b.pack_box([f.lo for f in wl.fits])
    hi = b.pack_box([f.hi for f in wl.fits])
    k = 6
    idx_np = np.array([[5, 0, 99, -1, 7, 3], [39, 1, 2, 3, 4, 5], [63, 62, 0, 1, -1, 9]])
    idx = torch.from_numpy(idx_np).cuda()
    rb = make_batch(wl.fits, [k] * 3)
    dst = S.sird_gather(b, src, lo, rb, idx, k)
    got = rb.unpack_theta(dst)
    for r in range(3):
        for q in range(k):
            exp = ths[r][idx_np[r, q]] if idx_np[r, q] >= 0 else wl.fits[r].lo
            assert np.array_equal(got[r][q], exp)
    # Adam: several steps against the oracle
    rng = np.random.default_rng(1)
    m = torch.zeros_like(dst)
    v = torch.zeros_like(dst)
    th_o = [g.copy() for g in got]
    m_o = [np.zeros_like(g) for g in got]
    v_o = [np.zeros_like(g) for g in got]
    for t in range(1, 6):
        grads = [rng.normal(0, 1, g.shape) for g in got]
        S.sird_adam_step(rb, dst, rb.pack_theta(grads), m, v, lo, hi, t, lr=1e-2)
        for r, f in enumerate(wl.fits):
            oracle.adam_step(th_o[r], grads[r], m_o[r], v_o[r], f.lo, f.hi, t, lr=1e-2)
    back = rb.unpack_theta(dst)
    for r in range(3):
        np.testing.assert_allclose(back[r], th_o[r], rtol=1e-14, atol=1e-14)
        assert np.all(back[r] >= wl.fits[r].lo) and np.all(back[r] <= wl.fits[r].hi)


@pytest.mark.parametrize("interval", [0, None])
def test_autograd_function_matches_oracle_gradient(interval):
    """SirdLoss: forward = sird_loss saving the adjoint's checkpoints,
    backward = the reverse sweep alone (sqrt(T) checkpoints, or the
    default 10-step ones)."""
    f = synth.c2().fits[0]
    P = 16
    th = random_theta(f, P, seed=6)
    th[:, :f.K] *= 0.5
    th[P - 4:] = near_truth(f, 4, seed=61)
    b = make_batch([f], [P])
    theta = b.pack_theta([th]).requires_grad_(True)
    obs = b.pack_obs([f.y])
    loss = SirdLoss.apply(theta, b, obs, "ssre", interval)
    w = torch.linspace(0.5, 2.0, P, dtype=torch.float64, device=theta.device)
    (loss[:P] * w).sum().backward()
    g = b.unpack_theta(theta.grad)[0]
    prob = oracle_problem(f)
    for p in range(P):
        gr, sc = oracle_grad(prob, th[p], f.y, "ssre")
        assert_grad_close(g[p], gr * w[p].item(), sc * abs(w[p].item()), f"particle {p}")
    # the same as the self-contained backward, bitwise
    g_full, L_full = S.sird_loss_backward(b, theta.detach(), obs, "ssre", grad_loss=w,
                                          loss_out=b.empty_particles())
    assert torch.equal(theta.grad, g_full) and torch.equal(loss.detach(), L_full)


def test_refine_topk_lowers_the_loss_on_noise_free_data():
    wl = synth.c1(n_part=128, iters=30)
    f = wl.fits[0]
    y = oracle.integrate(oracle_problem(f), f.truth)[3]
    b = make_batch([f], [128])
    params = S.PsoParams(b, [f.lo], [f.hi], wl.w, wl.c1, wl.c2, wl.seed)
    obs = b.pack_obs([y])
    sw = fit.run_swarm(b, params, obs, "ssre", iters=30, graph_chunk=10)
    g0 = sw.gbest_f[0].item()
    ref = fit.refine_topk(b, sw, params, obs, "ssre", k=8, max_steps=300, lr=1e-3)
    th, L = fit.best_per_problem(ref.batch, ref.theta, ref.loss)
    assert L[0] < g0
    # the refined losses are the oracle's losses at the refined parameters
    l_o = oracle.loss_batch(oracle_problem(f), ref.batch.unpack_theta(ref.theta)[0], y, "ssre")
    np.testing.assert_allclose(ref.loss.cpu().numpy()[:8], l_o, rtol=1e-10, atol=1e-14)


def test_forecast_extends_with_last_segment():
    wl = synth.c5(restarts=1, windows=[3])
    f = wl.fits[0]
    spec = S.ProblemSpec.from_fit(f, 5)
    th = random_theta(f, 5, seed=2)
    out = fit.forecast([spec], [th], 14)[0]
    assert out.shape == (5, 4, f.W + 15)
    for p in range(5):
        prob = oracle.Problem(f.W + 14, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0)
        assert_traj_close(out[p], oracle.integrate(prob, th[p]), TOL64)


def test_autotuner_candidates_agree_bitwise(tmp_path, monkeypatch):
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "cache.json"))
    wl = synth.c3(regions=list(range(64)))
    b = make_batch(wl.fits, [256] * 64)
    ths = [random_theta(f, 256, seed=r) for r, f in enumerate(wl.fits)]
    theta, obs = b.pack_theta(ths), b.pack_obs([f.y for f in wl.fits])
    b.configure(block=256, persistent=0)
    ref = S.sird_loss(b, theta, obs, "ssre").cpu().numpy()
    best = autotune.autotune(b, theta, obs, "ssre", reps=2, verbose=True)
    assert best in autotune.candidates(torch.cuda.get_device_properties(0).multi_processor_count)
    assert np.array_equal(S.sird_loss(b, theta, obs, "ssre").cpu().numpy(), ref)
    # a second call is served from the cache
    again = autotune.autotune(b, theta, obs, "ssre")
    assert again == best
    # the key separates costs; a cached shape the library refuses for this
    # batch is searched again instead of applied
    assert autotune.shape_key(b, "ssre") != autotune.shape_key(b, "mse")
    import json
    path = tmp_path / "cache.json"
    cache = json.loads(path.read_text())
    bad = dict(block=1024, persistent=0, waves_per_simd=1, ppl=1)
    cache[autotune.shape_key(b, "ssre")]["launch"] = bad
    path.write_text(json.dumps(cache))
    redo = autotune.autotune(b, theta, obs, "ssre", reps=2)
    assert redo != bad and redo in autotune.candidates(
        torch.cuda.get_device_properties(0).multi_processor_count)
    assert np.array_equal(S.sird_loss(b, theta, obs, "ssre").cpu().numpy(), ref)


def test_autotuner_of_the_fused_iteration_restores_the_swarm(tmp_path, monkeypatch):
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "cache.json"))
    wl = synth.c3(regions=list(range(16)))
    b = make_batch(wl.fits, [128] * 16)
    params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                         wl.c2, wl.seed)
    obs = b.pack_obs([f.y for f in wl.fits])
    names = ("x", "v", "pbest_x", "pbest_f", "gbest_x", "gbest_f", "gbest_idx", "iter")

    def fresh():
        sw = S.Swarm(b)
        S.pso_init(b, params, sw)
        S.sird_pso_iterate(b, params, sw, obs, "ssre", 2)
        return sw

    def bits(t):
        return t.view(torch.int64).cpu()

    b.configure(block=256, persistent=0)
    ref = fresh()
    S.sird_pso_iterate(b, params, ref, obs, "ssre", 3)
    sw = fresh()
    before = {n: bits(getattr(sw, n)) for n in names}
    best = autotune.autotune_iterate(b, params, sw, obs, "ssre", reps=2, verbose=True)
    assert best in autotune.candidates(torch.cuda.get_device_properties(0).multi_processor_count)
    for n in names:
        assert torch.equal(bits(getattr(sw, n)), before[n]), n
    # the tuned launch continues the run bitwise like the default one
    S.sird_pso_iterate(b, params, sw, obs, "ssre", 3)
    for n in names:
        assert torch.equal(bits(getattr(sw, n)), bits(getattr(ref, n))), n


@pytest.mark.parametrize("m,rounds,T", [(5, 12, 1), (32, 40, 1), (8, 16, 4)])
def test_lbfgs_rounds_match_oracle_in_lockstep(m, rounds, T):
    """Same (f, grad) inputs on both sides -> the same proposals and updates
    (the second case wraps the 32-pair memory; the third tries four steps
    per round, its trials laid out and evaluated as the trial batch's)."""
    f = synth.c2().fits[0]
    P = 40
    th = random_theta(f, P, seed=11)
    th[:, :f.K] *= 0.5
    b = make_batch([f], [P])
    lo, hi = b.pack_box([f.lo]), b.pack_box([f.hi])
    st = S.LbfgsState(b, b.pack_theta([th]), m=m, log_last=True, n_trials=T)
    tb = st.trial_batch
    assert tb.theta_len == T * b.theta_len and tb.total_particles == T * P
    ost = oracle.Lbfgs(th, m=m, log_last=True, n_trials=T)
    prob = oracle_problem(f)

    def fg(t):
        return oracle.loss_grad_fwd(prob, t, f.y, "ssre")

    for q in range(P):
        ost.f[q], ost.grad[q] = fg(th[q])
    st.f.copy_(torch.from_numpy(ost.f.copy()).cuda())
    st.grad.copy_(b.pack_theta([ost.grad]))
    kept = set()
    for rnd in range(rounds):
        S.sird_lbfgs_propose(b, st, lo, hi)
        ost.propose(f.lo, f.hi)
        tt = np.concatenate(tb.unpack_theta(st.theta_t))
        np.testing.assert_allclose(tt, ost.theta_t, rtol=1e-13, atol=1e-300, err_msg=f"round {rnd}")
        np.testing.assert_allclose(st.gp.cpu().numpy(), ost.gp, rtol=1e-12)
        # evaluate at the oracle's trial points, feed both sides the same values
        for i in range(T * P):
            ost.f_t[i], ost.grad_t[i] = fg(ost.theta_t[i])
        st.theta_t.copy_(tb.pack_theta(np.split(ost.theta_t, T)))
        st.f_t.copy_(torch.from_numpy(ost.f_t.copy()).cuda())
        st.grad_t.copy_(tb.pack_theta(np.split(ost.grad_t, T)))
        S.sird_lbfgs_accept(b, st, lo, hi, 1e-4)
        ost.accept(f.lo, f.hi, 1e-4)
        for t in range(T):
            kept |= {t for q in range(P) if np.array_equal(ost.theta_t[t * P + q], ost.theta[q])}
        np.testing.assert_allclose(b.unpack_theta(st.theta)[0], ost.theta, rtol=1e-13)
        assert np.array_equal(st.count.cpu().numpy(), ost.count)
        assert np.array_equal(st.head.cpu().numpy(), ost.head)
        np.testing.assert_allclose(st.alpha.cpu().numpy(), ost.alpha, rtol=1e-13)
    if T > 1:
        assert len(kept) > 1   # rounds kept trials other than the first


@pytest.mark.parametrize("counts,T", [((5, 17, 2), 1), ((70, 3, 40), 1), ((5, 17, 2), 4)])
def test_lbfgs_rounds_match_oracle_on_uneven_problems(counts, T):
    """Problems of different sizes and dimensions in one batch: the kernels
    run as many wavefronts per tile as the largest problem needs (below 64:
    that count; else 64), so every vector of every problem is proposed and
    accepted, in lockstep with the oracle fed the same (f, grad); with four
    trial steps, the trials of every problem in the trial batch's blocks
    and their losses from one gradient call on it."""
    wl = synth.c3(regions=[0, 1, 3])
    fits = wl.fits
    ths = [random_theta(f, n, seed=20 + i) for i, (f, n) in enumerate(zip(fits, counts))]
    b = make_batch(fits, list(counts))
    lo = b.pack_box([f.lo for f in fits])
    hi = b.pack_box([f.hi for f in fits])
    st = S.LbfgsState(b, b.pack_theta(ths), m=4, log_last=True, n_trials=T)
    tb = st.trial_batch
    osts = [oracle.Lbfgs(t, m=4, log_last=True, n_trials=T) for t in ths]
    obs = b.pack_obs([f.y for f in fits])
    probs = [oracle_problem(f) for f in fits]

    def fg(i, t):
        return oracle.loss_grad_fwd(probs[i], t, fits[i].y, "ssre")

    for i, o in enumerate(osts):
        for q in range(counts[i]):
            o.f[q], o.grad[q] = fg(i, ths[i][q])
    st.f.copy_(torch.from_numpy(np.concatenate([o.f for o in osts])).cuda())
    st.grad.copy_(b.pack_theta([o.grad for o in osts]))
    n_prob = len(fits)

    def blocks(arrs):   # oracle rows [T n][...] per problem -> trial batch order
        return [np.split(a, T)[t] for t in range(T) for a in arrs]

    for rnd in range(6):
        S.sird_lbfgs_propose(b, st, lo, hi)
        tts = tb.unpack_theta(st.theta_t)
        for i, o in enumerate(osts):
            o.propose(fits[i].lo, fits[i].hi)
            got = np.concatenate([tts[t * n_prob + i] for t in range(T)])
            np.testing.assert_allclose(got, o.theta_t, rtol=1e-13, atol=1e-300,
                                       err_msg=f"round {rnd}, problem {i}")
            for q in range(T * counts[i]):
                o.f_t[q], o.grad_t[q] = fg(i, o.theta_t[q])
        if T > 1 and rnd == 0:
            # one gradient call on the trial batch gives every trial's loss
            f_gpu = tb.empty_particles()
            S.sird_loss_backward(tb, st.theta_t, obs, "ssre", loss_out=f_gpu)
            f_split = tb.split_particles(f_gpu)
            for i, o in enumerate(osts):
                got = np.concatenate([f_split[t * n_prob + i] for t in range(T)])
                np.testing.assert_allclose(got, o.f_t, rtol=TOL64, err_msg=f"trial losses {i}")
        st.theta_t.copy_(tb.pack_theta(blocks([o.theta_t for o in osts])))
        st.f_t.copy_(torch.from_numpy(np.concatenate(blocks([o.f_t for o in osts]))).cuda())
        st.grad_t.copy_(tb.pack_theta(blocks([o.grad_t for o in osts])))
        S.sird_lbfgs_accept(b, st, lo, hi, 1e-4)
        got = b.unpack_theta(st.theta)
        for i, o in enumerate(osts):
            o.accept(fits[i].lo, fits[i].hi, 1e-4)
            np.testing.assert_allclose(got[i], o.theta, rtol=1e-13,
                                       err_msg=f"round {rnd}, problem {i}")
        assert np.array_equal(st.count.cpu().numpy(), np.concatenate([o.count for o in osts]))
        assert np.array_equal(st.head.cpu().numpy(), np.concatenate([o.head for o in osts]))
        np.testing.assert_allclose(st.alpha.cpu().numpy(),
                                   np.concatenate([o.alpha for o in osts]), rtol=1e-13)


def test_lbfgs_refinement_recovers_noise_free_truth():
    wl = synth.c1(n_part=64, iters=20)
    f = wl.fits[0]
    y = oracle.integrate(oracle_problem(f), f.truth)[3]
    b = make_batch([f], [64])
    params = S.PsoParams(b, [f.lo], [f.hi], wl.w, wl.c1, wl.c2, wl.seed)
    obs = b.pack_obs([y])
    sw = fit.run_swarm(b, params, obs, "ssre", iters=20)
    ref = fit.refine_lbfgs(b, sw, params, obs, "ssre", k=8, max_rounds=400)
    th, L = fit.best_per_problem(ref.batch, ref.theta, ref.loss)
    assert L[0] < 1e-14
    np.testing.assert_allclose(th[0], f.truth, rtol=1e-5)


def test_lbfgs_rejects_trials_outside_range():
    """The C entry points refuse n_trials outside 0..8 before any launch."""
    f = synth.c2().fits[0]
    b = make_batch([f], [8])
    lo, hi = b.pack_box([f.lo]), b.pack_box([f.hi])
    st = S.LbfgsState(b, b.pack_theta([random_theta(f, 8, seed=1)]))
    for T in (-1, 9):
        st.c.n_trials = T
        with pytest.raises(S.SirdError, match="n_trials"):
            S.sird_lbfgs_propose(b, st, lo, hi)
        with pytest.raises(S.SirdError, match="n_trials"):
            S.sird_lbfgs_accept(b, st, lo, hi)


@pytest.mark.parametrize("T", [1, 2])
def test_lbfgs_lockstep_beyond_sixteen_dimensions(T):
    """Dot products over more than 16 and more than 32 dimensions (the
    pairwise sum's levels across rows of lanes): a 22-parameter window and a
    50-parameter one (326 days in 7-day beta segments), in lockstep with the
    oracle fed the same (f, grad)."""
    import dataclasses
    wl = synth.c3(regions=[6, 7])
    base = wl.fits[0]
    K = -(-base.W // 7)
    lo, hi = synth.box(K)
    wide = dataclasses.replace(base, seg_days=7, K=K, lo=lo, hi=hi, truth=None)
    fits = [wl.fits[1], wide]
    assert [f.d for f in fits] == [22, 50]
    counts = (6, 5)
    ths = [random_theta(f, n, seed=40 + i) for i, (f, n) in enumerate(zip(fits, counts))]
    b = make_batch(fits, list(counts))
    blo = b.pack_box([f.lo for f in fits])
    bhi = b.pack_box([f.hi for f in fits])
    st = S.LbfgsState(b, b.pack_theta(ths), m=6, log_last=True, n_trials=T)
    tb = st.trial_batch
    osts = [oracle.Lbfgs(t, m=6, log_last=True, n_trials=T) for t in ths]
    probs = [oracle_problem(f) for f in fits]

    def fg(i, t):
        return oracle.loss_grad_fwd(probs[i], t, fits[i].y, "ssre")

    for i, o in enumerate(osts):
        for q in range(counts[i]):
            o.f[q], o.grad[q] = fg(i, ths[i][q])
    st.f.copy_(torch.from_numpy(np.concatenate([o.f for o in osts])).cuda())
    st.grad.copy_(b.pack_theta([o.grad for o in osts]))
    n_prob = len(fits)

    def blocks(arrs):
        return [np.split(a, T)[t] for t in range(T) for a in arrs]

    for rnd in range(8):
        S.sird_lbfgs_propose(b, st, blo, bhi)
        tts = tb.unpack_theta(st.theta_t)
        for i, o in enumerate(osts):
            o.propose(fits[i].lo, fits[i].hi)
            got = np.concatenate([tts[t * n_prob + i] for t in range(T)])
            np.testing.assert_allclose(got, o.theta_t, rtol=1e-13, atol=1e-300,
                                       err_msg=f"round {rnd}, problem {i}")
            np.testing.assert_allclose(st.gp.cpu().numpy()[b.table[i]["p_off"]:][:counts[i]],
                                       o.gp, rtol=1e-12, err_msg=f"gp, round {rnd}")
            for q in range(T * counts[i]):
                o.f_t[q], o.grad_t[q] = fg(i, o.theta_t[q])
        st.theta_t.copy_(tb.pack_theta(blocks([o.theta_t for o in osts])))
        st.f_t.copy_(torch.from_numpy(np.concatenate(blocks([o.f_t for o in osts]))).cuda())
        st.grad_t.copy_(tb.pack_theta(blocks([o.grad_t for o in osts])))
        S.sird_lbfgs_accept(b, st, blo, bhi, 1e-4)
        got = b.unpack_theta(st.theta)
        for i, o in enumerate(osts):
            o.accept(fits[i].lo, fits[i].hi, 1e-4)
            np.testing.assert_allclose(got[i], o.theta, rtol=1e-13,
                                       err_msg=f"round {rnd}, problem {i}")
        assert np.array_equal(st.count.cpu().numpy(), np.concatenate([o.count for o in osts]))
    assert int(st.count.max().item()) > 1   # the recursion ran over stored pairs
