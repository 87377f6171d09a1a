"""GPU parity of the paper's own scheme against the oracle, through the C
ABI: forward Euler with the ramp of eq. (beta) (Sec. 3.1, 3.3), the F_IRD
costs over I, R and D (Sec. 3.1), batches that mix it with the RK4 segment
model, and swarm runs that keep t1 <= t2."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2204_12346_amd as S
from gpu_helpers import (TOL32, TOL64, assert_loss_close, assert_traj_close,
                         assert_traj_close_f32, format_worst, kappa, kappa_ird, make_batch,
                         need_gpu, oracle_problem_model)
from gpu_helpers import compared_iterations, loss_discrepancy

pytestmark = pytest.mark.gpu

KINDS_D = ["ssre", "mse", "mxse", "mae", "mape"]
KINDS_IRD = ["ird_mxse", "ird_mse", "ird_mae", "ird_mape"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _thetas(f, P, seed):
    """Random vectors in the box, with rows where t1 > t2 and t1 == t2."""
    rng = np.random.default_rng(seed)
    th = f.lo + rng.uniform(0, 1, (P, f.d)) * (f.hi - f.lo)
    th[0, 2:4] = [40.0, 12.0]      # t1 > t2: beta1 until t1, then beta2
    th[1, 2:4] = [30.0, 30.0]      # a step instead of a ramp
    th[2, 2:4] = [0.0, 85.0]       # ramp over the whole window
    th[3, :2] = 0.0                # no transmission
    th[4, 2:4] = [17.5, 17.5 + 1e-13]
    return th


def _batch(fits, n_parts, **kw):
    return make_batch(fits, n_parts, obs_series=3, **kw)


@pytest.mark.parametrize("spd", [1, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ramp_trajectories(spd, dtype):
    f = synth.paper().fits[0]
    f.spd = spd
    P = 130
    th = _thetas(f, P, seed=1)
    b = make_batch([f], [P], dtype=dtype, with_traj=True)
    tr = b.unpack_traj(S.sird_integrate(b, b.pack_theta([th])))[0]
    prob = oracle_problem_model(f)
    worst = {}
    for p in range(P):
        ref = oracle.integrate_model(prob, th[p])
        if dtype == "f64":
            assert_traj_close(tr[p], ref, TOL64, f"particle {p}")
        else:
            assert_traj_close_f32(tr[p], ref, TOL32, f"particle {p}", worst, f"particle {p}")
    if worst:
        print(f"ramp model, {spd} steps per day, FP32 state: worst per-value relative error "
              + format_worst(worst))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ramp_losses_all_kinds(dtype):
    f = synth.paper().fits[0]
    P = 200  # three full tiles and a ragged one
    th = _thetas(f, P, seed=2)
    b = _batch([f], [P], dtype=dtype)
    theta = b.pack_theta([th])
    obs = b.pack_obs([f.obs3])
    prob = oracle_problem_model(f)
    trajs = [oracle.integrate_model(prob, t) for t in th]
    eps = TOL64 if dtype == "f64" else TOL32
    for kind in KINDS_D + KINDS_IRD:
        print(f"case ramp loss {dtype} {kind}", flush=True)
        got = S.sird_loss(b, theta, obs, kind).cpu().numpy()[:P]
        o = f.obs3 if kind.startswith("ird") else f.y
        ref = oracle.loss_batch_model(prob, th, o, kind)
        if kind.startswith("ird"):
            kap = [kappa_ird(kind, t, f.obs3) for t in trajs]
        else:
            kap = [kappa(kind, t[3], f.y) for t in trajs]
        assert_loss_close(got, ref, kap, eps, f"{dtype}/{kind}")


def _rk4_fit_with_three_series():
    """The constant-beta RK4 window with I, R, D observations (the truth's
    trajectory scaled by 1.02, so no particle fits exactly)."""
    f = synth.c1().fits[0]
    truth = oracle.integrate(oracle.Problem(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0),
                             f.truth)
    f.obs3 = (1.02 * truth[1:]).reshape(-1)
    return f


def test_rk4_model_with_ird_costs():
    f = _rk4_fit_with_three_series()
    P = 100
    rng = np.random.default_rng(3)
    th = f.lo + rng.uniform(0, 1, (P, f.d)) * (f.hi - f.lo)
    b = _batch([f], [P])
    prob = oracle_problem_model(f)
    trajs = [oracle.integrate(prob, t) for t in th]
    for kind in KINDS_IRD + ["ssre"]:
        print(f"case rk4 {kind}", flush=True)
        got = S.sird_loss(b, b.pack_theta([th]), b.pack_obs([f.obs3]), kind).cpu().numpy()[:P]
        o = f.obs3 if kind.startswith("ird") else f.obs3[-(f.W + 1):]
        ref = oracle.loss_batch_model(prob, th, o, kind)
        kap = ([kappa_ird(kind, t, f.obs3) for t in trajs] if kind.startswith("ird")
               else [kappa(kind, t[3], o) for t in trajs])
        assert_loss_close(got, ref, kap, TOL64, kind)


@pytest.mark.parametrize("persistent", [0, 24])
def test_mixed_model_batch_equals_single_batches(persistent):
    fr = synth.paper().fits[0]
    fk = _rk4_fit_with_three_series()
    fits = [fk, fr, fk, fr]
    n_parts = [70, 130, 1, 64]
    ths = []
    for r, (f, n) in enumerate(zip(fits, n_parts)):
        rng = np.random.default_rng(10 + r)
        ths.append(f.lo + rng.uniform(0, 1, (n, f.d)) * (f.hi - f.lo))
    b = _batch(fits, n_parts, persistent=persistent)
    assert b.c.models == 3
    obs = b.pack_obs([f.obs3 for f in fits])
    for kind in ("ird_mxse", "mae"):
        print(f"case mixed persistent={persistent} {kind}", flush=True)
        per = b.split_particles(S.sird_loss(b, b.pack_theta(ths), obs, kind))
        for r, f in enumerate(fits):
            one = _batch([f], [n_parts[r]])
            l1 = S.sird_loss(one, one.pack_theta([ths[r]]), one.pack_obs([f.obs3]), kind)
            assert np.array_equal(l1.cpu().numpy()[:n_parts[r]], per[r]), (kind, r)
    # a second launch reuses the persistent counters
    again = b.split_particles(S.sird_loss(b, b.pack_theta(ths), obs, "mae"))
    assert all(np.array_equal(x, y) for x, y in zip(again, per))


def test_swarm_init_orders_ramp_times_bitwise():
    f = synth.paper().fits[0]
    P = 300
    b = _batch([f], [P])
    params = S.PsoParams(b, [f.lo], [f.hi], 0.5, 0.5, 0.5, seed=6)
    sw = S.Swarm(b)
    S.pso_init(b, params, sw)
    ref = oracle.pso_init(P, f.lo, f.hi, 6, f.stream)
    oracle.pso_sort_pair(ref)
    x = b.unpack_theta(sw.x)[0]
    assert np.array_equal(x, ref.x)
    assert np.array_equal(b.unpack_theta(sw.pbest_x)[0], ref.x)
    assert np.all(x[:, 2] <= x[:, 3])


def _compare_runs_with_oracle(wl, fits, b, sw, min_compared):
    """Every fit's gbest sequence against the oracle's run of it, up to the
    first near-tie (threshold from the measured loss discrepancy at the
    personal bests)."""
    iters = wl.iters
    hist_i, hist_f = sw.hist_idx.cpu().numpy(), sw.hist_f.cpu().numpy()
    pbx, pbf = b.unpack_theta(sw.pbest_x), b.split_particles(sw.pbest_f)
    runs, delta = [], 0.0
    for r, f in enumerate(fits):
        prob = oracle_problem_model(f)
        runs.append(oracle.pso_run_model(prob, f.obs3, wl.loss, f.n_part, f.lo, f.hi, wl.w,
                                         wl.c1, wl.c2, wl.seed, f.stream, iters))
        at_pbest = oracle.loss_batch_model(prob, pbx[r], f.obs3, wl.loss)
        delta = max(delta, loss_discrepancy(pbf[r], at_pbest))
    assert delta < 1e-11, f"personal-best losses off the oracle's by {delta:.2e}"
    for r, (hf, hidx, hm, _) in enumerate(runs):
        upto, thr = compared_iterations(hm, delta, iters)
        print(f"fit {r}: loss discrepancy {delta:.2e}, near-tie threshold {thr:.1e}, "
              f"comparing {upto} of {iters} iterations", flush=True)
        assert upto >= min_compared, f"fit {r}: oracle near-tie too early ({upto})"
        np.testing.assert_array_equal(hist_i[:upto, r], hidx[:upto])
        np.testing.assert_allclose(hist_f[:upto, r], hf[:upto], rtol=1e-11)


@pytest.mark.parametrize("graph_chunk", [0, 5])
def test_swarm_run_matches_oracle(graph_chunk):
    """The paper's timing case as configured (Sec. 3.3): 10000 particles x
    100 iterations of the F_IRD^MXSE fit, forward Euler with the ramp."""
    wl = synth.paper()
    f = wl.fits[0]
    P, iters = f.n_part, wl.iters
    b = _batch([f], [P])
    params = S.PsoParams(b, [f.lo], [f.hi], wl.w, wl.c1, wl.c2, wl.seed)
    obs = b.pack_obs([f.obs3])
    from paper_2204_12346_amd import fit
    sw = S.Swarm(b, hist_len=iters)
    fit.run_swarm(b, params, obs, wl.loss, iters=iters, graph_chunk=graph_chunk, swarm=sw)
    torch.cuda.synchronize()
    x = b.unpack_theta(sw.x)[0]
    px = b.unpack_theta(sw.pbest_x)[0]
    assert np.all(x[:, 2] <= x[:, 3]) and np.all(px[:, 2] <= px[:, 3])
    assert np.all(x >= f.lo) and np.all(x <= f.hi)
    _compare_runs_with_oracle(wl, [f], b, sw, min_compared=50)


def test_repetitions_match_oracle():
    """Two fits of the repetition study (Sec. 4.2) as configured, 10000
    particles x 100 iterations each with their own Philox streams, in one
    batch, each against the oracle's run."""
    wl = synth.rep(n_rep=2)
    fits = wl.fits
    b = _batch(fits, [f.n_part for f in fits])
    params = S.PsoParams(b, [f.lo for f in fits], [f.hi for f in fits], wl.w, wl.c1, wl.c2,
                         wl.seed)
    sw = S.Swarm(b, hist_len=wl.iters)
    S.pso_init(b, params, sw)
    S.sird_pso_iterate(b, params, sw, b.pack_obs([f.obs3 for f in fits]), wl.loss, wl.iters)
    torch.cuda.synchronize()
    _compare_runs_with_oracle(wl, fits, b, sw, min_compared=40)


def test_repetition_batch_equals_single_fits():
    """The repetition study's batch (one window, fits with their own Philox
    streams) runs every fit exactly as a batch of that fit alone."""
    wl = synth.rep(n_rep=6, n_part=100, iters=12)
    fits = wl.fits
    b = _batch(fits, [f.n_part for f in fits])
    params = S.PsoParams(b, [f.lo for f in fits], [f.hi for f in fits], wl.w, wl.c1, wl.c2,
                         wl.seed)
    sw = S.Swarm(b, hist_len=wl.iters)
    obs = b.pack_obs([f.obs3 for f in fits])
    S.pso_init(b, params, sw)
    S.sird_pso_iterate(b, params, sw, obs, wl.loss, wl.iters)
    hist = sw.hist_f.cpu().numpy()
    for r, f in enumerate(fits):
        one = _batch([f], [f.n_part])
        p1 = S.PsoParams(one, [f.lo], [f.hi], wl.w, wl.c1, wl.c2, wl.seed)
        s1 = S.Swarm(one, hist_len=wl.iters)
        S.pso_init(one, p1, s1)
        S.sird_pso_iterate(one, p1, s1, one.pack_obs([f.obs3]), wl.loss, wl.iters)
        assert np.array_equal(s1.hist_f.cpu().numpy()[:, 0], hist[:, r]), r
        assert np.array_equal(one.unpack_box(s1.gbest_x)[0], b.unpack_box(sw.gbest_x)[r])
    # different streams explore differently
    assert len({tuple(h) for h in hist.T}) > 1


def test_ramp_extension_stays_at_beta2():
    from paper_2204_12346_amd import fit
    f = synth.rep(n_rep=1).fits[0]
    th = _thetas(f, 5, seed=4)
    th[:, 2:4] = np.sort(np.minimum(th[:, 2:4], f.W - 7.0), axis=1)
    spec = S.ProblemSpec.from_fit(f, 5)
    out = fit.forecast([spec], [th], 21)[0]
    prob = oracle.Problem(f.W + 21, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0, model=1)
    for p in range(5):
        assert_traj_close(out[p], oracle.integrate_model(prob, th[p]), TOL64, f"particle {p}")


def test_ramp_edge_cases_against_oracle():
    """One-day and ragged windows, several steps per day, a problem with no
    particles, a flat observed series (normalised by 1) and NaN parameters."""
    N = 1e6
    rng = np.random.default_rng(8)
    specs, ths, obs, probs = [], [], [], []
    for W, spd, n in ((1, 1, 3), (2, 3, 65), (5, 2, 0), (13, 1, 64)):
        specs.append(S.ProblemSpec(W, spd, 1, 4, N, R0=100.0, D0=10.0, n_part=n,
                                   model="euler_ramp"))
        lo = np.array([0, 0, 0, 0, 0, 0, 500.0])
        hi = np.array([1, 1, W, W, 0.5, 0.05, 500.0])
        ths.append(lo + rng.uniform(0, 1, (n, 7)) * (hi - lo))
        o = rng.uniform(0, 1000, (3, W + 1))
        o[2] = 7.0  # flat deceased series
        obs.append(o.reshape(-1))
        probs.append(oracle.Problem(W, spd, 1, 4, N, R0=100.0, D0=10.0, model=1))
    ths[3][5, 4] = np.nan
    b = S.Batch(specs, obs_series=3)
    theta, ob = b.pack_theta(ths), b.pack_obs(obs)
    for kind in KINDS_IRD + ["mse"]:
        print(f"case ramp edges {kind}", flush=True)
        got = b.split_particles(S.sird_loss(b, theta, ob, kind))
        for r, s in enumerate(specs):
            if s.n_part == 0:
                continue
            o = obs[r] if kind.startswith("ird") else obs[r][-(s.W + 1):]
            ref = oracle.loss_batch_model(probs[r], ths[r], o, kind)
            trajs = [oracle.integrate_model(probs[r], t) for t in ths[r]]
            kap = [kappa_ird(kind, t, obs[r]) if kind.startswith("ird") else kappa(kind, t[3], o)
                   for t in trajs]
            assert_loss_close(got[r], ref, np.nan_to_num(kap), TOL64, f"{kind}/problem {r}")
    assert np.isnan(got[3][5])
