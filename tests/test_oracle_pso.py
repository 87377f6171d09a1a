"""Pins of the oracle's particle swarm (Sec. 3.3).

Random numbers are re-derived from numpy's independent Philox generator; the
update is checked on a hand-worked step, on special cases that freeze parts
of the update, on invariants (box, monotone bests, lowest-index argmin) and
on convergence for a sphere function.
"""
import numpy as np
import pytest


def np_block(it, p, m, purpose, seed, stream):
    # numpy increments its counter before encrypting: start one below
    ctr = np.array([it, p, m, purpose], dtype=np.uint64)
    val = sum(int(w) << (64 * i) for i, w in enumerate(ctr)) - 1
    words = np.array([(val >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    return np.random.Philox(key=np.array([seed, stream], dtype=np.uint64),
                            counter=words).random_raw(4)


def u(w):
    return float(int(w) >> 11) * 2.0 ** -53


def test_init_uses_counter_blocks(orc):
    lo = np.array([0.0, 0.0, 0.0, 100.0, -2.0])
    hi = np.array([1.0, 0.5, 0.05, 1e5, 2.0])
    s = orc.pso_init(7, lo, hi, seed=1, stream=9)
    for p in range(7):
        for j in range(5):
            w = np_block(0, p, j // 2, 0, 1, 9)
            uj = u(w[2 * (j % 2)])
            assert s.x[p, j] == lo[j] + uj * (hi[j] - lo[j])
    assert np.all(s.v == 0) and np.all(s.pbest_x == s.x)
    assert np.all(np.isinf(s.pbest_f)) and np.isinf(s.gbest_f[0]) and s.gbest_idx[0] == -1


def test_one_step_by_hand(orc):
    # two particles in 6-D (two Philox blocks), hand-set state; r from
    # numpy's Philox, dimension j in slot (j + 3) mod d
    d = 6
    lo, hi = np.zeros(d), np.ones(d)
    s = orc.pso_init(2, lo, hi, seed=5, stream=2)
    s.x[:] = [[0.5, 0.25, 0.75, 0.125, 0.625, 0.375], [0.125, 0.5, 0.875, 0.25, 0.0, 1.0]]
    s.v[:] = [[0.0625, -0.125, 0.25, 0.5, -0.5, 0.0], [0.5, 0.0, -0.25, 0.125, 0.75, -1.0]]
    s.pbest_x[:] = [[0.25, 0.5, 1.0, 0.0, 0.75, 0.5], [0.0, 0.75, 0.5, 1.0, 0.25, 0.5]]
    s.gbest_x[:] = [0.0, 0.75, 0.5, 1.0, 0.25, 0.5]
    w, c1, c2, it = 0.7, 1.5, 1.5, 3
    x0, v0 = s.x.copy(), s.v.copy()
    orc.pso_move(s, it, w, c1, c2, lo, hi, seed=5, stream=2)
    for p in range(2):
        for j in range(d):
            slot = (j + 3) % d
            word = int(np_block(it, p, slot // 4, 1, 5, 2)[slot % 4])
            r1, r2 = (word >> 32) * 2.0 ** -32, (word & 0xFFFFFFFF) * 2.0 ** -32
            t = w * v0[p, j]
            t = t + (c1 * r1) * (s.pbest_x[p, j] - x0[p, j])
            t = t + (c2 * r2) * (s.gbest_x[j] - x0[p, j])
            assert s.v[p, j] == t
            assert s.x[p, j] == min(max(x0[p, j] + t, 0.0), 1.0)


def test_no_attraction_means_pure_inertia(orc):
    lo, hi = np.zeros(4), np.full(4, 10.0)
    s = orc.pso_init(5, lo, hi, seed=3)
    s.v[:] = 0.25
    s.pbest_x[:] = s.x
    s.gbest_x[:] = 5.0
    x0 = s.x.copy()
    orc.pso_move(s, 0, 0.5, 1.5, 0.0, lo, hi, seed=3)  # c2 = 0, pb == x
    assert np.all(s.v == 0.125)
    assert np.all(s.x == np.clip(x0 + 0.125, 0, 10))


def test_clamp_to_box(orc):
    lo, hi = np.array([0.0, 1.0]), np.array([1.0, 2.0])
    s = orc.pso_init(3, lo, hi, seed=1)
    s.v[:] = [[5.0, -5.0], [-5.0, 5.0], [0.0, 0.0]]
    s.pbest_x[:] = s.x
    s.gbest_x[:] = s.x[0]
    orc.pso_move(s, 0, 1.0, 0.0, 0.0, lo, hi, seed=1)
    assert list(s.x[0]) == [1.0, 1.0]
    assert list(s.x[1]) == [0.0, 2.0]


def test_degenerate_box_dimension_stays_fixed(orc):
    lo = np.array([0.0, 1000.0])
    hi = np.array([1.0, 1000.0])
    s = orc.pso_init(16, lo, hi, seed=1)
    assert np.all(s.x[:, 1] == 1000.0)
    for it in range(5):
        f = (s.x[:, 0] - 0.3) ** 2
        orc.pso_bests(s, f)
        orc.pso_move(s, it, 0.7, 1.5, 1.5, lo, hi, seed=1)
        assert np.all(s.x[:, 1] == 1000.0) and np.all(s.v[:, 1] == 0.0)


def test_bests_ties_nan_and_strictness(orc):
    lo, hi = np.zeros(2), np.ones(2)
    s = orc.pso_init(4, lo, hi, seed=2)
    orc.pso_bests(s, np.array([np.nan, 3.0, 1.0, 1.0]))
    assert np.isinf(s.pbest_f[0])                      # NaN counts as +inf
    assert s.gbest_idx[0] == 2 and s.gbest_f[0] == 1.0  # tie -> lowest index
    assert np.all(s.gbest_x == s.pbest_x[2])
    x2 = s.pbest_x[2].copy()
    s.x[:] = 0.5
    orc.pso_bests(s, np.array([5.0, 3.0, 1.0, 0.5]))  # equal f: no pbest change
    assert np.all(s.pbest_x[2] == x2)
    assert s.gbest_idx[0] == 3 and s.gbest_f[0] == 0.5
    orc.pso_bests(s, np.array([0.5, 9.0, 9.0, 9.0]))  # equal to gbest: keep old
    assert s.gbest_idx[0] == 3


def test_invariants_on_a_real_problem(orc):
    prob = orc.Problem(W=40, spd=5, seg_days=40, K=1, N=3.8e7)
    truth = orc.integrate(prob, [0.25, 0.1, 0.002, 1000.0])[3]
    lo = np.array([0.0, 0.0, 0.0, 1000.0])
    hi = np.array([1.0, 0.5, 0.05, 1000.0])
    s = orc.pso_init(32, lo, hi, seed=1)
    prev_pb, prev_g = s.pbest_f.copy(), np.inf
    for it in range(15):
        f = orc.loss_batch(prob, s.x, truth, "ssre")
        orc.pso_bests(s, f)
        assert np.all(s.pbest_f <= prev_pb)
        assert s.gbest_f[0] <= prev_g
        assert s.gbest_f[0] == s.pbest_f.min()
        assert s.gbest_idx[0] == int(np.argmin(s.pbest_f))
        prev_pb, prev_g = s.pbest_f.copy(), s.gbest_f[0]
        orc.pso_move(s, it, 0.7, 1.5, 1.5, lo, hi, seed=1)
        assert np.all(s.x >= lo) and np.all(s.x <= hi)


def test_sphere_convergence(orc):
    d = 4
    lo, hi = np.full(d, -5.0), np.full(d, 5.0)
    a = np.array([1.0, -2.0, 0.5, 3.0])
    s = orc.pso_init(64, lo, hi, seed=4)
    for it in range(150):
        f = ((s.x - a) ** 2).sum(axis=1)
        orc.pso_bests(s, f)
        orc.pso_move(s, it, 0.7, 1.5, 1.5, lo, hi, seed=4)
    assert s.gbest_f[0] < 1e-6
    np.testing.assert_allclose(s.gbest_x, a, atol=1e-3)


def test_run_equals_stepwise_and_resume(orc):
    prob = orc.Problem(W=30, spd=4, seg_days=14, K=3, N=3.8e7)
    th = [0.3, 0.2, 0.1, 0.1, 0.002, 1000.0]
    y = orc.integrate(prob, th)[3]
    lo = np.array([0, 0, 0, 0, 0, 1e2])
    hi = np.array([1, 1, 1, .5, .05, 1e5])
    hf, hidx, hm, final = orc.pso_run(prob, y, "ssre", 24, lo, hi, 0.7, 1.5, 1.5, 7, 3, 12)
    s = orc.pso_init(24, lo, hi, seed=7, stream=3)
    for it in range(12):
        if it == 6:  # "save and load" half-way: a copy continues identically
            s = s.copy()
        f = orc.loss_batch(prob, s.x, y, "ssre")
        orc.pso_bests(s, f)
        assert s.gbest_f[0] == hf[it] and s.gbest_idx[0] == hidx[it]
        if it < 11:
            orc.pso_move(s, it, 0.7, 1.5, 1.5, lo, hi, seed=7, stream=3)
    assert np.array_equal(s.x, final.x) and np.array_equal(s.pbest_f, final.pbest_f)
    assert np.all(np.diff(hf) <= 0)


def _bests_case(orc, pbest_f, f, gbest_f):
    """Swarm of len(pbest_f) particles in 2-D with the given personal bests
    and global best; returns (margin, swarm) after pso_bests(f)."""
    P = len(pbest_f)
    s = orc.pso_init(P, np.zeros(2), np.ones(2), seed=1)
    s.pbest_f[:] = pbest_f
    s.gbest_f[0] = gbest_f
    s.gbest_idx[0] = -1 if np.isinf(gbest_f) else 0
    m = orc.pso_bests(s, np.array(f, dtype=np.float64))
    return m, s


# The near-tie margin is the smallest relative gap |a - b| / max(|a|, |b|)
# over the comparisons that decided an outcome of the update (Sec. 3.3's
# personal and global bests).  Each case below makes one of the three kinds
# of comparison the smallest, with dyadic gaps whose value is exact.
def test_margin_personal_best_comparison_decides(orc):
    # f vs pbest: 4 vs 3 -> 1/4, 30 vs 32 -> 1/16 (improves); winner 3 vs
    # runner-ups 30, 100: 0.9, 0.97; the global best stays 3 (no decision)
    m, s = _bests_case(orc, [3.0, 32.0, 100.0], [4.0, 30.0, np.nan], 3.0)
    assert m == 0.0625
    assert list(s.pbest_f) == [3.0, 30.0, 100.0]


def test_margin_winner_vs_runner_up_decides(orc):
    # no finite f: no personal-best comparison; argmin 15 vs 16 -> 1/16,
    # vs 40 -> 0.625; no previous global best
    m, s = _bests_case(orc, [16.0, 15.0, 40.0], [np.nan] * 3, np.inf)
    assert m == 0.0625
    assert s.gbest_idx[0] == 1 and s.gbest_f[0] == 15.0


def test_margin_new_best_vs_previous_global_best_decides(orc):
    # winner 7 vs runner-up 50: 0.86; 7 replaces the global best 8: 1/8
    m, s = _bests_case(orc, [7.0, 50.0], [np.nan, np.nan], 8.0)
    assert m == 0.125
    assert s.gbest_idx[0] == 0 and s.gbest_f[0] == 7.0


def test_margin_excludes_equal_values_and_unchanged_best(orc):
    # f equal to pbest (both particles) and the exact tie 5 == 5 between
    # particles 0 and 1 decide identically in any implementation; the
    # global best equal to the winner is unchanged: only 5 vs 40 counts
    m, s = _bests_case(orc, [5.0, 5.0, 40.0], [5.0, 5.0, np.nan], 5.0)
    assert m == 0.875
    assert s.gbest_idx[0] == 0


def test_margin_excludes_non_finite_sides(orc):
    # pbest +inf (never evaluated) vs f = 3 is no near decision; 8 vs 4 ->
    # 0.5; afterwards 3 vs 4 -> 0.25
    m, _ = _bests_case(orc, [np.inf, 4.0], [3.0, 8.0], np.inf)
    assert m == 0.25
    # nothing finite decided anything
    m, _ = _bests_case(orc, [np.inf], [np.nan], np.inf)
    assert m == np.inf


def test_run_records_the_margin_of_each_update(orc):
    prob = orc.Problem(W=20, spd=2, seg_days=20, K=1, N=1e6)
    y = orc.integrate(prob, [0.3, 0.1, 0.01, 100.0])[3]
    lo, hi = np.array([0.0, 0.0, 0.0, 100.0]), np.array([1.0, 0.5, 0.05, 100.0])
    hf, hidx, hm, _ = orc.pso_run(prob, y, "ssre", 16, lo, hi, 0.7, 1.5, 1.5, 3, 0, 6)
    s = orc.pso_init(16, lo, hi, seed=3)
    for it in range(6):
        m = orc.pso_bests(s, orc.loss_batch(prob, s.x, y, "ssre"))
        assert m == hm[it] and s.gbest_idx[0] == hidx[it]
        orc.pso_move(s, it, 0.7, 1.5, 1.5, lo, hi, seed=3)
