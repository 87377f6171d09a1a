"""Pins of the oracle's costs (Sec. 3.1) on hand-computed toys.

Expected values are worked out by hand below (not by re-running the
formulas), so a wrong index range, a dropped guard or a wrong mean divisor
shows up as a mismatch.
"""
import math

import numpy as np
import pytest

# 3-day toy (days 0..3), observed cumulative deaths y and model Dhat.
Y = [0.0, 10.0, 20.0, 40.0]
DH = [0.0, 12.0, 17.0, 40.0]
# e = y - Dhat = [0, -2, 3, 0], n = 4


def test_ssre_toy(orc):
    # ((12-10)/10)^2 + ((17-20)/20)^2 + 0 = 0.04 + 0.0225
    assert orc.loss("ssre", DH, Y) == pytest.approx(0.0625, rel=1e-15)


def test_mse_toy(orc):
    # (0 + 4 + 9 + 0)/4
    assert orc.loss("mse", DH, Y) == pytest.approx(3.25, rel=1e-15)


def test_mxse_toy(orc):
    assert orc.loss("mxse", DH, Y) == 9.0


def test_mae_toy(orc):
    # (0 + 2 + 3 + 0)/4
    assert orc.loss("mae", DH, Y) == pytest.approx(1.25, rel=1e-15)


def test_mape_toy(orc):
    # 100/4 * (0 + 2/10 + 3/20 + 0) = 25 * 0.35
    assert orc.loss("mape", DH, Y) == pytest.approx(8.75, rel=1e-14)


def test_guard_for_small_observations(orc):
    # y = 0 and y = 0.5 are divided by max(y, 1) = 1
    y = [0.0, 0.0, 0.5]
    dh = [0.0, 3.0, 2.5]
    assert orc.loss("ssre", dh, y) == pytest.approx(9.0 + 4.0, rel=1e-15)
    assert orc.loss("mape", dh, y) == pytest.approx(100.0 / 3 * (3.0 + 2.0), rel=1e-14)


def test_ssre_skips_day_zero_others_include_it(orc):
    # an error on day 0 only: SSRE ignores it, the paper's costs count it
    y = [5.0, 10.0]
    dh = [3.0, 10.0]
    assert orc.loss("ssre", dh, y) == 0.0
    assert orc.loss("mse", dh, y) == pytest.approx(2.0, rel=1e-15)   # 4/2
    assert orc.loss("mxse", dh, y) == 4.0
    assert orc.loss("mae", dh, y) == pytest.approx(1.0, rel=1e-15)   # 2/2
    assert orc.loss("mape", dh, y) == pytest.approx(20.0, rel=1e-14)  # 100/2 * 2/5


def test_nan_propagates_for_every_kind(orc):
    dh = [0.0, 1.0, float("nan"), 3.0]
    y = [0.0, 1.0, 2.0, 3.0]
    for k in ("ssre", "mse", "mxse", "mae", "mape"):
        assert math.isnan(orc.loss(k, dh, y)), k


def test_losses_brute_force_random(orc):
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = int(rng.integers(2, 40))
        y = np.cumsum(rng.integers(0, 50, n)).astype(float)
        dh = y + rng.normal(0, 5, n)
        e = [float(a) - float(b) for a, b in zip(y, dh)]
        g = [max(float(a), 1.0) for a in y]
        # brute force over python floats, summing in a different order
        ssre = math.fsum(((float(dh[i]) - float(y[i])) / g[i]) ** 2 for i in range(1, n))
        mse = math.fsum(x * x for x in e) / n
        mxse = max(x * x for x in e)
        mae = math.fsum(abs(x) for x in e) / n
        mape = 100.0 * math.fsum(abs(e[i] / g[i]) for i in range(n)) / n
        assert orc.loss("ssre", dh, y) == pytest.approx(ssre, rel=1e-12)
        assert orc.loss("mse", dh, y) == pytest.approx(mse, rel=1e-12)
        assert orc.loss("mxse", dh, y) == mxse
        assert orc.loss("mae", dh, y) == pytest.approx(mae, rel=1e-12)
        assert orc.loss("mape", dh, y) == pytest.approx(mape, rel=1e-12)


def test_loss_batch_equals_single(orc):
    prob = orc.Problem(W=30, spd=10, seg_days=14, K=3, N=3.8e7)
    rng = np.random.default_rng(1)
    th = np.column_stack([rng.uniform(0, 1, (16, 3)), rng.uniform(0, .5, 16),
                          rng.uniform(0, .05, 16), rng.uniform(1e2, 1e5, 16)])
    y = np.cumsum(rng.integers(0, 30, 31)).astype(float)
    y[0] = 0
    for kind in ("ssre", "mse", "mxse", "mae", "mape"):
        lb = orc.loss_batch(prob, th, y, kind, nthreads=2)
        for p in range(16):
            assert lb[p] == orc.loss(kind, orc.integrate(prob, th[p])[3], y)
