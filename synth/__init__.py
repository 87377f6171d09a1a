"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds no arithmetic of the method: it draws parameters, shapes
and count noise, and loads the stored observation series.  Truth
trajectories are produced by the oracle in ``synth/make_series.py`` (a
committed script that calls only the oracle) and stored under
``synth/series/``; both sides read the same stored numbers.

The workloads stand in for the paper's Polish OxCOVID19 series (Sec. 2.1),
which is not available: "Poland-shaped" means a population of 3.8e7, daily
cumulative deaths, and fitting windows of weeks to a year (Sec. 3.1 uses
36-day windows; the batched workload spans 28..365 days).

Workloads (names follow the calibration setups they model):
  c1  constant beta, 60-day window, 256 particles x 200 iterations
  c2  13 two-week beta segments, 180-day window, 8192 x 1000
  c3  512 independent regions of uneven window and population, 1024 x 500
  c4  65536 parameter vectors on a 365-day window at dt = 0.05 (gradients)
  c5  52 weekly-shifted 42-day windows of a 414-day series with regime
      changes, 16 restarts x 4096 x 300, then refinement and a 14-day forecast
  paper  the paper's own timing case (Sec. 3.3): one 92-day window (93 daily
      observations of I, R and D), forward Euler at one step per day with the
      ramp of eq. (beta), cost F_IRD^MXSE, 10000 particles, coefficients
      0.5/0.5/0.5, 100 iterations, box of the paper's second run
  rep  the repetition study (Sec. 4.2): one 36-day window of the same series
      (tau = 35) fitted 1000 times with independent Philox streams, each fit
      with the paper's swarm (10000 particles, 100 iterations)
  windows  the window-wise calibration (Sec. 3.1, 4.1): a 450-day series of
      I, R, D with regime changes, cut into 139 windows of 36 days shifted
      by 3 days (tau = 35, delta = 3), each fitted with the paper's scheme,
      F_IRD^MXSE and the paper's swarm
"""
from __future__ import annotations

import dataclasses
import os
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SERIES_DIR = os.path.join(HERE, "series")

POLAND_N = 3.8e7
NB_DISPERSION = 10.0

# PSO coefficients of the synthetic workloads (inertia, cognitive, social)
PSO_W, PSO_C1, PSO_C2 = 0.7, 1.5, 1.5


@dataclasses.dataclass
class Fit:
    """One calibration window.  theta = (beta_1..beta_K, gamma, mu, I0)."""
    W: int
    spd: int
    seg_days: int
    K: int
    N: float
    R0: float
    D0: float
    lo: np.ndarray
    hi: np.ndarray
    y: np.ndarray                 # observed cumulative deaths, days 0..W
    n_part: int
    stream: int                   # Philox key word 1 of this fit
    truth: Optional[np.ndarray] = None
    obs3: Optional[np.ndarray] = None  # I, R, D observations (3 (W+1) values)
    model: str = "rk4"                 # or "euler_ramp"

    @property
    def d(self):
        return self.K + 3

    @property
    def T(self):
        return self.W * self.spd


@dataclasses.dataclass
class Workload:
    name: str
    fits: List[Fit]
    iters: int
    seed: int                     # Philox key word 0
    loss: str = "ssre"
    w: float = PSO_W
    c1: float = PSO_C1
    c2: float = PSO_C2

    @property
    def particles(self):
        return sum(f.n_part for f in self.fits)

    @property
    def particle_steps_per_iter(self):
        return sum(f.n_part * f.T for f in self.fits)


def box(K, I0_lo=1e2, I0_hi=1e5):
    """Search box: beta in [0,1], gamma in [0,0.5], mu in [0,0.05], I0 as given."""
    lo = np.array([0.0] * K + [0.0, 0.0, I0_lo])
    hi = np.array([1.0] * K + [0.5, 0.05, I0_hi])
    return lo, hi


def noisy_cumulative(D_truth, kind, rng, r=NB_DISPERSION):
    """Observed cumulative series from a truth cumulative series: daily
    increments m_i = D(i) - D(i-1) get Poisson(m_i) or negative-binomial
    (mean m_i, variance m_i + m_i^2/r) noise; y_0 = D(0)."""
    D = np.asarray(D_truth, dtype=np.float64)
    m = np.maximum(np.diff(D), 0.0)
    if kind == "poisson":
        inc = rng.poisson(m)
    elif kind == "negbin":
        inc = np.where(m > 0, rng.negative_binomial(r, r / (r + np.where(m > 0, m, 1.0))), 0)
    elif kind == "none":
        return D.copy()
    else:
        raise ValueError(kind)
    return np.concatenate([[D[0]], D[0] + np.cumsum(inc)]).astype(np.float64)


# ----------------------------------------------------------- draws only
def c1_truth():
    return np.array([0.25, 0.1, 0.002, 1000.0])


def c2_truth():
    rng = np.random.default_rng(2)
    return np.concatenate([rng.uniform(0.05, 0.4, 13), [0.1, 0.002, 1000.0]])


def c3_regions(n=512):
    """Per-region draws: N log-uniform [1e5,1e8], W uniform {28..365},
    K = ceil(W/14), beta_k ~ U[0.05,0.4], gamma ~ U[0.05,0.2],
    mu ~ U[0.001,0.01], I0 log-uniform [1e2, min(1e4, N/100)]."""
    out = []
    for child in np.random.SeedSequence(3).spawn(n):
        rng = np.random.default_rng(child)
        N = float(10 ** rng.uniform(5, 8))
        W = int(rng.integers(28, 366))
        K = -(-W // 14)
        beta = rng.uniform(0.05, 0.4, K)
        gamma = rng.uniform(0.05, 0.2)
        mu = rng.uniform(0.001, 0.01)
        I0 = float(10 ** rng.uniform(2, np.log10(min(1e4, N / 100))))
        out.append(dict(N=N, W=W, K=K, theta=np.concatenate([beta, [gamma, mu, I0]]),
                        noise_seed=rng.integers(0, 2**63)))
    return out


def c4_truth():
    rng = np.random.default_rng(4)
    return np.concatenate([rng.uniform(0.05, 0.4, 13), [0.1, 0.002, 1000.0]])


def c4_thetas(n=65536):
    """Parameter vectors uniform in the 13-segment box (seed 4)."""
    rng = np.random.default_rng([4, 1])
    lo, hi = box(13)
    return lo + rng.uniform(0, 1, (n, 16)) * (hi - lo)


def c5_regimes(days=414):
    """Daily beta of the rolling-window series: regimes of U{30..90} days,
    beta per regime ~ U[0.05,0.2]; gamma = 0.1, mu = 0.002, I0 = 1000.
    With gamma + mu = 0.102 the effective reproduction number stays near 1,
    so the 414 days show several rising and falling waves (about 8e4
    cumulative deaths) instead of one wave that exhausts S in 100 days."""
    rng = np.random.default_rng(5)
    beta = np.zeros(days)
    t = 0
    while t < days:
        L = int(rng.integers(30, 91))
        beta[t:t + L] = rng.uniform(0.05, 0.2)
        t += L
    return beta


def paper_truth():
    """Ramp parameters (beta1, beta2, t1, t2, gamma, mu, I0) of the paper
    workload and its window-start R and D: a wave that plateaus, then
    declines after a ramp between days 10 and 25 (R_eff from about 1.08
    to 0.45), starting from 3e5 active cases."""
    return np.array([0.12, 0.05, 10.0, 25.0, 0.1, 0.0025, 3.0e5]), 2.2e6, 5.5e4


def noisy_level(x, rng):
    """Observed level series (active cases): Poisson noise per day."""
    return rng.poisson(np.maximum(np.asarray(x, dtype=np.float64), 0.0)).astype(np.float64)


# ------------------------------------------------------------ loading
def _load(name):
    path = os.path.join(SERIES_DIR, name + ".npz")
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} missing: run `python synth/make_series.py` to regenerate it")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def c1(n_part=256, iters=200):
    z = _load("c1")
    lo, hi = box(1, 1000.0, 1000.0)
    f = Fit(W=60, spd=10, seg_days=60, K=1, N=POLAND_N, R0=0.0, D0=0.0, lo=lo, hi=hi,
            y=z["y"], n_part=n_part, stream=0, truth=c1_truth())
    return Workload("c1", [f], iters=iters, seed=1)


def c2(n_part=8192, iters=1000):
    z = _load("c2")
    lo, hi = box(13)
    f = Fit(W=180, spd=10, seg_days=14, K=13, N=POLAND_N, R0=0.0, D0=0.0, lo=lo, hi=hi,
            y=z["y"], n_part=n_part, stream=0, truth=c2_truth())
    return Workload("c2", [f], iters=iters, seed=2)


def c3(n_part=1024, iters=500, regions=None):
    z = _load("c3")
    regs = c3_regions()
    idx = range(len(regs)) if regions is None else regions
    fits = []
    for r in idx:
        g = regs[r]
        W, K = g["W"], g["K"]
        lo, hi = box(K, 1e2, min(1e5, g["N"]))
        y = z["y"][r, :W + 1]
        fits.append(Fit(W=W, spd=10, seg_days=14, K=K, N=g["N"], R0=0.0, D0=0.0, lo=lo,
                        hi=hi, y=y, n_part=n_part, stream=r, truth=g["theta"]))
    return Workload("c3", fits, iters=iters, seed=3)


def c4():
    """One 365-day problem (K = 13, last segment extended) and the theta set."""
    z = _load("c4")
    lo, hi = box(13)
    f = Fit(W=365, spd=20, seg_days=14, K=13, N=POLAND_N, R0=0.0, D0=0.0, lo=lo, hi=hi,
            y=z["y"], n_part=65536, stream=0, truth=c4_truth())
    return Workload("c4", [f], iters=1, seed=4), c4_thetas()


def c5_series():
    """Truth and observed series of the rolling-window workload."""
    return _load("c5")


def c5(restarts=16, n_part=4096, iters=300, windows=None):
    """52 windows [7w, 7w+42]; per window 16 restarts, each its own fit with
    Philox stream 16w + r.  The window starts from the truth's removed
    count and the observed deaths; I at the window start is fitted."""
    z = _load("c5")
    fits = []
    for w in (range(52) if windows is None else windows):
        t0 = 7 * w
        R0 = float(z["truth"][2, t0])
        D0 = float(z["y"][t0])
        lo = np.array([0.0] * 3 + [0.0, 0.0, 1.0])
        hi = np.array([1.0] * 3 + [0.5, 0.05, 1e7])
        y = z["y"][t0:t0 + 43].copy()
        for r in range(restarts):
            fits.append(Fit(W=42, spd=10, seg_days=14, K=3, N=POLAND_N, R0=R0, D0=D0,
                            lo=lo, hi=hi, y=y, n_part=n_part, stream=16 * w + r))
    return Workload("c5", fits, iters=iters, seed=5)


def paper_box(W, I0):
    """The paper's second search box (Sec. 3.1): beta1, beta2 in [0, 2],
    0 <= t1 <= t2 <= W - 7, gamma in [0, 1], mu in [0, 0.1]; the window's
    initial I is taken from the data (a fixed dimension)."""
    lo = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0, I0])
    hi = np.array([2.0, 2.0, W - 7.0, W - 7.0, 1.0, 0.1, I0])
    return lo, hi


def _paper_fit(W, t0, n_part, stream):
    z = _load("paper")
    obs = z["obs"]  # (3, 93): I, R, D
    I0, R0, D0 = (float(v) for v in obs[:, t0])
    lo, hi = paper_box(W, I0)
    o3 = obs[:, t0:t0 + W + 1].reshape(-1).copy()
    return Fit(W=W, spd=1, seg_days=1, K=4, N=POLAND_N, R0=R0, D0=D0, lo=lo, hi=hi,
               y=obs[2, t0:t0 + W + 1].copy(), n_part=n_part, stream=stream,
               truth=paper_truth()[0] if t0 == 0 else None, obs3=o3, model="euler_ramp")


def paper(n_part=10000, iters=100):
    """One 92-day window from the observed first day (Sec. 3.3 timing)."""
    return Workload("paper", [_paper_fit(92, 0, n_part, 0)], iters=iters, seed=6,
                    loss="ird_mxse", w=0.5, c1=0.5, c2=0.5)


def rep(n_rep=1000, n_part=10000, iters=100, t0=20):
    """n_rep independent fits of the 36-day window starting on day t0, each
    with its own Philox stream (the repetition study of Sec. 4.2)."""
    fits = [_paper_fit(35, t0, n_part, r) for r in range(n_rep)]
    return Workload("rep", fits, iters=iters, seed=7, loss="ird_mxse", w=0.5, c1=0.5, c2=0.5)
