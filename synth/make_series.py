"""Write the stored observation series under synth/series/.

Truth trajectories come from the oracle's RK4 (the same discrete model the
fits use, so a noise-free series has loss exactly zero at the truth); count
noise comes from ``synth.noisy_cumulative``.  This script calls only the
oracle and the input generators.  Run from the repository root:

    python synth/make_series.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def make_c1():
    prob = oracle.Problem(W=60, spd=10, seg_days=60, K=1, N=synth.POLAND_N)
    truth = oracle.integrate(prob, synth.c1_truth())
    y = synth.noisy_cumulative(truth[3], "poisson", np.random.default_rng(0))
    return dict(y=y, truth=truth)


def make_c2():
    prob = oracle.Problem(W=180, spd=10, seg_days=14, K=13, N=synth.POLAND_N)
    truth = oracle.integrate(prob, synth.c2_truth())
    y = synth.noisy_cumulative(truth[3], "negbin", np.random.default_rng(2))
    return dict(y=y, truth=truth)


def make_c3():
    regs = synth.c3_regions()
    Y = np.full((len(regs), 366), np.nan)
    for r, g in enumerate(regs):
        prob = oracle.Problem(W=g["W"], spd=10, seg_days=14, K=g["K"], N=g["N"])
        truth = oracle.integrate(prob, g["theta"])
        rng = np.random.default_rng(int(g["noise_seed"]))
        Y[r, :g["W"] + 1] = synth.noisy_cumulative(truth[3], "negbin", rng)
    return dict(y=Y)


def make_c4():
    prob = oracle.Problem(W=365, spd=20, seg_days=14, K=13, N=synth.POLAND_N)
    truth = oracle.integrate(prob, synth.c4_truth())
    y = synth.noisy_cumulative(truth[3], "negbin", np.random.default_rng([4, 2]))
    return dict(y=y, truth=truth)


def make_c5():
    beta = synth.c5_regimes(414)
    days = 413
    prob = oracle.Problem(W=days, spd=10, seg_days=1, K=days, N=synth.POLAND_N)
    theta = np.concatenate([beta[:days], [0.1, 0.002, 1000.0]])
    truth = oracle.integrate(prob, theta)
    y = synth.noisy_cumulative(truth[3], "negbin", np.random.default_rng([5, 2]))
    return dict(y=y, truth=truth, beta=beta)


def make_paper():
    """92 days of I, R, D from the ramp model (forward Euler, one step per
    day) with count noise: Poisson on the active cases, negative-binomial
    on the daily increments of R and D; day 0 is observed exactly."""
    theta, R0, D0 = synth.paper_truth()
    prob = oracle.Problem(W=92, spd=1, seg_days=1, K=4, N=synth.POLAND_N, R0=R0, D0=D0,
                          model=1)
    truth = oracle.integrate_model(prob, theta)
    rng = np.random.default_rng(6)
    yI = synth.noisy_level(truth[1], rng)
    yI[0] = truth[1, 0]
    yR = synth.noisy_cumulative(truth[2], "negbin", rng)
    yD = synth.noisy_cumulative(truth[3], "negbin", rng)
    return dict(obs=np.stack([yI, yR, yD]), truth=truth)


MAKERS = dict(c1=make_c1, c2=make_c2, c3=make_c3, c4=make_c4, c5=make_c5, paper=make_paper)


def main(names=None):
    os.makedirs(synth.SERIES_DIR, exist_ok=True)
    for name in names or MAKERS:
        data = MAKERS[name]()
        np.savez_compressed(os.path.join(synth.SERIES_DIR, name + ".npz"), **data)
        print("wrote", name, {k: v.shape for k, v in data.items()})


if __name__ == "__main__":
    main(sys.argv[1:] or None)
