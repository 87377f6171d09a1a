"""Helpers of the GPU parity tests: building batches from synthetic fits,
random parameter vectors in a box, and the parity criteria.

Parity criteria (FP64 unless stated):
  * trajectories, FP64: |x_gpu - x_ref| <= 1e-12 |x_ref| per compartment and
    day;
  * trajectories, FP32 state: R and D (never decreasing) per value,
    |x_gpu - x_ref| <= 1e-5 |x_ref|; S and I within 1e-5 of the largest value
    the compartment has held so far, |x_gpu - x_ref| <= 1e-5 max_{t' <= t}
    |x_ref(t')|.  Float rounding is relative to the values the state passed
    through: a compartment that has decayed by dozens of e-folds (I of a
    dying epidemic) carries the rounding of its earlier, larger values, and
    no float evaluation matches it per value to 1e-5; the tests print the
    worst per-value error of every compartment;
  * losses: |L_gpu - L_ref| <= eps max(L_ref, kappa), where kappa is the
    first-order sensitivity of the cost to relative changes of the model's
    deceased values (sum of |dl/dDhat_i| |Dhat_i|), so that a loss near zero
    (a noise-free fit) is judged by the size of its terms, not by itself;
  * gradients: per component |g_j - g_ref,j| <= 1e-6 |g_ref,j| + 1e-10 scale_j,
    scale_j the sum of the absolute terms the component adds up.
"""
import numpy as np
import torch

import oracle
import paper_2204_12346_amd as S

TOL64 = 1e-12
TOL32 = 1e-5


def need_gpu():
    import pytest
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_problem(f):
    return oracle.Problem(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0)


def random_theta(f, n, seed):
    rng = np.random.default_rng(seed)
    return f.lo + rng.uniform(0, 1, (n, f.d)) * (f.hi - f.lo)


def kappa(kind, Dhat, y):
    """Sum over days of |dl/dDhat_i| |Dhat_i| for the cost of this kind."""
    Dhat = np.asarray(Dhat, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    e = y - Dhat
    g = np.maximum(y, 1.0)
    if kind == "ssre":
        t = 2 * np.abs(Dhat - y) / g / g * np.abs(Dhat)
        t[0] = 0.0
        return float(t.sum())
    if kind == "mse":
        return float((2 * np.abs(e) * np.abs(Dhat)).sum() / n)
    if kind == "mxse":
        i = int(np.argmax(e * e))
        return float(2 * abs(e[i]) * abs(Dhat[i]))
    if kind == "mae":
        return float(np.abs(Dhat).sum() / n)
    if kind == "mape":
        return float(100 * (np.abs(Dhat) / g).sum() / n)
    raise ValueError(kind)


def assert_loss_close(got, ref, kap, eps, what=""):
    got = np.asarray(got)
    ref = np.asarray(ref)
    kap = np.asarray(kap)
    bound = eps * np.maximum(np.abs(ref), kap)
    bad = ~(np.abs(got - ref) <= bound)
    # identical non-finite values agree
    bad &= ~((~np.isfinite(ref)) & (np.isnan(got) == np.isnan(ref)) &
             ((got == ref) | np.isnan(ref)))
    if bad.any():
        i = int(np.argmax(bad))
        raise AssertionError(f"{what}: {bad.sum()} losses off, first #{i}: gpu={got[i]!r} "
                             f"ref={ref[i]!r} kappa={kap[i]!r} bound={bound[i]!r}")


def assert_traj_close(got, ref, eps, what=""):
    """got/ref: (4, W+1); relative per compartment over days with ref != 0."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    nz = ref != 0
    rel = np.zeros_like(ref)
    rel[nz] = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
    assert np.all(got[~nz] == 0) or np.all(np.abs(got[~nz]) < 1e-300 + eps), what
    worst = rel.max()
    assert worst <= eps, f"{what}: worst relative error {worst:.3e} > {eps:.0e}"


def assert_traj_close_running_max(got, ref, eps, what=""):
    """got/ref: (4, W+1); error relative to each compartment's running max."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = np.maximum.accumulate(np.abs(ref), axis=1)
    err = np.abs(got - ref)
    ok = err <= eps * scale
    if not ok.all():
        c, t = np.argwhere(~ok)[0]
        raise AssertionError(f"{what}: compartment {'SIRD'[c]} day {t}: gpu={got[c, t]!r} "
                             f"ref={ref[c, t]!r} running max={scale[c, t]!r}")


def assert_traj_close_f32(got, ref, eps, what="", worst=None, tag=None):
    """FP32 state against the FP64 oracle, got/ref (4, W+1): R and D (never
    decreasing) within eps per value; S and I within eps of their running
    max.  worst (a dict) collects, per compartment, the largest per-value
    relative error as (error, day, tag)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert_traj_close(got[2:], ref[2:], eps, f"{what} (R, D per value)")
    assert_traj_close_running_max(got, ref, eps, what)
    if worst is not None:
        for c in range(4):
            nz = ref[c] != 0
            if not nz.any():
                continue
            rel = np.zeros(ref.shape[1])
            rel[nz] = np.abs(got[c, nz] - ref[c, nz]) / np.abs(ref[c, nz])
            t = int(np.argmax(rel))
            if rel[t] > worst.get("SIRD"[c], (-1.0,))[0]:
                worst["SIRD"[c]] = (float(rel[t]), t, tag)


def format_worst(worst):
    return ", ".join(f"{c}: {e:.2e} (day {t}, {tag})" for c, (e, t, tag) in sorted(
        worst.items(), key=lambda kv: "SIRD".index(kv[0])))


def make_batch(fits, n_parts=None, **kw):
    specs = [S.ProblemSpec.from_fit(f, None if n_parts is None else n_parts[i])
             for i, f in enumerate(fits)]
    return S.Batch(specs, **kw)


def oracle_problem_model(f):
    """Oracle problem of a fit of either model."""
    return oracle.Problem(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0,
                          model=1 if getattr(f, "model", "rk4") == "euler_ramp" else 0)


def kappa_ird(kind, traj, obs3):
    """Sensitivity bound of an F_IRD cost: the largest over I, R, D of the
    low-level cost's kappa on the normalised values (MAPE unnormalised)."""
    low = kind[len("ird_"):]
    W1 = traj.shape[1]
    y = np.asarray(obs3, dtype=np.float64).reshape(3, W1)
    worst = 0.0
    for c in range(3):
        yh, yo = traj[c + 1], y[c]
        if low == "mape":
            k = kappa("mape", yh, yo)
        else:
            r = yo.max() - yo.min()
            r = r if r > 0 else 1.0
            k = kappa(low, yh / r, yo / r)
        worst = max(worst, k)
    return worst


GRAD_RTOL = 1e-6
# Floor of the per-component criterion, relative to the component's own
# scale: the sum over days of |dl/dDhat_i| |dDhat_i/dtheta_j| (the terms the
# component adds up).  Forward mode and the complex step agree to ~3e-14 of
# it on the segmented workload, near its truth included.
GRAD_SCALE_FLOOR = 1e-10


def oracle_grad(prob, theta, y, kind):
    """(gradient, per-component scale) of the oracle's forward mode."""
    _, g, sc = oracle.loss_grad_fwd(prob, theta, y, kind, with_scale=True)
    return g, sc


def assert_grad_close(got, ref, scale, what="", worst=None):
    """|g_j - g_ref,j| <= 1e-6 |g_ref,j| + 1e-10 scale_j for every component
    j; worst (a list) collects the largest |g_j - g_ref,j| / |g_ref,j|."""
    got, ref, scale = np.asarray(got), np.asarray(ref), np.asarray(scale)
    err = np.abs(got - ref)
    tol = GRAD_RTOL * np.abs(ref) + GRAD_SCALE_FLOOR * scale
    bad = ~(err <= tol)
    if bad.any():
        j = int(np.argmax(bad))
        raise AssertionError(f"{what}: component {j}: gpu={got[j]!r} ref={ref[j]!r} "
                             f"scale={scale[j]!r}")
    if worst is not None:
        nz = ref != 0
        worst.append(float(np.max(err[nz] / np.abs(ref[nz]))) if nz.any() else 0.0)


def near_truth(f, n, seed):
    """n parameter vectors within 1e-3 (relative) of the synthetic truth:
    every segment's beta then shapes the deaths and its gradient matters."""
    rng = np.random.default_rng(seed)
    t = np.asarray(f.truth, dtype=np.float64)
    return t * (1 + 1e-3 * rng.standard_normal((n, t.size)))


# A swarm decision (personal best, winner against runner-up, new against old
# global best) can only come out differently on the two sides when their
# losses differ by more than the decision's relative margin.  The gbest
# sequences are compared up to the first decision of the oracle's run whose
# margin is below max(NEAR_TIE_FLOOR, NEAR_TIE_FACTOR * delta), delta the
# worst relative difference between the GPU's personal-best losses and the
# oracle's loss at the same positions, measured after the run.
NEAR_TIE_FLOOR = 1e-12
NEAR_TIE_FACTOR = 100.0


def loss_discrepancy(got, ref):
    """Worst |got - ref| / |ref| over entries where ref is finite and
    nonzero; inf when the finite/non-finite pattern differs."""
    got, ref = np.asarray(got), np.asarray(ref)
    fin = np.isfinite(ref)
    if not np.array_equal(fin, np.isfinite(got)):
        return float("inf")
    m = fin & (ref != 0)
    if not m.any():
        return 0.0
    return float(np.max(np.abs(got[m] - ref[m]) / np.abs(ref[m])))


def compared_iterations(margins, delta, iters):
    """Iterations before the first near-tie of the oracle's run."""
    thr = max(NEAR_TIE_FLOOR, NEAR_TIE_FACTOR * delta)
    tie = np.nonzero(np.asarray(margins) < thr)[0]
    return (int(tie[0]) if len(tie) else iters), thr
