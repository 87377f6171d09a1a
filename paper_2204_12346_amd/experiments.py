"""Measured workloads beside the main throughput line: single-fit swarm
throughput, gradients per second, time-to-fit of plain swarm vs swarm +
adjoint refinement, the rolling-window fit + 14-day forecast, the paper's
own timing case (one swarm iteration of its Euler + ramp model under
F_IRD^MXSE) and its repetition study.

Each function builds its batch from ``synth`` inputs, times device work with
HIP events (or wall clock where the protocol is wall time) and returns a
plain dict for the benchmark's JSON line.
"""
from __future__ import annotations

import sys
import time
from typing import Dict, List

import numpy as np
import torch

from . import fit
from .core import (CKPT_SEGMENTS, Batch, Graph, ProblemSpec, PsoParams, Swarm, pso_init,
                   sird_integrate, sird_loss, sird_loss_backward, sird_loss_backward_workspace,
                   sird_pso_iterate)


def _events():
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _setup(wl, dtype="f64", launch=None, hist_len=0):
    """Batch, swarm parameters, swarm and observations of a workload; the
    F_IRD costs get the three observed series."""
    three = wl.loss.startswith("ird")
    specs = [ProblemSpec.from_fit(f) for f in wl.fits]
    b = Batch(specs, dtype=dtype, obs_series=3 if three else 1, **(launch or {}))
    params = PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                       wl.c2, wl.seed)
    sw = Swarm(b, hist_len=hist_len)
    obs = b.pack_obs([f.obs3 if three else f.y for f in wl.fits])
    return b, params, sw, obs


def r2(y, yhat):
    """Coefficient of determination 1 - sum (y - yhat)^2 / sum (y - mean y)^2
    (the goodness-of-fit measure the paper reports on D)."""
    y = np.asarray(y, dtype=np.float64)
    yhat = np.asarray(yhat, dtype=np.float64)
    return float(1.0 - np.sum((y - yhat) ** 2) / np.sum((y - y.mean()) ** 2))


def swarm_throughput(wl, dtype="f64", iters=200, warmup=10, graph_chunk=10,
                     launch=None) -> Dict:
    """particle-steps/s of whole swarm iterations of one workload, replayed
    as HIP graphs of graph_chunk iterations."""
    b, params, sw, obs = _setup(wl, dtype, launch)
    pso_init(b, params, sw)
    sird_pso_iterate(b, params, sw, obs, wl.loss, warmup)
    g = Graph(b, params, sw, obs, wl.loss, iters_per_launch=graph_chunk)
    n = max(1, iters // graph_chunk)
    e0, e1 = _events()
    g.launch(1)  # the first replay uploads the graph
    torch.cuda.synchronize()
    e0.record()
    g.launch(n)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    g.close()
    its = n * graph_chunk
    return {"particle_steps_per_s": b.particle_steps * its / (ms / 1e3),
            "ms_per_iteration": ms / its, "iterations": its, "dtype": dtype,
            "particles": b.total_particles, "graph_chunk": graph_chunk}


def gradients_per_s(wl, thetas, reps=10, ckpt_interval=0, warm_pairs=5) -> Dict:
    """Loss + gradient of every parameter vector, as the autograd path runs
    it: sird_loss saving the adjoint's checkpoints, then the reverse sweep
    alone (sird_loss_backward from_forward).  Also timed: the self-contained
    sird_loss_backward (both passes in one launch, as the refinement uses
    it) and the plain loss kernel.  warm_pairs loss + gradient pairs run
    first: the engine clock takes a few milliseconds of this load to settle
    (the first pairs of a cold start run up to 20 % slower)."""
    f = wl.fits[0]
    b = Batch([ProblemSpec.from_fit(f, len(thetas))])
    theta = b.pack_theta([thetas])
    obs = b.pack_obs([f.y])
    grad = b.empty_theta()
    loss = b.empty_particles()
    ws = torch.empty(sird_loss_backward_workspace(b, ckpt_interval), dtype=torch.uint8,
                     device=b.device)

    def timed(fn):
        fn()  # warm
        e0, e1 = _events()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def fwd_ckpt():
        sird_loss(b, theta, obs, wl.loss, loss, workspace=ws, ckpt_interval=ckpt_interval)

    def rev():
        sird_loss_backward(b, theta, obs, wl.loss, grad_theta=grad, ckpt_interval=ckpt_interval,
                           workspace=ws, from_forward=True)

    def pair():
        fwd_ckpt()
        rev()

    def full():
        sird_loss_backward(b, theta, obs, wl.loss, grad_theta=grad, loss_out=loss,
                           ckpt_interval=ckpt_interval, workspace=ws)

    for _ in range(warm_pairs):
        pair()
    ms_pair = timed(pair)
    ms_fc = timed(fwd_ckpt)
    fwd_ckpt()
    ms_rev = timed(rev)
    ms_full = timed(full)
    ms_f = timed(lambda: sird_loss(b, theta, obs, wl.loss, loss))
    n = len(thetas)
    return {"gradients_per_s": n / (ms_pair / 1e3), "ms_loss_and_gradient": ms_pair,
            "ms_forward_saving_checkpoints": ms_fc, "ms_reverse_sweep": ms_rev,
            "gradients_per_s_reverse_sweep": n / (ms_rev / 1e3),
            "ms_self_contained_backward": ms_full,
            "gradients_per_s_self_contained": n / (ms_full / 1e3),
            "ms_forward": ms_f, "reverse_over_forward": ms_rev / ms_f,
            "ckpt_interval": ckpt_interval or "default: whole days per LDS slice (one day here)",
            "particle_steps": b.particle_steps, "workspace_bytes": int(ws.numel())}


def refine_gradient_latency(wl, ks=(32, 1024), reps=30, seed=12) -> Dict:
    """Latency of one self-contained gradient call (forward + reverse sweep)
    at a refinement's size: k parameter vectors drawn in the workload's box,
    with the sequential sweep (default interval) and with the
    segment-parallel sweep (CKPT_SEGMENTS)."""
    f = wl.fits[0]
    rng = np.random.default_rng(seed)
    out = {}
    for k in ks:
        b = Batch([ProblemSpec.from_fit(f, k)])
        th = f.lo + rng.random((k, len(f.lo))) * (f.hi - f.lo)
        theta, obs = b.pack_theta([th]), b.pack_obs([f.y])
        grad = b.empty_theta()
        row = {}
        for name, ci in (("sequential", 0), ("segments", CKPT_SEGMENTS)):
            ws = torch.empty(max(sird_loss_backward_workspace(b, ci), 8), dtype=torch.uint8,
                             device=b.device)
            for _ in range(5):
                sird_loss_backward(b, theta, obs, wl.loss, grad_theta=grad, ckpt_interval=ci,
                                   workspace=ws)
            e0, e1 = _events()
            e0.record()
            for _ in range(reps):
                sird_loss_backward(b, theta, obs, wl.loss, grad_theta=grad, ckpt_interval=ci,
                                   workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            row[f"ms_{name}"] = e0.elapsed_time(e1) / reps
        out[f"k{k}"] = row
    return out


def time_to_fit(wl, seeds=(2, 3, 4, 5, 6), plain_cap=10000, pso_first=(50, 100, 200),
                ks=(64, 1024, 4096), refine_steps=2000, lr=1e-2, rels=(1e-2, 1e-3, 1e-4, 1e-6),
                chunk=50, method="lbfgs", adam_arms=(), adam_lr_end=None, trials=(1,)) -> Dict:
    """Wall time from pso_init until the loss is within rel of the best
    loss any run of either arm found (L_best), per seed:
      plain arm: swarm iterations (graph chunks of `chunk`), capped;
      adjoint arm: I' swarm iterations, then refinement of the k best
      personal bests with gradients from the discrete adjoint: projected
      L-BFGS rounds (method "lbfgs", I0 in log coordinates; one arm per
      number of trial steps per round in trials, named _t<T> when T > 1) or
      projected Adam steps ("adam"); one arm per (I', k), plus projected Adam arms
      for the (I', k) in adam_arms (judged against the same L_best).  Adam's
      step is lr, or decays geometrically from lr to adam_lr_end over the
      refine_steps steps when adam_lr_end is given.  A round on k vectors of
      one window costs about the same wall time for any k up to a few
      thousand (one wavefront per 64 vectors), so a larger k refines more
      starting points, and so more basins, at little extra cost.
    Every run's trajectory of (elapsed s, best loss) is recorded first and
    the thresholds applied afterwards, so both arms are judged against the
    same L_best.  Reports per threshold the median over seeds (None when
    the median run does not reach it) and the final losses."""
    f = wl.fits[0]
    spec = ProblemSpec.from_fit(f)

    def new(seed):
        b = Batch([spec], block=64)
        params = PsoParams(b, [f.lo], [f.hi], wl.w, wl.c1, wl.c2, seed)
        obs = b.pack_obs([f.y])
        return b, params, obs

    curves: Dict[str, Dict[int, List]] = {"plain": {}}
    for seed in seeds:
        b, params, obs = new(seed)
        sw = Swarm(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pso_init(b, params, sw)
        g = Graph(b, params, sw, obs, wl.loss, iters_per_launch=chunk)
        curve = []
        for i in range(plain_cap // chunk):
            g.launch(1)
            best = sw.gbest_f[0].item()  # synchronises
            curve.append((time.perf_counter() - t0, best, (i + 1) * chunk))
        g.close()
        curves["plain"][seed] = curve
        _progress(f"time_to_fit plain seed {seed}: {curve[-1][0]:.2f} s, loss {curve[-1][1]:.9g}")
    arms = [(I1, k, method, T) for k in ks for I1 in pso_first
            for T in (trials if method == "lbfgs" else (1,))]
    arms += [(I1, k, "adam", 1) for I1, k in adam_arms]
    for I1, k, meth, T in arms:
        arm = f"adjoint_I{I1}_k{k}" if meth == method else f"{meth}_I{I1}_k{k}"
        if T > 1:
            arm += f"_t{T}"
        curves[arm] = {}
        for seed in seeds:
            b, params, obs = new(seed)
            sw = Swarm(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pso_init(b, params, sw)
            sird_pso_iterate(b, params, sw, obs, wl.loss, I1)
            best = sw.gbest_f[0].item()  # synchronises
            curve = [(time.perf_counter() - t0, best, 0)]
            if meth == "adam":
                _adam_curve(b, sw, params, obs, wl.loss, k, refine_steps, lr, t0, curve,
                            lr_end=adam_lr_end)
            else:
                _lbfgs_curve(b, sw, params, obs, wl.loss, k, refine_steps, t0, curve,
                             n_trials=T)
            curves[arm][seed] = curve
            _progress(f"time_to_fit {arm} seed {seed}: {curve[-1][0]:.2f} s, "
                      f"loss {curve[-1][1]:.9g}")
    L_best = min(min(c[1] for c in cur) for arm in curves.values() for cur in arm.values())

    def reach(curve, thr):
        for t, l, it in curve:
            if l <= thr:
                return t
        return None

    res = {"L_best": L_best, "rels": list(rels), "seeds": list(seeds),
           "plain_cap_iterations": plain_cap, "refine": method,
           "refine_steps_cap": refine_steps, "k": list(ks), "pso_first": list(pso_first),
           "trials": list(trials)}
    if method == "adam" or adam_arms:
        res["lr"] = lr
        res["lr_end"] = adam_lr_end
    for arm, runs in curves.items():
        entry = {"final_loss": [runs[s][-1][1] for s in seeds],
                 "wall_s": [runs[s][-1][0] for s in seeds], "median_s": {}}
        for rel in rels:
            thr = L_best * (1 + rel)
            entry["median_s"][f"{rel:g}"] = _median([reach(runs[s], thr) for s in seeds])
        res[arm] = entry
    return res


def _progress(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _median(ts):
    """Median with 'not reached' counted as +inf; None if the median is."""
    v = sorted(np.inf if t is None else t for t in ts)
    m = float(np.median(v))
    return None if not np.isfinite(m) else m


def _adam_curve(b, sw, params, obs, kind, k, steps, lr, t0, curve, check_every=25,
                lr_end=None):
    """Projected Adam from the top-k personal bests, appending
    (elapsed s, best loss so far, Adam step) every check_every steps; the
    step decays geometrically from lr to lr_end when lr_end is given."""
    from .core import pso_topk, sird_adam_step, sird_gather
    idx = pso_topk(b, sw.pbest_f, k)
    specs = [s.with_particles(k) for s in b.specs]
    rb = Batch(specs, device=b.device, obs_series=b.obs_series)
    theta = sird_gather(b, sw.pbest_x, params.lo, rb, idx, k)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    loss = rb.empty_particles()
    ci = fit.default_ckpt_interval(rb)
    ws = torch.empty(max(sird_loss_backward_workspace(rb, ci), 8), dtype=torch.uint8,
                     device=b.device)
    best = curve[-1][1]
    for t in range(1, steps + 1):
        sird_loss_backward(rb, theta, obs, kind, grad_theta=grad, loss_out=loss,
                           ckpt_interval=ci, workspace=ws)
        lr_t = lr if lr_end is None else lr * (lr_end / lr) ** ((t - 1) / max(steps - 1, 1))
        sird_adam_step(rb, theta, grad, m, v, params.lo, params.hi, t, lr=lr_t)
        if t % check_every == 0:
            cur = float(torch.nan_to_num(loss, nan=float("inf")).min().item())
            best = min(best, cur)
            curve.append((time.perf_counter() - t0, best, t))
    final = float(torch.nan_to_num(sird_loss(rb, theta, obs, kind), nan=float("inf")).min().item())
    curve.append((time.perf_counter() - t0, min(best, final), steps))
    return rb


def _lbfgs_curve(b, sw, params, obs, kind, k, rounds, t0, curve, check_every=10, n_trials=1):
    """Projected L-BFGS from the top-k personal bests (n_trials trial steps
    per round), appending (elapsed s, best loss so far, round) every
    check_every rounds."""
    from .core import LbfgsState, pso_topk, sird_gather
    idx = pso_topk(b, sw.pbest_f, k)
    specs = [s.with_particles(k) for s in b.specs]
    rb = Batch(specs, device=b.device, obs_series=b.obs_series)
    theta = sird_gather(b, sw.pbest_x, params.lo, rb, idx, k)
    st = LbfgsState(rb, theta, n_trials=n_trials)
    ci = fit.default_ckpt_interval(st.trial_batch)
    ws = torch.empty(max(sird_loss_backward_workspace(st.trial_batch, ci), 8),
                     dtype=torch.uint8, device=b.device)
    sird_loss_backward(rb, st.theta, obs, kind, grad_theta=st.grad, loss_out=st.f,
                       ckpt_interval=ci, workspace=ws)
    best = [curve[-1][1]]

    def record(r):
        cur = float(torch.nan_to_num(st.f, nan=float("inf")).min().item())
        best[0] = min(best[0], cur)
        curve.append((time.perf_counter() - t0, best[0], r))
        return False

    fit.lbfgs_rounds(rb, st, params, obs, kind, rounds, ckpt_interval=ci, workspace=ws,
                     callback=record, check_every=check_every)
    record(rounds)
    return rb


def rolling_forecast(wl, truth, restarts, iters=300, k_per_restart=2, refine_rounds=300,
                     horizon=14, launch=None, method="lbfgs", lr=1e-2) -> Dict:
    """All windows x restarts in one batch: swarm, refinement of the best
    k_per_restart particles of every restart (projected L-BFGS, or projected
    Adam with step lr), best refined parameters per window, and a horizon-day
    forecast of cumulative deaths compared with the noise-free truth
    (relative error at 7 and 14 days, and of the 14-day increment);
    quantiles over windows.  A pass of one iteration and one refinement
    round runs untimed first, so that the timed run starts in a warm
    process (kernels loaded, workspaces cached)."""
    fits = wl.fits
    specs = [ProblemSpec.from_fit(f) for f in fits]
    b = Batch(specs, **(launch or {}))
    params = PsoParams(b, [f.lo for f in fits], [f.hi for f in fits], wl.w, wl.c1, wl.c2,
                       wl.seed)
    sw = Swarm(b)
    obs = b.pack_obs([f.y for f in fits])

    def swarm_and_refine(n_iters, n_rounds):
        pso_init(b, params, sw)
        sird_pso_iterate(b, params, sw, obs, wl.loss, n_iters)
        torch.cuda.synchronize()
        t_mid = time.perf_counter()
        if method == "adam":
            r = fit.refine_topk(b, sw, params, obs, wl.loss, k=k_per_restart,
                                max_steps=n_rounds, lr=lr, check_every=max(n_rounds, 1))
        else:
            r = fit.refine_lbfgs(b, sw, params, obs, wl.loss, k=k_per_restart,
                                 max_rounds=n_rounds, check_every=max(n_rounds, 1))
        torch.cuda.synchronize()
        return r, t_mid

    swarm_and_refine(1, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref, t_mid = swarm_and_refine(iters, refine_rounds)
    t_pso = t_mid - t0
    t_ref = time.perf_counter() - t_mid
    th, L = fit.best_per_problem(ref.batch, ref.theta, ref.loss)
    # best over the restarts of each window (problems come window-major)
    n_win = len(fits) // restarts
    win_theta, win_spec, starts = [], [], []
    for w in range(n_win):
        cand = [(L[w * restarts + r], w * restarts + r) for r in range(restarts)]
        Lb, pi = min(cand)
        win_theta.append(th[pi])
        win_spec.append(specs[pi])
        starts.append(7 * w)
    traj = fit.forecast([s.with_particles(1) for s in win_spec],
                        [t[None, :] for t in win_theta], horizon, device=b.device)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    e7, e14, einc = [], [], []
    for w, (tr, t0w) in enumerate(zip(traj, starts)):
        W = win_spec[w].W
        D = tr[0, 3]
        end = t0w + W
        true = truth[3]
        e7.append(abs(D[W + 7] - true[end + 7]) / true[end + 7])
        e14.append(abs(D[W + 14] - true[end + 14]) / true[end + 14])
        inc_true = true[end + 14] - true[end]
        inc_fit = D[W + 14] - D[W]
        einc.append(abs(inc_fit - inc_true) / max(inc_true, 1.0))

    def q(v):
        return {p: float(np.quantile(v, p / 100)) for p in (5, 50, 95)}

    return {"windows": n_win, "restarts": restarts, "particles": b.total_particles,
            "iterations": iters, "refine": method, "refine_rounds": refine_rounds,
            "particle_steps": b.particle_steps * iters,
            "seconds_swarm": t_pso, "seconds_refine": t_ref, "seconds_total": t_all,
            "particle_steps_per_s_swarm": b.particle_steps * iters / t_pso,
            "rel_err_cum_deaths_h7": q(e7), "rel_err_cum_deaths_h14": q(e14),
            "rel_err_14day_increment": q(einc)}


def paper_iteration(wl, dtype="f64", reps=20, launch=None) -> Dict:
    """The paper's timing protocol (Sec. 3.3): the mean and standard
    deviation over reps of one swarm iteration (every particle's model over
    the window, its F_IRD^MXSE cost, bests and move), each launched and
    timed on its own; then a whole run of wl.iters iterations from pso_init
    (wall clock) and the fit it reaches (loss, R^2 on D, I and R)."""
    b, params, sw, obs = _setup(wl, dtype, launch, hist_len=wl.iters)
    pso_init(b, params, sw)
    sird_pso_iterate(b, params, sw, obs, wl.loss, 3)  # warm-up
    ms = []
    for _ in range(reps):
        e0, e1 = _events()
        e0.record()
        sird_pso_iterate(b, params, sw, obs, wl.loss, 1)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    # a whole run, eager
    b, params, sw, obs = _setup(wl, dtype, launch, hist_len=wl.iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pso_init(b, params, sw)
    sird_pso_iterate(b, params, sw, obs, wl.loss, wl.iters)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    f = wl.fits[0]
    gx = b.unpack_box(sw.gbest_x)[0]
    tr = fit.forecast([b.specs[0]], [gx[None, :]], 0, device=b.device)[0][0]
    o = np.asarray(f.obs3).reshape(3, -1)
    return {"particles": b.total_particles, "days": f.W, "steps_per_day": f.spd,
            "dtype": dtype, "ms_per_iteration_mean": float(np.mean(ms)),
            "ms_per_iteration_std": float(np.std(ms)), "reps": reps,
            "particle_steps_per_s": b.particle_steps / (np.mean(ms) / 1e3),
            "iterations": wl.iters, "seconds_run": t_run,
            "final_loss": sw.gbest_f[0].item(), "r2_D": r2(o[2], tr[3]),
            "r2_I": r2(o[0], tr[1]), "r2_R": r2(o[1], tr[2])}


def repetition(wl, horizon=21, launch=None) -> Dict:
    """The repetition study (Sec. 4.2): every fit of the workload is the
    same window with its own Philox stream, all in one batch; returns the
    time, the spread of the fitted parameters (5/50/95 % quantiles), the
    spread of the losses and the 50/90/95 % bands of the horizon-day
    extension of D, I and R at the window end + horizon."""
    b, params, sw, obs = _setup(wl, "f64", launch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pso_init(b, params, sw)
    sird_pso_iterate(b, params, sw, obs, wl.loss, wl.iters)
    torch.cuda.synchronize()
    t_pso = time.perf_counter() - t0
    th = np.stack(b.unpack_box(sw.gbest_x))
    L = sw.gbest_f.cpu().numpy()
    trajs = fit.forecast(b.specs, [t[None, :] for t in th], horizon, device=b.device)
    end = np.stack([t[0, :, -1] for t in trajs])  # (n_rep, 4) at W + horizon
    t_all = time.perf_counter() - t0

    def q(v, ps=(5, 50, 95)):
        return {p: float(np.quantile(v, p / 100)) for p in ps}

    names = ["beta1", "beta2", "t1", "t2", "gamma", "mu"]
    bands = {}
    for c, name in ((1, "I"), (2, "R"), (3, "D")):
        bands[name] = {f"{lvl}%": [float(np.quantile(end[:, c], (1 - lvl / 100) / 2)),
                                   float(np.quantile(end[:, c], 1 - (1 - lvl / 100) / 2))]
                       for lvl in (50, 90, 95)}
    return {"fits": b.n_prob, "particles_per_fit": b.specs[0].n_part,
            "iterations": wl.iters, "particle_steps": b.particle_steps * wl.iters,
            "seconds_swarm": t_pso, "seconds_total": t_all,
            "particle_steps_per_s": b.particle_steps * wl.iters / t_pso,
            "loss": q(L), "params": {n: q(th[:, j]) for j, n in enumerate(names)},
            f"extension_day_{horizon}_bands": bands}
