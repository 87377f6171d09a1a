"""Measured workloads beside the main throughput line: single-fit swarm
throughput, gradients per second, time-to-fit of plain swarm vs swarm +
adjoint refinement, and the rolling-window fit + 14-day forecast.

Each function builds its batch from ``synth`` inputs, times device work with
HIP events (or wall clock where the protocol is wall time) and returns a
plain dict for the benchmark's JSON line.
"""
from __future__ import annotations

import time
from typing import Dict, List

import numpy as np
import torch

from . import fit
from .core import (Batch, Graph, ProblemSpec, PsoParams, Swarm, pso_init, sird_integrate,
                   sird_loss, sird_loss_backward, sird_loss_backward_workspace, sird_pso_iterate)


def _events():
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def swarm_throughput(wl, dtype="f64", iters=200, warmup=10, graph_chunk=10,
                     launch=None) -> Dict:
    """particle-RK4-steps/s of whole swarm iterations of one workload,
    replayed as HIP graphs of graph_chunk iterations."""
    specs = [ProblemSpec.from_fit(f) for f in wl.fits]
    b = Batch(specs, dtype=dtype, **(launch or {}))
    params = PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                       wl.c2, wl.seed)
    sw = Swarm(b)
    obs = b.pack_obs([f.y for f in wl.fits])
    pso_init(b, params, sw)
    sird_pso_iterate(b, params, sw, obs, wl.loss, warmup)
    g = Graph(b, params, sw, obs, wl.loss, iters_per_launch=graph_chunk)
    n = max(1, iters // graph_chunk)
    e0, e1 = _events()
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


def gradients_per_s(wl, thetas, reps=3, ckpt_interval=0) -> Dict:
    """Loss + gradient of every parameter vector (sird_loss_backward)."""
    f = wl.fits[0]
    b = Batch([ProblemSpec.from_fit(f, len(thetas))])
    theta = b.pack_theta([thetas])
    obs = b.pack_obs([f.y])
    grad = b.empty_theta()
    loss = b.empty_particles()
    ws = torch.empty(sird_loss_backward_workspace(b, ckpt_interval), dtype=torch.uint8,
                     device=b.device)
    sird_loss_backward(b, theta, obs, wl.loss, grad_theta=grad, loss_out=loss,
                       ckpt_interval=ckpt_interval, workspace=ws)
    e0, e1 = _events()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        sird_loss_backward(b, theta, obs, wl.loss, grad_theta=grad, loss_out=loss,
                           ckpt_interval=ckpt_interval, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        sird_loss(b, theta, obs, wl.loss, loss)
    e1.record()
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1) / reps
    return {"gradients_per_s": len(thetas) / (ms_b / 1e3), "ms_backward": ms_b,
            "ms_forward": ms_f, "backward_over_forward": ms_b / ms_f,
            "particle_steps": b.particle_steps, "workspace_bytes": int(ws.numel())}


def time_to_fit(wl, seeds=(2, 3, 4, 5, 6), plain_cap=10000, pso_first=(50, 100, 200),
                k=32, refine_steps=600, lr=1e-2, rel=1e-6, chunk=50,
                method="lbfgs") -> Dict:
    """Wall time from pso_init until the loss is within rel of the best
    loss any run of either arm found (L_best), per seed:
      plain arm: swarm iterations (graph chunks of `chunk`), capped;
      adjoint arm: I' swarm iterations, then refinement of the top-k
      personal bests with gradients from the discrete adjoint: projected
      L-BFGS rounds (method "lbfgs") or projected Adam steps ("adam").
    Every run's trajectory of (elapsed s, best loss) is recorded first, the
    threshold applied afterwards, so both arms are judged against the same
    L_best.  Reports the median over seeds for each arm (None if not
    reached)."""
    f = wl.fits[0]
    spec = ProblemSpec.from_fit(f)

    def new(seed):
        b = Batch([spec], block=64)
        params = PsoParams(b, [f.lo], [f.hi], wl.w, wl.c1, wl.c2, seed)
        obs = b.pack_obs([f.y])
        return b, params, obs

    plain: Dict[int, List] = {}
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
        plain[seed] = curve
    adj: Dict = {}
    for I1 in pso_first:
        for seed in seeds:
            b, params, obs = new(seed)
            sw = Swarm(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pso_init(b, params, sw)
            sird_pso_iterate(b, params, sw, obs, wl.loss, I1)
            curve = [(time.perf_counter() - t0, sw.gbest_f[0].item(), 0)]
            if method == "adam":
                _adam_curve(b, sw, params, obs, wl.loss, k, refine_steps, lr, t0, curve)
            else:
                _lbfgs_curve(b, sw, params, obs, wl.loss, k, refine_steps, t0, curve)
            adj[(I1, seed)] = curve
    L_best = min(min(c[1] for c in cur) for cur in list(plain.values()) + list(adj.values()))
    thr = L_best * (1 + rel)

    def reach(curve):
        for t, l, it in curve:
            if l <= thr:
                return t, it
        return None, None

    res = {"L_best": L_best, "threshold": thr, "rel": rel, "seeds": list(seeds),
           "plain_cap_iterations": plain_cap, "refine": method,
           "refine_steps_cap": refine_steps, "k": k}
    if method == "adam":
        res["lr"] = lr
    pt = [reach(plain[s]) for s in seeds]
    res["plain"] = {"times_s": [t for t, _ in pt], "iterations": [i for _, i in pt],
                    "final_loss": [plain[s][-1][1] for s in seeds]}
    res["plain"]["median_s"] = _median([t for t, _ in pt])
    best_arm = None
    for I1 in pso_first:
        at = [reach(adj[(I1, s)]) for s in seeds]
        m = _median([t for t, _ in at])
        res[f"adjoint_I{I1}"] = {"times_s": [t for t, _ in at],
                                 "refine_steps": [i for _, i in at],
                                 "final_loss": [adj[(I1, s)][-1][1] for s in seeds],
                                 "median_s": m}
        if m is not None and (best_arm is None or m < res[best_arm]["median_s"]):
            best_arm = f"adjoint_I{I1}"
    res["best_adjoint_arm"] = best_arm
    return res


def _median(ts):
    """Median with 'not reached' counted as +inf; None if the median is."""
    v = sorted(np.inf if t is None else t for t in ts)
    m = float(np.median(v))
    return None if not np.isfinite(m) else m


def _adam_curve(b, sw, params, obs, kind, k, steps, lr, t0, curve, check_every=25):
    """Projected Adam from the top-k personal bests, appending
    (elapsed s, best loss so far, Adam step) every check_every steps."""
    from .core import pso_topk, sird_adam_step, sird_gather
    idx = pso_topk(b, sw.pbest_f, k)
    specs = [ProblemSpec(s.W, s.spd, s.seg_days, s.K, s.N, s.R0, s.D0, k, s.stream)
             for s in b.specs]
    rb = Batch(specs, device=b.device)
    theta = sird_gather(b, sw.pbest_x, params.lo, rb, idx, k)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    loss = rb.empty_particles()
    ws = torch.empty(max(sird_loss_backward_workspace(rb, 0), 8), dtype=torch.uint8,
                     device=b.device)
    best = curve[-1][1]
    for t in range(1, steps + 1):
        sird_loss_backward(rb, theta, obs, kind, grad_theta=grad, loss_out=loss, workspace=ws)
        sird_adam_step(rb, theta, grad, m, v, params.lo, params.hi, t, lr=lr)
        if t % check_every == 0:
            cur = float(torch.nan_to_num(loss, nan=float("inf")).min().item())
            best = min(best, cur)
            curve.append((time.perf_counter() - t0, best, t))
    final = float(torch.nan_to_num(sird_loss(rb, theta, obs, kind), nan=float("inf")).min().item())
    curve.append((time.perf_counter() - t0, min(best, final), steps))
    return rb


def _lbfgs_curve(b, sw, params, obs, kind, k, rounds, t0, curve, check_every=10):
    """Projected L-BFGS from the top-k personal bests, appending
    (elapsed s, best loss so far, round) every check_every rounds."""
    from .core import LbfgsState, pso_topk, sird_gather
    idx = pso_topk(b, sw.pbest_f, k)
    specs = [ProblemSpec(s.W, s.spd, s.seg_days, s.K, s.N, s.R0, s.D0, k, s.stream)
             for s in b.specs]
    rb = Batch(specs, device=b.device)
    theta = sird_gather(b, sw.pbest_x, params.lo, rb, idx, k)
    st = LbfgsState(rb, theta)
    ws = torch.empty(max(sird_loss_backward_workspace(rb, 0), 8), dtype=torch.uint8,
                     device=b.device)
    sird_loss_backward(rb, st.theta, obs, kind, grad_theta=st.grad, loss_out=st.f, workspace=ws)
    best = [curve[-1][1]]

    def record(r):
        cur = float(torch.nan_to_num(st.f, nan=float("inf")).min().item())
        best[0] = min(best[0], cur)
        curve.append((time.perf_counter() - t0, best[0], r))
        return False

    fit.lbfgs_rounds(rb, st, params, obs, kind, rounds, workspace=ws, callback=record,
                     check_every=check_every)
    record(rounds)
    return rb


def rolling_forecast(wl, truth, restarts, iters=300, k_per_restart=2, refine_rounds=300,
                     horizon=14, launch=None) -> Dict:
    """All windows x restarts in one batch: swarm, refinement of the best
    k_per_restart particles of every restart, best refined parameters per
    window, and a horizon-day forecast of cumulative deaths compared with the
    noise-free truth (relative error at 7 and 14 days, and of the 14-day
    increment); quantiles over windows."""
    fits = wl.fits
    specs = [ProblemSpec.from_fit(f) for f in fits]
    b = Batch(specs, **(launch or {}))
    params = PsoParams(b, [f.lo for f in fits], [f.hi for f in fits], wl.w, wl.c1, wl.c2,
                       wl.seed)
    sw = Swarm(b)
    obs = b.pack_obs([f.y for f in fits])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pso_init(b, params, sw)
    sird_pso_iterate(b, params, sw, obs, wl.loss, iters)
    torch.cuda.synchronize()
    t_pso = time.perf_counter() - t0
    ref = fit.refine_lbfgs(b, sw, params, obs, wl.loss, k=k_per_restart,
                           max_rounds=refine_rounds, check_every=max(refine_rounds, 1))
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0 - t_pso
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
    traj = fit.forecast([ProblemSpec(s.W, s.spd, s.seg_days, s.K, s.N, s.R0, s.D0, 1, s.stream)
                         for s in win_spec], [t[None, :] for t in win_theta], horizon,
                        device=b.device)
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
            "iterations": iters, "particle_steps": b.particle_steps * iters,
            "seconds_swarm": t_pso, "seconds_refine": t_ref, "seconds_total": t_all,
            "particle_steps_per_s_swarm": b.particle_steps * iters / t_pso,
            "rel_err_cum_deaths_h7": q(e7), "rel_err_cum_deaths_h14": q(e14),
            "rel_err_14day_increment": q(einc)}
