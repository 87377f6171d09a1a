"""Throughput benchmark of the calibration hot path on one MI355X.

One step = one swarm iteration over the whole batch: the previous
iteration's Philox velocity/position update, RK4 over every particle's
window fused with the cost and the personal best (one kernel,
pso_evaluate), then the per-problem global best (pso_gbest).  Default
workload: 512 independent synthetic regions of uneven window (28..365
days) and population, 1024 particles each, 14-day beta segments, dt = 0.1
day, FP64, the K timed iterations captured in one HIP graph.

Prints one JSON line:
  * value: particle-RK4-steps/s of the K graph-replayed steps (M1), with
    the same K steps run eagerly beside it;
  * roofline: the fused integration kernel (timed per launch with HIP
    events on its stream in the eager pass) against the FP64 vector peak,
    at the algorithmic 49 flops per particle-step;
  * time_to_fit (M2): wall time to reach 1e-6 of the best loss on the
    8192-particle segmented fit, plain swarm vs swarm + adjoint refinement;
  * gradients: loss + gradient per second of 65536 parameter vectors over
    7300 steps;
  * other_workloads: the other configurations, one number each;
  * cpu_baseline: the oracle on the host cores on a bounded sample of the
    same workload, and per configuration (stated samples).
The full results of the other workloads go to stderr as one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c1|paper] [--dtype f64|f32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Launch configuration of the integration kernel for the batched workload
# (block size, cap on resident wavefronts per SIMD, persistent wavefronts);
# what the autotuner of the fused iteration (autotune.autotune_iterate,
# bench.py --autotune) picks.
C3_LAUNCH = dict(block=256, persistent=0, waves_per_simd=4)

# Algorithmic work of one particle-step of classical RK4 on eq. (SIRD)
# with the state (S, I, D): four right-hand sides (p = b S I, p - lam I,
# mu I) and the stage and update combinations, 8 mul + 3 add + 19 fma =
# 49 flops (an FMA counts 2).  The kernel issues fewer: on (s = b S, I, D)
# its step is 3 mul + 3 add + 16 fma = 22 VALU instructions = 38 flops.
FLOPS_PER_STEP = 49
FLOPS_ISSUED_PER_STEP = 38
VALU_PER_STEP = 22
# The paper's scheme (forward Euler with the beta ramp): the ramp costs a
# subtract and an fma (3 flops), the step 2 mul + 5 fma (12 flops).
FLOPS_PER_STEP_EULER_RAMP = 15
PEAK_FP64_VECTOR = 78.6e12  # MI355X, FLOP/s
# MI355X's published FP32 vector peak (counts packed FP32 issue, which this
# library is built without: unpacked FP32 issues at the FP64 rate)
PEAK_FP32_VECTOR = 157.3e12

# HBM bytes per fused k_forward launch from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs (KiB per dispatch, scaled by the copy-probe factors 2.0 /
# 1.0), recorded with the hash of the kernel sources they were taken on;
# reported only while the sources match.
MEASURED_TRAFFIC = {
    "c3": {"bytes": 2.0 * 125349.2 * 1024 + 1.0 * 166695.9 * 1024,
           "sources": "980b2bb7202c9493",
           "summary": "profiles/k_forward_fused_batched_512x1024.md"},
}

METRIC = ("particle·RK4-steps/sec and wall-time-to-fit at fixed loss, "
          "plain PSO vs PSO+adjoint")
UNIT = "particle·RK4-steps/s"


def kernel_source_hash():
    import hashlib
    files = [os.path.join(ROOT, "paper_2204_12346_amd", "csrc", f)
             for f in ("forward.hip", "device.h")]
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in files)).hexdigest()[:16]


def build_workload(name, dtype):
    import synth
    import paper_2204_12346_amd as S
    if name == "c3":
        wl = synth.c3()
        launch = C3_LAUNCH
    elif name == "c2":
        wl = synth.c2()
        launch = dict(block=64, persistent=0)
    elif name == "c1":
        wl = synth.c1()
        launch = dict(block=64, persistent=0)
    elif name == "paper":
        wl = synth.paper()
        launch = dict(block=64, persistent=0)
    else:
        raise SystemExit(f"unknown workload {name}")
    three = wl.loss.startswith("ird")
    specs = [S.ProblemSpec.from_fit(f) for f in wl.fits]
    b = S.Batch(specs, dtype=dtype, obs_series=3 if three else 1, **launch)
    params = S.PsoParams(b, [f.lo for f in wl.fits], [f.hi for f in wl.fits], wl.w, wl.c1,
                         wl.c2, wl.seed)
    sw = S.Swarm(b)
    obs = b.pack_obs([f.obs3 if three else f.y for f in wl.fits])
    return wl, b, params, sw, obs


def host_cpu():
    """Model name of the host CPU and its logical CPU count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs visible"


def _threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _progress(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def cpu_baseline(wl, budget_s):
    """Oracle throughput on the host cores (OpenMP over particles, as the
    oracle stands): whole-batch loss evaluations of the workload (every
    particle of every problem, parameters uniform in each box), repeated
    while the elapsed time is below budget_s (at least one)."""
    import oracle
    threads = _threads()
    rng = np.random.default_rng(0)
    thetas = [f.lo + rng.uniform(0, 1, (f.n_part, f.d)) * (f.hi - f.lo) for f in wl.fits]
    probs = [oracle.Problem(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0,
                            model=1 if f.model == "euler_ramp" else 0) for f in wl.fits]
    three = wl.loss.startswith("ird")
    work = 0
    t0 = time.perf_counter()
    while True:
        for f, th, prob in zip(wl.fits, thetas, probs):
            oracle.loss_batch_model(prob, th, f.obs3 if three else f.y, wl.loss,
                                    nthreads=threads)
            work += f.n_part * f.T
            if time.perf_counter() - t0 > budget_s:
                break
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    # the same oracle on one thread: 64 particles of each problem in turn
    w1 = 0
    t1 = time.perf_counter()
    for f, th, prob in zip(wl.fits, thetas, probs):
        oracle.loss_batch_model(prob, th[:64], f.obs3 if three else f.y, wl.loss, nthreads=1)
        w1 += min(64, f.n_part) * f.T
        if time.perf_counter() - t1 > budget_s / 5:
            break
    dt1 = time.perf_counter() - t1
    return {"value": work / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "host": host_cpu(),
            "sample": f"whole-batch loss evaluations of the same workload, stopped after "
                      f"{budget_s:.0f} s: {work:.3e} particle-steps in {dt:.1f} s",
            "single_thread_value": w1 / dt1,
            "single_thread_sample": f"64 particles of each problem in turn, one thread: "
                                    f"{w1:.3e} particle-steps in {dt1:.1f} s"}


def oracle_per_config():
    """The oracle beside every other configuration, on the host cores
    (OpenMP over particles; the gradient sample over a thread pool, since
    the oracle's forward mode takes one vector per call):
      constant beta: the whole swarm run (256 x 200 iterations);
      segmented: 100 of the 1000 iterations, extrapolated linearly;
      gradients: forward-mode gradients of 1024 of the 65536 vectors;
      rolling windows: one window's 16 restarts x 20 of the 300 iterations,
        extrapolated linearly to 300 iterations and 52 windows (swarm only);
      the paper's timing case: the whole run (10000 x 100 Euler iterations)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import synth
    threads = _threads()
    out = {"cores": threads, "host": host_cpu(), "kind": "oracle"}

    def prob_of(f):
        return oracle.Problem(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0,
                              model=1 if f.model == "euler_ramp" else 0)

    def run(wl, f, iters):
        t0 = time.perf_counter()
        if f.model == "euler_ramp":
            oracle.pso_run_model(prob_of(f), f.obs3, wl.loss, f.n_part, f.lo, f.hi, wl.w,
                                 wl.c1, wl.c2, wl.seed, f.stream, iters, nthreads=threads)
        else:
            oracle.pso_run(prob_of(f), f.y, wl.loss, f.n_part, f.lo, f.hi, wl.w, wl.c1, wl.c2,
                           wl.seed, f.stream, iters, nthreads=threads)
        return time.perf_counter() - t0

    wl = synth.c1()
    f = wl.fits[0]
    t = run(wl, f, wl.iters)
    out["c1_constant_beta_256x200"] = {
        "seconds": t, "particle_steps_per_s": f.n_part * f.T * wl.iters / t,
        "sample": "whole run"}
    _progress("oracle c1 done")
    wl = synth.c2()
    f = wl.fits[0]
    t = run(wl, f, 100)
    out["c2_segmented_8192x1000"] = {
        "seconds_extrapolated": t * wl.iters / 100,
        "particle_steps_per_s": f.n_part * f.T * 100 / t,
        "sample": "100 of 1000 iterations, extrapolated linearly"}
    _progress("oracle c2 done")
    wl, thetas = synth.c4()
    f = wl.fits[0]
    prob = prob_of(f)
    sample = thetas[np.linspace(0, len(thetas) - 1, 1024).astype(int)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda th: oracle.loss_grad_fwd(prob, th, f.y, "ssre"), sample))
    t = time.perf_counter() - t0
    out["c4_gradients_65536x7300"] = {
        "gradients_per_s": len(sample) / t, "seconds_extrapolated": t * len(thetas) / len(sample),
        "sample": "forward-mode gradients of 1024 vectors spread over the 65536"}
    _progress("oracle c4 done")
    wl = synth.c5(windows=[0])
    t = sum(run(wl, f, 20) for f in wl.fits)
    steps = sum(f.n_part * f.T for f in wl.fits) * 20
    out["c5_rolling_52x16x4096x300"] = {
        "seconds_extrapolated": t * (wl.iters / 20) * 52,
        "particle_steps_per_s": steps / t,
        "sample": "one window's 16 restarts x 20 of 300 iterations, extrapolated to 300 "
                  "iterations and 52 windows; swarm only"}
    _progress("oracle c5 done")
    wl = synth.paper()
    f = wl.fits[0]
    t = run(wl, f, wl.iters)
    out["paper_euler_ramp_10000x100"] = {
        "seconds": t, "seconds_per_iteration": t / wl.iters,
        "particle_steps_per_s": f.n_part * f.T * wl.iters / t, "sample": "whole run"}
    _progress("oracle paper case done")
    return out


def copy_probe(mib):
    """A plain device copy of known size (for scaling HBM byte counters)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "launches": 3}))


def extra_tasks():
    """The other configurations, each measured once (see experiments.py):
    (name, thunk) in run order."""
    import synth
    from paper_2204_12346_amd import experiments as X
    t = [("c1_constant_beta_256x60d",
          lambda: X.swarm_throughput(synth.c1(), "f64", iters=200, graph_chunk=20,
                                     launch=dict(block=64)))]
    for dt in ("f64", "f32"):
        t.append((f"c2_segmented_8192x180d_{dt}",
                  lambda dt=dt: X.swarm_throughput(synth.c2(), dt, iters=200, graph_chunk=20,
                                                   launch=dict(block=64))))
    t.append(("c4_gradients_65536x7300steps", lambda: X.gradients_per_s(*synth.c4())))
    # the ceil(sqrt(T)) interval of two-level checkpointing, rounded to 90:
    # longer than the reverse sweep's LDS slice, so every interval is
    # replayed twice
    t.append(("c4_gradients_65536x7300steps_interval90",
              lambda: X.gradients_per_s(*synth.c4(), ckpt_interval=90)))
    # a refinement's gradient call (32 and 1024 vectors of the segmented
    # fit): the sequential and the segment-parallel reverse sweep
    t.append(("c2_refine_gradient_latency", lambda: X.refine_gradient_latency(synth.c2())))
    # M2: plain swarm against swarm + refinement of the top k by the adjoint
    # (projected L-BFGS, and the projected Adam the protocol names, with a
    # decaying step)
    t.append(("time_to_fit_c2",
              lambda: X.time_to_fit(synth.c2(), pso_first=(50, 100), ks=(32, 128, 1024),
                                    adam_arms=((100, 32),), adam_lr_end=1e-5,
                                    trials=(1, 4))))
    for dt in ("f64", "f32"):
        t.append((f"paper_euler_ramp_ird_mxse_10000x92d_{dt}",
                  lambda dt=dt: X.paper_iteration(synth.paper(), dt)))
    t.append(("rep_1000x10000x36d", lambda: X.repetition(synth.rep())))
    t.append(("c5_rolling_52x16x4096",
              lambda: X.rolling_forecast(synth.c5(), synth.c5_series()["truth"], restarts=16,
                                         launch=dict(C3_LAUNCH))))
    # the configuration names Adam for the refinement
    t.append(("c5_rolling_52x16x4096_adam",
              lambda: X.rolling_forecast(synth.c5(), synth.c5_series()["truth"], restarts=16,
                                         launch=dict(C3_LAUNCH), method="adam")))
    return t


def extras(only=None):
    res = {}
    for name, fn in extra_tasks():
        if only is not None and name != only:
            continue
        _progress(f"extras: {name} ...")
        res[name] = fn()
    if only is not None and not res:
        raise SystemExit(f"unknown extra {only!r}: one of "
                         + ", ".join(n for n, _ in extra_tasks()))
    return res


def summarize(ex):
    """The compact blocks of the JSON line from the full extras."""
    out = {}
    ttf = ex.get("time_to_fit_c2")
    if ttf:
        arms = {k: v for k, v in ttf.items() if isinstance(v, dict) and "median_s" in v}
        rel = "1e-06"
        med = {k: v["median_s"].get(rel) for k, v in arms.items()}
        ref_arms = {k: m for k, m in med.items() if k != "plain" and m is not None}
        best = min(ref_arms, key=ref_arms.get) if ref_arms else None
        out["time_to_fit"] = {
            "workload": "one fit: 8192 particles, 180 days, 13 beta segments, dt 0.1, FP64; "
                        f"{len(ttf['seeds'])} Philox seeds, median wall seconds from pso_init",
            "L_best": ttf["L_best"], "target": "loss <= L_best (1 + 1e-6)",
            "plain_median_s": med.get("plain"),
            "plain_cap_iterations": ttf["plain_cap_iterations"],
            "best_adjoint_arm": best, "best_adjoint_median_s": ref_arms.get(best),
            "median_s_by_arm": med,
            "median_s_1e-3_by_arm": {k: v["median_s"].get("0.001") for k, v in arms.items()},
        }
    g = ex.get("c4_gradients_65536x7300steps")
    if g:
        g90 = ex.get("c4_gradients_65536x7300steps_interval90", {})
        out["gradients"] = {
            "workload": "65536 parameter vectors x 7300 RK4 steps (365 days, dt 0.05), "
                        "13 segments, SSRE, FP64",
            "gradients_per_s": g["gradients_per_s"],
            "ms_loss_and_gradient": g["ms_loss_and_gradient"],
            "ms_forward_saving_checkpoints": g["ms_forward_saving_checkpoints"],
            "ms_reverse_sweep": g["ms_reverse_sweep"],
            "gradients_per_s_self_contained": g["gradients_per_s_self_contained"],
            "ckpt_interval": g["ckpt_interval"],
            "gradients_per_s_interval90": g90.get("gradients_per_s"),
        }
    lat = ex.get("c2_refine_gradient_latency")
    if lat:
        out["gradients"] = out.get("gradients", {})
        out["gradients"]["refinement_latency_ms"] = {
            "workload": "one gradient call on k vectors of the segmented fit (180 days, "
                        "dt 0.1, 13 segments)",
            **{k: {n: round(v, 4) for n, v in row.items()} for k, row in lat.items()}}
    o = {}
    for k in ("c1_constant_beta_256x60d", "c2_segmented_8192x180d_f64",
              "c2_segmented_8192x180d_f32"):
        if k in ex:
            o[k] = {"ms_per_iteration": ex[k]["ms_per_iteration"],
                    "particle_steps_per_s": ex[k]["particle_steps_per_s"]}
    for k in ("paper_euler_ramp_ird_mxse_10000x92d_f64", "paper_euler_ramp_ird_mxse_10000x92d_f32"):
        if k in ex:
            o[k] = {"ms_per_iteration_mean": ex[k]["ms_per_iteration_mean"],
                    "ms_per_iteration_std": ex[k]["ms_per_iteration_std"]}
    if "rep_1000x10000x36d" in ex:
        r = ex["rep_1000x10000x36d"]
        o["rep_1000x10000x36d"] = {"seconds_swarm": r["seconds_swarm"],
                                   "particle_steps_per_s": r["particle_steps_per_s"]}
    for k in ("c5_rolling_52x16x4096", "c5_rolling_52x16x4096_adam"):
        if k in ex:
            r = ex[k]
            o[k] = {"seconds_swarm": r["seconds_swarm"], "seconds_refine": r["seconds_refine"],
                    "rel_err_cum_deaths_h14_median": r["rel_err_cum_deaths_h14"][50]}
    if o:
        out["other_workloads"] = o
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="search the launch shape before timing instead of the recorded one")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (single fits, gradients, time to fit, ...)")
    ap.add_argument("--extra", default=None,
                    help="run only this one of the other workloads and print its JSON")
    args = ap.parse_args()
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.extra:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        torch.cuda.set_device(0)
        print(json.dumps(extras(args.extra)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(independent fits would shard across GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2204_12346_amd as S
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl, b, params, sw, obs = build_workload(args.workload, args.dtype)
    stream = torch.cuda.current_stream()
    kind = wl.loss

    S.pso_init(b, params, sw)
    if args.autotune:
        from paper_2204_12346_amd import autotune
        tuned = autotune.autotune_iterate(b, params, sw, obs, kind, use_cache=False,
                                          verbose=True)
        _progress(f"autotuned launch: {tuned}")
    S.sird_pso_iterate(b, params, sw, obs, kind, args.warmup)
    # the K timed iterations captured in one HIP graph (uploaded when created)
    graph = S.Graph(b, params, sw, obs, kind, iters_per_launch=args.steps)
    torch.cuda.synchronize()
    _progress(f"warmup done: {args.warmup} steps; graph of {args.steps} iterations ready")

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    graph.launch(1, stream=stream)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    graph.close()

    # the same K iterations eagerly, each evaluate launch between HIP events
    # on its stream: the kernel time of the roofline
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        S.pso_evaluate(b, params, sw, obs, kind, move_first=(i > 0))
        ev[i][1].record(stream)
        S.pso_gbest(b, params, sw)
    S.pso_complete_move(b, params, sw)
    end.record(stream)
    torch.cuda.synchronize()
    eager_ms = start.elapsed_time(end)
    fwd_ms = float(np.mean([a.elapsed_time(c) for a, c in ev]))
    _progress(f"timed: graph {total_ms / args.steps:.4f} ms/step, eager "
              f"{eager_ms / args.steps:.4f} ms/step, evaluate kernel {fwd_ms:.4f} ms")

    steps_per_iter = b.particle_steps
    value = steps_per_iter * args.steps / (total_ms / 1e3)
    # the fused kernel reads x, v, pbest_x, pbest_f and the observations and
    # writes x, v and f; personal-best copies depend on the data and are not
    # counted
    alg_bytes = 8 * (5 * b.theta_len + 2 * b.total_particles + b.obs_len)
    meas = MEASURED_TRAFFIC.get(args.workload)
    traffic = None
    if meas and meas["sources"] == kernel_source_hash() and args.dtype == "f64":
        traffic = meas["bytes"]
    paper = args.workload == "paper"
    flops_step = FLOPS_PER_STEP_EULER_RAMP if paper else FLOPS_PER_STEP
    achieved = flops_step * steps_per_iter / (fwd_ms / 1e3)
    peak = PEAK_FP32_VECTOR if args.dtype == "f32" else PEAK_FP64_VECTOR
    roof = {
        "kernel": ("k_forward fused (pso_evaluate: move + Euler with the beta ramp + "
                   "F_IRD^MXSE + pbest)" if paper else
                   "k_forward fused (pso_evaluate: move + RK4 + cost + pbest)"),
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": peak / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": traffic,
        "traffic_unit": "bytes per launch",
        "algorithmic_bytes": alg_bytes,
        "kernel_ms": fwd_ms,
        "flops_per_particle_step": flops_step,
    }
    if not paper and args.dtype == "f64":
        issued = FLOPS_ISSUED_PER_STEP * steps_per_iter / (fwd_ms / 1e3)
        roof["issued_flops_per_particle_step"] = FLOPS_ISSUED_PER_STEP
        roof["frac_issued"] = issued / PEAK_FP64_VECTOR
        roof["valu_issue_frac"] = ((VALU_PER_STEP * steps_per_iter / (fwd_ms / 1e3)) /
                                   (256 * 4 * 16 * 2.4e9))
    workloads = {
        "c3": "batched uneven fits: 512 regions x 1024 particles, W 28..365 days, 14-day "
              "beta segments, dt 0.1 day, iterations replayed from one HIP graph",
        "c2": "one fit: 8192 particles, 180 days, 13 beta segments, dt 0.1",
        "c1": "one fit: 256 particles, 60 days, constant beta, dt 0.1",
        "paper": "the paper's timing case: one fit, 10000 particles, 92 days, forward Euler "
                 "at one step per day with the beta ramp, F_IRD^MXSE"}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": workloads[args.workload],
            "problems": b.n_prob,
            "particles": b.total_particles,
            "particle_steps_per_step": steps_per_iter,
            "loss": kind,
            "launch": {"block": b.c.block, "persistent": b.c.persistent,
                       "waves_per_simd": b.c.waves_per_simd, "timing": "hipGraph replay"},
        },
        "eager": {"ms_per_step": eager_ms / args.steps,
                  "value": steps_per_iter * args.steps / (eager_ms / 1e3)},
        "roofline": roof,
        "wall_s": wall,
    }
    if not args.no_extras and args.workload == "c3":
        ex = extras()
        print("# extras " + json.dumps(ex), file=sys.stderr, flush=True)
        out.update(summarize(ex))
    if not args.no_cpu_baseline:
        _progress("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        if not args.no_extras and args.workload == "c3":
            out["cpu_baseline"]["per_config"] = oracle_per_config()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
