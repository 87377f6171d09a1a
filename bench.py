"""Throughput benchmark of the calibration hot path on one MI355X.

One step = one swarm iteration over the whole batch, as sird_pso_iterate
runs it: pso_evaluate (the previous iteration's Philox velocity/position
update, RK4 over every particle's window fused with the cost, personal
bests -- one kernel) then pso_gbest (per-problem argmin, iteration
advance).  Default workload: 512 independent
synthetic regions of uneven window (28..365 days) and population, 1024
particles each, 14-day beta segments, dt = 0.1 day, FP64.

Prints one JSON line: particle-RK4-steps/s of the timed steps, the roofline
of the dominant kernel (the forward integration, timed per launch with HIP
events on the stream it runs on) and the oracle's throughput on the host
cores on a bounded sample of the same workload.

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

# Algorithmic work of one particle-step of the FP64 forward: the RK4 step
# on (s = b S, I, D) issues 3 mul + 3 add + 16 fma = 22 VALU instructions =
# 38 flops (an FMA counts 2).  The per-day cost and the swarm update fused
# into the same kernel are not counted.
FLOPS_PER_STEP = 38
VALU_PER_STEP = 22
# The paper's scheme (forward Euler with the beta ramp): the ramp costs a
# subtract and an fma (3 flops), the step 2 mul + 5 fma (12 flops).
FLOPS_PER_STEP_EULER_RAMP = 15
PEAK_FP64_VECTOR = 78.6e12  # MI355X, FLOP/s

# HBM bytes per fused k_forward launch from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs (KiB per dispatch, scaled by the copy-probe factors 2.0 /
# 1.0), recorded with the hash of the kernel sources they were taken on;
# reported only while the sources match.
MEASURED_TRAFFIC = {
    "c3": {"bytes": 2.0 * 131147.5 * 1024 + 1.0 * 172955.3 * 1024,
           "sources": "b572d9935b042b07",
           "summary": "profiles/k_forward_fused_batched_512x1024.md"},
}

METRIC = "particle·RK4-steps/sec"
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


def cpu_baseline(wl, budget_s):
    """Oracle throughput on the host cores (OpenMP over particles, as the
    oracle stands): whole-batch loss evaluations of the workload (every
    particle of every problem, parameters uniform in each box), repeated
    while the elapsed time is below budget_s (at least one)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(0)
    thetas = [f.lo + rng.uniform(0, 1, (f.n_part, f.d)) * (f.hi - f.lo) for f in wl.fits]
    probs = [oracle.Problem(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0,
                            model=1 if f.model == "euler_ramp" else 0) for f in wl.fits]
    three = wl.loss.startswith("ird")
    work = 0
    reps = 0
    t0 = time.perf_counter()
    while True:
        for f, th, prob in zip(wl.fits, thetas, probs):
            oracle.loss_batch_model(prob, th, f.obs3 if three else f.y, wl.loss,
                                    nthreads=threads)
            work += f.n_part * f.T
            if time.perf_counter() - t0 > budget_s:
                break
        reps += 1
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
    (group, name, thunk) in run order."""
    import synth
    from paper_2204_12346_amd import experiments as X
    t = [("single-fit swarms", "c1_constant_beta_256x60d",
          lambda: X.swarm_throughput(synth.c1(), "f64", iters=200, graph_chunk=20,
                                     launch=dict(block=64)))]
    for dt in ("f64", "f32"):
        t.append(("single-fit swarms", f"c2_segmented_8192x180d_{dt}",
                  lambda dt=dt: X.swarm_throughput(synth.c2(), dt, iters=200, graph_chunk=20,
                                                   launch=dict(block=64))))
    # the batched workload with its iterations captured in HIP graphs
    t.append(("single-fit swarms", "c3_batched_512x1024_graph",
              lambda: X.swarm_throughput(synth.c3(), "f64", iters=50, warmup=5, graph_chunk=10,
                                         launch=dict(C3_LAUNCH))))
    t.append(("gradients", "c4_gradients_65536x7300steps",
              lambda: X.gradients_per_s(*synth.c4())))
    t.append(("gradients", "c4_gradients_65536x7300steps_interval10",
              lambda: X.gradients_per_s(*synth.c4(), ckpt_interval=10)))
    # L-BFGS arms, and two arms with the Adam refinement the protocol names
    t.append(("time to fit", "time_to_fit_c2",
              lambda: X.time_to_fit(synth.c2(), adam_arms=((100, 64), (100, 1024)))))
    for dt in ("f64", "f32"):
        t.append(("the paper's own timing case", f"paper_euler_ramp_ird_mxse_10000x92d_{dt}",
                  lambda dt=dt: X.paper_iteration(synth.paper(), dt)))
    t.append(("repetition study", "rep_1000x10000x36d", lambda: X.repetition(synth.rep())))
    t.append(("window-wise calibration", "windows_139x10000x36d",
              lambda: X.window_wise(synth.windows())))
    t.append(("rolling windows", "c5_rolling_52x16x4096",
              lambda: X.rolling_forecast(synth.c5(), synth.c5_series()["truth"], restarts=16,
                                         launch=dict(C3_LAUNCH))))
    # the configuration names Adam for the refinement
    t.append(("rolling windows", "c5_rolling_52x16x4096_adam",
              lambda: X.rolling_forecast(synth.c5(), synth.c5_series()["truth"], restarts=16,
                                         launch=dict(C3_LAUNCH), method="adam")))
    return t


def extras(only=None):
    res = {}
    group = None
    for g, name, fn in extra_tasks():
        if only is not None and name != only:
            continue
        if g != group:
            print(f"# extras: {g} ...", file=sys.stderr, flush=True)
            group = g
        res[name] = fn()
    if only is not None and not res:
        raise SystemExit(f"unknown extra {only!r}: one of "
                         + ", ".join(n for _, n, _ in extra_tasks()))
    return res


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
                    help="skip the other workloads (single fits, gradients, rolling windows)")
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
    tuned = None
    if args.autotune:
        from paper_2204_12346_amd import autotune
        tuned = autotune.autotune_iterate(b, params, sw, obs, kind, use_cache=False,
                                          verbose=True)
        print(f"# autotuned launch: {tuned}", file=sys.stderr, flush=True)
    S.sird_pso_iterate(b, params, sw, obs, kind, args.warmup)
    torch.cuda.synchronize()
    print(f"# warmup done: {args.warmup} steps", file=sys.stderr, flush=True)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        S.pso_evaluate(b, params, sw, obs, kind, move_first=(i > 0))
        ev[i][1].record(stream)
        S.pso_gbest(b, params, sw)
    S.pso_complete_move(b, params, sw)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    fwd_ms = float(np.mean([a.elapsed_time(c) for a, c in ev]))

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
    flops_step = FLOPS_PER_STEP_EULER_RAMP if args.workload == "paper" else FLOPS_PER_STEP
    achieved = flops_step * steps_per_iter / (fwd_ms / 1e3)
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
            "workload": {"c3": "batched uneven fits: 512 regions x 1024 particles, "
                               "W 28..365 days, 14-day beta segments, dt 0.1 day",
                         "c2": "one fit: 8192 particles, 180 days, 13 beta segments, dt 0.1",
                         "c1": "one fit: 256 particles, 60 days, constant beta, dt 0.1",
                         "paper": "the paper's timing case: one fit, 10000 particles, 92 days, "
                                  "forward Euler at one step per day with the beta ramp, "
                                  "F_IRD^MXSE"
                         }[args.workload],
            "problems": b.n_prob,
            "particles": b.total_particles,
            "particle_steps_per_step": steps_per_iter,
            "loss": kind,
            "launch": {"block": b.c.block, "persistent": b.c.persistent,
                       "waves_per_simd": b.c.waves_per_simd},
        },
        "roofline": {
            "kernel": ("k_forward fused (pso_evaluate: move + Euler with the beta ramp + "
                       "F_IRD^MXSE + pbest)" if args.workload == "paper" else
                       "k_forward fused (pso_evaluate: move + RK4 + cost + pbest)"),
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP64_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VECTOR,
            "traffic": traffic,
            "traffic_unit": "bytes per launch",
            "algorithmic_bytes": alg_bytes,
            "kernel_ms": fwd_ms,
            "flops_per_particle_step": flops_step,
            "valu_issue_frac": None if args.workload == "paper" else
                               (VALU_PER_STEP * steps_per_iter / (fwd_ms / 1e3)) /
                               (256 * 4 * 16 * 2.4e9),
        },
        "wall_s": wall,
    }
    if not args.no_extras and args.workload == "c3":
        out["extras"] = extras()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
