"""Autotuner of the integration kernel's launch shape.

Searches threads per block (1, 2, 4 or 8 wavefronts, each on its own
64-particle tile) and the persistent-queue size (0 = one wavefront per tile
dispatched longest-first; otherwise that many resident wavefronts pulling
tiles from a device counter), times sird_loss with HIP events, and checks
that every candidate returns bitwise the same losses as the first -- the
launch shape must never change results.  Choices are cached in a JSON file
keyed by device, precision and workload shape.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional

import torch

from .core import Batch, sird_loss

CACHE_ENV = "SIRD_AUTOTUNE_CACHE"


def _cache_path():
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache",
                                                   "sird_autotune.json"))


def shape_key(batch: Batch) -> str:
    dev = torch.cuda.get_device_name(batch.device)
    steps = [s.T for s in batch.specs]
    return (f"{dev}|{'f32' if batch.c.dtype else 'f64'}|probs={batch.n_prob}|"
            f"particles={batch.total_particles}|maxT={max(steps)}|sumT={sum(steps)}")


def candidates(n_cu: int) -> List[Dict[str, int]]:
    out = []
    for block in (64, 128, 256, 512):
        out.append(dict(block=block, persistent=0))
    for wpc in (4, 6, 8, 10, 12, 16):  # resident wavefronts per CU
        out.append(dict(block=64, persistent=n_cu * wpc))
    out.append(dict(block=256, persistent=n_cu * 8))
    return out


def time_config(batch: Batch, theta, obs, kind, reps=5, stream=None):
    s = stream or torch.cuda.current_stream()
    out = torch.empty(max(batch.total_particles, 1), dtype=torch.float64, device=batch.device)
    sird_loss(batch, theta, obs, kind, out)  # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        sird_loss(batch, theta, obs, kind, out)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def autotune(batch: Batch, theta, obs, kind="ssre", reps=5, use_cache=True,
             verbose=False) -> Dict[str, int]:
    """Pick and apply the fastest launch shape for this batch; returns it."""
    key = shape_key(batch)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        best = cache[key]["launch"]
        batch.configure(**best)
        return best
    n_cu = torch.cuda.get_device_properties(batch.device).multi_processor_count
    ref = None
    results = []
    for cand in candidates(n_cu):
        lds = (cand["block"] // 64) * 2 * (batch.c.max_days + 1) * 8
        if lds > 65536:
            continue
        batch.configure(**cand)
        ms, out = time_config(batch, theta, obs, kind, reps)
        h = out.cpu()
        if ref is None:
            ref = h
        elif not torch.equal(h.view(torch.int64), ref.view(torch.int64)):
            raise RuntimeError(f"launch shape {cand} changed the losses: kernel bug")
        results.append((ms, cand))
        if verbose:
            print(f"autotune {cand}: {ms:.4f} ms", flush=True)
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    batch.configure(**best)
    if use_cache:
        cache[key] = {"launch": best, "ms": results[0][0],
                      "all": [[c, m] for m, c in results]}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(cache, fh, indent=1)
        except OSError:
            pass
    return best
