"""Calibration drivers built on the C ABI: a whole swarm run (Sec. 3.3) with
graph-captured iterations, gradient refinement of the swarm's best
particles, and the forecast that extends a fitted window (Sec. 4.2).

Every arithmetic step runs in the library's kernels; these functions only
sequence the calls and read back small results (losses, indices).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from .core import (CKPT_SEGMENTS, Batch, Graph, LbfgsState, ProblemSpec, PsoParams, Swarm,
                   pso_init, pso_topk, sird_adam_step, sird_gather, sird_integrate,
                   sird_lbfgs_accept, sird_lbfgs_propose, sird_loss, sird_loss_backward,
                   sird_loss_backward_workspace, sird_pso_iterate)


# Days per piece of the segment-parallel sweep (the library walks each beta
# segment in pieces of at most this many days, one wavefront per tile and
# piece).
SEG_PIECE_DAYS = 7


def default_ckpt_interval(batch: Batch) -> int:
    """Checkpoint interval of a refinement's gradients: the segment-parallel
    sweep (CKPT_SEGMENTS) when all its transfer wavefronts (tiles times the
    bound on pieces per vector, ceil(days / 7) + segments) fit in one
    wavefront per SIMD, the residency their LDS slices allow; there the
    sequential sweep (one wavefront per tile) would leave most SIMDs idle
    and the call's latency is what counts.  Else the sequential sweep's
    default (0): with more wavefronts than SIMDs the transfers run in
    rounds and walk more steps than the sequential sweep."""
    simds = 4 * torch.cuda.get_device_properties(batch.device).multi_processor_count
    c = batch.c
    pieces = -(-c.max_days // SEG_PIECE_DAYS) + (c.max_d - 3)
    return CKPT_SEGMENTS if batch.n_tiles * pieces <= simds else 0


def run_swarm(batch: Batch, params: PsoParams, obs, kind="ssre", iters=100, hist=True,
              graph_chunk=0, swarm: Optional[Swarm] = None, init=True) -> Swarm:
    """iters swarm iterations from pso_init.  graph_chunk > 0 replays a HIP
    graph of graph_chunk iterations (the remainder runs eagerly)."""
    sw = swarm if swarm is not None else Swarm(batch, hist_len=iters if hist else 0)
    if init:
        pso_init(batch, params, sw)
    done = 0
    if graph_chunk > 0 and iters >= graph_chunk:
        g = Graph(batch, params, sw, obs, kind, iters_per_launch=graph_chunk)
        n = iters // graph_chunk
        g.launch(n)
        done = n * graph_chunk
        torch.cuda.current_stream().synchronize()
        g.close()
    if iters > done:
        sird_pso_iterate(batch, params, sw, obs, kind, iters - done)
    return sw


@dataclasses.dataclass
class Refined:
    batch: Batch          # k particles per problem
    theta: torch.Tensor   # theta-shaped, refined parameters
    loss: torch.Tensor    # particle-indexed losses at theta
    idx: torch.Tensor     # [n_prob, k] source particles (local indices)
    steps: int


def refine_topk(batch: Batch, swarm: Swarm, params: PsoParams, obs, kind="ssre", k=32,
                max_steps=2000, lr=1e-3, rel_tol=1e-12, check_every=25,
                ckpt_interval=None) -> Refined:
    """Projected Adam (Kingma & Ba 2015) from the k best personal bests of
    every problem, in box-normalised coordinates, with gradients from the
    discrete adjoint.  Stops after max_steps, or when no refined particle's
    loss changed by more than rel_tol (relative) over check_every steps."""
    idx = pso_topk(batch, swarm.pbest_f, k)
    specs = [s.with_particles(k) for s in batch.specs]
    rb = Batch(specs, dtype="f64", device=batch.device, obs_series=batch.obs_series)
    theta = sird_gather(batch, swarm.pbest_x, params.lo, rb, idx, k)
    if ckpt_interval is None:
        ckpt_interval = default_ckpt_interval(rb)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    loss = rb.empty_particles()
    ws = torch.empty(max(sird_loss_backward_workspace(rb, ckpt_interval), 8), dtype=torch.uint8,
                     device=batch.device)
    prev = None
    t = 0
    for t in range(1, max_steps + 1):
        sird_loss_backward(rb, theta, obs, kind, grad_theta=grad, loss_out=loss,
                           ckpt_interval=ckpt_interval, workspace=ws)
        sird_adam_step(rb, theta, grad, m, v, params.lo, params.hi, t, lr=lr)
        if t % check_every == 0:
            cur = loss.clone()
            if prev is not None:
                change = ((cur - prev).abs() <= rel_tol * cur.abs()) | ~torch.isfinite(cur)
                if bool(change.all().item()):
                    break
            prev = cur
    final = sird_loss(rb, theta, obs, kind)
    return Refined(rb, theta, final, idx, t)


def lbfgs_rounds(rb: Batch, st: LbfgsState, params: PsoParams, obs, kind="ssre", rounds=200,
                 c1=1e-4, ckpt_interval=None, workspace=None, callback=None, check_every=0):
    """Run projected L-BFGS rounds on every parameter vector of rb: each
    round is sird_lbfgs_propose, the adjoint at the trial points
    (sird_loss_backward on st.trial_batch: all st.n_trials trials of every
    vector in one call), sird_lbfgs_accept.  st.f / st.grad must hold the
    loss and gradient at st.theta.  ckpt_interval and workspace serve the
    trial batch.  callback(round) every check_every rounds may return True
    to stop."""
    tb = st.trial_batch
    if ckpt_interval is None:
        ckpt_interval = default_ckpt_interval(tb)
    ws = workspace
    if ws is None:
        ws = torch.empty(max(sird_loss_backward_workspace(tb, ckpt_interval), 8),
                         dtype=torch.uint8, device=rb.device)
    for r in range(1, rounds + 1):
        sird_lbfgs_propose(rb, st, params.lo, params.hi)
        sird_loss_backward(tb, st.theta_t, obs, kind, grad_theta=st.grad_t, loss_out=st.f_t,
                           ckpt_interval=ckpt_interval, workspace=ws)
        sird_lbfgs_accept(rb, st, params.lo, params.hi, c1)
        if callback is not None and check_every and r % check_every == 0:
            if callback(r):
                return r
    return rounds


def refine_lbfgs(batch: Batch, swarm: Swarm, params: PsoParams, obs, kind="ssre", k=32,
                 max_rounds=500, rel_tol=1e-12, check_every=25, m=32,
                 ckpt_interval=None, n_trials=1) -> Refined:
    """Projected L-BFGS from the k best personal bests of every problem, in
    box-normalised coordinates, with gradients from the discrete adjoint
    and n_trials trial steps per round.  Stops after max_rounds, or when no
    vector's loss changed by more than rel_tol (relative) over check_every
    rounds."""
    idx = pso_topk(batch, swarm.pbest_f, k)
    specs = [s.with_particles(k) for s in batch.specs]
    rb = Batch(specs, dtype="f64", device=batch.device, obs_series=batch.obs_series)
    theta = sird_gather(batch, swarm.pbest_x, params.lo, rb, idx, k)
    st = LbfgsState(rb, theta, m=m, n_trials=n_trials)
    if ckpt_interval is None:
        ckpt_interval = default_ckpt_interval(st.trial_batch)
    # the trial batch's workspace also serves the k vectors themselves
    ws = torch.empty(max(sird_loss_backward_workspace(st.trial_batch, ckpt_interval), 8),
                     dtype=torch.uint8, device=batch.device)
    sird_loss_backward(rb, st.theta, obs, kind, grad_theta=st.grad, loss_out=st.f,
                       ckpt_interval=ckpt_interval, workspace=ws)
    prev = [st.f.clone()]

    def converged(r):
        cur = st.f.clone()
        done = bool((((cur - prev[0]).abs() <= rel_tol * cur.abs()) |
                     ~torch.isfinite(cur)).all().item())
        prev[0] = cur
        return done

    steps = lbfgs_rounds(rb, st, params, obs, kind, max_rounds, ckpt_interval=ckpt_interval,
                         workspace=ws, callback=converged, check_every=check_every)
    return Refined(rb, st.theta, st.f.clone(), idx, steps)


def best_per_problem(batch: Batch, theta: torch.Tensor, loss: torch.Tensor):
    """(theta_best (n_prob, d) list, loss_best array) of the lowest loss of
    every problem (lowest index on ties, NaN never wins)."""
    th = batch.unpack_theta(theta)
    ls = batch.split_particles(loss)
    outs, vals = [], []
    for a, l in zip(th, ls):
        l = np.where(np.isnan(l), np.inf, l)
        i = int(np.argmin(l)) if len(l) else -1
        outs.append(a[i] if i >= 0 else None)
        vals.append(l[i] if i >= 0 else np.inf)
    return outs, np.array(vals)


def forecast(specs: Sequence[ProblemSpec], thetas: Sequence[np.ndarray], horizon_days: int,
             device="cuda") -> List[np.ndarray]:
    """Integrate every parameter vector over its window plus horizon_days
    (the last beta segment continues past the window, and the ramp model
    stays at beta2, as the paper extends a window with its last
    transmission rate); returns per problem an array (n, 4, W + horizon + 1)
    of S, I, R, D."""
    ext = [s.with_particles(len(th), W=s.W + horizon_days) for s, th in zip(specs, thetas)]
    # segments are anchored at the window start; the last one extends
    b = Batch(ext, with_traj=True, device=device)
    traj = sird_integrate(b, b.pack_theta([np.asarray(t) for t in thetas]))
    return b.unpack_traj(traj)
