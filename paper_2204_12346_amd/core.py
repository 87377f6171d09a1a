"""Python face of the C ABI: batches of calibration problems, swarm state,
and one function per entry point with the C name.

Only argument marshalling happens here; the arithmetic of every call runs in
the HIP kernels of ``libsird.so``.  PyTorch provides device memory and the
stream (torch's current stream unless one is given).

Layouts (see ``include/sird.h``):
  * theta-shaped arrays: per problem a ``[d][n_part]`` block at ``theta_off``;
  * particle-indexed arrays: ``total_particles`` entries, problem r at
    ``[p_off, p_off + n_part)``;
  * box-shaped arrays: ``d`` values per problem at ``box_off``.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import LOSS, MODEL, SIRD_F32, SIRD_F64, check, lib, ptr, stream_handle


def _kind(kind):
    return LOSS[kind] if isinstance(kind, str) else int(kind)


class Args:
    """Device array arguments of one call, checked before their addresses
    reach the C ABI.  Calling the object checks one argument -- a torch
    tensor (not a host array) of the given dtype, contiguous, holding at
    least n elements; None passes only where the argument is optional --
    and returns its address; device() then checks that every argument and
    its batch are on one GPU.  Raises TypeError or ValueError, so a bad
    argument never reaches a kernel."""

    def __init__(self, batch: "Batch"):
        self.batch = batch
        self.seen = []

    def __call__(self, t, n, name, dtype=torch.float64, optional=False, batch=None):
        if t is None:
            if optional:
                return None
            raise ValueError(f"{name}: a device tensor is required")
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: expected a torch tensor on the batch's GPU, "
                            f"got {type(t).__name__}")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: tensor is not contiguous")
        if t.numel() < n:
            raise ValueError(f"{name}: {t.numel()} elements, the call needs {n}")
        self.seen.append((t, name, batch or self.batch))
        return t.data_ptr()

    def workspace(self, ws, nbytes, name="workspace"):
        """(address, size in bytes) of a workspace tensor of any dtype
        holding at least nbytes."""
        ptr_ = self(ws, 0, name, dtype=None)
        size = ws.numel() * ws.element_size()
        if size < nbytes:
            raise ValueError(f"{name}: {size} bytes, the call needs {nbytes}")
        return ptr_, size

    def device(self):
        for t, name, b in self.seen:
            if b.device.type != "cuda":
                raise ValueError(f"{name}: the batch lives on {b.device}, not on a GPU")
            if t.device != b.device:
                raise ValueError(f"{name}: tensor on {t.device}, the batch on {b.device}")


class ProblemSpec:
    """One calibration window.  model "rk4": theta = (beta_1..beta_K, gamma,
    mu, I0) with beta piecewise constant on K segments of seg_days;
    model "euler_ramp" (K = 4): theta = (beta1, beta2, t1, t2, gamma, mu,
    I0), forward Euler with the ramp of eq. (beta)."""

    def __init__(self, W, spd, seg_days, K, N, R0=0.0, D0=0.0, n_part=0, stream=0,
                 model="rk4"):
        self.W, self.spd, self.seg_days, self.K = int(W), int(spd), int(seg_days), int(K)
        self.N, self.R0, self.D0 = float(N), float(R0), float(D0)
        self.n_part, self.stream = int(n_part), int(stream)
        self.model = MODEL[model] if isinstance(model, str) else int(model)

    def with_particles(self, n_part, W=None):
        """Same window (or one of W days) with n_part parameter vectors."""
        return ProblemSpec(self.W if W is None else W, self.spd, self.seg_days, self.K, self.N,
                           self.R0, self.D0, n_part, self.stream, self.model)

    @property
    def d(self):
        return self.K + 3

    @property
    def T(self):
        return self.W * self.spd

    @classmethod
    def from_fit(cls, f, n_part=None):
        return cls(f.W, f.spd, f.seg_days, f.K, f.N, f.R0, f.D0,
                   f.n_part if n_part is None else n_part, f.stream,
                   getattr(f, "model", "rk4"))


class Batch:
    """A planned batch of problems resident on one device.  obs_series = 3
    lays out I, R and D observations per problem (the F_IRD costs).
    replicas = T > 1 repeats the problems T times, replica-major: replica t
    of problem r has its own parameter vectors (theta and particle offsets
    shifted by t theta_len and t total_particles of one replica) and shares
    the observations and box of replica 0 -- the layout of the L-BFGS trial
    points, T theta-shaped blocks back to back."""

    def __init__(self, specs: Sequence[ProblemSpec], dtype="f64", block=0, persistent=0,
                 with_traj=False, device="cuda", obs_series=1, waves_per_simd=0, ppl=1,
                 replicas=1):
        base = list(specs)
        self.replicas = int(replicas)
        if self.replicas < 1 or (self.replicas > 1 and with_traj):
            raise ValueError("replicas must be >= 1, and 1 with trajectories")
        specs = base * self.replicas
        n = len(specs)
        self.obs_series = int(obs_series)
        tab = np.zeros(n, dtype=_lib.PROBLEM_DTYPE)
        p_off = theta_off = obs_off = traj_off = box_off = 0
        shared = []   # (obs_off, box_off) of replica 0
        for r, s in enumerate(specs):
            if r < len(base):
                shared.append((obs_off, box_off))
            o_off, b_off = shared[r % len(base)]
            tab[r] = (s.W, s.spd, s.seg_days, s.K, s.n_part, s.model, s.N, s.R0, s.D0,
                      p_off, theta_off, o_off, traj_off if with_traj else 0, b_off, s.stream)
            p_off += s.n_part
            theta_off += s.d * s.n_part
            if r < len(base):
                obs_off += self.obs_series * (s.W + 1)
                box_off += s.d
            if with_traj:
                traj_off += 4 * (s.W + 1) * s.n_part
        self.specs = specs
        self.table = tab
        self.total_particles = p_off
        self.theta_len = theta_off
        self.obs_len = obs_off
        self.traj_len = traj_off
        self.box_len = box_off
        n_tiles_max = sum((s.n_part + 63) // 64 for s in specs)
        tiles = np.zeros(max(n_tiles_max, 1), dtype=_lib.TILE_DTYPE)
        nt = lib().sird_plan_tiles(tab.ctypes.data, n, tiles.ctypes.data, len(tiles))
        check(nt if nt < 0 else 0, "sird_plan_tiles")
        self.n_tiles = nt
        self.tiles_host = tiles[:nt]
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.probs_dev = torch.from_numpy(tab.view(np.uint8).copy()).to(self.device)
        self.tiles_dev = torch.from_numpy(tiles.view(np.uint8).copy()).to(self.device)
        pairs = np.zeros(max(nt, 1), dtype=np.int32)
        npairs = lib().sird_plan_pairs(tiles.ctypes.data, nt, pairs.ctypes.data, len(pairs))
        check(npairs if npairs < 0 else 0, "sird_plan_pairs")
        self.n_pairs = npairs
        self.pairs_host = pairs[:npairs]
        self.pairs_dev = torch.from_numpy(pairs.copy()).to(self.device)
        self.sched_dev = torch.zeros(2, dtype=torch.int32, device=self.device)
        b = _lib.sird_batch()
        b.dtype = SIRD_F32 if dtype in ("f32", SIRD_F32) else SIRD_F64
        b.block = int(block)
        b.persistent = int(persistent)
        b.waves_per_simd = int(waves_per_simd)
        b.ppl = int(ppl)
        check(lib().sird_batch_plan(ctypes.byref(b), tab.ctypes.data, n, p_off, theta_off,
                                    obs_off, traj_off, box_off, self.obs_series, nt,
                                    ptr(self.probs_dev),
                                    ptr(self.tiles_dev), ptr(self.sched_dev)),
              "sird_batch_plan")
        b.n_pairs = npairs
        b.pair_tiles = ptr(self.pairs_dev)
        self.c = b

    # ------------------------------------------------------------ config
    def configure(self, block=None, persistent=None, dtype=None, waves_per_simd=None,
                  ppl=None):
        if ppl is not None:
            self.c.ppl = int(ppl)
        if block is not None:
            self.c.block = int(block)
        if persistent is not None:
            self.c.persistent = int(persistent)
        if waves_per_simd is not None:
            self.c.waves_per_simd = int(waves_per_simd)
        if dtype is not None:
            self.c.dtype = SIRD_F32 if dtype in ("f32", SIRD_F32) else SIRD_F64
        return self

    @property
    def n_prob(self):
        return len(self.specs)

    @property
    def particle_steps(self):
        return sum(s.n_part * s.T for s in self.specs)

    # ------------------------------------------------------------ layout
    def pack_theta(self, per_problem: Sequence[np.ndarray]) -> torch.Tensor:
        """List of (n_part, d) arrays -> theta-shaped device tensor."""
        out = np.zeros(self.theta_len)
        for s, row, a in zip(self.specs, self.table, per_problem):
            a = np.asarray(a, dtype=np.float64)
            assert a.shape == (s.n_part, s.d), (a.shape, s.n_part, s.d)
            o = int(row["theta_off"])
            out[o:o + s.d * s.n_part] = a.T.reshape(-1)
        return torch.from_numpy(out).to(self.device)

    def unpack_theta(self, t: torch.Tensor) -> List[np.ndarray]:
        h = t.detach().cpu().numpy()
        res = []
        for s, row in zip(self.specs, self.table):
            o = int(row["theta_off"])
            res.append(h[o:o + s.d * s.n_part].reshape(s.d, s.n_part).T.copy())
        return res

    def pack_obs(self, per_problem: Sequence[np.ndarray]) -> torch.Tensor:
        """Per problem obs_series x (W+1) values: D, or I, R, D concatenated."""
        out = np.zeros(self.obs_len)
        for s, row, y in zip(self.specs, self.table, per_problem):
            y = np.asarray(y, dtype=np.float64).reshape(-1)
            n = self.obs_series * (s.W + 1)
            assert y.shape == (n,), (y.shape, n)
            o = int(row["obs_off"])
            out[o:o + n] = y
        return torch.from_numpy(out).to(self.device)

    def pack_box(self, per_problem: Sequence[np.ndarray]) -> torch.Tensor:
        out = np.zeros(self.box_len)
        for s, row, v in zip(self.specs, self.table, per_problem):
            v = np.asarray(v, dtype=np.float64)
            assert v.shape == (s.d,)
            o = int(row["box_off"])
            out[o:o + s.d] = v
        return torch.from_numpy(out).to(self.device)

    def unpack_box(self, t: torch.Tensor) -> List[np.ndarray]:
        h = t.detach().cpu().numpy()
        return [h[int(r["box_off"]):int(r["box_off"]) + s.d].copy()
                for s, r in zip(self.specs, self.table)]

    def split_particles(self, t: torch.Tensor) -> List[np.ndarray]:
        h = t.detach().cpu().numpy()
        return [h[int(r["p_off"]):int(r["p_off"]) + s.n_part].copy()
                for s, r in zip(self.specs, self.table)]

    def unpack_traj(self, t: torch.Tensor) -> List[np.ndarray]:
        """traj tensor -> list of (n_part, 4, W+1) arrays."""
        h = t.detach().cpu().numpy()
        res = []
        for s, row in zip(self.specs, self.table):
            o = int(row["traj_off"])
            blk = h[o:o + 4 * (s.W + 1) * s.n_part].reshape(4, s.W + 1, s.n_part)
            res.append(np.transpose(blk, (2, 0, 1)).copy())
        return res

    def empty_theta(self):
        return torch.empty(self.theta_len, dtype=torch.float64, device=self.device)

    def empty_particles(self):
        return torch.empty(max(self.total_particles, 1), dtype=torch.float64,
                           device=self.device)


class Swarm:
    """Device swarm state of a batch (pso_state)."""

    def __init__(self, batch: Batch, hist_len=0):
        dev = batch.device
        th = max(batch.theta_len, 1)
        P = max(batch.total_particles, 1)
        f64 = dict(dtype=torch.float64, device=dev)
        self.x = torch.zeros(th, **f64)
        self.v = torch.zeros(th, **f64)
        self.pbest_x = torch.zeros(th, **f64)
        self.pbest_f = torch.zeros(P, **f64)
        self.gbest_x = torch.zeros(max(batch.box_len, 1), **f64)
        self.gbest_f = torch.zeros(batch.n_prob, **f64)
        self.gbest_idx = torch.zeros(batch.n_prob, dtype=torch.int64, device=dev)
        self.iter = torch.zeros(2, dtype=torch.int64, device=dev)
        self.f = torch.zeros(P, **f64)
        self.hist_len = int(hist_len)
        if hist_len:
            self.hist_f = torch.full((hist_len, batch.n_prob), float("nan"), **f64)
            self.hist_idx = torch.full((hist_len, batch.n_prob), -2, dtype=torch.int64,
                                       device=dev)
        else:
            self.hist_f = self.hist_idx = None
        s = _lib.pso_state()
        s.x, s.v, s.pbest_x, s.pbest_f = ptr(self.x), ptr(self.v), ptr(self.pbest_x), ptr(self.pbest_f)
        s.gbest_x, s.gbest_f, s.gbest_idx = ptr(self.gbest_x), ptr(self.gbest_f), ptr(self.gbest_idx)
        s.iter, s.f = ptr(self.iter), ptr(self.f)
        s.hist_f, s.hist_idx, s.hist_len = ptr(self.hist_f), ptr(self.hist_idx), self.hist_len
        self.c = s


class PsoParams:
    def __init__(self, batch: Batch, lo, hi, w=0.7, c1=1.5, c2=1.5, seed=0):
        """lo, hi: box-shaped device tensors (or per-problem lists)."""
        self.lo = lo if isinstance(lo, torch.Tensor) else batch.pack_box(lo)
        self.hi = hi if isinstance(hi, torch.Tensor) else batch.pack_box(hi)
        p = _lib.pso_params()
        p.w, p.c1, p.c2, p.seed = float(w), float(c1), float(c2), int(seed)
        a = Args(batch)
        p.lo = a(self.lo, batch.box_len, "lo")
        p.hi = a(self.hi, batch.box_len, "hi")
        a.device()
        self.c = p


# ------------------------------------------------------------------ calls
def sird_integrate(batch: Batch, theta, traj=None, stream=None):
    if traj is None:
        traj = torch.empty(max(batch.traj_len, 1), dtype=torch.float64, device=batch.device)
    a = Args(batch)
    args = (a(theta, batch.theta_len, "theta"), a(traj, batch.traj_len, "traj"))
    a.device()
    check(lib().sird_integrate(ctypes.byref(batch.c), *args, stream_handle(stream)),
          "sird_integrate")
    return traj


def sird_loss(batch: Batch, theta, obs, kind="ssre", loss=None, stream=None,
              workspace=None, ckpt_interval=0):
    """Losses of every particle.  With a workspace (a device tensor of at
    least sird_loss_backward_workspace(batch, ckpt_interval) bytes) the
    adjoint's forward pass computes them and saves its checkpoints there for
    sird_loss_backward(..., from_forward=True)."""
    if loss is None:
        loss = batch.empty_particles()
    a = Args(batch)
    args = (a(theta, batch.theta_len, "theta"), a(obs, batch.obs_len, "obs"), _kind(kind),
            a(loss, batch.total_particles, "loss"))
    if workspace is None:
        ws, nbytes = None, 0
    else:
        ws, nbytes = a.workspace(workspace, sird_loss_backward_workspace(batch, ckpt_interval))
    a.device()
    check(lib().sird_loss(ctypes.byref(batch.c), *args, int(ckpt_interval), ws, nbytes,
                          stream_handle(stream)), "sird_loss")
    return loss


def pso_init(batch: Batch, params: PsoParams, swarm: Swarm, stream=None):
    check(lib().pso_init(ctypes.byref(batch.c), ctypes.byref(params.c), ctypes.byref(swarm.c),
                         stream_handle(stream)), "pso_init")


def pso_step(batch: Batch, params: PsoParams, swarm: Swarm, stream=None):
    check(lib().pso_step(ctypes.byref(batch.c), ctypes.byref(params.c), ctypes.byref(swarm.c),
                         stream_handle(stream)), "pso_step")


def sird_pso_iterate(batch: Batch, params: PsoParams, swarm: Swarm, obs, kind="ssre",
                     n_iters=1, stream=None):
    a = Args(batch)
    o = a(obs, batch.obs_len, "obs")
    a.device()
    check(lib().sird_pso_iterate(ctypes.byref(batch.c), ctypes.byref(params.c),
                                 ctypes.byref(swarm.c), o, _kind(kind), int(n_iters),
                                 stream_handle(stream)), "sird_pso_iterate")


def pso_evaluate(batch: Batch, params: PsoParams, swarm: Swarm, obs, kind="ssre",
                 move_first=False, stream=None):
    a = Args(batch)
    o = a(obs, batch.obs_len, "obs")
    a.device()
    check(lib().pso_evaluate(ctypes.byref(batch.c), ctypes.byref(params.c),
                             ctypes.byref(swarm.c), o, _kind(kind), int(bool(move_first)),
                             stream_handle(stream)), "pso_evaluate")


def pso_gbest(batch: Batch, params: PsoParams, swarm: Swarm, stream=None):
    check(lib().pso_gbest(ctypes.byref(batch.c), ctypes.byref(params.c), ctypes.byref(swarm.c),
                          stream_handle(stream)), "pso_gbest")


def pso_complete_move(batch: Batch, params: PsoParams, swarm: Swarm, stream=None):
    check(lib().pso_complete_move(ctypes.byref(batch.c), ctypes.byref(params.c),
                                  ctypes.byref(swarm.c), stream_handle(stream)),
          "pso_complete_move")


# ckpt_interval of the segment-parallel reverse sweep (SIRD_CKPT_SEGMENTS):
# every beta segment of every vector at once, for batches too small to fill
# the GPU; the gradient equals the sequential sweep's up to rounding.
CKPT_SEGMENTS = -1


def sird_loss_backward_workspace(batch: Batch, ckpt_interval=0):
    return int(lib().sird_loss_backward_workspace(ctypes.byref(batch.c), int(ckpt_interval)))


def sird_loss_backward(batch: Batch, theta, obs, kind="ssre", grad_loss=None,
                       grad_theta=None, loss_out=None, ckpt_interval=0, workspace=None,
                       stream=None, from_forward=False):
    """Returns (grad_theta, loss_out).  from_forward: the workspace holds
    the forward pass of sird_loss(..., workspace=workspace) on the same
    theta, obs, kind and interval; only the reverse sweep runs."""
    if grad_theta is None:
        grad_theta = batch.empty_theta()
    nbytes = sird_loss_backward_workspace(batch, ckpt_interval)
    if workspace is None:
        if from_forward:
            raise ValueError("from_forward needs the workspace sird_loss filled")
        workspace = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=batch.device)
    a = Args(batch)
    args = (a(theta, batch.theta_len, "theta"), a(obs, batch.obs_len, "obs"), _kind(kind),
            a(grad_loss, batch.total_particles, "grad_loss", optional=True),
            a(grad_theta, batch.theta_len, "grad_theta"),
            a(loss_out, batch.total_particles, "loss_out", optional=True))
    ws, size = a.workspace(workspace, nbytes)
    a.device()
    check(lib().sird_loss_backward(ctypes.byref(batch.c), *args, int(ckpt_interval),
                                   int(bool(from_forward)), ws, size, stream_handle(stream)),
          "sird_loss_backward")
    return grad_theta, loss_out


# Bytes of the static device scratch behind sird_loss_backward_static.
STATIC_SCRATCH_BYTES = 64 << 20


def sird_loss_backward_static(batch: Batch, theta, obs, kind="ssre", grad_loss=None,
                              grad_theta=None, loss_out=None, ckpt_interval=0, stream=None):
    """sird_loss_backward with the library's static per-GPU workspace: the
    C call allocates nothing (pass grad_theta, and loss_out if wanted, to
    allocate nothing here either).  Returns (grad_theta, loss_out)."""
    if grad_theta is None:
        grad_theta = batch.empty_theta()
    a = Args(batch)
    args = (a(theta, batch.theta_len, "theta"), a(obs, batch.obs_len, "obs"), _kind(kind),
            a(grad_loss, batch.total_particles, "grad_loss", optional=True),
            a(grad_theta, batch.theta_len, "grad_theta"),
            a(loss_out, batch.total_particles, "loss_out", optional=True))
    a.device()
    check(lib().sird_loss_backward_static(ctypes.byref(batch.c), *args, int(ckpt_interval),
                                          stream_handle(stream)),
          "sird_loss_backward_static")
    return grad_theta, loss_out


def pso_topk(batch: Batch, pbest_f, k, idx_out=None, stream=None):
    if idx_out is None:
        idx_out = torch.empty((batch.n_prob, k), dtype=torch.int64, device=batch.device)
    a = Args(batch)
    args = (a(pbest_f, batch.total_particles, "pbest_f"), int(k),
            a(idx_out, batch.n_prob * int(k), "idx_out", dtype=torch.int64))
    a.device()
    check(lib().pso_topk(ctypes.byref(batch.c), *args, stream_handle(stream)), "pso_topk")
    return idx_out


def sird_gather(src: Batch, src_theta, src_lo, dst: Batch, idx, k, dst_theta=None,
                stream=None):
    if dst_theta is None:
        dst_theta = dst.empty_theta()
    a = Args(src)
    sa = (a(src_theta, src.theta_len, "src_theta"), a(src_lo, src.box_len, "src_lo"))
    da = (a(dst_theta, dst.theta_len, "dst_theta", batch=dst),
          a(idx, src.n_prob * int(k), "idx", dtype=torch.int64))
    a.device()
    check(lib().sird_gather(ctypes.byref(src.c), *sa, ctypes.byref(dst.c), *da, int(k),
                            stream_handle(stream)), "sird_gather")
    return dst_theta


def sird_adam_step(batch: Batch, theta, grad, m, v, lo, hi, t, lr=1e-3, beta1=0.9,
                   beta2=0.999, eps=1e-8, stream=None):
    p = _lib.adam_params(lr, beta1, beta2, eps)
    a = Args(batch)
    args = [a(t_, batch.theta_len, n)
            for t_, n in ((theta, "theta"), (grad, "grad"), (m, "m"), (v, "v"))]
    args += [a(lo, batch.box_len, "lo"), a(hi, batch.box_len, "hi")]
    a.device()
    check(lib().sird_adam_step(ctypes.byref(batch.c), *args, int(t), ctypes.byref(p),
                               stream_handle(stream)), "sird_adam_step")


class LbfgsState:
    """Device state of projected L-BFGS over the parameter vectors of a
    batch (lbfgs_state); theta is copied in, f/grad are evaluated by the
    caller before the first round.  n_trials > 1 trial points per round:
    theta_t, grad_t and f_t hold n_trials blocks, and trial_batch (the
    batch with that many replicas) evaluates them in one call."""

    def __init__(self, batch: Batch, theta, m=32, log_last=True, n_trials=1):
        dev = batch.device
        th = max(batch.theta_len, 1)
        P = max(batch.total_particles, 1)
        f64 = dict(dtype=torch.float64, device=dev)
        self.m = int(m)
        self.n_trials = int(n_trials)
        if not 1 <= self.n_trials <= 8:
            raise ValueError("n_trials must be in 1..8")
        T = self.n_trials
        self.trial_batch = batch if T == 1 else Batch(
            batch.specs[:batch.n_prob // batch.replicas], dtype="f64", device=dev,
            obs_series=batch.obs_series, replicas=T * batch.replicas)
        a = Args(batch)
        a(theta, batch.theta_len, "theta")
        a.device()
        self.theta = theta.detach().clone()
        self.grad = torch.zeros(th, **f64)
        self.f = torch.zeros(P, **f64)
        self.theta_t = torch.zeros(T * th, **f64)
        self.grad_t = torch.zeros(T * th, **f64)
        self.f_t = torch.zeros(T * P, **f64)
        self.S = torch.zeros(self.m * th, **f64)
        self.Y = torch.zeros(self.m * th, **f64)
        self.rho = torch.zeros(self.m * P, **f64)
        self.alpha = torch.ones(P, **f64)
        self.gp = torch.zeros(P, **f64)
        self.count = torch.zeros(P, dtype=torch.int32, device=dev)
        self.head = torch.zeros(P, dtype=torch.int32, device=dev)
        c = _lib.lbfgs_state()
        for name in ("theta", "grad", "f", "theta_t", "grad_t", "f_t", "S", "Y", "rho",
                     "alpha", "gp", "count", "head"):
            setattr(c, name, ptr(getattr(self, name)))
        c.m = self.m
        c.log_last = int(bool(log_last))
        c.n_trials = T
        self.c = c


def sird_lbfgs_propose(batch: Batch, st: LbfgsState, lo, hi, stream=None):
    a = Args(batch)
    box = (a(lo, batch.box_len, "lo"), a(hi, batch.box_len, "hi"))
    a.device()
    check(lib().sird_lbfgs_propose(ctypes.byref(batch.c), ctypes.byref(st.c), *box,
                                   stream_handle(stream)), "sird_lbfgs_propose")


def sird_lbfgs_accept(batch: Batch, st: LbfgsState, lo, hi, c1=1e-4, stream=None):
    a = Args(batch)
    box = (a(lo, batch.box_len, "lo"), a(hi, batch.box_len, "hi"))
    a.device()
    check(lib().sird_lbfgs_accept(ctypes.byref(batch.c), ctypes.byref(st.c), *box,
                                  float(c1), stream_handle(stream)), "sird_lbfgs_accept")


class Graph:
    """HIP graph of iters_per_launch [sird_loss -> pso_step] iterations."""

    def __init__(self, batch: Batch, params: PsoParams, swarm: Swarm, obs, kind="ssre",
                 iters_per_launch=1):
        h = ctypes.c_void_p()
        a = Args(batch)
        o = a(obs, batch.obs_len, "obs")
        a.device()
        check(lib().sird_graph_create(ctypes.byref(batch.c), ctypes.byref(params.c),
                                      ctypes.byref(swarm.c), o, _kind(kind),
                                      int(iters_per_launch), ctypes.byref(h)),
              "sird_graph_create")
        self.h = h
        self.iters_per_launch = int(iters_per_launch)
        self._keep = (batch, params, swarm, obs)

    def launch(self, n=1, stream=None):
        check(lib().sird_graph_launch(self.h, int(n), stream_handle(stream)), "sird_graph_launch")

    def close(self):
        if self.h is not None and self.h.value:
            check(lib().sird_graph_destroy(self.h), "sird_graph_destroy")
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
