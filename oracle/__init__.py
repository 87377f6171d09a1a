"""Plain FP64 CPU oracle for the SIRD calibration hot path (test infrastructure).

This package is the independent reference the GPU library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path never does.  It shares no code
with the GPU library: the arithmetic lives in ``sird_oracle.c`` (plain C,
``-ffp-contract=off``), and this module only marshals numpy arrays.

Citations (sections and equations of the paper):
  * eq. (SIRD), Sec. 2.2 -- the model integrated by :func:`integrate`;
  * eq. (beta), Sec. 2.2 -- the ramp of :func:`integrate_euler_ramp`;
  * Sec. 3.1 -- the low-level costs of :func:`loss`;
  * Sec. 3.3 -- the PSO of :func:`pso_init`, :func:`pso_bests`,
    :func:`pso_move` and :func:`pso_run`.

Parameter vectors are row-major ``(P, d)`` with
``theta = (beta_1..beta_K, gamma, mu, I0)`` and ``d = K + 3``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sird_oracle.c")
_LIB = os.path.join(_HERE, "libsird_oracle.so")

LOSS_KINDS = {"ssre": 0, "mse": 1, "mxse": 2, "mae": 3, "mape": 4,
              "ird_mxse": 5, "ird_mse": 6, "ird_mae": 7, "ird_mape": 8}

_D = ctypes.POINTER(ctypes.c_double)
_U64 = ctypes.POINTER(ctypes.c_uint64)
_I64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_philox4x64_10.argtypes = [_U64, _U64, _U64]
        L.orc_u01.argtypes = [ctypes.c_uint64]
        L.orc_u01.restype = ctypes.c_double
        L.orc_beta_ramp.argtypes = [ctypes.c_double] * 5
        L.orc_beta_ramp.restype = ctypes.c_double
        prob = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_integrate.argtypes = prob + [_D, _D, _D]
        L.orc_integrate_euler_ramp.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D,
                                               ctypes.c_double, _D]
        L.orc_loss.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_loss.restype = ctypes.c_double
        L.orc_loss_batch.argtypes = prob + [ctypes.c_int, _D, _D, ctypes.c_int, _D, ctypes.c_int]
        L.orc_pso_init.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_uint64,
                                   ctypes.c_uint64, _D, _D, _D, _D, _D, _D, _I64]
        L.orc_pso_bests.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D,
                                    _I64, _D]
        L.orc_pso_move.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   _D, _D, ctypes.c_uint64, ctypes.c_uint64, _D, _D, _D, _D]
        L.orc_pso_run.argtypes = prob + [_D, ctypes.c_int, ctypes.c_int, _D, _D,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                         _D, _I64, _D, _D, _D, _D, _D, _D, ctypes.c_int]
        L.orc_loss_grad_fwd.argtypes = prob + [_D, _D, ctypes.c_int, _D, _D, _D]
        _IP = ctypes.POINTER(ctypes.c_int)
        L.orc_lbfgs_propose.argtypes = [ctypes.c_int] * 5 + [_D, _D, _D, _D, _D, _D, _D, _IP,
                                                             _IP, _D, _D, _D, _D]
        L.orc_lbfgs_accept.argtypes = [ctypes.c_int] * 5 + [_D, _D, ctypes.c_double, _D, _D, _D,
                                                            _D, _D, _D, _D, _D, _D, _D, _IP,
                                                            _IP, _D]
        L.orc_integrate_model.argtypes = [ctypes.c_int] + prob + [_D, _D]
        L.orc_loss_ird.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D]
        L.orc_loss_ird.restype = ctypes.c_double
        L.orc_loss_batch_model.argtypes = [ctypes.c_int] + prob + [ctypes.c_int, _D, _D,
                                                                   ctypes.c_int, _D, ctypes.c_int]
        L.orc_pso_sort_pair.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
        L.orc_pso_run_model.argtypes = [ctypes.c_int] + prob + [
            _D, ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _D, _I64, _D, _D,
            _D, _D, _D, _D, ctypes.c_int]
        L.orc_adam_step.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _kind(kind):
    return LOSS_KINDS[kind] if isinstance(kind, str) else int(kind)


class Problem:
    """One calibration window: W days at spd steps per day, population N,
    fixed initial removed R0 and deceased D0.  model 0: RK4 with K beta
    segments of seg_days days (the last one extends to the window end),
    theta = (beta_1..beta_K, gamma, mu, I0); model 1: forward Euler with the
    ramp of eq. (beta), K = 4, theta = (beta1, beta2, t1, t2, gamma, mu, I0)."""

    def __init__(self, W, spd, seg_days, K, N, R0=0.0, D0=0.0, model=0):
        self.W, self.spd, self.seg_days, self.K = int(W), int(spd), int(seg_days), int(K)
        self.N, self.R0, self.D0 = float(N), float(R0), float(D0)
        self.model = int(model)
        assert self.model in (0, 1) and (self.model == 0 or self.K == 4)

    @property
    def d(self):
        return self.K + 3

    @property
    def T(self):
        return self.W * self.spd

    def args(self):
        return (self.W, self.spd, self.seg_days, self.K, self.N, self.R0, self.D0)


# ----------------------------------------------------------------- Philox
def philox4x64_10(ctr, key):
    """Philox4x64-10 block of counter ``ctr`` (4 words) under ``key`` (2 words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(c.ctypes.data_as(_U64), k.ctypes.data_as(_U64),
                            out.ctypes.data_as(_U64))
    return out


def u01(word):
    return lib().orc_u01(ctypes.c_uint64(int(word)))


# ---------------------------------------------------------------- model
def integrate(prob: Problem, theta, steps=False):
    """RK4 trajectory of one parameter vector: S, I, R, D at every day,
    shape (4, W+1); with ``steps=True`` also the state after every step,
    shape (4, T+1)."""
    th = _f64(theta)
    assert th.shape == (prob.d,)
    days = np.zeros((4, prob.W + 1))
    st = np.zeros((4, prob.T + 1)) if steps else None
    lib().orc_integrate(*prob.args(), _dp(th), _dp(days), _dp(st))
    return (days, st) if steps else days


def integrate_euler_ramp(W, spd, theta6, y0, N):
    """Forward-Euler trajectory with the ramp of eq. (beta):
    theta6 = (beta1, beta2, t1, t2, gamma, mu), start state y0 = (S, I, R, D)."""
    th = _f64(theta6)
    y = _f64(y0)
    days = np.zeros((4, W + 1))
    lib().orc_integrate_euler_ramp(int(W), int(spd), _dp(th), _dp(y), float(N), _dp(days))
    return days


def beta_ramp(t, b1, b2, t1, t2):
    return lib().orc_beta_ramp(float(t), float(b1), float(b2), float(t1), float(t2))


def loss(kind, Dhat, y):
    """Cost of one deceased trajectory Dhat (days 0..W) against y."""
    Dh, yy = _f64(Dhat), _f64(y)
    assert Dh.shape == yy.shape
    return lib().orc_loss(_kind(kind), len(yy) - 1, _dp(Dh), _dp(yy))


def loss_batch(prob: Problem, theta, y, kind="ssre", nthreads=0):
    """Losses of every row of theta (P, d) on one problem (OpenMP over rows)."""
    th = _f64(theta)
    P = th.shape[0]
    assert th.shape == (P, prob.d)
    yy = _f64(y)
    assert yy.shape == (prob.W + 1,)
    out = np.zeros(P)
    lib().orc_loss_batch(*prob.args(), P, _dp(th), _dp(yy), _kind(kind), _dp(out), int(nthreads))
    return out


# ------------------------------------------------------------------ PSO
class Swarm:
    """Swarm state of one problem, row-major (P, d)."""

    def __init__(self, P, d):
        self.x = np.zeros((P, d))
        self.v = np.zeros((P, d))
        self.pbest_x = np.zeros((P, d))
        self.pbest_f = np.zeros(P)
        self.gbest_x = np.zeros(d)
        self.gbest_f = np.zeros(1)
        self.gbest_idx = np.zeros(1, dtype=np.int64)

    def copy(self):
        s = Swarm(*self.x.shape)
        for k, v in self.__dict__.items():
            setattr(s, k, v.copy())
        return s


def pso_init(P, lo, hi, seed, stream=0):
    lo, hi = _f64(lo), _f64(hi)
    d = lo.shape[0]
    s = Swarm(P, d)
    lib().orc_pso_init(P, d, _dp(lo), _dp(hi), seed, stream, _dp(s.x), _dp(s.v),
                       _dp(s.pbest_x), _dp(s.pbest_f), _dp(s.gbest_x), _dp(s.gbest_f),
                       s.gbest_idx.ctypes.data_as(_I64))
    return s


def pso_bests(s: Swarm, f):
    """Update personal and global bests in place; returns the near-tie margin."""
    f = _f64(f)
    P, d = s.x.shape
    m = np.zeros(1)
    lib().orc_pso_bests(P, d, _dp(f), _dp(s.x), _dp(s.pbest_x), _dp(s.pbest_f),
                        _dp(s.gbest_x), _dp(s.gbest_f), s.gbest_idx.ctypes.data_as(_I64),
                        _dp(m))
    return float(m[0])


def pso_move(s: Swarm, it, w, c1, c2, lo, hi, seed, stream=0):
    """Velocity/position update of iteration ``it`` in place."""
    lo, hi = _f64(lo), _f64(hi)
    P, d = s.x.shape
    lib().orc_pso_move(P, d, it, w, c1, c2, _dp(lo), _dp(hi), seed, stream,
                       _dp(s.pbest_x), _dp(s.gbest_x), _dp(s.x), _dp(s.v))


def pso_run(prob: Problem, y, kind, P, lo, hi, w, c1, c2, seed, stream, iters, nthreads=0):
    """Whole PSO run; returns (hist_f, hist_idx, hist_margin, final Swarm)."""
    lo, hi, yy = _f64(lo), _f64(hi), _f64(y)
    d = prob.d
    s = Swarm(P, d)
    hf = np.zeros(iters)
    hi_ = np.zeros(iters, dtype=np.int64)
    hm = np.zeros(iters)
    lib().orc_pso_run(*prob.args(), _dp(yy), _kind(kind), P, _dp(lo), _dp(hi), w, c1, c2,
                      seed, stream, iters, _dp(hf), hi_.ctypes.data_as(_I64), _dp(hm),
                      _dp(s.x), _dp(s.v), _dp(s.pbest_x), _dp(s.pbest_f), _dp(s.gbest_x),
                      int(nthreads))
    s.gbest_f[0] = hf[-1] if iters else np.inf
    s.gbest_idx[0] = hi_[-1] if iters else -1
    return hf, hi_, hm, s


# ------------------------------------------------------------- gradient
def loss_grad_fwd(prob: Problem, theta, y, kind="ssre", with_scale=False):
    """(loss, dloss/dtheta) of one parameter vector by forward-mode tangents;
    with_scale also returns per component the sum over days of the absolute
    terms the gradient adds up (the size its rounding is relative to)."""
    th, yy = _f64(theta), _f64(y)
    L = np.zeros(1)
    g = np.zeros(prob.d)
    sc = np.zeros(prob.d) if with_scale else None
    lib().orc_loss_grad_fwd(*prob.args(), _dp(th), _dp(yy), _kind(kind), _dp(L), _dp(g),
                            _dp(sc))
    return (float(L[0]), g, sc) if with_scale else (float(L[0]), g)


def adam_step(theta, grad, m, v, lo, hi, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One projected Adam step in place on theta (n, d) with moments m, v."""
    n, d = theta.shape
    for a in (theta, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == (n, d)
    lo, hi = _f64(lo), _f64(hi)
    lib().orc_adam_step(n, d, _dp(theta), _dp(grad), _dp(m), _dp(v), _dp(lo), _dp(hi),
                        int(t), lr, b1, b2, eps)


# --------------------------------------------------------------- L-BFGS
class Lbfgs:
    """State of the oracle's projected L-BFGS over n vectors of dimension d
    (row-major [n][d]; memory [n][m][d]); log_last optimises the last
    dimension as its logarithm within [log lo, log hi].  n_trials trial
    points per round: trial t of vector q in row t n + q of theta_t,
    grad_t and f_t."""

    def __init__(self, theta, m=8, log_last=False, n_trials=1):
        self.log_last = int(bool(log_last))
        self.theta = _f64(theta).copy()
        n, d = self.theta.shape
        self.m = m
        self.n_trials = int(n_trials)
        assert 1 <= self.n_trials <= 8
        self.grad = np.zeros((n, d))
        self.f = np.zeros(n)
        self.theta_t = np.zeros((self.n_trials * n, d))
        self.grad_t = np.zeros((self.n_trials * n, d))
        self.f_t = np.zeros(self.n_trials * n)
        self.p = np.zeros((n, d))
        self.gp = np.zeros(n)
        self.S = np.zeros((n, m, d))
        self.Y = np.zeros((n, m, d))
        self.rho = np.zeros((n, m))
        self.alpha = np.ones(n)
        self.count = np.zeros(n, dtype=np.intc)
        self.head = np.zeros(n, dtype=np.intc)

    def propose(self, lo, hi):
        lo, hi = _f64(lo), _f64(hi)
        n, d = self.theta.shape
        ip = ctypes.POINTER(ctypes.c_int)
        lib().orc_lbfgs_propose(n, d, self.m, self.log_last, self.n_trials, _dp(lo), _dp(hi),
                                _dp(self.theta), _dp(self.grad), _dp(self.S), _dp(self.Y), _dp(self.rho),
                                self.count.ctypes.data_as(ip), self.head.ctypes.data_as(ip),
                                _dp(self.alpha), _dp(self.p), _dp(self.gp), _dp(self.theta_t))

    def accept(self, lo, hi, c1=1e-4):
        lo, hi = _f64(lo), _f64(hi)
        n, d = self.theta.shape
        ip = ctypes.POINTER(ctypes.c_int)
        lib().orc_lbfgs_accept(n, d, self.m, self.log_last, self.n_trials, _dp(lo), _dp(hi),
                               c1, _dp(self.theta), _dp(self.grad), _dp(self.f), _dp(self.theta_t), _dp(self.grad_t),
                               _dp(self.f_t), _dp(self.gp), _dp(self.S), _dp(self.Y),
                               _dp(self.rho), self.count.ctypes.data_as(ip),
                               self.head.ctypes.data_as(ip), _dp(self.alpha))


# ------------------------------------------------ the paper's own variant
def integrate_model(prob: Problem, theta):
    """S, I, R, D at every day for either model, shape (4, W+1)."""
    th = _f64(theta)
    assert th.shape == (prob.d,)
    days = np.zeros((4, prob.W + 1))
    lib().orc_integrate_model(prob.model, *prob.args(), _dp(th), _dp(days))
    return days


def loss_ird(kind, Ihat, Rhat, Dhat, yI, yR, yD):
    """F_IRD of Sec. 3.1 with low-level cost kind (mse, mxse, mae, mape)."""
    arrs = [_f64(a) for a in (Ihat, Rhat, Dhat, yI, yR, yD)]
    W = len(arrs[0]) - 1
    return lib().orc_loss_ird(_kind(kind), W, *[_dp(a) for a in arrs])


def loss_batch_model(prob: Problem, theta, obs, kind, nthreads=0):
    """Losses of every row of theta for either model; obs = y_D for the
    D-only costs, [y_I; y_R; y_D] (3 (W+1) values) for the ird_* costs."""
    th = _f64(theta)
    P = th.shape[0]
    ob = _f64(obs).reshape(-1)
    k = _kind(kind)
    assert ob.shape == ((3 if k >= 5 else 1) * (prob.W + 1),)
    out = np.zeros(P)
    lib().orc_loss_batch_model(prob.model, *prob.args(), P, _dp(th), _dp(ob), k, _dp(out),
                               int(nthreads))
    return out


def pso_sort_pair(s: Swarm, j=2):
    """Order the pair (j, j+1) of every position (the ramp's t1 <= t2)."""
    P, d = s.x.shape
    lib().orc_pso_sort_pair(P, d, j, _dp(s.x))


def pso_run_model(prob: Problem, obs, kind, P, lo, hi, w, c1, c2, seed, stream, iters,
                  nthreads=0):
    lo, hi, ob = _f64(lo), _f64(hi), _f64(obs).reshape(-1)
    d = prob.d
    s = Swarm(P, d)
    hf = np.zeros(iters)
    hi_ = np.zeros(iters, dtype=np.int64)
    hm = np.zeros(iters)
    lib().orc_pso_run_model(prob.model, *prob.args(), _dp(ob), _kind(kind), P, _dp(lo), _dp(hi),
                            w, c1, c2, seed, stream, iters, _dp(hf),
                            hi_.ctypes.data_as(_I64), _dp(hm), _dp(s.x), _dp(s.v),
                            _dp(s.pbest_x), _dp(s.pbest_f), _dp(s.gbest_x), int(nthreads))
    s.gbest_f[0] = hf[-1] if iters else np.inf
    s.gbest_idx[0] = hi_[-1] if iters else -1
    return hf, hi_, hm, s
