"""ctypes binding of the C ABI in ``include/sird.h``.

Argument marshalling only: every step of the path runs in the HIP kernels
of ``libsird.so``.  Functions carry the C names; each raises ``SirdError``
on a negative status.  Device arrays are passed as torch tensors (their
``data_ptr()``) and the stream defaults to torch's current stream.

The library must have been built (``python -m paper_2204_12346_amd.build``); there is no
fallback path: a missing library raises ``ImportError`` when first used.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsird.so")

SIRD_OK, SIRD_EINVAL, SIRD_ENOSPACE, SIRD_EHIP = 0, -1, -2, -3
SIRD_F64, SIRD_F32 = 0, 1
LOSS = {"ssre": 0, "mse": 1, "mxse": 2, "mae": 3, "mape": 4,
        "ird_mxse": 5, "ird_mse": 6, "ird_mae": 7, "ird_mape": 8}
MODEL = {"rk4": 0, "euler_ramp": 1}


class SirdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


# numpy mirror of struct sird_problem (96 bytes)
PROBLEM_DTYPE = np.dtype([
    ("n_days", "<i4"), ("steps_per_day", "<i4"), ("seg_days", "<i4"), ("n_seg", "<i4"),
    ("n_part", "<i4"), ("model", "<i4"),
    ("N", "<f8"), ("R0", "<f8"), ("D0", "<f8"),
    ("p_off", "<i8"), ("theta_off", "<i8"), ("obs_off", "<i8"), ("traj_off", "<i8"),
    ("box_off", "<i8"), ("stream", "<u8"),
])
assert PROBLEM_DTYPE.itemsize == 96

TILE_DTYPE = np.dtype([("prob", "<i4"), ("p0", "<i4")])


class sird_batch(ctypes.Structure):
    _fields_ = [
        ("n_prob", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
        ("max_days", ctypes.c_int32), ("max_d", ctypes.c_int32),
        ("max_steps", ctypes.c_int64), ("total_particles", ctypes.c_int64),
        ("theta_len", ctypes.c_int64), ("obs_len", ctypes.c_int64),
        ("traj_len", ctypes.c_int64), ("box_len", ctypes.c_int64),
        ("probs", ctypes.c_void_p), ("tiles", ctypes.c_void_p), ("sched", ctypes.c_void_p),
        ("dtype", ctypes.c_int32), ("block", ctypes.c_int32),
        ("persistent", ctypes.c_int32), ("obs_series", ctypes.c_int32),
        ("models", ctypes.c_int32), ("max_part", ctypes.c_int32),
        ("waves_per_simd", ctypes.c_int32), ("ppl", ctypes.c_int32),
        ("n_pairs", ctypes.c_int32), ("pair_tiles", ctypes.c_void_p),
    ]


class pso_params(ctypes.Structure):
    _fields_ = [("w", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p)]


class pso_state(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("pbest_x", ctypes.c_void_p),
                ("pbest_f", ctypes.c_void_p), ("gbest_x", ctypes.c_void_p),
                ("gbest_f", ctypes.c_void_p), ("gbest_idx", ctypes.c_void_p),
                ("iter", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("hist_f", ctypes.c_void_p), ("hist_idx", ctypes.c_void_p),
                ("hist_len", ctypes.c_int64)]


class adam_params(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class lbfgs_state(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("theta", "grad", "f", "theta_t", "grad_t", "f_t", "S", "Y", "rho", "alpha",
                 "gp", "count", "head")] + [("m", ctypes.c_int32), ("log_last", ctypes.c_int32),
                                            ("n_trials", ctypes.c_int32)]


_P = ctypes.c_void_p
_B = ctypes.POINTER(sird_batch)
_PP = ctypes.POINTER(pso_params)
_PS = ctypes.POINTER(pso_state)
_I = ctypes.c_int
_I64 = ctypes.c_int64

# name -> (restype, argtypes); mirrors include/sird.h
SIGNATURES = {
    "sird_status_string": (ctypes.c_char_p, [_I]),
    "sird_last_error": (ctypes.c_char_p, []),
    "sird_problem_validate": (_I, [_P, _I, _I64, _I64, _I64, _I64, _I64, _I]),
    "sird_plan_tiles": (_I, [_P, _I, _P, _I]),
    "sird_batch_plan": (_I, [_B, _P, _I, _I64, _I64, _I64, _I64, _I64, _I, _I, _P, _P, _P]),
    "sird_integrate": (_I, [_B, _P, _P, _P]),
    "sird_loss": (_I, [_B, _P, _P, _I, _P, _I, _P, ctypes.c_size_t, _P]),
    "pso_init": (_I, [_B, _PP, _PS, _P]),
    "pso_step": (_I, [_B, _PP, _PS, _P]),
    "sird_pso_iterate": (_I, [_B, _PP, _PS, _P, _I, _I, _P]),
    "pso_evaluate": (_I, [_B, _PP, _PS, _P, _I, _I, _P]),
    "pso_gbest": (_I, [_B, _PP, _PS, _P]),
    "pso_complete_move": (_I, [_B, _PP, _PS, _P]),
    "sird_loss_backward": (_I, [_B, _P, _P, _I, _P, _P, _P, _I, _I, _P, ctypes.c_size_t, _P]),
    "sird_loss_backward_workspace": (ctypes.c_size_t, [_B, _I]),
    "sird_plan_pairs": (_I, [_P, _I, _P, _I]),
    "sird_loss_backward_static": (_I, [_B, _P, _P, _I, _P, _P, _P, _I, _P]),
    "pso_topk": (_I, [_B, _P, _I, _P, _P]),
    "sird_gather": (_I, [_B, _P, _P, _B, _P, _P, _I, _P]),
    "sird_adam_step": (_I, [_B, _P, _P, _P, _P, _P, _P, _I64,
                            ctypes.POINTER(adam_params), _P]),
    "sird_lbfgs_propose": (_I, [_B, ctypes.POINTER(lbfgs_state), _P, _P, _P]),
    "sird_lbfgs_accept": (_I, [_B, ctypes.POINTER(lbfgs_state), _P, _P, ctypes.c_double, _P]),
    "sird_graph_create": (_I, [_B, _PP, _PS, _P, _I, _I, ctypes.POINTER(ctypes.c_void_p)]),
    "sird_graph_launch": (_I, [_P, _I, _P]),
    "sird_graph_destroy": (_I, [_P]),
}

_lib = None


def lib():
    """Load libsird.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} not built: run python -m paper_2204_12346_amd.build "
                "(hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, who=""):
    if status != SIRD_OK:
        msg = lib().sird_last_error().decode() or lib().sird_status_string(status).decode()
        raise SirdError(status, f"{who}: {msg}" if who else msg)
    return status


def ptr(t):
    """Device (or host) address of a tensor/ndarray, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)
