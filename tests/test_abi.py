"""CPU checks of the C ABI: the library loads, exports every function that
include/sird.h declares, its structs have the layout the binding assumes,
and host-side argument checks reject bad input before any HIP call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sird.h")


@pytest.fixture(scope="module")
def L():
    from paper_2204_12346_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2204_12346_amd import build
        build.build()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(n for n in set(names) if n not in ("defined",))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sird_integrate", "sird_loss", "pso_step", "sird_loss_backward"):
        assert required in names
    assert len(names) == 25, names


def test_library_exports_every_declared_symbol(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(L.SIGNATURES)


def test_struct_layout_matches_binding(tmp_path, L):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "sird.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(sird_problem), sizeof(sird_tile),
         sizeof(sird_batch), sizeof(pso_params), sizeof(pso_state), sizeof(adam_params));
  printf("%zu %zu %zu %zu %zu\n", offsetof(sird_problem, N), offsetof(sird_problem, p_off),
         offsetof(sird_problem, stream), offsetof(sird_batch, probs), offsetof(sird_batch, dtype));
  printf("%zu %zu\n", offsetof(pso_state, f), offsetof(pso_state, hist_len));
  printf("%zu %zu %zu\n", offsetof(sird_batch, ppl), offsetof(sird_batch, n_pairs),
         offsetof(sird_batch, pair_tiles));
  printf("%zu %zu %zu\n", sizeof(lbfgs_state), offsetof(lbfgs_state, m),
         offsetof(lbfgs_state, n_trials));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    vals = [int(x) for x in out]
    assert vals[0] == L.PROBLEM_DTYPE.itemsize == 96
    assert vals[1] == L.TILE_DTYPE.itemsize == 8
    assert vals[2] == ctypes.sizeof(L.sird_batch)
    assert vals[3] == ctypes.sizeof(L.pso_params)
    assert vals[4] == ctypes.sizeof(L.pso_state)
    assert vals[5] == ctypes.sizeof(L.adam_params)
    assert vals[6] == L.PROBLEM_DTYPE.fields["N"][1]
    assert vals[7] == L.PROBLEM_DTYPE.fields["p_off"][1]
    assert vals[8] == L.PROBLEM_DTYPE.fields["stream"][1]
    assert vals[9] == L.sird_batch.probs.offset
    assert vals[10] == L.sird_batch.dtype.offset
    assert vals[13:16] == [L.sird_batch.ppl.offset, L.sird_batch.n_pairs.offset,
                           L.sird_batch.pair_tiles.offset]
    assert vals[2] == 136
    assert vals[11] == L.pso_state.f.offset
    assert vals[12] == L.pso_state.hist_len.offset
    assert vals[16:19] == [ctypes.sizeof(L.lbfgs_state), L.lbfgs_state.m.offset,
                           L.lbfgs_state.n_trials.offset]


def _table(rows):
    from paper_2204_12346_amd import _lib
    t = np.zeros(len(rows), dtype=_lib.PROBLEM_DTYPE)
    for i, r in enumerate(rows):
        for k, v in r.items():
            t[i][k] = v
    return t


def _good(**kw):
    r = dict(n_days=10, steps_per_day=4, seg_days=7, n_seg=2, n_part=70, N=1e6,
             p_off=0, theta_off=0, obs_off=0, traj_off=0, box_off=0)
    r.update(kw)
    return r


def test_status_strings_and_last_error(L):
    lib = L.lib()
    for s in (0, -1, -2, -3, 7):
        assert lib.sird_status_string(s)
    assert lib.sird_status_string(-2).startswith(b"SIRD_ENOSPACE")


@pytest.mark.parametrize("bad,msg", [
    (dict(n_days=0), b"n_days"), (dict(steps_per_day=0), b"steps_per_day"),
    (dict(seg_days=0), b"seg_days"), (dict(n_seg=0), b"n_seg"), (dict(n_part=-1), b"n_part"),
    (dict(N=0.0), b"N must"), (dict(N=float("nan")), b"N must"), (dict(R0=-1.0), b"R0"),
    (dict(model=3), b"unknown model"), (dict(model=1), b"ramp model needs n_seg = 4"),
    (dict(p_off=1), b"particle"),
    (dict(theta_off=1), b"theta"), (dict(obs_off=1), b"obs"), (dict(box_off=1), b"box"),
])
def test_validate_rejects(L, bad, msg):
    lib = L.lib()
    t = _table([_good(**bad)])
    st = lib.sird_problem_validate(t.ctypes.data, 1, 70, 5 * 70, 11, 0, 5, 1)
    assert st == L.SIRD_EINVAL
    assert msg in lib.sird_last_error()


def test_validate_accepts_and_checks_lengths(L):
    lib = L.lib()
    t = _table([_good(), _good(p_off=70, theta_off=350, obs_off=11, box_off=5, n_part=0)])
    assert lib.sird_problem_validate(t.ctypes.data, 2, 70, 350, 22, 0, 10, 1) == 0
    assert lib.sird_problem_validate(t.ctypes.data, 2, 70, 349, 22, 0, 10, 1) == L.SIRD_EINVAL
    assert lib.sird_problem_validate(None, 2, 70, 350, 22, 0, 10, 1) == L.SIRD_EINVAL
    assert lib.sird_problem_validate(t.ctypes.data, 0, 70, 350, 22, 0, 10, 1) == L.SIRD_EINVAL
    for series in (0, 2, 4):
        assert lib.sird_problem_validate(t.ctypes.data, 2, 70, 350, 22, 0, 10,
                                         series) == L.SIRD_EINVAL
    # three observed series: blocks of 3 (W+1) values
    assert lib.sird_problem_validate(t.ctypes.data, 2, 70, 350, 22, 0, 10, 3) == L.SIRD_EINVAL
    t3 = _table([_good(), _good(p_off=70, theta_off=350, obs_off=33, box_off=5, n_part=0)])
    assert lib.sird_problem_validate(t3.ctypes.data, 2, 70, 350, 66, 0, 10, 3) == 0
    assert lib.sird_problem_validate(t3.ctypes.data, 2, 70, 350, 65, 0, 10, 3) == L.SIRD_EINVAL
    # the ramp model with its four parameters of beta
    tr = _table([_good(model=1, n_seg=4)])
    assert lib.sird_problem_validate(tr.ctypes.data, 1, 70, 7 * 70, 11, 0, 7, 1) == 0


def test_plan_tiles_longest_first(L):
    lib = L.lib()
    t = _table([_good(n_days=10, n_part=130), _good(n_days=30, n_part=64),
                _good(n_days=20, n_part=1), _good(n_days=50, n_part=0)])
    out = np.zeros(10, dtype=L.TILE_DTYPE)
    n = lib.sird_plan_tiles(t.ctypes.data, 4, out.ctypes.data, 10)
    assert n == 5
    got = [(int(a), int(b)) for a, b in out[:n]]
    assert got == [(1, 0), (2, 0), (0, 0), (0, 64), (0, 128)]
    assert lib.sird_plan_tiles(t.ctypes.data, 4, out.ctypes.data, 4) == L.SIRD_ENOSPACE


def test_device_calls_reject_bad_arguments_without_a_gpu(L):
    lib = L.lib()
    null = ctypes.c_void_p()
    # NULL batch
    assert lib.sird_loss(None, null, null, 0, null, 0, None, 0, None) == L.SIRD_EINVAL
    assert lib.sird_integrate(None, null, null, None) == L.SIRD_EINVAL
    assert lib.pso_step(None, None, None, None) == L.SIRD_EINVAL
    assert lib.sird_loss_backward(None, null, null, 0, null, null, null, 0, 0, null, 0,
                                  None) == L.SIRD_EINVAL
    assert lib.sird_graph_launch(None, 1, None) == L.SIRD_EINVAL
    assert lib.sird_graph_destroy(None) == 0
    # an unplanned batch
    b = L.sird_batch()
    assert lib.sird_loss(ctypes.byref(b), null, null, 0, null, 0, None, 0, None) == L.SIRD_EINVAL
    assert b"not planned" in lib.sird_last_error() or b"n_prob" in lib.sird_last_error()
    assert lib.sird_loss_backward_workspace(ctypes.byref(b), 0) == 0


def test_batch_plan_and_per_call_checks_on_host(L):
    import torch
    from paper_2204_12346_amd import core
    specs = [core.ProblemSpec(30, 10, 14, 3, 1e6, n_part=100, stream=0),
             core.ProblemSpec(12, 5, 7, 2, 1e5, n_part=0, stream=1),
             core.ProblemSpec(45, 2, 14, 4, 1e7, n_part=65, stream=2)]
    b = core.Batch(specs, device="cpu", with_traj=True)
    assert b.n_tiles == 2 + 0 + 2
    assert b.c.max_days == 45 and b.c.max_d == 7 and b.c.max_steps == 300
    assert b.total_particles == 165 and b.theta_len == 6 * 100 + 7 * 65
    assert b.obs_len == 31 + 13 + 46 and b.box_len == 6 + 5 + 7
    assert b.c.obs_series == 1 and b.c.models == 1 and b.c.max_part == 100
    lib = L.lib()
    dummy = torch.zeros(8, dtype=torch.float64)
    for kind in (-1, 9):
        assert lib.sird_loss(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), kind,
                             dummy.data_ptr(), 0, None, 0, None) == L.SIRD_EINVAL
        assert b"unknown loss_kind" in lib.sird_last_error()
    # the F_IRD kinds need the I and R series too
    for kind in (5, 8):
        assert lib.sird_loss(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), kind,
                             dummy.data_ptr(), 0, None, 0, None) == L.SIRD_EINVAL
        assert b"obs_series = 3" in lib.sird_last_error()
    b.c.models = 0
    assert lib.sird_loss(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 0,
                         dummy.data_ptr(), 0, None, 0, None) == L.SIRD_EINVAL
    b.c.models = 1
    b.c.dtype = 7
    assert lib.sird_loss(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 0,
                         dummy.data_ptr(), 0, None, 0, None) == L.SIRD_EINVAL
    b.c.dtype = 0
    b.c.block = 96
    assert lib.sird_loss(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 0,
                         dummy.data_ptr(), 0, None, 0, None) == L.SIRD_EINVAL
    b.c.block = 0
    assert b.c.waves_per_simd == 0
    for w in (-1, 9):
        b.c.waves_per_simd = w
        assert lib.sird_loss(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 0,
                             dummy.data_ptr(), 0, None, 0, None) == L.SIRD_EINVAL
        assert b"waves_per_simd" in lib.sird_last_error()
    b.c.waves_per_simd = 0
    ws = lib.sird_loss_backward_workspace(ctypes.byref(b.c), 0)
    # steps of the LDS sub-interval: what fits 40 KiB next to the observations
    # (2 x 46 doubles), 64 lanes' betas (4 segments), a parked checkpoint
    # (3 x 64) and two slack rows of (s, I) at either end
    lc = (40960 - 8 * (2 * 46 + 64 * (4 + 3 + 8))) // (2 * 64 * 8)
    assert lc == 31
    # the default interval is a whole number of days per problem that fits lc
    # steps: at least (lc + 1)/2 steps, at most one checkpoint a day; 3 slots
    # per checkpoint (s, I, S), Dhat of days 0..45, S at the start of each of
    # 4 segments, the sum of J of days 0..44, the day MXSE peaks on and the
    # loss
    n_ck = max(int(np.ceil(300 / lc)), min(45, (2 * 300 + lc) // (lc + 1)))
    assert n_ck == 19
    assert ws == (3 * n_ck + 46 + 4 + 45 + 2) * 165 * 8
    # an interval longer than the sub-interval adds 3 slots per sub-interval
    ws100 = lib.sird_loss_backward_workspace(ctypes.byref(b.c), 100)
    assert ws100 == (3 * 3 + 3 * int(np.ceil(100 / lc)) + 46 + 4 + 45 + 2) * 165 * 8
    # the segment-parallel sweep: a checkpoint per day (3 x 45), Dhat, S at
    # every segment start, the sums of J, the tail and 16 slots per piece
    # (segments walked in pieces of at most 7 days: at most ceil(45 / 7) + 4)
    text = open(HEADER).read()
    m = re.search(r"#define SIRD_CKPT_SEGMENTS \((-?\d+)\)", text)
    assert m and int(m.group(1)) == core.CKPT_SEGMENTS
    wseg = lib.sird_loss_backward_workspace(ctypes.byref(b.c), core.CKPT_SEGMENTS)
    assert wseg == (3 * 45 + 46 + 4 + 45 + 2 + 16 * (7 + 4)) * 165 * 8
    assert lib.sird_loss_backward_workspace(ctypes.byref(b.c), -2) == 0
    st = lib.sird_loss_backward(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 0, None,
                                dummy.data_ptr(), None, -2, 0, ctypes.c_void_p(4096), 1 << 30,
                                None)
    assert st == L.SIRD_EINVAL and b"SIRD_CKPT_SEGMENTS" in lib.sird_last_error()
    # too small a workspace is reported before anything is enqueued
    st = lib.sird_loss_backward(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 0, None,
                                dummy.data_ptr(), None, 0, 0, ctypes.c_void_p(4096), 16, None)
    assert st == L.SIRD_ENOSPACE


def test_ramp_model_and_three_series_batches_on_host(L):
    import torch
    from paper_2204_12346_amd import core
    specs = [core.ProblemSpec(92, 1, 1, 4, 3.8e7, n_part=100, model="euler_ramp"),
             core.ProblemSpec(30, 4, 10, 3, 1e6, n_part=10)]
    b = core.Batch(specs, device="cpu", obs_series=3)
    assert b.c.models == 3 and b.c.obs_series == 3
    assert b.obs_len == 3 * 93 + 3 * 31
    y = [np.arange(3 * 93.0), np.arange(3 * 31.0)]
    o = b.pack_obs(y).numpy()
    assert o[3 * 93] == 0.0 and o[-1] == 3 * 31 - 1
    lib = L.lib()
    dummy = torch.zeros(8, dtype=torch.float64)
    # gradients exist for the RK4 model with a deceased-count cost only
    st = lib.sird_loss_backward(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 0, None,
                                dummy.data_ptr(), None, 0, 0, ctypes.c_void_p(4096), 1 << 40, None)
    assert st == L.SIRD_EINVAL and b"RK4 segment model" in lib.sird_last_error()
    b.c.models = 1
    st = lib.sird_loss_backward(ctypes.byref(b.c), dummy.data_ptr(), dummy.data_ptr(), 5, None,
                                dummy.data_ptr(), None, 0, 0, ctypes.c_void_p(4096), 1 << 40, None)
    assert st == L.SIRD_EINVAL and b"deceased-count" in lib.sird_last_error()


def test_layout_round_trip_on_host():
    from paper_2204_12346_amd import core
    specs = [core.ProblemSpec(5, 2, 3, 2, 1e4, n_part=7), core.ProblemSpec(4, 1, 2, 1, 1e4, n_part=3)]
    b = core.Batch(specs, device="cpu")
    rng = np.random.default_rng(0)
    th = [rng.normal(size=(7, 5)), rng.normal(size=(3, 4))]
    t = b.pack_theta(th)
    back = b.unpack_theta(t)
    for a, c in zip(th, back):
        np.testing.assert_array_equal(a, c)
    # SoA: parameter j of particle p of problem 0 is at j*7 + p
    assert t[2 * 7 + 4].item() == th[0][4, 2]


def test_loss_with_checkpoint_workspace_checks_on_host(L):
    """sird_loss with a workspace is the adjoint's forward pass: it takes
    what sird_loss_backward takes, and refuses the rest before enqueueing."""
    import torch
    from paper_2204_12346_amd import core
    specs = [core.ProblemSpec(30, 10, 14, 3, 1e6, n_part=100, stream=0)]
    b = core.Batch(specs, device="cpu")
    lib = L.lib()
    d = torch.zeros(8, dtype=torch.float64).data_ptr()
    big = ctypes.c_void_p(4096)
    need = lib.sird_loss_backward_workspace(ctypes.byref(b.c), 10)
    assert lib.sird_loss(ctypes.byref(b.c), d, d, 0, d, 10, big, need - 1, None) == L.SIRD_ENOSPACE
    assert b"workspace too small" in lib.sird_last_error()
    assert lib.sird_loss(ctypes.byref(b.c), d, d, 0, d, -2, big, 1 << 40, None) == L.SIRD_EINVAL
    assert lib.sird_loss(ctypes.byref(b.c), d, d, 5, d, 10, big, 1 << 40, None) == L.SIRD_EINVAL
    assert lib.sird_loss(ctypes.byref(b.c), d, d, 1, d, 10, ctypes.c_void_p(4096 + 8), 1 << 40,
                         None) == L.SIRD_EINVAL
    assert b"256-byte aligned" in lib.sird_last_error()
    b.c.dtype = L.SIRD_F32
    assert lib.sird_loss(ctypes.byref(b.c), d, d, 0, d, 10, big, 1 << 40, None) == L.SIRD_EINVAL
    assert b"SIRD_F64" in lib.sird_last_error()
    b.c.dtype = L.SIRD_F64
    # the reverse sweep alone takes from_forward = 1, nothing else
    assert lib.sird_loss_backward(ctypes.byref(b.c), d, d, 0, None, d, None, 10, 2, big,
                                  1 << 40, None) == L.SIRD_EINVAL
    assert b"from_forward" in lib.sird_last_error()


def test_static_gradient_entry_checks_on_host(L):
    """sird_loss_backward_static: argument checks and the scratch limit are
    reported before any HIP call (so they run without a GPU)."""
    import torch
    from paper_2204_12346_amd import core
    text = open(HEADER).read()
    m = re.search(r"#define SIRD_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == core.STATIC_SCRATCH_BYTES
    lib = L.lib()
    d = torch.zeros(8, dtype=torch.float64).data_ptr()
    assert lib.sird_loss_backward_static(None, d, d, 0, None, d, None, 0, None) == L.SIRD_EINVAL
    # 65536 vectors over 7300 steps need about 180 MiB of workspace
    big = core.Batch([core.ProblemSpec(365, 20, 14, 13, 3.8e7, n_part=65536)], device="cpu")
    need = lib.sird_loss_backward_workspace(ctypes.byref(big.c), 0)
    assert need > core.STATIC_SCRATCH_BYTES
    assert lib.sird_loss_backward_static(ctypes.byref(big.c), d, d, 0, None, d, None, 0,
                                         None) == L.SIRD_ENOSPACE
    assert b"static scratch" in lib.sird_last_error()
    small = core.Batch([core.ProblemSpec(30, 10, 14, 3, 1e6, n_part=100)], device="cpu")
    for args, what in (((d, d, 5, None, d, None, 0), b"deceased-count"),
                       ((d, d, 0, None, None, None, 0), b"grad_theta"),
                       ((None, d, 0, None, d, None, 0), b"NULL"),
                       ((d, d, 0, None, d, None, -2), b"ckpt_interval")):
        assert lib.sird_loss_backward_static(ctypes.byref(small.c), *args, None) == L.SIRD_EINVAL
        assert what in lib.sird_last_error()
    small.c.dtype = L.SIRD_F32
    assert lib.sird_loss_backward_static(ctypes.byref(small.c), d, d, 0, None, d, None, 0,
                                         None) == L.SIRD_EINVAL


def test_tile_pairs_on_host(L):
    """sird_plan_pairs: a problem's tiles 0-1, 2-3, ... pair up, an odd last
    tile stands alone, table order kept; ppl = 2 without the table is
    refused before any HIP call."""
    import torch
    from paper_2204_12346_amd import core
    specs = [core.ProblemSpec(30, 10, 14, 3, 1e6, n_part=300, stream=0),   # 5 tiles
             core.ProblemSpec(60, 10, 14, 5, 1e6, n_part=128, stream=1),   # 2 tiles
             core.ProblemSpec(12, 5, 7, 2, 1e5, n_part=0, stream=2),
             core.ProblemSpec(45, 2, 14, 4, 1e7, n_part=65, stream=3)]     # 2 tiles
    b = core.Batch(specs, device="cpu", ppl=2)
    tiles = b.tiles_host
    # longest window first: problem 1 (600 steps), then 0 (300), then 3 (90)
    assert [int(t["prob"]) for t in tiles] == [1, 1, 0, 0, 0, 0, 0, 3, 3]
    assert list(b.pairs_host) == [0, 2, 4, 6, 7]
    assert b.c.ppl == 2 and b.c.n_pairs == 5
    lib = L.lib()
    out = np.zeros(2, dtype=np.int32)
    assert lib.sird_plan_pairs(tiles.ctypes.data, len(tiles), out.ctypes.data, 2) == L.SIRD_ENOSPACE
    d = torch.zeros(8, dtype=torch.float64).data_ptr()
    b.c.pair_tiles = None
    assert lib.sird_loss(ctypes.byref(b.c), d, d, 0, d, 0, None, 0, None) == L.SIRD_EINVAL
    assert b"pair table" in lib.sird_last_error()
    b.c.ppl = 3
    assert lib.sird_loss(ctypes.byref(b.c), d, d, 0, d, 0, None, 0, None) == L.SIRD_EINVAL
