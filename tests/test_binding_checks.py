"""The Python binding checks every device array argument before its address
reaches the C ABI: a host array, a wrong dtype, a non-contiguous view, a
tensor shorter than the batch's layout needs, or a tensor away from the
batch's GPU raises here, with nothing enqueued (CPU only: these checks run
before any HIP call)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2204_12346_amd import _lib, core
from paper_2204_12346_amd.autograd import SirdLoss


@pytest.fixture(scope="module")
def batch():
    specs = [core.ProblemSpec(30, 10, 14, 3, 1e6, n_part=100, stream=0),
             core.ProblemSpec(45, 2, 14, 4, 1e7, n_part=65, stream=2)]
    return core.Batch(specs, device="cpu", with_traj=True)


def f64(n):
    return torch.zeros(n, dtype=torch.float64)


def test_host_arrays_and_wrong_dtypes_raise(batch):
    obs = f64(batch.obs_len)
    with pytest.raises(TypeError, match="torch tensor"):
        core.sird_loss(batch, np.zeros(batch.theta_len), obs)
    with pytest.raises(TypeError, match="float32"):
        core.sird_loss(batch, torch.zeros(batch.theta_len, dtype=torch.float32), obs)
    with pytest.raises(TypeError, match="int64"):
        core.pso_topk(batch, f64(batch.total_particles), 4,
                      idx_out=torch.zeros(8, dtype=torch.int32))


def test_short_and_strided_tensors_raise(batch):
    obs = f64(batch.obs_len)
    with pytest.raises(ValueError, match="theta: .* elements"):
        core.sird_loss(batch, f64(batch.theta_len - 1), obs)
    with pytest.raises(ValueError, match="obs: .* elements"):
        core.sird_loss(batch, f64(batch.theta_len), f64(batch.obs_len - 1))
    with pytest.raises(ValueError, match="loss: .* elements"):
        core.sird_loss(batch, f64(batch.theta_len), obs, loss=f64(batch.total_particles - 1))
    strided = f64(2 * batch.theta_len)[::2]
    with pytest.raises(ValueError, match="not contiguous"):
        core.sird_loss(batch, strided, obs)
    with pytest.raises(ValueError, match="traj"):
        core.sird_integrate(batch, f64(batch.theta_len), traj=f64(batch.traj_len - 1))
    with pytest.raises(ValueError, match="grad_theta"):
        core.sird_loss_backward(batch, f64(batch.theta_len), obs,
                                grad_theta=f64(batch.theta_len - 2),
                                workspace=torch.zeros(1 << 20, dtype=torch.uint8))
    with pytest.raises(ValueError, match="grad_loss"):
        core.sird_loss_backward(batch, f64(batch.theta_len), obs, grad_loss=f64(3),
                                workspace=torch.zeros(1 << 20, dtype=torch.uint8))
    with pytest.raises(ValueError, match="idx_out"):
        core.pso_topk(batch, f64(batch.total_particles), 4,
                      idx_out=torch.zeros(7, dtype=torch.int64))
    for name in ("theta", "grad", "m", "v"):
        args = {n: f64(batch.theta_len) for n in ("theta", "grad", "m", "v")}
        args[name] = f64(batch.theta_len - 1)
        with pytest.raises(ValueError, match=name):
            core.sird_adam_step(batch, args["theta"], args["grad"], args["m"], args["v"],
                                f64(batch.box_len), f64(batch.box_len), 1)
    with pytest.raises(ValueError, match="hi"):
        core.sird_adam_step(batch, *[f64(batch.theta_len)] * 4, f64(batch.box_len),
                            f64(batch.box_len - 1), 1)


def test_workspace_size_counts_bytes_of_any_dtype(batch):
    need = core.sird_loss_backward_workspace(batch, 0)
    assert need > 0
    obs = f64(batch.obs_len)
    short = torch.zeros((need - 8) // 8, dtype=torch.float64)  # 8 bytes short
    with pytest.raises(ValueError, match="bytes"):
        core.sird_loss(batch, f64(batch.theta_len), obs, workspace=short)
    with pytest.raises(ValueError, match="from_forward"):
        core.sird_loss_backward(batch, f64(batch.theta_len), obs, from_forward=True)


def test_host_resident_batch_and_tensors_are_refused(batch):
    # every size and dtype right: what is left is that nothing is on a GPU
    with pytest.raises(ValueError, match="not on a GPU"):
        core.sird_loss(batch, f64(batch.theta_len), f64(batch.obs_len))
    with pytest.raises(ValueError, match="not on a GPU"):
        core.PsoParams(batch, f64(batch.box_len), f64(batch.box_len))


def test_autograd_rejects_float32_theta(batch):
    th = torch.zeros(batch.theta_len, dtype=torch.float32, requires_grad=True)
    with pytest.raises(TypeError, match="float64"):
        SirdLoss.apply(th, batch, f64(batch.obs_len), "ssre", 0)


def test_replicated_batch_layout():
    """Batch(replicas=T), the layout of the L-BFGS trial points: replica t of
    problem r has its own parameters and particles at t theta_len and t
    total_particles past replica 0's (one replica's sizes), and shares replica
    0's observations and box; the plan sees T times the problems and tiles."""
    specs = [core.ProblemSpec(30, 10, 14, 3, 1e6, n_part=100, stream=0),
             core.ProblemSpec(45, 2, 14, 4, 1e7, n_part=65, stream=2)]
    one = core.Batch(specs, device="cpu")
    T = 3
    rep = core.Batch(specs, device="cpu", replicas=T)
    assert rep.n_prob == T * one.n_prob and rep.n_tiles == T * one.n_tiles
    assert rep.theta_len == T * one.theta_len
    assert rep.total_particles == T * one.total_particles
    assert rep.obs_len == one.obs_len and rep.box_len == one.box_len
    for t in range(T):
        for r in range(one.n_prob):
            a, b = one.table[r], rep.table[t * one.n_prob + r]
            assert b["theta_off"] == a["theta_off"] + t * one.theta_len
            assert b["p_off"] == a["p_off"] + t * one.total_particles
            assert b["obs_off"] == a["obs_off"] and b["box_off"] == a["box_off"]
            assert b["n_part"] == a["n_part"] and b["n_seg"] == a["n_seg"]
    # pack/unpack see the replicas as problems of their own
    th = [np.full((s.n_part, s.d), 10.0 * t + r) for t in range(T) for r, s in enumerate(specs)]
    flat = rep.pack_theta(th).cpu().numpy()
    for t in range(T):
        np.testing.assert_array_equal(flat[t * one.theta_len:(t + 1) * one.theta_len],
                                      one.pack_theta(th[t * 2:(t + 1) * 2]).cpu().numpy())


def test_replicas_and_trials_are_validated():
    specs = [core.ProblemSpec(30, 10, 14, 3, 1e6, n_part=10)]
    with pytest.raises(ValueError, match="replicas"):
        core.Batch(specs, device="cpu", replicas=0)
    with pytest.raises(ValueError, match="replicas"):
        core.Batch(specs, device="cpu", replicas=2, with_traj=True)
    b = core.Batch(specs, device="cpu")
    for T in (0, 9):
        with pytest.raises(ValueError, match="n_trials"):
            core.LbfgsState(b, f64(b.theta_len), n_trials=T)
