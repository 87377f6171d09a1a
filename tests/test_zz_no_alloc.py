"""The allocation-free gradient entry point (sird_loss_backward_static)
against sird_loss_backward with a caller's workspace, through the C ABI:
bitwise the same gradients and losses on two calls in a row on one GPU,
the second on a smaller batch (the static scratch keeps the first call's
contents), and an oversized batch refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth
import paper_2204_12346_amd as S
from gpu_helpers import make_batch, need_gpu, random_theta

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _both(b, theta, obs, kind, interval, grad_loss=None):
    g_ref, L_ref = S.sird_loss_backward(b, theta, obs, kind, grad_loss=grad_loss,
                                        loss_out=b.empty_particles(), ckpt_interval=interval)
    g = b.empty_theta()
    L = b.empty_particles()
    S.sird_loss_backward_static(b, theta, obs, kind, grad_loss=grad_loss, grad_theta=g,
                                loss_out=L, ckpt_interval=interval)
    torch.cuda.synchronize()
    return g, L, g_ref, L_ref


def test_static_scratch_gradient_equals_workspace_gradient():
    # call 1: one fit of 8192 particles over 1800 steps (about 36 MiB of
    # workspace)
    f = synth.c2().fits[0]
    assert S.sird_loss_backward_workspace(make_batch([f]), 0) <= S.core.STATIC_SCRATCH_BYTES
    b1 = make_batch([f])
    th = random_theta(f, f.n_part, seed=5)
    th[:, :f.K] *= 0.5
    print("case static scratch: 8192 particles, ssre", flush=True)
    g, L, g_ref, L_ref = _both(b1, b1.pack_theta([th]), b1.pack_obs([f.y]), "ssre", 0)
    assert torch.equal(g, g_ref) and torch.equal(L, L_ref)
    # call 2: a smaller uneven batch, another cost, interval and upstream
    # gradient, on the scratch the first call left behind
    wl = synth.c3(regions=list(range(6)))
    n_parts = [100, 64, 1, 150, 33, 70]
    ths = [random_theta(fr, n, seed=50 + r) for r, (fr, n) in enumerate(zip(wl.fits, n_parts))]
    b2 = make_batch(wl.fits, n_parts)
    scale = torch.linspace(-1, 2, b2.total_particles, dtype=torch.float64, device="cuda")
    print("case static scratch: uneven batch, mse", flush=True)
    g, L, g_ref, L_ref = _both(b2, b2.pack_theta(ths), b2.pack_obs([fr.y for fr in wl.fits]),
                               "mse", 13, grad_loss=scale)
    assert torch.equal(g, g_ref) and torch.equal(L, L_ref)
    assert np.all(np.isfinite(g.cpu().numpy()))
    # call 3: the segment-parallel sweep on the same scratch
    print("case static scratch: uneven batch, segment-parallel sweep", flush=True)
    g, L, g_ref, L_ref = _both(b2, b2.pack_theta(ths), b2.pack_obs([fr.y for fr in wl.fits]),
                               "mse", S.CKPT_SEGMENTS, grad_loss=scale)
    assert torch.equal(g, g_ref) and torch.equal(L, L_ref)


def test_static_scratch_refuses_an_oversized_batch():
    wl, thetas = synth.c4()
    f = wl.fits[0]
    b = make_batch([f])
    g = b.empty_theta()
    g.fill_(7.0)
    with pytest.raises(S.SirdError, match="static scratch"):
        S.sird_loss_backward_static(b, b.pack_theta([thetas]), b.pack_obs([f.y]), "ssre",
                                    grad_theta=g)
    torch.cuda.synchronize()
    assert bool((g == 7.0).all())
