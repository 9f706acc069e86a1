"""The allocation-free MLP backward (ss_mlp_backward_noalloc, buffers in the library's
fixed scratch array) against the workspace entry point (ss_mlp_backward) on the same
inputs: identical gradients and loss (the same deterministic kernels run), on two calls
in a row, the second with a smaller batch, plus the FP64 BF16-emulating oracle's bar."""
import numpy as np
import pytest
import torch

from paper_2606_28581_amd import _lib
from oracle import mlp as om
from paper_2606_28581_amd import surrogate as sg
from paper_2606_28581_amd._lib import SatSplatError
from gpu_common import context, to_np

pytestmark = pytest.mark.gpu

CENTRE = np.array([-4.0, 2.5, 9.0], np.float32)
INV_HALF = np.float32(1.0 / 60.0)


def cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def inputs(M, seed):
    rng = np.random.default_rng(seed)
    pts = (rng.uniform(-60, 60, size=(M, 3)) + CENTRE).astype(np.float32)
    sun = np.stack([rng.uniform(0, 2 * np.pi, M), rng.uniform(0.5, 1.2, M)], 1).astype(np.float32)
    labels = (rng.uniform(size=M) > 0.4).astype(np.float32)
    dl = rng.normal(size=M).astype(np.float32)
    return pts, sun, labels, dl


def test_noalloc_backward_matches_workspace_entry_point_on_two_calls():
    ctx = context()
    w = om.init_params(21)
    tw = cuda(w)
    ref_net = sg.Mlp(ctx, CENTRE, INV_HALF, max_points=_lib.SS_NOALLOC_MAX_POINTS)
    free_net = sg.Mlp(ctx, CENTRE, INV_HALF, max_points=None)    # no workspace at all
    assert free_net.workspace is None
    for M, mode, seed in ((12000, "bce", 1), (777, "dlogit", 2)):
        print(f"[no-alloc] M={M} mode={mode} seed={seed}", flush=True)
        pts, sun, labels, dl = inputs(M, seed)
        args = dict(labels=cuda(labels), scale=1.0 / M) if mode == "bce" else \
            dict(d_logits=cuda(dl), scale=1.0)
        loss_a = torch.full((1,), -1.0, device="cuda")
        loss_b = torch.full((1,), -2.0, device="cuda")
        ga = to_np(ref_net.backward(tw, cuda(pts), cuda(sun), loss=loss_a, **args))
        gb = to_np(free_net.backward_noalloc(tw, cuda(pts), cuda(sun), loss=loss_b, **args))
        torch.cuda.synchronize()
        assert np.array_equal(ga, gb), np.abs(ga - gb).max()
        assert float(loss_a.item()) == float(loss_b.item())
        if mode == "bce":
            ref_loss, gref, _ = om.bce_grad(w.astype(np.float64), pts, sun, labels, CENTRE, INV_HALF)
            assert abs(float(loss_b.item()) - ref_loss) < 1e-3 * max(1.0, ref_loss)
        else:
            _, cache = om.forward(w.astype(np.float64), pts, sun, CENTRE, INV_HALF)
            gref = om.backward(cache, dl.astype(np.float64))
        G, R = om.unpack(gb), om.unpack(gref)
        for k in om.SIZES:
            rel = np.linalg.norm(G[k] - R[k]) / max(np.linalg.norm(R[k]), 1e-30)
            assert rel <= 1e-2, (M, k, rel)


def test_noalloc_backward_refuses_batches_beyond_its_scratch():
    ctx = context()
    net = sg.Mlp(ctx, CENTRE, INV_HALF, max_points=None)
    M = _lib.SS_NOALLOC_MAX_POINTS + 1
    pts, sun, labels, _ = inputs(M, 3)
    with pytest.raises(SatSplatError) as e:
        net.backward_noalloc(cuda(om.init_params(1)), cuda(pts), cuda(sun), labels=cuda(labels))
    assert e.value.code == -2      # SS_ERR_CAPACITY, nothing launched
