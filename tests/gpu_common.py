"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the oracle)."""
import functools

import numpy as np
import torch

import oracle
import synth
import paper_2606_28581_amd as ss


@functools.lru_cache(maxsize=1)
def context():
    return ss.Context(0)


def oracle_settings(ts=16, mode=0, S=1024):
    return oracle.Settings(lowpass_mode=mode, tile_size=ts, sun_map_size=S)


def make_plan(scene, ts=16, batch=64, mode=0, S=1024, with_sun=False):
    surf, views = ss.scene_to_device(scene, with_sun=with_sun)
    s = ss.default_settings(tile_size=ts, batch_depth=batch, lowpass_mode=mode, sun_map_size=S)
    plan = ss.Plan(context(), surf.mean.shape[0], views.width, views.height, s)
    plan.ensure_capacity(surf, views)
    return plan, surf, views


def to_np(t):
    return t.detach().cpu().numpy()


def expand3(mask, W, H):
    """Per-pixel mask (concatenated views) -> mask of the 3-channel planar layout."""
    out = []
    off = 0
    for w, h in zip(W, H):
        P = int(w) * int(h)
        out.append(np.tile(mask[off:off + P], 3))
        off += P
    return np.concatenate(out)


# Gradients are FP32 sums whose order the hardware's float atomics decide (LDS and global).
# Reordering a sum of K terms moves it by about sqrt(K) * 6e-8 * sum|x_i|; rel_err floors
# its denominator at 1e-2 rms, so a nearly cancelling element can magnify that up to 100x.
# Per-record K stays in the hundreds here: 1e-4 bounds run-to-run differences.
ATOMIC_ORDER_TOL = 1e-4


def rel_err(a, b):
    """max_i |a_i - b_i| / max(|b_i|, 1e-2 rms(b)): the per-tensor gradient metric."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    rms = np.sqrt(np.mean(b ** 2)) if b.size else 0.0
    den = np.maximum(np.abs(b), 1e-2 * rms + 1e-30)
    return float(np.max(np.abs(a - b) / den)) if b.size else 0.0


GRAD_KEYS = ("mean", "t_u", "t_v", "scale", "opacity", "albedo", "dF", "colC", "colc", "ambient")
