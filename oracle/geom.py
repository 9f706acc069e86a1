"""FP64 oracle of the geometric regularisers on rendered maps: the depth-gradient world
normal and the normal-consistency loss (Sec. 3.2 "Normal Definition", Eq.
surface_normal).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.

Readings (the paper gives the equation and the loss's weight, Supp. B, but not these
details; the same readings are implemented on the GPU):
* the depth map that is back-projected is the expected depth zbar = D / (1 - T) of a
  pixel (D = sum w z, T the final transmittance), with the accumulated opacity 1 - T
  treated as a constant (no gradient flows into T);
* a pixel is valid when 1 - T >= tau for it and its four neighbours, and it is not on
  the view's border; only valid pixels enter the loss;
* back-projection through the affine camera F' = F + dF with the fixed depth row
  B_z = (0, 0, -1), b_z: the world point p_s of pixel centre x and depth zbar solves
  B_xy p + b_xy = x, b_z - p_z = zbar;
* the gradients of the point map are central differences p_s(i+1, j) - p_s(i-1, j) and
  p_s(i, j+1) - p_s(i, j-1); N = normalise(grad_x x grad_y), oriented like the rendered
  normals (against d = B_x x B_y with d_z < 0);
* per view, L = (1 / P) sum over valid pixels of (1 - N_r . N), N_r the rendered normal
  (the composited sum w n, not renormalised), P the view's pixel count.
"""
from __future__ import annotations

import numpy as np


def _camera(Fxy, dF, v):
    F = np.asarray(Fxy, np.float32)[v].astype(np.float64)
    if dF is not None:
        F = F + np.asarray(dF, np.float32)[v].astype(np.float64)
    return F[:, :3], F[:, 3]


def _view_dir(B):
    d = np.cross(B[0], B[1])
    return -d if d[2] > 0 else d


def _slices(W, H, v_off):
    return v_off, v_off + W * H


def depth_normals_view(B, b, bz, D, T, tau):
    """Depth-gradient normals of one view.  D, T [H, W] float64.  Returns N [3, H, W]
    (zero where invalid), valid [H, W] bool, and the intermediates of the adjoint."""
    H, W = D.shape
    M = np.array([B[0], B[1], [0.0, 0.0, -1.0]])
    Minv = np.linalg.inv(M)
    cover = (1.0 - T) >= tau
    zbar = np.where(cover, D / np.where(cover, 1.0 - T, 1.0), 0.0)
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    rhs = np.stack([xs - b[0], ys - b[1], zbar - bz], 0)               # [3, H, W]
    ps = np.einsum("rk,khw->rhw", Minv, rhs)
    valid = np.zeros((H, W), bool)
    if H >= 3 and W >= 3:
        valid[1:-1, 1:-1] = (cover[1:-1, 1:-1] & cover[1:-1, 2:] & cover[1:-1, :-2] &
                             cover[2:, 1:-1] & cover[:-2, 1:-1])
    gx = np.zeros((3, H, W))
    gy = np.zeros((3, H, W))
    gx[:, 1:-1, 1:-1] = ps[:, 1:-1, 2:] - ps[:, 1:-1, :-2]
    gy[:, 1:-1, 1:-1] = ps[:, 2:, 1:-1] - ps[:, :-2, 1:-1]
    n = np.cross(gx, gy, axis=0)
    nn = np.linalg.norm(n, axis=0)
    d = _view_dir(B)
    sgn = np.where(np.einsum("k,khw->hw", d, n) > 0, -1.0, 1.0)
    N = np.where(valid[None], sgn[None] * n / np.where(valid, nn, 1.0)[None], 0.0)
    return N, valid, dict(Minv=Minv, zbar=zbar, cover=cover, gx=gx, gy=gy, n=n, nn=nn,
                          sgn=sgn, rhs=rhs)


def normal_loss(scene, depth, T, normal, tau=0.5):
    """Normal-consistency loss of every view and its adjoint.  depth, T [P] and normal
    [3P] in the forward's planar per-view layout.  Returns (loss [V], N_d [3P],
    d_depth [P], d_normal [3P], d_dF [V, 2, 4]), gradients of sum_v loss[v]."""
    W = np.asarray(scene["width"], np.int64)
    H = np.asarray(scene["height"], np.int64)
    V = W.shape[0]
    depth = np.asarray(depth, np.float64)
    T = np.asarray(T, np.float64)
    normal = np.asarray(normal, np.float64)
    P_all = int(np.sum(W * H))
    loss = np.zeros(V)
    Nd_all = np.zeros(3 * P_all)
    g_depth = np.zeros(P_all)
    g_normal = np.zeros(3 * P_all)
    g_dF = np.zeros((V, 2, 4))
    off = 0
    for v in range(V):
        w, h = int(W[v]), int(H[v])
        P = w * h
        B, b = _camera(scene["Fxy"], scene.get("dF"), v)
        D = depth[off:off + P].reshape(h, w)
        Tv = T[off:off + P].reshape(h, w)
        Nr = normal[3 * off:3 * off + 3 * P].reshape(3, h, w)
        Nd, valid, c = depth_normals_view(B, b, float(scene["b_z"]), D, Tv, tau)
        dot = np.einsum("khw,khw->hw", Nr, Nd)
        loss[v] = np.sum(np.where(valid, 1.0 - dot, 0.0)) / P
        Nd_all[3 * off:3 * off + 3 * P] = Nd.reshape(-1)
        # adjoint: dL/dN_r = -N_d / P, dL/dN_d = -N_r / P (valid pixels)
        g_normal[3 * off:3 * off + 3 * P] = np.where(valid[None], -Nd / P, 0.0).reshape(-1)
        gNd = np.where(valid[None], -Nr / P, 0.0)
        # N_d = sgn n / |n|  ->  dL/dn = sgn (gNd - N_d (N_d . gNd)) / |n|
        proj = np.einsum("khw,khw->hw", Nd, gNd)
        gn = np.where(valid[None], c["sgn"][None] * (gNd - Nd * proj[None]) /
                      np.where(valid, c["nn"], 1.0)[None], 0.0)
        # n = gx x gy  ->  dL/dgx = gy x gn, dL/dgy = gn x gx
        ggx = np.cross(c["gy"], gn, axis=0)
        ggy = np.cross(gn, c["gx"], axis=0)
        # gx = p(i+1) - p(i-1), gy = p(j+1) - p(j-1)
        gps = np.zeros((3, h, w))
        gps[:, 1:-1, 2:] += ggx[:, 1:-1, 1:-1]
        gps[:, 1:-1, :-2] -= ggx[:, 1:-1, 1:-1]
        gps[:, 2:, 1:-1] += ggy[:, 1:-1, 1:-1]
        gps[:, :-2, 1:-1] -= ggy[:, 1:-1, 1:-1]
        # p_s = Minv rhs, rhs_2 = zbar - b_z, zbar = D / (1 - T) with 1 - T constant
        grhs = np.einsum("rk,rhw->khw", c["Minv"], gps)
        gz = np.where(c["cover"], grhs[2] / np.where(c["cover"], 1.0 - Tv, 1.0), 0.0)
        g_depth[off:off + P] = gz.reshape(-1)
        # camera: dL/dMinv = sum gps rhs^T; Minv = M^-1 -> dL/dM = -Minv^T dL/dMinv Minv^T;
        # rhs_0,1 = x - b -> dL/db = -grhs_0,1
        gMinv = np.einsum("rhw,khw->rk", gps, c["rhs"])
        gM = -c["Minv"].T @ gMinv @ c["Minv"].T
        g_dF[v, :, :3] = gM[:2]
        g_dF[v, :, 3] = -grhs[:2].sum(axis=(1, 2))
        off += P
    return loss, Nd_all, g_depth, g_normal, g_dF
