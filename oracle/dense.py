"""Dense torch-FP64 definition of the forward render, for tiny scenes only.

TEST INFRASTRUCTURE ONLY.  A second, independently written statement of the same
definition as satsplat_oracle.c (Sec. 3.2 of the paper: affine ray-splat intersection,
lower-bounded Gaussian, centre-depth order, Eq. rasterization; Sec. 3.1 Eq.
image_formation), evaluated for every (pixel, surfel) pair at once with tensor ops and
differentiated by torch autograd.  Discrete decisions (skip below alpha_min, stop below
T_min, low-pass branch, clamp at alpha_max, degenerate test) are taken on detached
values, so they carry zero derivative, as in the analytic adjoint.
"""
from __future__ import annotations

import numpy as np
import torch


def render(params, scene, settings, vis=None):
    """params: dict of float64 tensors mean [n,3], t_u, t_v, scale [n,2], opacity [n],
    albedo [n,3], dF [V,2,4], colC [V,3,3], colc [V,3], ambient [V,3].
    Returns per-view lists of image [3,H,W], A, V [H,W], D, N [3,H,W], T."""
    dt = torch.float64
    W = [int(w) for w in scene["width"]]
    H = [int(h) for h in scene["height"]]
    Fxy = torch.as_tensor(np.asarray(scene["Fxy"], np.float64))
    bz = float(scene["b_z"])
    p, tu, tv = params["mean"], params["t_u"], params["t_v"]
    s, o, a = params["scale"], params["opacity"], params["albedo"]
    n = p.shape[0]
    # order: FP32 key b_z - p_z, ties by index (np.lexsort: last key is primary)
    kap = (np.float32(bz) - np.asarray(scene["surfels"]["mean"], np.float32)[:, 2]).astype(np.float32)
    order = torch.as_tensor(np.lexsort((np.arange(n), kap)))
    inv_s2 = 1.0 / settings.sigma ** 2
    out = []
    for v in range(len(W)):
        F = Fxy[v] + params["dF"][v]
        B, b = F[:, :3], F[:, 3]
        M = torch.stack([s[:, 0:1] * tu, s[:, 1:2] * tv], dim=2)          # [n,3,2]
        T = torch.einsum("rj,njq->nrq", B, M)                              # [n,2,2]
        c = p @ B.T + b                                                    # [n,2]
        det = T[:, 0, 0] * T[:, 1, 1] - T[:, 0, 1] * T[:, 1, 0]
        deg = ~(det.detach().abs() > settings.det_rel_eps * (T.detach() ** 2).sum((1, 2)))
        Tsafe = torch.where(deg[:, None, None], torch.eye(2, dtype=dt).expand(n, 2, 2), T)
        Q = torch.linalg.inv(Tsafe)
        filt = torch.ones(n, dtype=torch.bool) if settings.lowpass_mode == 0 else deg
        m = torch.cross(tu, tv, dim=1)
        nrm = m / m.norm(dim=1, keepdim=True)
        d = torch.cross(B[0], B[1], dim=0).detach()
        if d[2] > 0:
            d = -d
        nrm = torch.where(((m.detach() @ d) > 0)[:, None], -nrm, nrm)
        ys, xs = torch.meshgrid(torch.arange(H[v], dtype=dt) + 0.5,
                                torch.arange(W[v], dtype=dt) + 0.5, indexing="ij")
        X = torch.stack([xs.reshape(-1), ys.reshape(-1)], 1)               # [P,2]
        cc, QQ = c[order], Q[order]
        dlt = X[:, None, :] - cc[None]                                     # [P,n,2]
        u = torch.einsum("nrq,pnq->pnr", QQ, dlt)
        rho_u = (u ** 2).sum(-1)
        rho_u = torch.where(deg[order][None], torch.full_like(rho_u, float("inf")), rho_u)
        rho_f = (dlt ** 2).sum(-1) * inv_s2
        rho_f = torch.where(filt[order][None], rho_f, torch.full_like(rho_f, float("inf")))
        ub = (rho_u <= rho_f).detach()
        rho = torch.where(ub, rho_u, rho_f)
        finite = torch.isfinite(rho.detach())
        rho = torch.where(finite, rho, torch.zeros_like(rho))
        G = torch.exp(-0.5 * rho)
        oG = o[order][None] * G
        alpha = torch.where(oG.detach() < settings.alpha_max, oG,
                            torch.full_like(oG, settings.alpha_max))
        keep = finite & (alpha.detach() >= settings.alpha_min)
        al = torch.where(keep, alpha, torch.zeros_like(alpha))
        T_after = torch.cumprod(1.0 - al.detach(), dim=1)
        keep = keep & (T_after >= settings.T_min)
        al = torch.where(keep, alpha, torch.zeros_like(alpha))
        one_m = 1.0 - al
        Tb = torch.cat([torch.ones_like(one_m[:, :1]), torch.cumprod(one_m, dim=1)[:, :-1]], 1)
        w = al * Tb                                                        # [P,n]
        k = M[:, 2, :][order]                                              # [n,2]
        z0 = (bz - p[:, 2])[order]
        z = torch.where(ub, z0[None] - (u * k[None]).sum(-1), z0[None].expand_as(w))
        A = w @ a[order]
        D = (w * z).sum(1)
        N = w @ nrm[order]
        Tf = torch.prod(one_m, dim=1)
        if vis is not None:
            vv = torch.as_tensor(np.asarray(vis, np.float64)[v])
            Vp = w @ vv[order]
        else:
            Vp = torch.ones(X.shape[0], dtype=dt)
        Cm = params["colC"][v] if params.get("colC") is not None else torch.eye(3, dtype=dt)
        cb = params["colc"][v] if params.get("colc") is not None else torch.zeros(3, dtype=dt)
        La = params["ambient"][v] if params.get("ambient") is not None else torch.zeros(3, dtype=dt)
        I = (A @ Cm.T + cb) * (Vp[:, None] + (1 - Vp[:, None]) * La)
        # depth distortion, half the double sum over all ordered pairs of
        # w_i w_j (m_i - m_j)^2, in its moment form (sum w)(sum w m^2) - (sum w m)^2
        m = z * getattr(settings, "depth_scale", 1.0)
        dist = w.sum(1) * (w * m * m).sum(1) - (w * m).sum(1) ** 2
        hw = (H[v], W[v])
        out.append(dict(image=I.T.reshape(3, *hw), albedo=A.T.reshape(3, *hw),
                        vis=Vp.reshape(hw), depth=D.reshape(hw), normal=N.T.reshape(3, *hw),
                        T=Tf.reshape(hw), dist=dist.reshape(hw)))
    return out


def params_from_scene(scene, requires_grad=True):
    s = scene["surfels"]
    V = len(scene["width"])
    t = lambda x: torch.tensor(np.asarray(x, np.float64), requires_grad=requires_grad)
    P = dict(mean=t(s["mean"]), t_u=t(s["t_u"]), t_v=t(s["t_v"]), scale=t(s["scale"]),
             opacity=t(s["opacity"]), albedo=t(s["albedo"]),
             dF=t(scene["dF"] if scene.get("dF") is not None else np.zeros((V, 2, 4))))
    for k in ("colC", "colc", "ambient"):
        P[k] = t(scene[k]) if scene.get(k) is not None else None
    return P


def normal_loss(depth, T, normal, Fxy, dF, b_z, tau=0.5):
    """Normal-consistency loss of one view (Sec. 3.2 "Normal Definition", Eq.
    surface_normal), dense torch statement: depth, T [H, W], normal [3, H, W], dF [2, 4]
    torch tensors; T is used as a constant.  Same readings as oracle.geom."""
    dt = torch.float64
    H, W = depth.shape
    F = torch.as_tensor(np.asarray(Fxy, np.float64)) + dF
    Bxy, b = F[:, :3], F[:, 3]
    M = torch.cat([Bxy, torch.tensor([[0.0, 0.0, -1.0]], dtype=dt)], 0)
    a = (1.0 - T).detach()
    cover = a >= tau
    zbar = torch.where(cover, depth / torch.where(cover, a, torch.ones_like(a)), torch.zeros_like(a))
    ys, xs = torch.meshgrid(torch.arange(H, dtype=dt) + 0.5, torch.arange(W, dtype=dt) + 0.5,
                            indexing="ij")
    rhs = torch.stack([xs - b[0], ys - b[1], zbar - b_z], -1)               # [H, W, 3]
    ps = torch.linalg.solve(M.expand(H, W, 3, 3), rhs.unsqueeze(-1)).squeeze(-1)
    gx = ps[1:-1, 2:] - ps[1:-1, :-2]
    gy = ps[2:, 1:-1] - ps[:-2, 1:-1]
    n = torch.linalg.cross(gx, gy, dim=-1)
    d = torch.linalg.cross(Bxy[0].detach(), Bxy[1].detach(), dim=0)
    if d[2] > 0:
        d = -d
    flip = ((n.detach() @ d) > 0)
    Nd = n / n.norm(dim=-1, keepdim=True)
    Nd = torch.where(flip[..., None], -Nd, Nd)
    ok = cover[1:-1, 1:-1] & cover[1:-1, 2:] & cover[1:-1, :-2] & cover[2:, 1:-1] & cover[:-2, 1:-1]
    dot = (normal[:, 1:-1, 1:-1].permute(1, 2, 0) * Nd).sum(-1)
    return torch.where(ok, 1.0 - dot, torch.zeros_like(dot)).sum() / (H * W)
