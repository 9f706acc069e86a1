"""Train and evaluate the learned shadow surrogate on the GPU with the library's kernels.

Labels come from the geometric shadow pass (ss_shadow_plain): for each training sun,
the visibility of sampled surfels, label = [vis >= 0.5].  Training uses the library's
MLP forward/backward (BCE with logits) and Adam.  Evaluation compares, on held-out suns,
the surrogate shadow pass (with the geometric pass as fallback inside the confidence
band) against the plain pass, in agreement of the lit/shadow decision and in time per
view.  The surrogate and this protocol are not in the paper; they follow the stated
workload (4-layer 64-wide BF16 MLP, 16-frequency features, 10M labels from 1000 suns,
200 held-out suns, fallback band 0.1).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import surrogate as sg
from .raster import Context, Plan, SurfelTensors, ViewTensors, default_settings


@dataclass
class TrainConfig:
    train_suns: int = 1000
    points_per_sun: int = 10_000
    eval_suns: int = 200
    sun_elev_deg: tuple = (30.0, 70.0)
    train_seed: int = 2004
    eval_seed: int = 3004
    batch: int = 65_536
    epochs: int = 30
    lr: float = 1e-2
    band: float = 0.1
    chunk: int = 20            # suns per geometric-pass call
    init_seed: int = 0


def draw_suns(n, elev, seed, exclude=None, min_sep_deg=0.5):
    """Suns (phi, theta) in radians; with `exclude`, redraw any sun within min_sep_deg of
    an excluded one (great-circle distance of the sun directions)."""
    rng = np.random.default_rng(seed)
    out = []
    ex = None
    if exclude is not None:
        e = np.asarray(exclude, np.float64)
        ex = np.stack([np.cos(e[:, 1]) * np.cos(e[:, 0]), np.cos(e[:, 1]) * np.sin(e[:, 0]),
                       np.sin(e[:, 1])], 1)
    while len(out) < n:
        phi = rng.uniform(0, 2 * np.pi)
        th = np.deg2rad(rng.uniform(*elev))
        if ex is not None:
            d = np.array([np.cos(th) * np.cos(phi), np.cos(th) * np.sin(phi), np.sin(th)])
            if np.degrees(np.arccos(np.clip(ex @ d, -1, 1))).min() < min_sep_deg:
                continue
        out.append((phi, th))
    return np.asarray(out, np.float32)


class ShadowLab:
    """A scene plus plans that render many suns with one camera."""

    def __init__(self, ctx: Context, surf: SurfelTensors, Fxy: torch.Tensor, b_z: float,
                 chunk: int, sun_map=1024, tile=16):
        self.ctx, self.surf, self.chunk = ctx, surf, chunk
        self.Fxy1 = Fxy[:1].contiguous()
        self.b_z = b_z
        n = surf.mean.shape[0]
        st = default_settings(tile_size=tile, sun_map_size=sun_map)
        # the main-view size does not matter for the sun maps (fixed S x S)
        self.plan = Plan(ctx, n, [64] * chunk, [64] * chunk, st)
        self.views = None

    def _views(self, sun):
        k = sun.shape[0]
        F = self.Fxy1.expand(k, 2, 4).contiguous()
        return ViewTensors(np.full(k, 64, np.int32), np.full(k, 64, np.int32), F, self.b_z,
                           sun=sun)

    def plain(self, sun):
        """Geometric visibility [len(sun), N] (chunks of `chunk` suns)."""
        out = []
        for s0 in range(0, sun.shape[0], self.chunk):
            s = sun[s0:s0 + self.chunk]
            if s.shape[0] < self.chunk:
                s = torch.cat([s, s[-1:].expand(self.chunk - s.shape[0], 2)], 0)
            v = self._views(s.contiguous())
            self.plan.ensure_capacity(self.surf, v)
            vis = self.plan.shadow(self.surf, v)
            out.append(vis[:min(self.chunk, sun.shape[0] - s0)].clone())
        return torch.cat(out, 0)


def train(lab: ShadowLab, net: sg.Mlp, cfg: TrainConfig, log=print):
    dev = lab.surf.mean.device
    n = lab.surf.mean.shape[0]
    suns = draw_suns(cfg.train_suns, cfg.sun_elev_deg, cfg.train_seed)
    rng = np.random.default_rng(cfg.train_seed + 1)
    t0 = time.time()
    P, S, Y = [], [], []
    sun_t = torch.as_tensor(suns, device=dev)
    for s0 in range(0, cfg.train_suns, lab.chunk):
        vis = lab.plain(sun_t[s0:s0 + lab.chunk])
        for j in range(vis.shape[0]):
            idx = torch.as_tensor(rng.choice(n, cfg.points_per_sun, replace=False), device=dev)
            P.append(lab.surf.mean[idx])
            S.append(sun_t[s0 + j].expand(cfg.points_per_sun, 2))
            Y.append((vis[j, idx] >= 0.5).float())
    P, S, Y = torch.cat(P).contiguous(), torch.cat(S).contiguous(), torch.cat(Y).contiguous()
    torch.cuda.synchronize()
    t_label = time.time() - t0
    log(f"[surrogate] {Y.numel()} labels from {cfg.train_suns} suns in {t_label:.1f} s, lit {Y.mean().item():.3f}")
    w = torch.as_tensor(init_params(cfg.init_seed), device=dev)
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    if net.max_points < cfg.batch:
        net.bind(cfg.batch)
    M = Y.numel()
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg.train_seed + 2)
    step = 0
    steps_total = cfg.epochs * ((M + cfg.batch - 1) // cfg.batch)
    loss = torch.zeros(1, device=dev)
    t1 = time.time()
    for ep in range(cfg.epochs):
        perm = torch.randperm(M, device=dev, generator=gen)
        for b0 in range(0, M, cfg.batch):
            idx = perm[b0:b0 + cfg.batch]
            step += 1
            lr = cfg.lr * 0.5 * (1 + np.cos(np.pi * (step - 1) / steps_total))
            g = net.backward(w, P[idx].contiguous(), S[idx].contiguous(),
                             labels=Y[idx].contiguous(), scale=1.0 / idx.numel(), loss=loss)
            sg.adam(w, m, v, g, lr=lr, step=step)
        log(f"[surrogate] epoch {ep + 1}/{cfg.epochs} loss {loss.item():.4f}")
    torch.cuda.synchronize()
    t_train = time.time() - t1
    # training accuracy on a sample
    k = min(M, 1_000_000)
    acc = ((net.forward(w, P[:k], S[:k]) > 0).float() == Y[:k]).float().mean().item()
    return w, dict(labels=M, label_s=round(t_label, 2), train_s=round(t_train, 2), steps=step,
                   train_acc=round(acc, 4), final_loss=round(loss.item(), 4))


def init_params(seed):
    """He-uniform weights, zero biases, seeded: [W1, b1, W2, b2, W3, b3, w4, b4]."""
    rng = np.random.default_rng(seed)
    he = lambda shape, fan_in: rng.uniform(-np.sqrt(6.0 / fan_in), np.sqrt(6.0 / fan_in), size=shape)
    parts = [he((64, 128), 128), np.zeros(64), he((64, 64), 64), np.zeros(64),
             he((64, 64), 64), np.zeros(64), he((64,), 64), np.zeros(1)]
    w = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert w.size == sg.N_PARAMS
    return w


def evaluate(lab: ShadowLab, net: sg.Mlp, w, cfg: TrainConfig, train_suns=None, log=print,
             bands=(0.0, 0.02, 0.05, 0.1, 0.2, 0.3)):
    """Held-out suns: agreement of the surrogate (with fallback) and of the bare network
    with the plain pass, fallback fraction, and ms per view of both passes; `curve` gives
    agreement, fallback fraction and ms per view of the surrogate pass for each
    fallback band."""
    dev = lab.surf.mean.device
    if train_suns is None:
        train_suns = draw_suns(cfg.train_suns, cfg.sun_elev_deg, cfg.train_seed)
    suns = draw_suns(cfg.eval_suns, cfg.sun_elev_deg, cfg.eval_seed, exclude=train_suns)
    sun_t = torch.as_tensor(suns, device=dev)
    agree = agree_net = fallback = total = lit = 0
    t_plain = t_sur = 0.0
    cur = {b: dict(agree=0, fallback=0, ms=0.0) for b in bands}
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan = lab.plan
    for s0 in range(0, cfg.eval_suns, lab.chunk):
        s = sun_t[s0:s0 + lab.chunk]
        nv = s.shape[0]
        if nv < lab.chunk:
            s = torch.cat([s, s[-1:].expand(lab.chunk - nv, 2)], 0)
        v = lab._views(s.contiguous())
        plan.ensure_capacity(lab.surf, v)
        plan.shadow(lab.surf, v)                       # warm
        ev_a.record(); ref = plan.shadow(lab.surf, v, check=False); ev_b.record()
        torch.cuda.synchronize()
        t_plain += ev_a.elapsed_time(ev_b)
        ref = ref.clone()
        sg.shadow_surrogate(plan, net, w, lab.surf, v, band=cfg.band)   # warm
        ev_a.record(); vis = sg.shadow_surrogate(plan, net, w, lab.surf, v, band=cfg.band); ev_b.record()
        torch.cuda.synchronize()
        t_sur += ev_a.elapsed_time(ev_b)
        fallback += plan.stats()["fallback"] * nv // lab.chunk
        agree_main = ((vis[:nv] >= 0.5) == (ref[:nv] >= 0.5)).sum().item()
        for b in bands:
            sg.shadow_surrogate(plan, net, w, lab.surf, v, band=b)      # warm
            ev_a.record(); vb = sg.shadow_surrogate(plan, net, w, lab.surf, v, band=b); ev_b.record()
            torch.cuda.synchronize()
            cur[b]["ms"] += ev_a.elapsed_time(ev_b)
            cur[b]["fallback"] += plan.stats()["fallback"] * nv // lab.chunk
            cur[b]["agree"] += ((vb[:nv] >= 0.5) == (ref[:nv] >= 0.5)).sum().item()
        p = net.forward(w, lab.surf.mean, s.contiguous(), all_pairs=True, prob=True).view(lab.chunk, -1)
        agree += agree_main
        agree_net += ((p[:nv] >= 0.5) == (ref[:nv] >= 0.5)).sum().item()
        lit += (ref[:nv] >= 0.5).sum().item()
        total += ref[:nv].numel()
    nviews = (cfg.eval_suns + lab.chunk - 1) // lab.chunk * lab.chunk
    res = dict(eval_suns=cfg.eval_suns, points=total,
               agreement=round(agree / total, 5), agreement_network_only=round(agree_net / total, 5),
               fallback_fraction=round(fallback / total, 5), lit_fraction=round(lit / total, 5),
               plain_ms_per_view=round(t_plain / nviews, 4),
               surrogate_ms_per_view=round(t_sur / nviews, 4),
               curve=[dict(band=b, agreement=round(c["agree"] / total, 5),
                           fallback_fraction=round(c["fallback"] / total, 5),
                           ms_per_view=round(c["ms"] / nviews, 4)) for b, c in cur.items()])
    log(f"[surrogate] eval: {res}")
    return res
