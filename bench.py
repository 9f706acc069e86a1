"""Benchmark of the SatSplat hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
  sun-view shadow pass for every view (sun cameras, depth-only sun maps, per-surfel
  soft visibility) -> forward render of every view with that visibility, colour
  correction and camera deltas -> backward to every surfel parameter, camera delta
  and colour term.
Default workload: 2M surfels on a 1x1 km synthetic city, 40 affine views of uneven
sides in [1024, 2048] px, a 1024^2 sun map per view.

Prints ONE JSON line.  `value` is fwd+bwd throughput in Mpix/s over the timed steps
(inputs resident in HBM).  `roofline` reports the dominant kernel, timed live with HIP
events on the stream its kernels run on; `cpu_baseline` times the FP64 oracle on a
bounded pixel sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# Published FP32 vector peak of the MI355X: 256 CU x 2.4 GHz x 256 flop/clk (it counts
# packed dual-FP32 FMAs).  The library is compiled with packed FP32 operations disabled,
# so its own issue ceiling is half of that (64 FMA lanes per CU and clock):
VALU_PEAK_TFLOPS = 157.3
VALU_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# Algorithmic FP32 flops per contributing (pixel, surfel) pair: ~30 operations and one
# exponential (counted as 4) in the forward, ~80 in the backward.
FLOPS_FWD_PAIR = 34
FLOPS_BWD_PAIR = 80


def raster_kernel_bytes(kernel, P, K):
    """Algorithmic HBM bytes of one launch of a raster kernel over all views (P pixels,
    K (tile, surfel) pairs): the forward reads a 72-byte record (and its list entry) per
    pair and writes 52 bytes per pixel (image, albedo, V, depth, normal, T, last); the
    backward reads 68 bytes per pixel (upstream image, depth and normal gradients, saved
    albedo, V, T, last), re-reads each pair's record and adds its 64-byte record gradient."""
    if kernel == "raster_fwd":
        return 72 * K + 52 * P
    return 68 * P + (72 + 64) * K


# HBM bytes per launch measured with the profiler's byte counters (FETCH_SIZE, WRITE_SIZE,
# each scaled by what it reads for a plain copy of known size).  The record names the
# digest of the kernel sources it was taken with; any change to them makes it stale and
# `traffic` is then reported as null.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_c3_2M_40views_tile8_batch64.json")


def kernel_source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for rel in files:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, tile, batch):
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if (rec.get("workload"), rec.get("tile"), rec.get("batch_depth")) != (workload, tile, batch):
        return None
    if kernel not in rec.get("kernels", {}):
        return None
    if rec.get("source_sha256") != kernel_source_digest(rec.get("source_files", [])):
        return None
    return rec["kernels"][kernel]["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--tile-order", type=int, default=0, choices=(0, 1),
                    help="raster dispatch order: 0 static XCD chunks (default), 1 heavy tiles first per XCD")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="eager steps instead of a HIP graph")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=512)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip training / evaluating the learned shadow surrogate")
    ap.add_argument("--surrogate-epochs", type=int, default=30)
    ap.add_argument("--no-camera", action="store_true",
                    help="skip the camera-robustness experiment")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the training-step-scale run (5M surfels, 50 views of 2048^2)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this many MiB (5 times) and exit; "
                         "used to calibrate the profiler's FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_step_bytes(N, V, P, K, Ks, S, Nv=None, Nvs=None):
    """Bytes the method's structure must move per step (surfels read/written once,
    per-view records, pair lists, per-pixel images, record gradients, sun maps)."""
    Nv = N if Nv is None else Nv
    Nvs = N if Nvs is None else Nvs
    per_step = 60 * N + 16 * N + 60 * N
    fwd = 68 * Nv * V + 16 * K + 72 * K + 52 * P
    bwd = 68 * P + 72 * K + 64 * K + 64 * Nv * V
    sun = 44 * Nvs * V + 64 * Ks + 8 * S * S * V + 4 * N * V
    return per_step + fwd + bwd + sun


def copy_bandwidth(mib=2048, reps=10):
    """Achievable HBM bandwidth: a plain device-to-device copy, bytes read + written per
    second, timed with HIP events."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    return 2 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, n_pix, seed=5, n_pix_1t=16):
    import numpy as np
    import oracle
    oracle.build(force=False)
    W, H = int(scene["width"][0]), int(scene["height"][0])
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(W * H, size=n_pix, replace=False)).astype(np.int64)
    scene1 = dict(scene, width=scene["width"][:1], height=scene["height"][:1],
                  Fxy=scene["Fxy"][:1], dF=scene["dF"][:1],
                  colC=None if scene["colC"] is None else scene["colC"][:1],
                  colc=None if scene["colc"] is None else scene["colc"][:1],
                  ambient=None if scene["ambient"] is None else scene["ambient"][:1])
    st = oracle.Settings()
    g = np.random.default_rng(seed + 1)
    dI = g.standard_normal(3 * n_pix).astype(np.float32)
    dD = g.standard_normal(n_pix).astype(np.float32)
    dN = g.standard_normal(3 * n_pix).astype(np.float32)
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.forward(scene1, st, sel=sel)
    t1 = time.perf_counter()
    oracle.backward(scene1, dI, dD, dN, st, sel=sel)
    t2 = time.perf_counter()
    # one thread, on the first n_pix_1t pixels of the same sample
    s1 = sel[:n_pix_1t]
    oracle.set_threads(1)
    t3 = time.perf_counter()
    oracle.forward(scene1, st, sel=s1)
    oracle.backward(scene1, dI[:3 * n_pix_1t], dD[:n_pix_1t], dN[:3 * n_pix_1t], st, sel=s1)
    t4 = time.perf_counter()
    oracle.set_threads(cores)
    return dict(value=n_pix / (t2 - t0) / 1e6, unit="Mpix/s", cores=cores,
                kind="oracle", cpu=cpu_model(),
                one_thread=dict(value=n_pix_1t / (t4 - t3) / 1e6, unit="Mpix/s",
                                sample=f"first {n_pix_1t} pixels of the sample, {t4 - t3:.1f} s"),
                sample=f"{n_pix} seeded pixels of view 0 ({W}x{H}), forward {t1 - t0:.1f} s + "
                       f"backward {t2 - t1:.1f} s, FP64 brute force over all {scene['surfels']['mean'].shape[0]} "
                       f"surfels per pixel, no shadow pass")


def surrogate_eval(ctx, args):
    """Learned shadow surrogate on the 1M-surfel city: 10M labels from 1000 suns by the
    geometric pass, GPU training, then 200 held-out suns: agreement of the lit/shadow
    decision with the geometric pass (fallback band |p - 0.5| < 0.1) and ms per view of
    both passes."""
    import numpy as np
    import torch
    import synth
    import paper_2606_28581_amd as ss
    from paper_2606_28581_amd import surrogate as sg
    from paper_2606_28581_amd import surrogate_train as st
    t0 = time.time()
    spec = synth.config(2)
    scene = synth.make_scene(spec)
    surf, views = ss.scene_to_device(scene, with_sun=False)
    half = spec.extent / 2
    zc = float(np.mean(scene["surfels"]["mean"][:, 2]))
    net = sg.Mlp(ctx, np.array([0.0, 0.0, zc], np.float32), np.float32(1.0 / half))
    cfg = st.TrainConfig(epochs=args.surrogate_epochs)
    lab = st.ShadowLab(ctx, surf, views.Fxy, views.b_z, cfg.chunk)
    w, tr = st.train(lab, net, cfg, log=log)
    ev = st.evaluate(lab, net, w, cfg, log=log)
    out = dict(workload="c4_surrogate_1M_city", **ev, training=tr,
               total_s=round(time.time() - t0, 1))
    out["surrogate_faster"] = ev["surrogate_ms_per_view"] < ev["plain_ms_per_view"]
    return out


def training_scale(args, tile=None, batch=None):
    """Full training step at scale: 5M surfels on a 2x2 km city, 50 views of 2048^2.  Per
    step the learned shadow surrogate (plain-pass fallback for |p - 0.5| < 0.1) gives
    every view's surfel visibility; then the forward of all views with colour correction,
    camera deltas and the depth-distortion channel, the L1 image loss (0.8) against a
    fixed target, the depth-normal consistency loss (0.05) and the distortion (0.05), the
    backward, and Adam over the surfels, camera deltas and colour terms (the paper's loss
    weights; learning rates small enough that the pair count stays within the plan's
    capacity over the timed steps).  The surrogate is first trained with the library's
    kernels on this scene's own plain-pass labels.  Reports steps/s, Mpix/s and peak
    device memory."""
    import numpy as np
    import torch
    import synth
    import paper_2606_28581_amd as ss
    from paper_2606_28581_amd import surrogate as sg
    from paper_2606_28581_amd import surrogate_train as st
    t0 = time.time()
    spec = synth.config(5)
    scene = synth.make_scene(spec)
    log(f"[bench] scene {spec.name}: {spec.n_surfels} surfels, {len(spec.view_sizes)} views, "
        f"generated in {time.time() - t0:.1f} s")
    ctx = ss.Context(0)
    surf, views = ss.scene_to_device(scene, with_sun=True)
    N, V, P = surf.mean.shape[0], len(views.width), views.pixels
    settings = ss.default_settings(tile_size=tile or args.tile, batch_depth=batch or args.batch,
                                   tile_order=args.tile_order)
    plan = ss.Plan(ctx, N, views.width, views.height, settings)
    K, Ks = plan.ensure_capacity(surf, views)
    log(f"[bench] pairs main {K}, sun {Ks}, pixels {P}, workspace {plan.workspace.numel() / 2**30:.1f} GiB")
    zc = float(np.mean(scene["surfels"]["mean"][:, 2]))
    net = sg.Mlp(ctx, np.array([0.0, 0.0, zc], np.float32), np.float32(2.0 / spec.extent))
    cfg = st.TrainConfig(epochs=args.surrogate_epochs)
    lab = st.ShadowLab(ctx, surf, views.Fxy, views.b_z, cfg.chunk)
    w, tr = st.train(lab, net, cfg, log=log)
    del lab
    torch.cuda.empty_cache()
    from paper_2606_28581_amd import train as trn
    dev = "cuda:0"
    vis = torch.empty(V, N, dtype=torch.float32, device=dev)
    shade = lambda: sg.shadow_surrogate(plan, net, w, surf, views, band=0.1, vis_out=vis)
    # target: the first render with 10 % less light (set up once, outside the timing)
    target = (plan.forward(surf, views, shade())["image"] * 0.9).contiguous()
    cfg = trn.adam_config(lr_mean=1e-3, lr_dF=1e-5, camera_start=1)
    trainer = trn.Trainer(plan, surf, views, target, depth_scale=2.0 / spec.extent, cfg=cfg,
                          vis=shade)
    trainer.check = False      # the overflow flag is read once after the timed steps

    def step():
        trainer.step()

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    if plan.check()[0]:
        raise RuntimeError("pair capacity overflow during warmup")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    if plan.check()[0]:
        raise RuntimeError("pair capacity overflow in the timed region")
    fallback = plan.stats()["fallback"] / float(N * V)
    plan.read_timing()
    plan.set_timing(True)
    step()
    torch.cuda.synchronize()
    stages = plan.read_timing()
    plan.set_timing(False)
    ms_step = 1e3 * t_total / args.steps
    return {
        "metric": "fwd+bwd Mpix/s (2DGS affine raster); shadow ms/view plain vs MLP surrogate",
        "value": round(P * args.steps / t_total / 1e6, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "steps_per_s": round(1e3 / ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "surfels": N, "views": V, "pixels": P,
                   "tile": settings.tile_size, "batch_depth": settings.batch_depth,
                   "shadow": "MLP surrogate, plain-pass fallback |p-0.5|<0.1",
                   "step": "surrogate shadows + forward (with distortion) + L1 + normal "
                           "consistency + backward + Adam (surfels, camera deltas, colour)",
                   "launch": "eager", "parallelism": "single GPU"},
        "loss_l1_last": float(trainer.loss_l1.sum()),
        "peak_hbm_GB": round(torch.cuda.max_memory_allocated() / 1e9, 2),
        "pairs": {"main": K, "sun_full": Ks},
        "surrogate": {"fallback_fraction": round(fallback, 5), "training": tr},
        "kernels": {k: round(ms / n, 4) for k, (ms, n) in stages.items() if n},
    }


def dsm_init_timing(reps=5):
    """Geometry-aware initialisation of the 5M surfels of the 2 x 2 km city from its DSM
    (Sec. 3.4): weights, prefix sum and sampling, HIP events around the whole call."""
    import numpy as np
    import torch
    import synth
    from synth.scene import _streams, make_dsm
    from paper_2606_28581_amd import init as gi
    spec = synth.config(5)
    coords, z = make_dsm(spec, _streams(spec.seed)["scene"])
    zt = torch.as_tensor(z.astype(np.float32), device="cuda")
    x0 = float(coords[0])
    gi.dsm_init(zt, x0, x0, spec.gsd, spec.n_surfels, seed=1)      # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        gi.dsm_init(zt, x0, x0, spec.gsd, spec.n_surfels, seed=1 + r)
    e1.record()
    e1.synchronize()
    return dict(workload="c5 DSM 4001^2 nodes -> 5M surfels", ms=round(e0.elapsed_time(e1) / reps, 3),
                cells=int((z.shape[0] - 1) * (z.shape[1] - 1)), surfels=spec.n_surfels)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 (over "
                                   "several GPUs the path would shard views and all-reduce the "
                                   "surfel gradients once per step)"}))
        sys.exit(2)
    import numpy as np
    import torch
    import synth
    import paper_2606_28581_amd as ss

    torch.cuda.set_device(0)
    if args.config == 5:
        print(json.dumps(training_scale(args)))
        return
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 5}))
        return
    t0 = time.time()
    spec = synth.config(args.config)
    scene = synth.make_scene(spec)
    log(f"[bench] scene {spec.name}: {spec.n_surfels} surfels, {len(spec.view_sizes)} views, "
        f"generated in {time.time() - t0:.1f} s")
    ctx = ss.Context(0)
    surf, views = ss.scene_to_device(scene, with_sun=True)
    has_sun = views.sun is not None
    settings = ss.default_settings(tile_size=args.tile, batch_depth=args.batch,
                                   tile_order=args.tile_order)
    plan = ss.Plan(ctx, surf.mean.shape[0], views.width, views.height, settings)
    K, Ks = plan.ensure_capacity(surf, views)
    P = views.pixels
    N = surf.mean.shape[0]
    V = len(views.width)
    S = settings.sun_map_size
    log(f"[bench] pairs main {K}, sun {Ks}, pixels {P}, workspace {plan.workspace.numel() / 2**30:.1f} GiB")
    dev = "cuda:0"
    gen = torch.Generator(device=dev)
    gen.manual_seed(spec.seed)
    dI = torch.randn(3 * P, generator=gen, device=dev)
    dD = torch.randn(P, generator=gen, device=dev)
    dN = torch.randn(3 * P, generator=gen, device=dev)
    bufs = ss.StepBuffers(N, views.width, views.height, device=dev, with_sun=has_sun,
                          upstream=(dI, dD, dN))
    tune = None
    if not args.no_autotune:
        t0 = time.time()
        best, best_ms, table = ss.autotune(plan, surf, views, bufs, reps=2)
        tune = dict(tile=best.tile_size, batch_depth=best.batch_depth, ms=round(best_ms, 3),
                    table=[[int(a), int(b), round(c, 3)] for a, b, c in table])
        log(f"[bench] autotune in {time.time() - t0:.1f} s: tile {best.tile_size}, batch "
            f"{best.batch_depth}, {best_ms:.2f} ms/step")
        K, Ks = plan.ensure_capacity(surf, views)
    graph = None if args.no_graph else ss.Graph(plan, surf, views, bufs)

    def step():
        if graph is not None:
            graph.launch()
        else:
            ss.step(plan, surf, views, bufs)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    over, K_now, Ks_now = plan.check()
    if over:
        raise RuntimeError("pair capacity overflow during warmup")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    log(f"[bench] timed {args.steps} steps in {t_total:.3f} s")
    over, _, _ = plan.check()
    if over:
        raise RuntimeError("pair capacity overflow in the timed region")
    stats = plan.stats()
    # per-stage timing pass (HIP events recorded by the library on the same stream)
    plan.read_timing()
    plan.set_timing(True)
    for i in range(args.steps):
        ss.step(plan, surf, views, bufs)      # same kernels, eager so events can be recorded
    torch.cuda.synchronize()
    stages = plan.read_timing()
    plan.set_timing(False)
    ms_step = 1e3 * t_total / args.steps
    value = P * args.steps / t_total / 1e6
    kern = {}
    for name, (ms, n) in stages.items():
        if n:
            kern[name] = dict(avg_ms=ms / n, launches=n, share=ms / n / ms_step)
    log("[bench] stages (avg ms / launch): " + ", ".join(f"{k} {v['avg_ms']:.3f}" for k, v in kern.items()))
    C = stats["contrib"]
    Kp = stats["pairs"]
    cands = {k: kern[k]["avg_ms"] for k in ("raster_fwd", "raster_bwd")}
    dom = max(cands, key=cands.get)
    dom_ms = cands[dom]
    dom_bytes = raster_kernel_bytes(dom, P, Kp)
    dom_flops = (FLOPS_FWD_PAIR if dom == "raster_fwd" else FLOPS_BWD_PAIR) * C
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    copy_gbps = copy_bandwidth()
    traffic = measured_traffic(dom, spec.name, plan.settings.tile_size, plan.settings.batch_depth)
    tflops = dom_flops / (dom_ms * 1e-3) / 1e12
    roofline = dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBPS, 4), traffic=traffic,
                    avg_ms=round(dom_ms, 4),
                    work=f"{dom_bytes} algorithmic bytes per launch "
                         f"({'72 K + 52 P' if dom == 'raster_fwd' else '68 P + 136 K'}, "
                         f"P = {P} pixels, K = {Kp} tile-surfel pairs)",
                    copy=dict(GBps=round(copy_gbps, 1), frac=round(achieved / copy_gbps, 4)),
                    alu=dict(achieved=round(tflops, 3), peak=VALU_PEAK_TFLOPS, unit="TFLOP/s",
                             frac=round(tflops / VALU_PEAK_TFLOPS, 4),
                             nonpacked_issue_ceiling=round(VALU_NONPACKED_TFLOPS, 1),
                             work=f"{FLOPS_FWD_PAIR if dom == 'raster_fwd' else FLOPS_BWD_PAIR} "
                                  f"flop x {C} contributing pairs per launch"))
    step_bytes = algorithmic_step_bytes(N, V, P, stats["pairs"], stats["sun_pairs"] if has_sun else 0,
                                        S if has_sun else 0)
    result = {
        "metric": "fwd+bwd Mpix/s (2DGS affine raster); shadow ms/view plain vs MLP surrogate",
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "surfels": N, "views": V, "pixels": P,
                   "sun_map": S if has_sun else 0, "tile": plan.settings.tile_size,
                   "batch_depth": plan.settings.batch_depth,
                   "launch": "hipGraph" if graph is not None else "eager",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "step_hbm": dict(algorithmic_bytes=step_bytes,
                         achieved_GBps=round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
                         peak_GBps=HBM_PEAK_GBPS,
                         frac=round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)),
        "shadow_ms_per_view": round(sum(kern.get(k, {}).get("avg_ms", 0.0) for k in
                                        ("sun_camera", "sun_project", "sun_bin", "sun_raster",
                                         "shadow_query")) / V, 4) if has_sun else None,
        "work": dict(pairs=stats["pairs"], contributing=C, evaluated=stats["evaluated"],
                     sun_pairs=stats["sun_pairs"], sun_contributing=stats["sun_contrib"]),
        "kernels": {k: round(v["avg_ms"], 4) for k, v in kern.items()},
        "autotune": tune,
    }
    if not args.no_surrogate:
        log("[bench] learned shadow surrogate (train + held-out evaluation)")
        del bufs, graph
        plan = None
        torch.cuda.empty_cache()
        result["shadow_surrogate"] = surrogate_eval(ctx, args)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host")
        result["cpu_baseline"] = cpu_baseline(scene, args.cpu_pixels)
    if not args.no_camera and args.config == 3:
        log("[bench] camera-robustness experiment (c1 scene, 4 views of 256^2)")
        from paper_2606_28581_amd import experiments
        t0 = time.time()
        csc = synth.make_scene(synth.config(1, views=[(256, 256)] * 4))
        rows = experiments.camera_robustness(csc, steps=300, ctx=ctx, log=log)
        result["camera_robustness"] = dict(workload="c1_20k_4views_256", steps=300,
                                           seconds=round(time.time() - t0, 1),
                                           rows=[{k: (round(v, 6) if isinstance(v, float) else v)
                                                  for k, v in r.items()} for r in rows])
    if not args.no_c5 and args.config == 3:
        log("[bench] training-step scale: 5M surfels, 50 views of 2048^2")
        bufs = graph = plan = None
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        result["dsm_init"] = dsm_init_timing()
        torch.cuda.empty_cache()
        c5 = training_scale(args, tile=8, batch=64)
        result["training_step_c5"] = {k: c5[k] for k in ("value", "unit", "ms_per_step", "steps_per_s",
                                                         "steps", "peak_hbm_GB", "config", "pairs",
                                                         "surrogate", "kernels", "loss_l1_last")}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
