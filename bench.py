"""Benchmark: interlaced light-field frames/s on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--cluster-size 8]
                    [--no-cpu-baseline] [--no-plain] [--workload outdoor]

Workload (default ``outdoor``): 3,000,000 Gaussians (64-cluster mixture plus a
far shell, SH degree 3), 100 views over 50 degrees, 3840x2160 panel, slant
1/5, pitch 31/5; rendered with cross-view reuse (cluster size 8) and the
view-coherent remapped blend.  A step is one interlaced frame: projection,
key generation, sorting, ranges and blending, with the scene and cameras
already resident.  The plain baseline renders every view at full resolution
and interlaces.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "interlaced LF frames/s (4K, 100 views) reuse+remap vs plain; fwd+bwd ms"
PEAK_FP32_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12   # 78.6: 256 CUs x 64 lanes x FMA x 2.4 GHz
HBM_PEAK_GBS = 8000.0
FLOPS_PER_EVAL = 14      # alpha: dx,dy (2) + w fma (2) + A'w, G'dy, *dy (3) + fma (2) + exp2 (1)
                         #        + o*e (1) + min (1) + cutoff test (1)
FLOPS_PER_BLEND = 6      # 1-a, T*(1-a), stop test, c*a, fma (2)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="outdoor")
    ap.add_argument("--cluster-size", type=int, default=8)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--bwd-steps", type=int, default=10)
    ap.add_argument("--bwd-workload", default="display")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-shapes", action="store_true")
    ap.add_argument("--batch-poses", type=int, default=16)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=96)
    ap.add_argument("--tile", default=None, help="WxH tile shape; default: autotuned")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run three 256 MiB device copies (a known-size reference for HBM counters)")
    return ap.parse_args()


def kernel_source_hash():
    """Hash of the sources the blend kernel is built from; counter summaries
    in profiles/ apply only to the kernel they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("blend.hip", "lfr_internal.h"):
        with open(os.path.join(ROOT, "paper_2605_04509_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, tile):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if there is none for this workload, tile shape and kernel source."""
    path = os.path.join(ROOT, "profiles", "blend_remap_outdoor_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if (t.get("kernel") != kernel or t.get("workload_name") != workload or t.get("tile") != list(tile)
            or t.get("source_sha256") != kernel_source_hash()):
        return None
    return t["hbm_bytes_per_launch"]


def fwd_bwd(args, torch, lfr, sync):
    """Forward + backward at the differentiable configuration: the
    ``display`` workload (200k Gaussians, SH3, 45 views, 1920x1080) on the
    exact path (cluster size 1); loss = MSE against the same scene with the
    means perturbed by N(0, 0.01), rendered by the exact path.  A step is the
    forward (lists kept for the backward), the loss gradient and the
    backward into all 59 parameters of every Gaussian."""
    import numpy as np
    from workloads import get_workload
    from workloads.cameras import pack_cameras
    from workloads.scenes import perturb_means
    w = get_workload(args.bwd_workload)
    scene = w.make_scene()
    cams = lfr.cameras_array(pack_cameras(w.cameras()))
    ctx = lfr.Context(0)
    ds = lfr.DeviceScene.from_numpy(scene, device="cuda:0")
    tgt_scene = lfr.DeviceScene.from_numpy(perturb_means(scene, 5, 0.01), device="cuda:0")
    n_sub = 3 * w.display.width * w.display.height
    best = None
    for tile in ((16, 16), (32, 16), (32, 32), (64, 32)):
        d = lfr.Display(ctx, w.display.with_tile(*tile))
        target = lfr.render(ctx, d, tgt_scene, cams, cluster_size=1).clone()
        grads = {k: torch.empty_like(getattr(ds, k)) for k in lfr.GRAD_NAMES}

        def step(timing=False, d=d, target=target, grads=grads):
            img = lfr.render(ctx, d, ds, cams, cluster_size=1, save_for_backward=True, timing=timing)
            gout = (img - target).mul_(2.0 / n_sub)
            lfr.render_backward(ctx, d, ds, gout, grads)
            return img

        step()
        t = timed(step, 2, sync)
        log(f"fwd+bwd tile {tile}: {t * 1e3:.2f} ms")
        if best is None or t < best[1]:
            if best is not None:
                best[0][0].close()
            best = ((d, target, grads, step, tile), t)
        else:
            d.close()
    (d, target, grads, step, tile), _ = best
    for _ in range(2):
        step()
    sync()
    # per-stage split from the library's HIP events (separate, untimed run)
    img = step(timing=True)
    st = ctx.stats()
    t = timed(step, args.bwd_steps, sync)
    fwd = timed(lambda: lfr.render(ctx, d, ds, cams, cluster_size=1, out=img), args.bwd_steps, sync)
    loss = float(((img - target) ** 2).mean())
    d.close()
    ctx.close()
    return {"ms": t * 1e3, "forward_only_ms": fwd * 1e3, "tile": list(tile), "cluster_size": 1,
            "workload": (f"{w.name}: {scene.num_gaussians} Gaussians (SH{scene.sh_degree}), "
                         f"{w.display.num_views} views, {w.display.width}x{w.display.height}, exact path"),
            "ms_forward_saved": st["ms_total"], "ms_bwd_blend": st["ms_bwd_blend"],
            "ms_bwd_project": st["ms_bwd_project"], "ms_bwd_total": st["ms_bwd_total"],
            "pairs": st["pairs"], "loss": loss, "steps": args.bwd_steps}


def psnr_db(torch, img, ref):
    """PSNR (dB, peak 1) of an interlaced image against a reference image, both
    clamped to [0, 1] as a display shows them, over every subpixel."""
    mse = float(((img.clamp(0.0, 1.0) - ref.clamp(0.0, 1.0)).double() ** 2).mean())
    return float("inf") if mse == 0.0 else 10.0 * math.log10(1.0 / mse)


def paper_shapes(args, torch, lfr, sync):
    """The paper's two display shapes on the 3M-Gaussian scene: 71 views over
    53 degrees at 3840x2160 with reuse groups of 18, and 63 views over 53
    degrees at 1440x2560 with groups of 16.  For each: reuse + remap, the exact
    path (S = 1, remap), and the plain full-frame-then-interlace baseline over
    all views at its best view batch; tile shapes autotuned."""
    from workloads import get_workload
    from workloads.cameras import pack_cameras
    res = {}
    for name, S in (("landscape71", 18), ("portrait63", 16)):
        w = get_workload(name)
        ctx = lfr.Context(0)
        ds = lfr.DeviceScene.from_numpy(w.make_scene(), device="cuda:0")
        cams = lfr.cameras_array(pack_cameras(w.cameras()))
        imgs = {}
        r = {"display": [w.display.width, w.display.height, w.display.num_views], "span_deg": w.span_deg}
        for label, cs in (("reuse+remap", S), ("exact", 1)):
            out = torch.empty((w.display.height, w.display.width, 3), dtype=torch.float32, device="cuda:0")
            imgs[label] = out
            best, _ = lfr.autotune(ctx, w.display, ds, cams, cluster_sizes=(cs,), reps=1)
            d = lfr.Display(ctx, w.display.with_tile(best["tile_w"], best["tile_h"]))
            fn = lambda: lfr.render(ctx, d, ds, cams, cluster_size=cs, out=out)
            fn()
            t = timed(fn, 5, sync)
            r[label] = {"cluster_size": cs, "tile": [best["tile_w"], best["tile_h"]], "ms": t * 1e3,
                        "frames_per_s": 1.0 / t}
            if label == "exact":
                sync()
                r["reuse+remap"]["psnr_vs_exact_db"] = psnr_db(torch, imgs["reuse+remap"], imgs["exact"])
                plain = None
                for vb in (18, 36):
                    fp = lambda vb=vb: lfr.render_fullframe_interlace(ctx, d, ds, cams, view_batch=vb, out=out,
                                                                      tile=32)
                    try:
                        fp()
                    except lfr.LfrError as e:
                        log(f"{name} plain batch {vb}: {e}")
                        continue
                    tp = timed(fp, 1, sync)
                    if plain is None or tp < plain[1]:
                        plain = (vb, tp)
                if plain:
                    r["plain"] = {"view_batch": plain[0], "ms": plain[1] * 1e3, "frames_per_s": 1.0 / plain[1]}
            d.close()
        if "plain" in r:
            r["speedup_vs_plain"] = r["plain"]["ms"] / r["reuse+remap"]["ms"]
        log(name, r)
        res[name] = r
        ctx.close()
    return res


def batched(args, torch, lfr, sync):
    """The serving batch: three outdoor-style scenes (0.5M, 1M, 3M Gaussians)
    on 1920x1080/45-view, 2560x1440/64-view and 3840x2160/100-view panels,
    each seen from 16 head poses (rig offsets U[-0.05, 0.05]^3), cluster size
    8.  The tile shape of each display is autotuned on its first pose.  A
    step is one lfr_render_batch call over all 48 frames (planned frames,
    replayed from captured hipGraphs, one synchronization); the first calls,
    which plan the slots and capture the graphs, are warm-up."""
    from workloads.cameras import orbit_rig, pack_cameras
    from workloads.configs import batched_frames
    from workloads.scenes import mixture_scene
    S = 8
    ctx = lfr.Context(0)
    frames, tiles, keep = [], [], []
    for seed_i, m, disp, radius, span, offs in batched_frames(num_poses=args.batch_poses):
        ds = lfr.DeviceScene.from_numpy(mixture_scene(seed_i, m, 3), device="cuda:0")
        rig = lambda o: pack_cameras(orbit_rig(disp.num_views, disp.width, disp.height, radius, span, 60.0,
                                               centre=(0.0, 0.0, radius), rig_offset=tuple(o)))
        best, _ = lfr.autotune(ctx, disp, ds, rig(offs[0]), cluster_sizes=(S,), reps=1)
        d = lfr.Display(ctx, disp.with_tile(best["tile_w"], best["tile_h"]))
        tiles.append([disp.width, disp.height, disp.num_views, best["tile_w"], best["tile_h"], m])
        keep.append((d, ds))
        for o in offs:
            out = torch.empty((disp.height, disp.width, 3), dtype=torch.float32, device="cuda:0")
            frames.append(lfr.Frame(d, ds, rig(o), out, cluster_size=S))
    n = len(frames)
    res = {"frames": n, "cluster_size": S, "displays": tiles}
    for label, graph in (("graph", True), ("planned", False)):
        bctx = lfr.Context(0)
        for _ in range(3):
            st = lfr.render_batch(bctx, frames, graph=graph)
        t = timed(lambda: lfr.render_batch(bctx, frames, graph=graph), args.batch_steps, sync)
        st = lfr.render_batch(bctx, frames, graph=graph)
        res[label] = {"ms_per_batch": t * 1e3, "frames_per_s": n / t, "last_batch": st}
        log(f"batch {label}: {t * 1e3:.1f} ms per {n} frames ({n / t:.1f} frames/s) {st}")
        bctx.close()
    # the same frames one lfr_render call at a time (one host readback per chunk)
    def unbatched():
        for f in frames:
            lfr.render(ctx, f.display, f.scene, f.cams, cluster_size=S, out=f.out)
    unbatched()
    t = timed(unbatched, max(1, args.batch_steps - 1), sync)
    res["unbatched"] = {"ms_per_batch": t * 1e3, "frames_per_s": n / t}
    log(f"unbatched: {t * 1e3:.1f} ms per {n} frames ({n / t:.1f} frames/s)")
    res["frames_per_s"] = res["graph"]["frames_per_s"]
    for d, ds in keep:
        d.close()
    ctx.close()
    return res


def timed(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def cpu_baseline(w, scene, cams, n_samples):
    """The oracle, single-threaded, on a bounded sample of the same frame:
    one projection of all Gaussians (timed alone) plus a blend of n_samples
    subpixels of one view inside one cluster; extrapolated to a full frame as
    (clusters + views) projections + 3WH subpixel blends."""
    import numpy as np
    import oracle
    V = oracle.view_map(w.display)
    S = 8
    _, rep = oracle.cluster_table(w.display.num_views, S)
    ref_views = np.unique(V)
    j = int(ref_views[len(ref_views) // 2])
    r = int(rep[j // S])
    if j == r:
        j = int(ref_views[len(ref_views) // 2 + 1])
    t0 = time.perf_counter()
    oracle.project(scene, cams[r], w.display.width, w.display.height)
    t_proj = time.perf_counter() - t0
    flat = V.reshape(-1)
    idx = np.flatnonzero(flat == j)
    samples = np.sort(np.random.default_rng(0).choice(idx, n_samples, replace=False))
    t0 = time.perf_counter()
    oracle.render_subpixels(scene, cams, w.display, V, S, samples)
    t_call = time.perf_counter() - t0
    t_sub = max(t_call - 2 * t_proj, 1e-9) / n_samples
    n_proj = len(ref_views) + len({int(rep[v // S]) for v in ref_views})
    frame_s = n_proj * t_proj + flat.size * t_sub
    return {
        "value": 1.0 / frame_s, "unit": "frames/s", "cores": 1, "kind": "oracle",
        "sample": (f"1 projection of all {scene.num_gaussians} Gaussians ({t_proj:.2f} s) + {n_samples} subpixels of "
                   f"view {j} at cluster size {S} ({t_call:.2f} s incl. 2 projections); extrapolated to "
                   f"{n_proj} projections + {flat.size} subpixels per frame"),
        "host": platform.processor() or platform.machine(),
        "host_cores_available": os.cpu_count(),
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_04509_amd import lfr
    from workloads import get_workload
    from workloads.cameras import pack_cameras

    if args.copy_probe:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    w = get_workload(args.workload)
    log("generating", w.name)
    scene = w.make_scene()
    cams_np = pack_cameras(w.cameras())
    cams = lfr.cameras_array(cams_np)
    ctx = lfr.Context(0)
    ds = lfr.DeviceScene.from_numpy(scene, device="cuda:0")
    out = torch.empty((w.display.height, w.display.width, 3), dtype=torch.float32, device="cuda:0")
    sync = torch.cuda.synchronize
    S = args.cluster_size
    # tile shape: the image does not depend on it, so pick the fastest (untimed)
    if args.tile:
        tw, th = (int(v) for v in args.tile.lower().split("x"))
        tune = None
    else:
        best, tune = lfr.autotune(ctx, w.display, ds, cams, cluster_sizes=(S,), reps=2)
        log("autotune", best)
        tw, th = best["tile_w"], best["tile_h"]
    params = w.display.with_tile(tw, th)
    disp = lfr.Display(ctx, params)

    def frame(cs=S, remap=True, timing=False):
        lfr.render(ctx, disp, ds, cams, cluster_size=cs, remap=remap, timing=timing, out=out)

    # work counts of the blend (separate counting launch, outside any timed region)
    frame()
    lfr.render(ctx, disp, ds, cams, cluster_size=S, remap=True, out=out, count_work=True)
    work = ctx.stats()
    log("work", work)

    for _ in range(args.warmup):
        frame(timing=True)
    sync()
    # timed region: K frames; per-stage HIP events on the library's stream
    stages = {k: 0.0 for k in ("ms_project", "ms_depth_sort", "ms_keygen", "ms_sort", "ms_ranges", "ms_blend",
                               "ms_sort_scatter")}
    scatter_launches = 0
    blend_launches = 0
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        frame(timing=True)
        st = ctx.stats()
        for k in stages:
            stages[k] += st[k]
        scatter_launches += st["sort_scatter_launches"]
        blend_launches += st["blend_launches"]
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    stages = {k: v / args.steps for k, v in stages.items()}
    fps = 1.0 / sec
    log(f"reuse+remap S={S}: {sec * 1e3:.3f} ms/frame, {fps:.1f} frames/s, stages {stages}")

    # the dominant kernel: the blend (one launch per frame) or the scatter of
    # the tile sort (one launch per radix pass)
    # blend: one launch per blended depth chunk; flops per launch = the
    # frame's algorithmic flops over its launches
    flops = FLOPS_PER_EVAL * work["evals"] + FLOPS_PER_BLEND * work["blended"]
    bl = max(blend_launches / args.steps, 1.0)
    blend_ms = stages["ms_blend"] / bl
    blend_alu = {"bound": "alu", "kernel": "blend_remap_kernel<false>", "launch_ms": blend_ms,
                 "launches_per_frame": bl, "flops_per_launch": flops / bl,
                 "achieved": flops / bl / (blend_ms * 1e-3) / 1e12, "peak": PEAK_FP32_NONPACKED_TFLOPS,
                 "unit": "TFLOP/s", "evals": work["evals"], "blended": work["blended"],
                 "wave_steps": work["wave_steps"], "wave_steps_live": work["wave_steps_live"],
                 # lane slots the kernel walks (staged Gaussians x 64) per alpha the
                 # method evaluates: below 1 where the per-batch culling drops entries
                 "lane_slots_per_eval": 64 * work["wave_steps"] / max(1, work["evals"]),
                 "traffic": measured_traffic("blend_remap_kernel<false>", w.name,
                                               (params.tile_w, params.tile_h))}
    blend_alu["frac"] = blend_alu["achieved"] / blend_alu["peak"]
    # tile sort: every chunk's pairs pass through ceil(tile_bits / 8) scatter
    # launches, each reading and writing (key, value) = 16 B per pair
    d = params
    n_tiles = -(-d.width // d.tile_w) * -(-d.height // d.tile_h)
    passes = -(-max(1, (n_tiles - 1).bit_length()) // 8)
    launches = max(scatter_launches / args.steps, 1.0)
    per_launch = stages["ms_sort_scatter"] / launches
    bytes_per_launch = 16.0 * work["pairs"] * passes / launches
    scatter = {"bound": "hbm", "kernel": "sort_scatter_kernel<uint32_t> (tile sort)", "launch_ms": per_launch,
               "launches_per_frame": launches, "achieved": bytes_per_launch / (per_launch * 1e-3) / 1e9,
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "bytes_per_launch": bytes_per_launch, "traffic": None}
    scatter["frac"] = scatter["achieved"] / scatter["peak"]
    dominant_is_sort = stages["ms_sort_scatter"] > stages["ms_blend"]
    roofline = scatter if dominant_is_sort else blend_alu
    other = blend_alu if dominant_is_sort else scatter

    result = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{w.name}: {scene.num_gaussians} Gaussians (SH{scene.sh_degree}), "
                                f"{w.display.num_views} views over {w.span_deg:g} deg, "
                                f"{w.display.width}x{w.display.height}, slant {w.display.tan_slant.num}/"
                                f"{w.display.tan_slant.den}, pitch {w.display.pitch.num}/{w.display.pitch.den}"),
                   "cluster_size": S, "remap": True, "tile": [params.tile_w, params.tile_h],
                   "parallelism": "single GPU"},
        "autotune": tune, "kernel_source_sha256": kernel_source_hash(),
        "stages_ms": stages, "pairs": work["pairs"], "chunks": work["chunks"], "clusters": work["clusters"],
        "views": work["views"],
        "roofline": roofline, "roofline_other": other, "fwd_bwd_ms": None,
    }

    # image quality of the reuse path: PSNR of the cluster-size-S image (and of
    # the paper's other group sizes) against the exact path (S = 1)
    exact = torch.empty_like(out)
    lfr.render(ctx, disp, ds, cams, cluster_size=1, out=exact)
    psnr = {}
    for cs in sorted({2, 4, 8, S}):
        img = torch.empty_like(out)
        lfr.render(ctx, disp, ds, cams, cluster_size=cs, out=img)
        sync()
        psnr[str(cs)] = psnr_db(torch, img, exact)
        del img
    result["psnr_vs_exact_db"] = psnr
    log("PSNR vs exact (dB) by cluster size", psnr)

    if not args.no_ablation:
        # the paper's ablation modes, each on its own fastest tile shape
        modes = {}
        for name, cs, rm in (("reuse_only", S, False), ("remap_only", 1, True), ("neither", 1, False)):
            b, _ = lfr.autotune(ctx, w.display, ds, cams, cluster_sizes=(cs,), reps=1, remap=rm,
                                tiles=((16, 16), (32, 16), (32, 32), (32, 64)))
            dm = lfr.Display(ctx, w.display.with_tile(b["tile_w"], b["tile_h"]))
            run = lambda: lfr.render(ctx, dm, ds, cams, cluster_size=cs, remap=rm, out=out)
            run()
            t = timed(run, 3, sync)
            modes[name] = {"cluster_size": cs, "remap": rm, "tile": [b["tile_w"], b["tile_h"]],
                           "frames_per_s": 1.0 / t, "ms": t * 1e3}
            dm.close()
            log(name, modes[name])
        modes["reuse+remap"] = {"cluster_size": S, "remap": True, "tile": [params.tile_w, params.tile_h],
                                "frames_per_s": fps, "ms": sec * 1e3}
        result["modes"] = modes

    if not args.no_plain:
        plain = {}
        for label, cull in (("all_views", False), ("referenced_views", True)):
            best_p = None
            for tile in (16, 32):
                for vb in (10, 20):
                    def pf(vb=vb, cull=cull, tile=tile):
                        lfr.render_fullframe_interlace(ctx, disp, ds, cams, view_batch=vb, cull=cull, out=out,
                                                       tile=tile)
                    try:
                        pf()
                    except lfr.LfrError as e:         # e.g. more pairs than 32-bit offsets hold
                        log(f"plain {label} tile {tile} batch {vb}: {e}")
                        continue
                    t = timed(pf, 1, sync)
                    log(f"plain {label} tile {tile} batch {vb}: {t * 1e3:.1f} ms")
                    if best_p is None or t < best_p[2]:
                        best_p = (vb, tile, t)
            vb, tile = best_p[0], best_p[1]
            t = timed(lambda: lfr.render_fullframe_interlace(ctx, disp, ds, cams, view_batch=vb, cull=cull, out=out,
                                                             tile=tile), args.plain_steps, sync)
            plain[label] = {"view_batch": vb, "tile": tile, "frames_per_s": 1.0 / t, "ms": t * 1e3}
        result["plain"] = plain
        result["speedup_vs_plain"] = fps / plain["all_views"]["frames_per_s"]
        result["speedup_vs_plain_referenced"] = fps / plain["referenced_views"]["frames_per_s"]

    if not args.no_shapes:
        result["paper_shapes"] = paper_shapes(args, torch, lfr, sync)

    if not args.no_batch:
        result["batched"] = batched(args, torch, lfr, sync)
        result["batched_frames_per_s"] = result["batched"]["frames_per_s"]

    if not args.no_backward:
        fb = fwd_bwd(args, torch, lfr, sync)
        log("fwd+bwd", fb)
        result["fwd_bwd_ms"] = fb["ms"]
        result["fwd_bwd"] = fb

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, scene, cams_np, args.cpu_samples)

    disp.close()
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
