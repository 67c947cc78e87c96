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
# VALU issue roof: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-operations/s
# (one vector instruction slot per lane per clock, FMA counted once; packed
# FP32 is not used by the library (it is compiled with packed FP32 off), so
# this is the roof of its plain ALU path)
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
OPS_PER_EVAL = 14        # alpha per (subpixel, Gaussian): dx, dy (2) + w = dx + beta dy (1) + w^2, dy^2 (2)
                         # + E = A'w^2 + G'dy^2 (2) + exp2 (quarter rate: 4) + o 2^-E (1) + clamp (1)
                         # + cutoff test (1)
OPS_PER_PROJ = 250       # per (Gaussian, cluster): covariance, EWA, inverse, SH3 colour
OPS_PER_MEAN = 20        # per (Gaussian, view): transform + pinhole


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


def stage_roofline(work, stages, M, deg, n_tiles, n_sub, frame_s):
    """Roofline time of each stage of the frame and of the whole frame.

    Algorithmic bytes B and VALU lane-operations O of each stage are counted
    from this frame's sizes: M Gaussians with (d+1)^2 SH coefficients, K'
    clusters and N' views in use, P Gaussian-(tile, cluster) pairs over all
    depth chunks, n_eval alphas the method evaluates, T tiles.
      project    B = M 4 (11 + 3 (d+1)^2) + 28 M K' + 8 M N'   O = 250 M K' + 20 M N'
      keygen     B = M (28 K' + 8 N') + 12 P
      sort       B = 24 P ceil((32 + bits(K') + bits(T)) / 8)   (one stable sort of the
                 (tile, cluster, depth) keys with 8-bit digits; the design's own passes
                 are three passes over the M K' depth keys that split off the near set, a
                 4-pass sort of the near set (at most R items per cluster, R the start rank
                 of the last chunk), 2 tile-bit passes per ranked chunk and one 64-bit sort
                 of the last chunk's pairs)
      ranges     B = 8 P + 8 T K'
      blend      B = P (36 + 8 N'/K') + 10 n_sub              O = 14 n_eval
    roofline time = max(B / 8 TB/s, O / 39.3 T lane-ops/s); fraction = roofline
    time / measured time.  The frame fraction is the sum of the stage roofline
    times over the measured frame time."""
    P, K, N, ne = work["pairs"], work["clusters"], work["views"], work["evals"]
    bits = lambda n: max(1, (int(n) - 1).bit_length())
    model = {
        "project": (M * 4 * (11 + 3 * (deg + 1) ** 2) + 28 * M * K + 8 * M * N, OPS_PER_PROJ * M * K + OPS_PER_MEAN * M * N,
                    stages["ms_project"]),
        "keygen": (M * (28 * K + 8 * N) + 12 * P, 0, stages["ms_keygen"]),
        "sort": (24 * P * -(-(32 + bits(K) + bits(n_tiles)) // 8), 0, stages["ms_depth_sort"] + stages["ms_sort"]),
        "ranges": (8 * P + 8 * n_tiles * K, 0, stages["ms_ranges"]),
        "blend": (P * (36 + 8 * N / max(K, 1)) + 10 * n_sub, OPS_PER_EVAL * ne, stages["ms_blend"]),
    }
    out, total = {}, 0.0
    for name, (B, O, ms) in model.items():
        t_hbm = B / (HBM_PEAK_GBS * 1e9) * 1e3
        t_alu = O / (PEAK_VALU_TOPS * 1e12) * 1e3
        roof = max(t_hbm, t_alu)
        total += roof
        out[name] = {"bytes": B, "ops": O, "bound": "hbm" if t_hbm >= t_alu else "alu", "roofline_ms": roof,
                     "ms": ms, "frac": roof / ms if ms > 0 else None}
    return {"stages": out, "frame_roofline_ms": total, "frame_frac": total / (frame_s * 1e3)}


def display_bytes(p, clusters):
    """Device memory the display holds for one cluster size: the view map
    (2 B per subpixel), the remap LUT (4 B per subpixel), the blend work
    items (32 B per at most 64 subpixels) and the per-(tile, cluster)
    subpixel counts."""
    n_sub = 3 * p.width * p.height
    n_tiles = -(-p.width // p.tile_w) * -(-p.height // p.tile_h)
    cb = max(1, (int(clusters) - 1).bit_length())
    return 2 * n_sub + 4 * n_sub + 32 * -(-n_sub // 64) + 4 * (n_tiles << cb)


def finite_json(v):
    """v with every non-finite float replaced by None (strict JSON has no inf or nan)."""
    if isinstance(v, dict):
        return {k: finite_json(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [finite_json(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def psnr_per_view(torch, img, ref, V, n_views):
    """PSNR (dB, peak 1, images clamped to [0, 1]) of the subpixels of each
    view of the display (V == j), like a per-view image metric: mean, min and
    max over the views the display uses, and every view's value."""
    err = (img.clamp(0.0, 1.0) - ref.clamp(0.0, 1.0)).double().square().reshape(-1)
    v = V.reshape(-1)
    sse = torch.bincount(v, weights=err, minlength=n_views)
    cnt = torch.bincount(v, minlength=n_views).double()
    used = cnt > 0
    mse = (sse[used] / cnt[used]).cpu().numpy()
    views = torch.nonzero(used).reshape(-1).cpu().numpy()
    db = [None if m == 0.0 else 10.0 * math.log10(1.0 / m) for m in mse]
    finite = [x for x in db if x is not None]
    # (a view equal to the exact path, e.g. a cluster's representative, has no
    # finite PSNR: reported as null and counted in `identical`)
    return {"mean": sum(finite) / len(finite) if finite else None, "min": min(finite) if finite else None,
            "max": max(finite) if finite else None, "identical": len(db) - len(finite),
            "views": {int(j): x for j, x in zip(views, db)}}


def psnr_db(torch, img, ref):
    """PSNR (dB, peak 1) of an interlaced image against a reference image, both
    clamped to [0, 1] as a display shows them, over every subpixel."""
    mse = float(((img.clamp(0.0, 1.0) - ref.clamp(0.0, 1.0)).double() ** 2).mean())
    return None if mse == 0.0 else 10.0 * math.log10(1.0 / mse)


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
                        "frames_per_s": 1.0 / t, "pairs": ctx.stats()["pairs"]}
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


BATCH_PSNR_FLOOR_DB = 35.0
BATCH_CLUSTER_SIZES = (4, 8, 12, 16)


def batched(args, torch, lfr, sync):
    """The serving batch: three outdoor-style scenes (0.5M, 1M, 3M Gaussians)
    on 1920x1080/45-view, 2560x1440/64-view and 3840x2160/100-view panels,
    each seen from 16 head poses (rig offsets U[-0.05, 0.05]^3).  Per panel,
    on its first pose, the autotuner times every (tile shape, cluster size)
    candidate; the cluster size is the fastest one whose image keeps a PSNR
    of at least 35 dB against the exact path (cluster size 1), with its
    fastest tile.  A step is one lfr_render_batch call over all 48 frames:
    the 16 poses of a panel merge into groups rendered as one render each,
    planned and replayed from captured hipGraphs, one synchronization.  The
    first calls, which plan the slots and capture the graphs, are warm-up.
    Also timed: the same batch with every frame rendered on its own (graphs,
    no merging) and frame by frame with lfr_render."""
    from workloads.cameras import orbit_rig, pack_cameras
    from workloads.configs import batched_frames
    from workloads.scenes import mixture_scene
    ctx = lfr.Context(0)
    frames, panels, keep = [], [], []
    for seed_i, m, disp, radius, span, offs in batched_frames(num_poses=args.batch_poses):
        ds = lfr.DeviceScene.from_numpy(mixture_scene(seed_i, m, 3), device="cuda:0")
        rig = lambda o: pack_cameras(orbit_rig(disp.num_views, disp.width, disp.height, radius, span, 60.0,
                                               centre=(0.0, 0.0, radius), rig_offset=tuple(o)))
        cams0 = rig(offs[0])
        _, res = lfr.autotune(ctx, disp, ds, cams0, cluster_sizes=BATCH_CLUSTER_SIZES, reps=1)
        # PSNR of each cluster size against the exact path, at its fastest tile
        d1 = lfr.Display(ctx, disp.with_tile(32, 32))
        exact = lfr.render(ctx, d1, ds, cams0, cluster_size=1).clone()
        choice, tried = None, {}
        for S in BATCH_CLUSTER_SIZES:
            best_s = min((r for r in res if r["cluster_size"] == S), key=lambda r: r["ms"])
            img = lfr.render(ctx, d1, ds, cams0, cluster_size=S)
            sync()
            tried[str(S)] = {"ms": best_s["ms"], "tile": [best_s["tile_w"], best_s["tile_h"]],
                             "psnr_vs_exact_db": psnr_db(torch, img, exact)}
            del img
            q = tried[str(S)]["psnr_vs_exact_db"]   # None: identical to the exact path
            if (q is None or q >= BATCH_PSNR_FLOOR_DB) and (choice is None or best_s["ms"] < choice["ms"]):
                choice = best_s
        if choice is None:                  # no size keeps the floor: the smallest
            choice = min((r for r in res if r["cluster_size"] == BATCH_CLUSTER_SIZES[0]), key=lambda r: r["ms"])
        d1.close()
        del exact
        S = choice["cluster_size"]
        d = lfr.Display(ctx, disp.with_tile(choice["tile_w"], choice["tile_h"]))
        panels.append({"panel": [disp.width, disp.height, disp.num_views], "gaussians": m, "cluster_size": S,
                       "tile": [choice["tile_w"], choice["tile_h"]], "candidates": tried})
        log("batch panel", panels[-1])
        keep.append((d, ds))
        for o in offs:
            out = torch.empty((disp.height, disp.width, 3), dtype=torch.float32, device="cuda:0")
            frames.append(lfr.Frame(d, ds, rig(o), out, cluster_size=S))
    n = len(frames)
    res = {"frames": n, "psnr_floor_db": BATCH_PSNR_FLOOR_DB, "panels": panels}
    for label, graph, merge in (("merged", True, True), ("per_frame_graphs", True, False)):
        bctx = lfr.Context(0)
        for _ in range(3):
            st = lfr.render_batch(bctx, frames, graph=graph, merge=merge)
        t = timed(lambda: lfr.render_batch(bctx, frames, graph=graph, merge=merge), args.batch_steps, sync)
        st = lfr.render_batch(bctx, frames, graph=graph, merge=merge)
        res[label] = {"ms_per_batch": t * 1e3, "frames_per_s": n / t, "last_batch": st,
                      "workspace_bytes": bctx.stats()["workspace_bytes"]}
        log(f"batch {label}: {t * 1e3:.1f} ms per {n} frames ({n / t:.1f} frames/s) {st}")
        bctx.close()

    # the same frames one lfr_render call at a time (one host readback per chunk)
    def unbatched():
        for f in frames:
            lfr.render(ctx, f.display, f.scene, f.cams, cluster_size=f.opts.cluster_size, out=f.out)
    unbatched()
    t = timed(unbatched, max(1, args.batch_steps - 1), sync)
    res["unbatched"] = {"ms_per_batch": t * 1e3, "frames_per_s": n / t}
    log(f"unbatched: {t * 1e3:.1f} ms per {n} frames ({n / t:.1f} frames/s)")
    res["frames_per_s"] = res["merged"]["frames_per_s"]
    res["gain_vs_unbatched"] = res["merged"]["frames_per_s"] / res["unbatched"]["frames_per_s"]
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _tile_samples(V, tw, th, n_tiles, per_tile, seed):
    """per_tile random subpixels in each of n_tiles random tw x th tiles."""
    import numpy as np
    H, W, _ = V.shape
    rng = np.random.default_rng(seed)
    TX, TY = -(-W // tw), -(-H // th)
    tiles = rng.choice(TX * TY, n_tiles, replace=False)
    out = []
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        ys = rng.integers(ty * th, min(H, (ty + 1) * th), per_tile)
        xs = rng.integers(tx * tw, min(W, (tx + 1) * tw), per_tile)
        us = rng.integers(0, 3, per_tile)
        out.append((ys * W + xs) * 3 + us)
    return np.unique(np.concatenate(out))


def _timed_call(fn):
    t0 = time.perf_counter()
    r = fn()
    return time.perf_counter() - t0, r


def cpu_baseline(w, scene, cams, S):
    """The oracle (test infrastructure: a plain CPU renderer, never tuned) on
    the host cores, on bounded samples of the same frame, extrapolated:

    threaded (the baseline value): every host thread the run may use, on
    subpixels in 256 random 16x16 tiles of the frame (4 each).  A first call
    with one subpixel of every view the panel uses costs what any frame costs
    once (every cluster's projection and depth sort, every view's means);
    the sample call adds the blends, so per frame = fixed + 3WH x (blend per
    subpixel).  Bit-identity with one thread is checked on a small sample.

    single-threaded (the oracle's correctness form): the tiny frame in full,
    and the display and outdoor frames extrapolated from one projection and
    a few dozen subpixels of one view."""
    import numpy as np
    import oracle
    from workloads import get_workload
    from workloads.cameras import pack_cameras
    res = {"kind": "oracle", "unit": "frames/s", "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    V = oracle.view_map(w.display)
    n_sub = V.size
    flat = V.reshape(-1)
    views = np.unique(flat)
    rng = np.random.default_rng(1)
    one_per_view = np.sort(np.array([rng.choice(np.flatnonzero(flat == j)) for j in views]))
    samples = _tile_samples(V, 16, 16, 256, 4, 2)
    nt = oracle.host_threads()
    with oracle.threads(nt):
        t_fixed, _ = _timed_call(lambda: oracle.render_subpixels(scene, cams, w.display, V, S, one_per_view))
        t_samp, _ = _timed_call(lambda: oracle.render_subpixels(scene, cams, w.display, V, S, samples))
    per_sub = max(t_samp - t_fixed, 1e-9) / max(1, samples.size - one_per_view.size)
    frame_s = t_fixed + n_sub * per_sub
    res.update({"value": 1.0 / frame_s, "cores": nt, "threads": nt, "frame_s_extrapolated": frame_s,
                "sample": (f"{w.name} frame at cluster size {S}: {samples.size} subpixels in 256 random 16x16 "
                           f"tiles ({t_samp:.1f} s) and one subpixel of each of the {views.size} views "
                           f"({t_fixed:.1f} s: every projection and depth sort a frame needs) on {nt} threads; "
                           f"extrapolated to {n_sub} subpixels")})
    # single thread (the correctness form); bit-identical to the threaded run
    j = int(views[len(views) // 2])
    idx = np.flatnonzero(flat == j)
    small = np.sort(rng.choice(idx, 48, replace=False))
    t_one, single = _timed_call(lambda: oracle.render_subpixels(scene, cams, w.display, V, S, small))
    with oracle.threads(nt):
        threaded = oracle.render_subpixels(scene, cams, w.display, V, S, small)
    res["bit_identical_to_single_thread"] = all(np.array_equal(a, b) for a, b in zip(single, threaded))
    t_proj, _ = _timed_call(lambda: oracle.project(scene, cams[j], w.display.width, w.display.height))
    _, rep = oracle.cluster_table(w.display.num_views, S)
    n_proj = views.size + len({int(rep[v // S]) for v in views})
    # the 48-subpixel call projects the cluster's representative and view j and sorts once
    per_sub1 = max(t_one - 2 * t_proj, 1e-9) / small.size
    single_frame = n_proj * t_proj + n_sub * per_sub1
    st = {"outdoor_frame_s_extrapolated": single_frame,
          "outdoor_sample": (f"1 projection of {scene.num_gaussians} Gaussians ({t_proj:.2f} s) + 48 subpixels "
                             f"of view {j} ({t_one:.1f} s incl. 2 projections and a sort); {n_proj} projections "
                             f"+ {n_sub} subpixels per frame")}
    tiny = get_workload("tiny")
    tsc, tcams = tiny.make_scene(), pack_cameras(tiny.cameras())
    tV = oracle.view_map(tiny.display)
    st["tiny_full_frame_s"], _ = _timed_call(lambda: oracle.render_frame(tsc, tcams, tiny.display, tV, 1))
    disp = get_workload("display")
    dsc, dcams = disp.make_scene(), pack_cameras(disp.cameras())
    dV = oracle.view_map(disp.display)
    dflat = dV.reshape(-1)
    dviews = np.unique(dflat)
    dj = int(dviews[len(dviews) // 2])
    ds = np.sort(rng.choice(np.flatnonzero(dflat == dj), 64, replace=False))
    t_d, _ = _timed_call(lambda: oracle.render_subpixels(dsc, dcams, disp.display, dV, 1, ds))
    t_dp, _ = _timed_call(lambda: oracle.project(dsc, dcams[dj], disp.display.width, disp.display.height))
    st["display_frame_s_extrapolated"] = dviews.size * t_dp + dflat.size * max(t_d - t_dp, 1e-9) / ds.size
    st["display_sample"] = (f"exact path: 1 projection of {dsc.num_gaussians} Gaussians ({t_dp:.3f} s) + 64 "
                            f"subpixels of view {dj} ({t_d:.2f} s); {dviews.size} projections + {dflat.size} "
                            "subpixels per frame")
    res["single_thread"] = st
    return res


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
        frame()
    sync()
    # timed region: K frames as a caller renders them (no per-stage events, no
    # host synchronization between frames)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        frame()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    # the per-stage breakdown: K more frames of the same work with the
    # library's HIP events between its stages, read back after each frame
    stages = {k: 0.0 for k in ("ms_project", "ms_depth_sort", "ms_keygen", "ms_sort", "ms_ranges", "ms_blend",
                               "ms_sort_scatter")}
    scatter_launches = 0
    blend_launches = 0
    frame_ms = []
    for _ in range(args.steps):
        frame(timing=True)
        st = ctx.stats()
        frame_ms.append(st["ms_total"])
        for k in stages:
            stages[k] += st[k]
        scatter_launches += st["sort_scatter_launches"]
        blend_launches += st["blend_launches"]
    sync()
    stages = {k: v / args.steps for k, v in stages.items()}
    fps = 1.0 / sec
    log(f"reuse+remap S={S}: {sec * 1e3:.3f} ms/frame, {fps:.1f} frames/s, stages {stages}")

    # per-stage roofline of the frame (algorithmic bytes / operations of each
    # stage, counted from this frame's sizes) and the dominant kernel
    d = params
    n_tiles = -(-d.width // d.tile_w) * -(-d.height // d.tile_h)
    rl = stage_roofline(work, stages, scene.num_gaussians, scene.sh_degree, n_tiles, d.width * d.height * 3, sec)
    bl = max(blend_launches / args.steps, 1.0)
    blend_ms = stages["ms_blend"] / bl
    ops_per_launch = OPS_PER_EVAL * work["evals"] / bl
    roofline = {"bound": "alu", "kernel": "blend_remap_kernel<false, false>",
                "achieved": ops_per_launch / (blend_ms * 1e-3) / 1e12, "peak": PEAK_VALU_TOPS, "unit": "T lane-ops/s",
                "traffic": measured_traffic("blend_remap_kernel<false, false>", w.name,
                                            (params.tile_w, params.tile_h)),
                "launch_ms": blend_ms, "launches_per_frame": bl, "ops_per_launch": ops_per_launch,
                "ops_per_eval": OPS_PER_EVAL, "evals": work["evals"], "blended": work["blended"],
                "wave_steps": work["wave_steps"], "wave_steps_live": work["wave_steps_live"],
                # lane slots the kernel walks (staged Gaussians x 64) per alpha the
                # method evaluates: below 1 where the per-batch culling drops entries
                "lane_slots_per_eval": 64 * work["wave_steps"] / max(1, work["evals"])}
    roofline["frac"] = roofline["achieved"] / roofline["peak"]
    roofline["stages"] = rl["stages"]
    roofline["frame_roofline_ms"] = rl["frame_roofline_ms"]
    roofline["frame_frac"] = rl["frame_frac"]
    # the tile sort's scatter: every chunk's pairs pass through ceil(tile_bits / 8)
    # scatter launches, each reading and writing (key, value) = 16 B per pair
    passes = -(-max(1, (n_tiles - 1).bit_length()) // 8)
    launches = max(scatter_launches / args.steps, 1.0)
    per_launch = stages["ms_sort_scatter"] / launches
    bytes_per_launch = 16.0 * work["pairs"] * passes / launches
    scatter = {"bound": "hbm", "kernel": "sort_scatter_kernel<uint32_t> (tile sort)", "launch_ms": per_launch,
               "launches_per_frame": launches, "achieved": bytes_per_launch / (per_launch * 1e-3) / 1e9,
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "bytes_per_launch": bytes_per_launch, "traffic": None}
    scatter["frac"] = scatter["achieved"] / scatter["peak"]
    frame_ms = sorted(frame_ms)
    pct = lambda q: frame_ms[min(len(frame_ms) - 1, int(round(q * (len(frame_ms) - 1))))]

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
        "frame_ms": {"median": pct(0.5), "p10": pct(0.1), "p90": pct(0.9), "n": len(frame_ms),
                     "clock": "HIP events on the library stream, projection to blend, in the instrumented frames"},
        "stages_ms": stages, "pairs": work["pairs"], "chunks": work["chunks"], "clusters": work["clusters"],
        "views": work["views"],
        "roofline": roofline, "roofline_sort_scatter": scatter, "fwd_bwd_ms": None,
        "device_memory": {"lfr_workspace_bytes": ctx.stats()["workspace_bytes"],
                          "display_bytes": display_bytes(params, work["clusters"]),
                          "torch_peak_allocated_bytes": int(torch.cuda.max_memory_allocated())},
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
    lfr.render(ctx, disp, ds, cams, cluster_size=S, out=out)
    Vd = torch.from_numpy(disp.view_map().astype(np.int64)).to("cuda:0")
    pv = psnr_per_view(torch, out, exact, Vd, w.display.num_views)
    result["psnr_per_view_db"] = pv
    log("per-view PSNR", {k: v for k, v in pv.items() if k != "views"})
    del Vd

    if not args.no_ablation:
        # the paper's ablation modes, each on its own fastest tile shape
        modes = {}
        for name, cs, rm in (("reuse_only", S, False), ("remap_only", 1, True), ("neither", 1, False)):
            b, _ = lfr.autotune(ctx, w.display, ds, cams, cluster_sizes=(cs,), reps=1, remap=rm,
                                tiles=((16, 16), (32, 16), (32, 32), (32, 64), (64, 64), (64, 128)))
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
        result["cpu_baseline"] = cpu_baseline(w, scene, cams_np, S)

    disp.close()
    ctx.close()
    print(json.dumps(finite_json(result)), flush=True)


if __name__ == "__main__":
    main()
