"""Batched frames (lfr_render_batch): every path a frame can take -- first use
(synchronizing, builds the plan), planned (no host synchronization), replayed
from a captured hipGraph, re-rendered after its pairs exceeded the plan --
must give exactly the image lfr_render gives, which the forward parity tests
check against the oracle.  One frame is also checked against the oracle
directly."""
import sys

import numpy as np
import pytest

import oracle
from tests._parity import colour_bound, compare
from workloads import DisplayParams, Rational
from workloads.cameras import orbit_rig, pack_cameras
from workloads.scenes import mixture_scene

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_04509_amd import lfr
    ctx = lfr.Context(0)
    yield lfr, ctx
    torch.cuda.synchronize()
    ctx.close()


# three panels of different shapes (one with ragged tiles), three scenes
PANELS = [
    (DisplayParams(256, 144, 16, Rational(1, 6), Rational(5, 1), tile_w=16, tile_h=16), 4000, 4, True),
    (DisplayParams(320, 180, 24, Rational(1, 6), Rational(5, 1), tile_w=32, tile_h=16), 9000, 8, True),
    (DisplayParams(200, 120, 10, Rational(1, 5), Rational(31, 5), tile_w=16, tile_h=32), 6000, 1, False),
]


def _rig(p, offset):
    return pack_cameras(orbit_rig(p.num_views, p.width, p.height, 12.0, 50.0, 60.0, centre=(0.0, 0.0, 12.0),
                                  rig_offset=offset))


def _setup(lfr, ctx, poses=3, seed=9):
    rng = np.random.Generator(np.random.PCG64(seed))
    frames, ref_args = [], []
    displays, scenes = [], []
    for k, (p, m, S, remap) in enumerate(PANELS):
        d = lfr.Display(ctx, p)
        sc = mixture_scene(41 + k, m, 3)
        ds = lfr.DeviceScene.from_numpy(sc, device="cuda:0")
        displays.append(d)
        scenes.append((sc, ds))
        for _ in range(poses):
            cams = _rig(p, tuple(rng.uniform(-0.05, 0.05, 3)))
            out = torch.zeros((p.height, p.width, 3), device="cuda:0")
            frames.append(lfr.Frame(d, ds, cams, out, cluster_size=S, remap=remap))
            ref_args.append((d, ds, S, remap, p, sc))
    return frames, ref_args, displays, scenes


def _reference(lfr, ctx, frames, ref_args):
    refs = []
    for f, (d, ds, S, remap, p, sc) in zip(frames, ref_args):
        refs.append(lfr.render(ctx, d, ds, f.cams, cluster_size=S, remap=remap).clone())
    torch.cuda.synchronize()
    return refs


def _check_equal(frames, refs):
    for i, (f, r) in enumerate(zip(frames, refs)):
        assert torch.equal(f.out, r), f"frame {i} differs"


@pytest.mark.parametrize("graph,merge", [(True, True), (False, True), (True, False), (False, False)])
def test_batch_matches_individual_renders(lib, graph, merge):
    """Merged groups: the three poses of each of the first two panels (same
    display, scene and options, remapped blend) render as one group each;
    the third panel's frames (row-major blend) render one by one."""
    lfr, ctx = lib
    bctx = lfr.Context(0)
    frames, ref_args, displays, scenes = _setup(lfr, ctx)
    refs = _reference(lfr, ctx, frames, ref_args)
    n = len(frames)
    say("batch of", n, "frames, graph", graph, "merge", merge)
    st = lfr.render_batch(bctx, frames, graph=graph, merge=merge)
    torch.cuda.synchronize()
    assert st["batch_frames"] == n and st["batch_unplanned"] == n
    assert st["batch_groups"] == (5 if merge else n)
    _check_equal(frames, refs)
    seen_graphs = 0
    for rep in range(3):
        for f in frames:
            f.out.zero_()
        st = lfr.render_batch(bctx, frames, graph=graph, merge=merge)
        torch.cuda.synchronize()
        say(" repeat", rep, st)
        assert st["batch_unplanned"] == 0
        seen_graphs = max(seen_graphs, st["batch_graphs"])
        _check_equal(frames, refs)
    if graph:
        assert seen_graphs == n
    else:
        assert seen_graphs == 0
    # new head poses: cameras change, slots keep their plans (and graphs)
    rng = np.random.Generator(np.random.PCG64(123))
    for f, (d, ds, S, remap, p, sc) in zip(frames, ref_args):
        f.set_cameras(_rig(p, tuple(rng.uniform(-0.05, 0.05, 3))))
        f.out.zero_()
    refs = _reference(lfr, ctx, frames, ref_args)
    st = lfr.render_batch(bctx, frames, graph=graph, merge=merge)
    torch.cuda.synchronize()
    say(" new poses", st)
    assert st["batch_unplanned"] == 0
    _check_equal(frames, refs)
    bctx.close()
    for d in displays:
        d.close()


def test_tight_plans_overflow_is_rerendered(lib):
    lfr, ctx = lib
    bctx = lfr.Context(0)
    frames, ref_args, displays, scenes = _setup(lfr, ctx, poses=2)
    lfr.render_batch(bctx, frames, graph=True, tight_plans=True)
    lfr.render_batch(bctx, frames, graph=True, tight_plans=True)
    # move every rig well away from its planned pose: with exact plans some
    # depth chunks need more pairs than planned
    rng = np.random.Generator(np.random.PCG64(7))
    for f, (d, ds, S, remap, p, sc) in zip(frames, ref_args):
        f.set_cameras(_rig(p, tuple(rng.uniform(-0.6, 0.6, 3))))
        f.out.zero_()
    refs = _reference(lfr, ctx, frames, ref_args)
    st = lfr.render_batch(bctx, frames, graph=True, tight_plans=True)
    torch.cuda.synchronize()
    say("tight plans after a pose change", st)
    assert st["batch_rerendered"] > 0
    _check_equal(frames, refs)
    # the re-rendered slots have new plans: the next batch is planned again
    for f in frames:
        f.out.zero_()
    st = lfr.render_batch(bctx, frames, graph=True, tight_plans=True)
    torch.cuda.synchronize()
    _check_equal(frames, refs)
    bctx.close()
    for d in displays:
        d.close()


def test_batch_frame_against_oracle(lib):
    lfr, ctx = lib
    bctx = lfr.Context(0)
    frames, ref_args, displays, scenes = _setup(lfr, ctx, poses=1)
    for _ in range(3):
        lfr.render_batch(bctx, frames, graph=True)
    torch.cuda.synchronize()
    f, (d, ds, S, remap, p, sc) = frames[1], ref_args[1]
    V = oracle.view_map(p)
    rng = np.random.Generator(np.random.PCG64(5))
    samples = np.sort(rng.choice(V.size, 3000, replace=False))
    cams = np.frombuffer(bytes(f.cams), dtype=np.float32).reshape(-1, 16)
    r = oracle.render_subpixels_ranged(sc, cams, p, V, S, samples)
    got = f.out.cpu().numpy().reshape(-1)[samples]
    say("batch frame vs oracle, S", S)
    say(compare(got, r, colour_bound(sc), label='batch frame'))
    bctx.close()
    for d in displays:
        d.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("S", [8])
def test_full_size_serving_batch_against_oracle(lib, S):
    """The serving configuration at full size: three outdoor-style scenes
    (0.5M / 1M / 3M Gaussians) on 1920x1080/45-view, 2560x1440/64-view and
    3840x2160/100-view panels, two head poses each, on the tiles the
    benchmark's autotuner picks for them (32x64, 32x64 and 64x128), rendered
    by lfr_render_batch (planned, replayed from captured graphs).  Every
    frame equals lfr_render's image; one frame of each panel is checked
    against the oracle on about 1024 subpixels spread over all its views."""
    from workloads.configs import batched_frames
    lfr, ctx = lib
    bctx = lfr.Context(0)
    frames, refs, keep = [], [], []
    for seed_i, m, disp, radius, span, offs in batched_frames(num_poses=2):
        say("panel", disp.width, disp.height, disp.num_views, "scene", seed_i, m)
        sc = mixture_scene(seed_i, m, 3)
        ds = lfr.DeviceScene.from_numpy(sc, device="cuda:0")
        d = lfr.Display(ctx, disp.with_tile(*((64, 128) if disp.width >= 3840 else (32, 64))))
        keep.append((d, ds, sc, disp, radius, span))
        for o in offs:
            cams = pack_cameras(orbit_rig(disp.num_views, disp.width, disp.height, radius, span, 60.0,
                                          centre=(0.0, 0.0, radius), rig_offset=tuple(o)))
            out = torch.zeros((disp.height, disp.width, 3), device="cuda:0")
            frames.append(lfr.Frame(d, ds, cams, out, cluster_size=S))
            refs.append((len(keep) - 1, cams))
    for rep in range(3):
        st = lfr.render_batch(bctx, frames, graph=True)
        torch.cuda.synchronize()
        say(" batch", rep, st)
    assert st["batch_unplanned"] == 0
    assert st["batch_groups"] == 3              # the two poses of each panel merge
    for i, (f, (k, cams)) in enumerate(zip(frames, refs)):
        d, ds, sc, disp, radius, span = keep[k]
        one = lfr.render(ctx, d, ds, cams, cluster_size=S)
        torch.cuda.synchronize()
        assert torch.equal(one, f.out), f"frame {i} differs from lfr_render"
        del one
    for k, (d, ds, sc, disp, radius, span) in enumerate(keep):
        i = 2 * k + 1                               # the second pose of each panel
        f, cams = frames[i], refs[i][1]
        V = oracle.view_map(disp)
        views = np.unique(V)
        rng = np.random.default_rng(k)
        flat = V.reshape(-1)
        samples = np.sort(np.concatenate([rng.choice(np.flatnonzero(flat == j), -(-1024 // len(views)),
                                                     replace=False) for j in views]))
        with oracle.threads():
            r = oracle.render_subpixels_ranged(sc, cams, disp, V, S, samples)
        got = f.out.cpu().numpy().reshape(-1)[samples]
        say(" panel", disp.width, disp.height, compare(got, r, colour_bound(sc), label=f"batch panel {k}"))
    bctx.close()
    for d, *_ in keep:
        d.close()


def test_batch_errors_and_empty(lib):
    lfr, ctx = lib
    import ctypes
    say("batch error paths")
    assert lfr.render_batch(ctx, [])["batch_frames"] == 0
    frames, ref_args, displays, scenes = _setup(lfr, ctx, poses=1)
    frames[0].opts.flags |= lfr.LFR_SAVE_FOR_BACKWARD
    with pytest.raises(lfr.LfrError):
        lfr.render_batch(ctx, frames)
    rc = lfr.library().lfr_render_batch(ctx.handle, None, -1, 0)
    assert rc == lfr.LFR_ERR_INVALID_ARG
    for d in displays:
        d.close()
