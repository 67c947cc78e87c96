"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Integer and index work (view map, remap LUT, sort) must be bit-exact;
projected attributes are computed in double precision on both sides and
must round to the same float32 values; rendered subpixels follow the rule
in tests/_parity.py.  Every test prints what it runs before it runs it."""
import sys

import numpy as np
import pytest

import oracle
from tests._parity import colour_bound, compare
from workloads import DisplayParams, Rational, Scene, get_workload
from workloads.cameras import orbit_rig, pack_cameras

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


def _display(lfr, ctx, params):
    return lfr.Display(ctx, params)


# --------------------------------------------------------------------------
# display precompute: bit-exact
# --------------------------------------------------------------------------

DISPLAYS = [
    get_workload("tiny").display,
    get_workload("display").display,
    get_workload("outdoor").display,
    DisplayParams(250, 139, 7, Rational(-3, 11), Rational(17, 3), Rational(-5, 7), 8, 8),
    DisplayParams(250, 139, 11, Rational(1, 6), Rational(23, 5), Rational(1, 2), 32, 32),
    DisplayParams(250, 139, 9, Rational(1, 5), Rational(31, 5), Rational(0), 64, 32),
    DisplayParams(77, 41, 9, Rational(2, 7), Rational(9, 2), Rational(0), 16, 8),
    DisplayParams(1, 1, 3, Rational(1, 6), Rational(5), Rational(0), 8, 8),
]


@pytest.mark.parametrize("k", range(len(DISPLAYS)))
def test_view_map_and_remap_bit_exact(lib, k):
    lfr, ctx = lib
    p = DISPLAYS[k]
    say("display", p)
    d = _display(lfr, ctx, p)
    V = d.view_map()
    Vo = oracle.view_map(p)
    np.testing.assert_array_equal(V, Vo)
    psi = d.remap()
    np.testing.assert_array_equal(psi, oracle.remap(p, Vo))
    n, mask = d.referenced_views()
    assert n == len(np.unique(Vo)) and mask[np.unique(Vo)].all()
    d.close()


def test_display_from_map_and_errors(lib):
    lfr, ctx = lib
    p = DisplayParams(33, 17, 5, Rational(1, 6), Rational(23, 5), tile_w=8, tile_h=8)
    Vo = oracle.view_map(p)
    d = lfr.Display(ctx, view_map=Vo, width=33, height=17, num_views=5, tile=(8, 8))
    np.testing.assert_array_equal(d.view_map(), Vo)
    np.testing.assert_array_equal(d.remap(), oracle.remap(p, Vo))
    d.close()
    bad = Vo.copy()
    bad[0, 0, 0] = 5
    with pytest.raises(lfr.LfrError) as ei:
        lfr.Display(ctx, view_map=bad, width=33, height=17, num_views=5, tile=(8, 8))
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG
    with pytest.raises(lfr.LfrError) as ei:
        lfr.Display(ctx, DisplayParams(33, 17, 5, Rational(1, 6), Rational(23, 5), tile_w=12, tile_h=8))
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG
    with pytest.raises(lfr.LfrError) as ei:                # 16384 pixels per tile: too many
        lfr.Display(ctx, DisplayParams(33, 17, 5, Rational(1, 6), Rational(23, 5), tile_w=128, tile_h=128))
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG
    # the largest tiles (24576 subpixels each, sorted in 128 KB of LDS), with
    # ragged edge tiles, against the oracle's remap table
    for tw, th in ((128, 64), (64, 128)):
        q = DisplayParams(300, 170, 7, Rational(1, 6), Rational(23, 5), tile_w=tw, tile_h=th)
        Vq = oracle.view_map(q)
        dq = lfr.Display(ctx, view_map=Vq, width=300, height=170, num_views=7, tile=(tw, th))
        np.testing.assert_array_equal(dq.remap(), oracle.remap(q, Vq))
        dq.close()


# --------------------------------------------------------------------------
# device sort: bit-exact against a stable argsort
# --------------------------------------------------------------------------

# The digit-count scans run in one launch up to 16384 counts (64 sort tiles of
# 256 digits), in two above that: 262144 keys sit at the boundary, 262145
# and the larger cases past it.
@pytest.mark.parametrize("n,bits,wide", [(1, 32, False), (1000, 32, False), (123457, 19, False),
                                         (300001, 13, False), (200003, 40, True), (65536, 64, True),
                                         (4097, 7, False), (262144, 32, False), (262145, 32, False),
                                         (2000003, 24, False), (300001, 64, True)])
def test_radix_sort_stable(lib, n, bits, wide):
    lfr, ctx = lib
    say("sort", n, bits, wide)
    rng = np.random.default_rng(n + bits)
    hi = 1 << min(bits, 63)
    keys = rng.integers(0, hi, n, dtype=np.uint64)
    keys[: n // 3] = keys[n // 2]                    # plenty of ties
    if not wide:
        keys = keys.astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    kd = torch.from_numpy(keys.view(np.int64 if wide else np.int32).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    lfr.sort_pairs(ctx, kd, vd, 0, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(kd.cpu().numpy().view(keys.dtype), keys[order])
    np.testing.assert_array_equal(vd.cpu().numpy().view(np.uint32), vals[order])


def test_radix_sort_stable_large(lib):
    """More than 2048 scan tiles of digit counts (32770 sort tiles x 256
    digits): the scans take their three-launch form.  Checked on the device
    by the properties that define a stable sort: keys non-decreasing, each
    output key the input key at its output index, indices a permutation,
    increasing within runs of equal keys."""
    lfr, ctx = lib
    n = 32770 * 4096 - 3
    say("sort large", n)
    g = torch.Generator(device="cuda").manual_seed(7)
    keys = torch.randint(0, 1 << 20, (n,), device="cuda", dtype=torch.int32, generator=g)
    keys[: n // 4] = 12345                            # a long run of ties
    kd = keys.clone()
    vd = torch.arange(n, device="cuda", dtype=torch.int32)
    lfr.sort_pairs(ctx, kd, vd, 0, 32)
    torch.cuda.synchronize()
    idx = vd.long()
    assert bool((kd[1:] >= kd[:-1]).all())
    assert bool((keys[idx] == kd).all())
    assert bool((torch.bincount(idx, minlength=n) == 1).all())
    tie = kd[1:] == kd[:-1]
    assert bool((vd[1:][tie] > vd[:-1][tie]).all())
    del keys, kd, vd, idx, tie
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# projection: float32 roundings of the double-precision projection agree
# --------------------------------------------------------------------------

def _check_projection(gpu, ref, label):
    np.testing.assert_array_equal(gpu["valid"], ref["valid"], err_msg=label)
    np.testing.assert_array_equal(gpu["valid_mean"], ref["valid_mean"], err_msg=label)
    np.testing.assert_array_equal(gpu["depth"], ref["depth"], err_msg=label)
    vm = ref["valid_mean"] == 1
    v = ref["valid"] == 1
    mism = 0
    for f, mask in (("mean2d", vm), ("conic", v), ("color", v)):
        a, b = gpu[f][mask], ref[f][mask]
        mism += int((a != b).sum())
        ulp = np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))
        assert ulp.max(initial=0) <= 1, f"{label}: {f} differs by {ulp.max()} ulp"
    total = int(vm.sum() * 2 + v.sum() * 6)
    assert mism <= max(2, 1e-5 * total), f"{label}: {mism} of {total} float32 values differ by an ulp"
    return mism


@pytest.mark.parametrize("name,views", [("tiny", (0, 7, 15)), ("display", (0, 22)), ("outdoor", (50,))])
def test_projection_matches_oracle(lib, name, views):
    lfr, ctx = lib
    w = get_workload(name)
    say("projection", name, views)
    scene = w.make_scene()
    cams = pack_cameras(w.cameras())
    ds = lfr.DeviceScene.from_numpy(scene)
    for j in views:
        gpu = lfr.project(ctx, ds, cams[j], w.display.width, w.display.height)
        ref = oracle.project(scene, cams[j], w.display.width, w.display.height)
        _check_projection(gpu, ref, f"{name} view {j}")


def test_projection_edge_cases(lib):
    lfr, ctx = lib
    say("projection edge cases")
    m = [[0, 0, 4], [0, 0, -4], [0, 0, 0.1], [0, 0, 4], [np.nan, 0, 4], [50, 0, 1], [0, 0, 4]]
    o = [0.5, 0.5, 0.5, 1 / 255 * 0.999, 0.5, 0.5, 0.9]
    ls = [[-3] * 3] * 6 + [[-30, -30, -30]]
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    sc = Scene(f32(m), f32(ls), f32([[1, 0, 0, 0]] * 7), f32(o), f32(np.zeros((7, 16, 3))), 3)
    cam = pack_cameras(orbit_rig(1, 64, 36, 4.0, 0.0))[0]
    gpu = lfr.project(ctx, lfr.DeviceScene.from_numpy(sc), cam, 64, 36)
    ref = oracle.project(sc, cam, 64, 36)
    _check_projection(gpu, ref, "edge")


# --------------------------------------------------------------------------
# rendering
# --------------------------------------------------------------------------

def _render(lfr, ctx, disp, dscene, cams, **kw):
    out = lfr.render(ctx, disp, dscene, cams, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def tiny_setup(lib):
    lfr, ctx = lib
    w = get_workload("tiny")
    scene = w.make_scene()
    cams = pack_cameras(w.cameras())
    V = oracle.view_map(w.display)
    return w, scene, cams, V, lfr.DeviceScene.from_numpy(scene)


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_tiny_full_frame_parity(lib, tiny_setup, S):
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("tiny full frame S =", S)
    d = _display(lfr, ctx, w.display)
    img = _render(lfr, ctx, d, ds, cams, cluster_size=S, remap=True)
    with oracle.threads():
        r = oracle.render_frame_ranged(scene, cams, w.display, V, S)
    info = compare(img, r, colour_bound(scene), label=f"tiny S={S}")
    say(info)
    # remap changes only the thread order, never a value
    img2 = _render(lfr, ctx, d, ds, cams, cluster_size=S, remap=False)
    np.testing.assert_array_equal(img, img2)
    # culling unreferenced views changes nothing either
    img3 = _render(lfr, ctx, d, ds, cams, cluster_size=S, remap=True, cull=False)
    np.testing.assert_array_equal(img, img3)
    d.close()


@pytest.mark.parametrize("S,remap", [(1, True), (4, True), (4, False)])
def test_depth_chunking_does_not_change_the_image(lib, tiny_setup, S, remap):
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("depth chunks: first chunk 1 / 7 / 64 / all, S =", S, "remap", remap)
    d = _display(lfr, ctx, w.display)
    whole = _render(lfr, ctx, d, ds, cams, cluster_size=S, remap=remap, first_chunk=1 << 20)
    assert ctx.stats()["chunks"] == 1
    for fc in (1, 7, 64):
        img = _render(lfr, ctx, d, ds, cams, cluster_size=S, remap=remap, first_chunk=fc)
        st = ctx.stats()
        say(fc, st["chunks"], st["pairs"])
        assert st["chunks"] > 1
        np.testing.assert_array_equal(img, whole)
    d.close()


def test_equal_depths_keep_index_order_across_depth_chunks(lib, tiny_setup):
    """Every Gaussian of the tiny scene gets a twin at the same mean (hence the
    same depth in every cluster) but with another colour and opacity, so the
    blend order of equal depths decides the image.  Rendered in several depth
    chunks (only the ranks before the last chunk depth-sorted, the last chunk
    binned in index order and sorted with the depth in its pair keys), the
    image must be bit-identical to one chunk from a single full depth sort,
    and that one must match the oracle, which orders equal depths by index."""
    lfr, ctx = lib
    w, scene, cams, V, _ = tiny_setup
    rng = np.random.default_rng(11)
    perm = rng.permutation(scene.num_gaussians)
    twin = Scene(scene.means.copy(), scene.log_scales[perm].copy(), scene.quats[perm].copy(),
                 scene.opacities[perm].copy(), scene.sh[perm].copy(), scene.sh_degree)
    both = Scene(*(np.concatenate([a, b]) for a, b in zip(
        (scene.means, scene.log_scales, scene.quats, scene.opacities, scene.sh),
        (twin.means, twin.log_scales, twin.quats, twin.opacities, twin.sh))), scene.sh_degree)
    ds = lfr.DeviceScene.from_numpy(both)
    d = _display(lfr, ctx, w.display)
    for S in (1, 4):
        whole = _render(lfr, ctx, d, ds, cams, cluster_size=S, first_chunk=1 << 20)
        assert ctx.stats()["chunks"] == 1
        if S == 4:
            r = oracle.render_frame_ranged(both, cams, w.display, V, S)
            say(compare(whole, r, colour_bound(both), label="twins S=4"))
        for fc in (1, 5, 64):
            img = _render(lfr, ctx, d, ds, cams, cluster_size=S, first_chunk=fc)
            st = ctx.stats()
            say("twins S =", S, "first chunk", fc, "chunks", st["chunks"], "pairs", st["pairs"])
            assert st["chunks"] > 1
            np.testing.assert_array_equal(img, whole)
    d.close()


@pytest.mark.parametrize("case", ["one_mean", "mostly_behind"])
def test_split_depth_order_edge_cases(lib, tiny_setup, case):
    """The two ends of the split depth order, against one chunk from a full
    sort.  one_mean: every Gaussian at the tiny scene's first mean (colours,
    opacities and shapes kept), so each cluster's keys are all equal and fall
    in one histogram bin holding more than the ranked chunks' ranks: the near
    set is empty and every item lies in the last chunk, whose 64-bit sort must
    keep equal depths in index order (checked against the oracle too).
    mostly_behind: nine Gaussians in ten moved behind the cameras, so fewer
    valid keys than ranked ranks: the last chunk is empty."""
    lfr, ctx = lib
    w, scene, cams, V, _ = tiny_setup
    means = scene.means.copy()
    if case == "one_mean":
        means[:] = means[0]
    else:
        means[np.arange(len(means)) % 10 != 0, 2] = -50.0
    sc = Scene(means, scene.log_scales, scene.quats, scene.opacities, scene.sh, scene.sh_degree)
    ds = lfr.DeviceScene.from_numpy(sc)
    d = _display(lfr, ctx, w.display)
    for S in (1, 4):
        whole = _render(lfr, ctx, d, ds, cams, cluster_size=S, first_chunk=1 << 20)
        assert ctx.stats()["chunks"] == 1
        if case == "one_mean" and S == 4:
            r = oracle.render_frame_ranged(sc, cams, w.display, V, S)
            say(compare(whole, r, colour_bound(sc), label=f"{case} S={S}"))
        for fc in (5, 64):
            img = _render(lfr, ctx, d, ds, cams, cluster_size=S, first_chunk=fc)
            st = ctx.stats()
            say(case, "S =", S, "first chunk", fc, "chunks", st["chunks"], "pairs", st["pairs"])
            assert st["chunks"] > 1
            np.testing.assert_array_equal(img, whole)
    d.close()


@pytest.mark.parametrize("S,first_chunk", [(1, 0), (4, 0), (4, 64), (8, 7)])
def test_work_counts_agree_across_blend_orders(lib, tiny_setup, S, first_chunk):
    """The counting renders report the method's work on the binned lists: the
    alphas each subpixel evaluates up to and including its stop, and the
    contributions it blends.  Both depend only on the lists, not on the thread
    order: the remapped blend (which culls staged entries and counts from list
    positions) and the row-major blend (which walks every entry) must agree
    exactly, with one depth chunk or several."""
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("work counts, S =", S, "first chunk", first_chunk)
    d = _display(lfr, ctx, w.display)
    counts = {}
    for remap in (True, False):
        out = torch.empty((w.display.height, w.display.width, 3), device="cuda:0")
        lfr.render(ctx, d, ds, cams, cluster_size=S, remap=remap, out=out, count_work=True,
                   first_chunk=first_chunk)
        torch.cuda.synchronize()
        st = ctx.stats()
        counts[remap] = (st["evals"], st["blended"], st["pairs"], st["chunks"])
        say(" remap" if remap else " row-major", counts[remap], "wave steps", st["wave_steps"])
        if remap:
            assert 0 < st["wave_steps_live"] <= st["wave_steps"]
    assert counts[True] == counts[False]
    assert counts[True][0] >= counts[True][1] > 0
    d.close()


@pytest.mark.parametrize("tile", [(8, 8), (32, 32), (16, 8), (64, 32), (32, 64), (64, 64), (128, 64), (64, 128)])
def test_tiling_does_not_change_the_image(lib, tiny_setup, tile):
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("tiling", tile)
    d16 = _display(lfr, ctx, w.display)
    dt = _display(lfr, ctx, w.display.with_tile(*tile))
    for S in (1, 4):
        a = _render(lfr, ctx, d16, ds, cams, cluster_size=S)
        b = _render(lfr, ctx, dt, ds, cams, cluster_size=S)
        np.testing.assert_array_equal(a, b)
    d16.close()
    dt.close()


def test_autotune_reports_every_candidate(lib, tiny_setup):
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("autotune")
    tiles = ((16, 16), (32, 32), (64, 32))
    best, res = lfr.autotune(ctx, w.display, ds, cams, cluster_sizes=(2, 8), tiles=tiles, reps=2)
    assert len(res) == 6
    assert [(r["tile_w"], r["tile_h"], r["cluster_size"]) for r in res] == [
        (tw, th, S) for (tw, th) in tiles for S in (2, 8)]
    assert all(r["ms"] > 0 and r["pairs"] > 0 for r in res)
    assert best["ms"] == min(r["ms"] for r in res)
    with pytest.raises(lfr.LfrError) as ei:
        lfr.autotune(ctx, w.display, ds, cams, tiles=((12, 16),))
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG


def test_fullframe_interlace_equals_exact_path(lib, tiny_setup):
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("full-frame + interlace vs exact path")
    d = _display(lfr, ctx, w.display)
    exact = _render(lfr, ctx, d, ds, cams, cluster_size=1)
    for vb, tile in ((1, 16), (5, 8), (16, 32)):
        ff = lfr.render_fullframe_interlace(ctx, d, ds, cams, view_batch=vb, tile=tile)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ff.cpu().numpy(), exact)
    ff_all = lfr.render_fullframe_interlace(ctx, d, ds, cams, view_batch=7, cull=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ff_all.cpu().numpy(), exact)
    d.close()


def test_ragged_panel_and_background(lib):
    lfr, ctx = lib
    say("ragged panel 250x139, tiles 32x32 / 8x8, background")
    w = get_workload("tiny")
    scene = w.make_scene().subset(np.arange(0, 2000, 2))
    bg = (0.25, 0.5, 1.0)
    for tile in ((32, 32), (8, 8)):
        p = DisplayParams(250, 139, 11, Rational(1, 6), Rational(23, 5), Rational(1, 2), *tile)
        cams = pack_cameras(orbit_rig(11, 250, 139, 4.0, 30.0))
        V = oracle.view_map(p)
        d = _display(lfr, ctx, p)
        ds = lfr.DeviceScene.from_numpy(scene)
        for S in (1, 3):
            img = _render(lfr, ctx, d, ds, cams, cluster_size=S, background=bg)
            rng = np.random.default_rng(S)
            samples = rng.choice(V.size, 4000, replace=False)
            r = oracle.render_subpixels_ranged(scene, cams, p, V, S, samples, bg)
            say(compare(img.reshape(-1)[samples], r, colour_bound(scene) + 1.0, label=f"ragged {tile} S={S}"))
        d.close()


def test_degenerate_scenes(lib):
    lfr, ctx = lib
    say("degenerate scenes")
    p = DisplayParams(40, 24, 5, Rational(1, 6), Rational(23, 5))
    cams = pack_cameras(orbit_rig(5, 40, 24, 4.0, 20.0))
    d = _display(lfr, ctx, p)
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    bg = (0.1, 0.2, 0.3)
    # empty scene -> background everywhere
    empty = Scene(f32(np.zeros((0, 3))), f32(np.zeros((0, 3))), f32(np.zeros((0, 4))), f32(np.zeros(0)),
                  f32(np.zeros((0, 1, 3))), 0)
    img = _render(lfr, ctx, d, lfr.DeviceScene.from_numpy(empty), cams, cluster_size=2, background=bg)
    np.testing.assert_array_equal(img, np.broadcast_to(np.float32(bg), img.shape))
    # everything behind the cameras or transparent -> background
    behind = Scene(f32([[0, 0, -5], [0, 0, 4]]), f32([[-2] * 3] * 2), f32([[1, 0, 0, 0]] * 2),
                   f32([0.9, 0.001]), f32(np.ones((2, 1, 3))), 0)
    img = _render(lfr, ctx, d, lfr.DeviceScene.from_numpy(behind), cams, cluster_size=1, background=bg)
    np.testing.assert_array_equal(img, np.broadcast_to(np.float32(bg), img.shape))
    # one large opaque Gaussian, cluster size larger than the view count
    one = Scene(f32([[0, 0, 4]]), f32([[-0.5] * 3]), f32([[1, 0, 0, 0]]), f32([0.97]), f32([[[0.7, 0.1, 0.3]]]), 0)
    V = oracle.view_map(p)
    for S in (1, 8):
        img = _render(lfr, ctx, d, lfr.DeviceScene.from_numpy(one), cams, cluster_size=S, background=bg)
        r = oracle.render_frame_ranged(one, cams, p, V, S, bg)
        compare(img, r, 2.0, label=f"one S={S}")
    d.close()


def test_capacity_limit_and_recovery(lib, tiny_setup):
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("capacity limit")
    c2 = lfr.Context(0)
    d = _display(lfr, c2, w.display)
    c2.set_limit(1 << 16)
    with pytest.raises(lfr.LfrError) as ei:
        lfr.render(c2, d, ds, cams, cluster_size=2)
    assert ei.value.code == lfr.LFR_ERR_CAPACITY
    c2.set_limit(0)
    img = lfr.render(c2, d, ds, cams, cluster_size=2)
    torch.cuda.synchronize()
    ref = _render(lfr, ctx, d, ds, cams, cluster_size=2)
    np.testing.assert_array_equal(img.cpu().numpy(), ref)
    d.close()
    c2.close()


def test_invalid_arguments_rejected(lib, tiny_setup):
    lfr, ctx = lib
    w, scene, cams, V, ds = tiny_setup
    say("invalid arguments")
    d = _display(lfr, ctx, w.display)
    with pytest.raises(lfr.LfrError) as ei:
        lfr.render(ctx, d, ds, cams[:5], cluster_size=2)      # wrong camera count
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG
    bad = cams.copy()
    bad[3, 12] = 0.0                                          # fx = 0
    with pytest.raises(lfr.LfrError) as ei:
        lfr.render(ctx, d, ds, bad, cluster_size=2)
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG
    with pytest.raises(lfr.LfrError) as ei:
        lfr.render(ctx, d, ds, cams, cluster_size=0)
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG
    with pytest.raises(lfr.LfrError) as ei:
        lfr.render(ctx, d, ds, cams, cluster_size=33)
    assert ei.value.code == lfr.LFR_ERR_UNSUPPORTED
    d.close()


def _sample_in_views(V, views, per_view, seed):
    rng = np.random.default_rng(seed)
    flat = V.reshape(-1)
    out = []
    for j in views:
        idx = np.flatnonzero(flat == j)
        out.append(rng.choice(idx, min(per_view, idx.size), replace=False))
    return np.sort(np.concatenate(out))


def _sample_every_view(V, total, seed):
    """About `total` subpixels spread evenly over every view the panel uses
    (so over every cluster, the padded last one included)."""
    views = np.unique(V)
    return _sample_in_views(V, views, -(-total // len(views)), seed), views


@pytest.mark.parametrize("S", [1, 8])
def test_display_workload_sampled(lib, S):
    lfr, ctx = lib
    w = get_workload("display")
    say("display workload (200k Gaussians, 1920x1080, 45 views) S =", S)
    scene = w.make_scene()
    cams = pack_cameras(w.cameras())
    V = oracle.view_map(w.display)
    d = _display(lfr, ctx, w.display.with_tile(32, 32))
    ds = lfr.DeviceScene.from_numpy(scene)
    img = _render(lfr, ctx, d, ds, cams, cluster_size=S)
    samples, views = _sample_every_view(V, 2048, S)
    with oracle.threads():
        r = oracle.render_subpixels_ranged(scene, cams, w.display, V, S, samples)
    info = compare(img.reshape(-1)[samples], r, colour_bound(scene), label=f"display S={S}")
    say(len(views), "views", info)
    if S == 1:
        ff = lfr.render_fullframe_interlace(ctx, d, ds, cams, view_batch=10)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ff.cpu().numpy(), img)
    d.close()


def test_display_workload_tilings_and_chunks_agree(lib):
    """The display workload in several depth chunks (the split depth order,
    the alive tables between chunks) on three tilings that take different
    code paths: 8x8 tiles (135 tile rows, a 136 x 241 summed-area table:
    no row/column masks, the table built outside LDS), 32x32, 32x64 and 64x64
    (masks and the LDS table) and 64x128 (24576 subpixels per tile, the remap
    table's largest sort, in 128 KB of LDS).  Coverage is conservative, so every rendering must be
    bit-identical, and equal to one chunk from a single full depth sort."""
    lfr, ctx = lib
    w = get_workload("display")
    scene = w.make_scene()
    cams = pack_cameras(w.cameras())
    ds = lfr.DeviceScene.from_numpy(scene)
    ref = None
    for tile in ((32, 32), (8, 8), (32, 64), (64, 128)):
        d = _display(lfr, ctx, w.display.with_tile(*tile))
        for S, fc in ((4, 2048), (4, 1 << 20), (1, 4096)):
            img = _render(lfr, ctx, d, ds, cams, cluster_size=S, first_chunk=fc)
            st = ctx.stats()
            say("display tiling", tile, "S =", S, "first chunk", fc, "chunks", st["chunks"], "pairs", st["pairs"])
            if fc != 1 << 20:
                assert st["chunks"] > 1
            if ref is None:
                ref = {}
            if S not in ref:
                ref[S] = img
            else:
                np.testing.assert_array_equal(img, ref[S])
        d.close()


# the tile shapes the benchmark's autotuner chooses among
BENCH_TILES = ((16, 16), (32, 16), (16, 32), (32, 32), (64, 32), (32, 64), (64, 64), (128, 64), (64, 128))


@pytest.fixture(scope="module")
def outdoor(lib):
    w = get_workload("outdoor")
    say("generating the outdoor scene (3M Gaussians)")
    scene = w.make_scene()
    cams = pack_cameras(w.cameras())
    V = oracle.view_map(w.display)
    return w, scene, cams, V


@pytest.mark.timeout(900)
@pytest.mark.parametrize("S,n_samples", [(8, 4096), (1, 1024)])
def test_outdoor_workload_bench_configuration(lib, outdoor, S, n_samples):
    """3M Gaussians, 100 views, 3840x2160, remap on, default depth chunks:
    the frame the benchmark times (cluster size 8) and its exact-path
    ablation (cluster size 1).  The image is rendered on every tile shape the
    autotuner picks from and must be bit-identical across them; subpixels
    spread over all 31 views the panel uses (all clusters, the padded last
    one included) are checked against the oracle."""
    lfr, ctx = lib
    w, scene, cams, V = outdoor
    ds = lfr.DeviceScene.from_numpy(scene)
    imgs = {}
    for tile in BENCH_TILES:
        say("outdoor S =", S, "tile", tile)
        d = _display(lfr, ctx, w.display.with_tile(*tile))
        imgs[tile] = _render(lfr, ctx, d, ds, cams, cluster_size=S)
        st = ctx.stats()
        say(" pairs", st["pairs"], "chunks", st["chunks"], "clusters", st["clusters"])
        assert st["chunks"] > 1
        d.close()
    img = imgs[(32, 64)]
    for tile, im in imgs.items():
        np.testing.assert_array_equal(im, img, err_msg=f"tile {tile}")
    assert np.isfinite(img).all()
    samples, views = _sample_every_view(V, n_samples, 3)
    if S == 8:
        assert len(views) == 31 and {int(v) // 8 for v in views} == set(range(13))
        assert any(v >= 96 for v in views)            # the padded last cluster
    say(f"oracle on {samples.size} subpixels of {len(views)} views")
    with oracle.threads():
        r = oracle.render_subpixels_ranged(scene, cams, w.display, V, S, samples)
    info = compare(img.reshape(-1)[samples], r, colour_bound(scene), label=f"outdoor S={S}")
    say(info)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,S", [("landscape71", 18), ("portrait63", 16)])
def test_paper_display_shapes(lib, outdoor, name, S):
    """The paper's two display shapes (71 views over 53 degrees at 3840x2160
    with reuse groups of 18; 63 views over 53 degrees at 1440x2560 with groups
    of 16, the last group padded) on the 3M-Gaussian scene, on the tile shapes
    the benchmark picks among (64x32, 32x64, 64x64, 128x64, 64x128; bit-identical): subpixels spread
    over every view against the oracle, and the exact path's image against
    full-frame-then-interlace on the same display."""
    lfr, ctx = lib
    w = get_workload(name)
    say(name, "S =", S)
    scene = outdoor[1]
    cams = pack_cameras(w.cameras())
    V = oracle.view_map(w.display)
    assert len(np.unique(V)) == w.display.num_views
    ds = lfr.DeviceScene.from_numpy(scene)
    imgs = {}
    for tile in ((64, 32), (32, 64), (64, 64), (128, 64), (64, 128)):
        d = _display(lfr, ctx, w.display.with_tile(*tile))
        imgs[tile] = _render(lfr, ctx, d, ds, cams, cluster_size=S)
        say(" tile", tile, ctx.stats()["pairs"], "pairs")
        if tile == (64, 32):
            exact = _render(lfr, ctx, d, ds, cams, cluster_size=1)
            ff = lfr.render_fullframe_interlace(ctx, d, ds, cams, view_batch=18, tile=32)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(ff.cpu().numpy(), exact)
        d.close()
    np.testing.assert_array_equal(imgs[(64, 32)], imgs[(32, 64)])
    for tile in ((64, 64), (128, 64), (64, 128)):
        np.testing.assert_array_equal(imgs[(64, 32)], imgs[tile], err_msg=f"tile {tile}")
    img = imgs[(64, 32)]
    samples, views = _sample_every_view(V, 2048, 3)
    assert w.display.num_views - 1 in views            # the padded last cluster
    with oracle.threads():
        r = oracle.render_subpixels_ranged(scene, cams, w.display, V, S, samples)
    info = compare(img.reshape(-1)[samples], r, colour_bound(scene), label=f"{name} S={S}")
    say(info)


def test_elongated_splats_cull_exactly(lib):
    """Strongly anisotropic splats (axis ratios up to 200:1) at random
    rotations: the remapped blend drops staged Gaussians whose cutoff box
    misses every unfinished lane of its wavefront, which must not change a
    single bit.  Checked against the row-major and full-frame kernels (which
    drop nothing), against the oracle, and at S = 1 and 4."""
    lfr, ctx = lib
    rng = np.random.Generator(np.random.PCG64(31))
    m = 3000
    means = np.c_[rng.uniform(-1.2, 1.2, m), rng.uniform(-0.7, 0.7, m), rng.uniform(3.0, 6.0, m)]
    ls = np.c_[rng.uniform(-5.5, -1.5, m), rng.uniform(-6.5, -4.5, m), rng.uniform(-6.5, -4.5, m)]
    q = rng.standard_normal((m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    o = 1.0 / (1.0 + np.exp(-rng.normal(0.5, 1.5, m)))
    sh = np.zeros((m, 1, 3))
    sh[:, 0] = rng.uniform(-1.0, 1.5, (m, 3))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    scene = Scene(f(means), f(ls), f(q), f(o), f(sh), 0)
    p = DisplayParams(160, 96, 12, Rational(1, 6), Rational(23, 5), tile_w=32, tile_h=16)
    cams = pack_cameras(orbit_rig(12, 160, 96, 4.0, 24.0, 60.0, centre=(0.0, 0.0, 4.0)))
    V = oracle.view_map(p)
    d = _display(lfr, ctx, p)
    ds = lfr.DeviceScene.from_numpy(scene)
    say("elongated splats, 3000 Gaussians, 160x96, 12 views")
    for S in (1, 4):
        a = _render(lfr, ctx, d, ds, cams, cluster_size=S, remap=True)
        b = _render(lfr, ctx, d, ds, cams, cluster_size=S, remap=False)
        np.testing.assert_array_equal(a, b)
        if S == 1:
            ff = lfr.render_fullframe_interlace(ctx, d, ds, cams, view_batch=6)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(ff.cpu().numpy(), a)
        samples = np.sort(np.random.default_rng(S).choice(V.size, 4000, replace=False))
        r = oracle.render_subpixels_ranged(scene, cams, p, V, S, samples)
        say(compare(a.reshape(-1)[samples], r, colour_bound(scene), label=f"elongated S={S}"))
    d.close()
