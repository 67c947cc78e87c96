"""Pins for the oracle's front-to-back blend (section 4.3, Eq. 9-10), the
reuse rule (section 4.2) and the subpixel path's equivalence with
full-frame-then-interlace (sections 1 and 4)."""
import math

import numpy as np
import pytest

import oracle
from workloads import DisplayParams, Rational, Scene, get_workload
from workloads.cameras import Camera, orbit_rig, pack_cameras


def _scene(means, log_scales, opac, colours, quats=None):
    m = len(means)
    C0 = 0.5 / math.sqrt(math.pi)
    sh = ((np.asarray(colours, np.float64) - 0.5) / C0).reshape(m, 1, 3)
    if quats is None:
        quats = [[1, 0, 0, 0]] * m
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means), f(log_scales), f(quats), f(opac), f(sh), 0)


def _one_view_display(W=24, H=16):
    # tan = 0, pitch = 3, N = 1: every subpixel belongs to view 0.
    return DisplayParams(W, H, 1, Rational(0), Rational(3))


def _front_cam(W, H, f=40.0):
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f, W / 2, H / 2).packed()[None]


def _render(scene, cams, disp, S=1, bg=(0, 0, 0)):
    V = oracle.view_map(disp)
    img, flags, tflag = oracle.render_frame(scene, cams, disp, V, S, bg)
    return img, flags


def test_single_gaussian_closed_form():
    W, H, f, z, s, o = 24, 16, 40.0, 4.0, 0.2, 0.7
    col = [0.9, 0.4, 0.1]
    sc = _scene([[0, 0, z]], [[math.log(s)] * 3], [o], [col])
    img, _ = _render(sc, _front_cam(W, H, f), _one_view_display(W, H))
    var = (f * s / z) ** 2 + 0.3
    x = np.arange(W) + 0.5 - W / 2
    y = np.arange(H) + 0.5 - H / 2
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    a = np.minimum(0.99, o * np.exp(-0.5 * r2 / var))
    a[a < 1 / 255] = 0.0
    want = a[..., None] * np.array(col)
    np.testing.assert_allclose(img, want, rtol=0, atol=2e-6)
    assert img[0, 0].max() == 0.0                 # far corner is below the cutoff


def test_two_gaussians_front_to_back():
    W, H, f = 24, 16, 40.0
    cols = [[1, 0, 0], [0, 1, 0]]
    # same footprint, different depth: C = c1 a1 + c2 a2 (1 - a1)
    sc = _scene([[0, 0, 4], [0, 0, 8]], [[math.log(0.2)] * 3, [math.log(0.4)] * 3], [0.6, 0.5], cols)
    img, _ = _render(sc, _front_cam(W, H, f), _one_view_display(W, H))
    var = (f * 0.2 / 4) ** 2 + 0.3
    a1 = 0.6 * np.exp(-0.5 * 0.5 / var)            # pixel (12, 8) is at r^2 = 0.5
    a2 = 0.5 * np.exp(-0.5 * 0.5 / var)
    np.testing.assert_allclose(img[8, 12], [a1, a2 * (1 - a1), 0.0], atol=2e-6)
    # reversing the depths swaps the roles
    sc2 = _scene([[0, 0, 8], [0, 0, 4]], [[math.log(0.4)] * 3, [math.log(0.2)] * 3], [0.5, 0.6],
                 [cols[1], cols[0]])
    img2, _ = _render(sc2, _front_cam(W, H, f), _one_view_display(W, H))
    np.testing.assert_array_equal(img, img2)


def test_equal_depth_ties_by_index():
    W, H = 8, 8
    sc = _scene([[0, 0, 4], [0, 0, 4]], [[-1.6] * 3] * 2, [0.5, 0.5], [[1, 0, 0], [0, 1, 0]])
    img, _ = _render(sc, _front_cam(W, H), _one_view_display(W, H))
    p = img[4, 4]
    assert p[0] > p[1] > 0          # Gaussian 0 (lower index) is in front


def test_stop_rule_and_full_occlusion():
    # Four coincident splats with alpha 0.95 at the centre: T goes
    # 1 -> 0.05 -> 0.0025 -> 1.25e-4 -> 6.25e-6 < 1e-4, so the fourth stops
    # the traversal without contributing; anything behind is invisible.
    W, H = 8, 8
    z = [4.0, 4.1, 4.2, 4.3]
    cols = [[0.2, 0.2, 0.2], [0.4, 0.4, 0.4], [0.6, 0.6, 0.6], [1.0, 0.0, 0.0]]
    big = math.log(2.0)
    sc = _scene([[0, 0, zz] for zz in z], [[big] * 3] * 4, [0.95] * 4, cols)
    img, flags = _render(sc, _front_cam(W, H), _one_view_display(W, H))
    a = [0.95 * math.exp(-0.5 * 0.5 / ((40 * 2.0 / zz) ** 2 + 0.3)) for zz in z]  # nearly flat
    want = 0.2 * a[0] + 0.4 * a[1] * (1 - a[0]) + 0.6 * a[2] * (1 - a[0]) * (1 - a[1])
    # the centre pixel
    assert flags[4, 4, 0] == 0
    np.testing.assert_allclose(img[4, 4], [want] * 3, atol=2e-6)
    # add a bright splat behind: bit-identical output everywhere it is occluded
    sc2 = _scene([[0, 0, zz] for zz in z] + [[0, 0, 5.0]], [[big] * 3] * 5, [0.95] * 5,
                 cols + [[1.0, 1.0, 1.0]])
    img2, _ = _render(sc2, _front_cam(W, H), _one_view_display(W, H))
    np.testing.assert_array_equal(img2, img)


def test_sub_cutoff_gaussians_are_irrelevant(tiny):
    w, scene, cams, V = tiny
    d = DisplayParams(40, 24, 16, Rational(1, 6), Rational(23, 5))
    V = oracle.view_map(d)
    cams = pack_cameras(orbit_rig(16, 40, 24, 4.0, 30.0))
    base = scene.subset(np.arange(300))
    img, _ = _render(base, cams, d)
    rng = np.random.default_rng(0)
    extra = scene.subset(np.arange(300, 400))
    extra.opacities[:] = rng.uniform(0.0, 1.0 / 255.0 * 0.999, 100).astype(np.float32)
    both = Scene(*[np.concatenate([a, b]) for a, b in zip(base.arrays(), extra.arrays())], 0)
    img2, _ = _render(both, cams, d)
    np.testing.assert_array_equal(img, img2)


def test_transmittance_invariants(tiny):
    w, scene, cams, V = tiny
    d = DisplayParams(48, 27, 16, Rational(1, 6), Rational(23, 5))
    cams = pack_cameras(orbit_rig(16, 48, 27, 4.0, 30.0))
    sc = scene.subset(np.arange(800))
    c0, _ = _render(sc, cams, d, bg=(0, 0, 0))
    c1, _ = _render(sc, cams, d, bg=(1, 1, 1))
    T = c1.astype(np.float64) - c0                   # final transmittance
    assert (T >= -1e-6).all() and (T <= 1 + 1e-6).all()
    cmax = 0.5 + 0.5 / math.sqrt(math.pi)            # SH0 colours with DC in [0, 1]
    assert (c0 >= 0).all()
    assert (c0 <= cmax * (1 - T) + 1e-5).all()


def test_exact_path_equals_fullframe_then_interlace():
    # Subpixel rasterization reaches the full-frame-then-interlace image.
    w = get_workload("tiny")
    d = DisplayParams(40, 24, 16, Rational(1, 6), Rational(23, 5))
    scene = w.make_scene().subset(np.arange(0, 2000, 4))
    cams = pack_cameras(orbit_rig(16, 40, 24, 4.0, 30.0))
    V = oracle.view_map(d)
    sub, _, _ = oracle.render_frame(scene, cams, d, V, 1)
    ff = oracle.render_interlaced_fullframe(scene, cams, d, V)
    np.testing.assert_array_equal(sub, ff)
    assert sub.max() > 0.1


def test_reuse_is_exact_when_views_coincide():
    # With all views at one pose, sharing covariance/colour/depth inside a
    # cluster changes nothing.
    w = get_workload("tiny")
    d = DisplayParams(40, 24, 16, Rational(1, 6), Rational(23, 5))
    scene = w.make_scene().subset(np.arange(0, 2000, 4))
    cams = pack_cameras(orbit_rig(16, 40, 24, 4.0, 0.0))
    V = oracle.view_map(d)
    exact, _, _ = oracle.render_frame(scene, cams, d, V, 1)
    for S in (2, 4, 16):
        reuse, _, _ = oracle.render_frame(scene, cams, d, V, S)
        np.testing.assert_array_equal(reuse, exact)


def test_reuse_rule_single_gaussian():
    # One Gaussian: a subpixel of view j under cluster size S gets
    # c_r * min(.99, o 2^-E(mu_j, conic_r)) with r the cluster representative.
    d = DisplayParams(32, 18, 8, Rational(1, 6), Rational(23, 5))
    cams = pack_cameras(orbit_rig(8, 32, 18, 4.0, 40.0))
    sc = _scene([[0.1, 0.05, 4.0]], [[-1.7, -2.2, -1.9]], [0.8], [[0.7, 0.5, 0.3]],
                quats=[[0.8, 0.3, -0.2, 0.4]])
    V = oracle.view_map(d)
    S = 4
    _, rep = oracle.cluster_table(8, S)
    img, _, _ = oracle.render_frame(sc, cams, d, V, S)
    hits = 0
    for (y, x, u), j in np.ndenumerate(V):
        r = rep[j // S]
        pr = oracle.project(sc, cams[r], 32, 18)[0]
        pj = oracle.project(sc, cams[j], 32, 18)[0]
        dx = x + 0.5 - np.float64(pj["mean2d"][0])
        dy = y + 0.5 - np.float64(pj["mean2d"][1])
        A, b, G = (np.float64(c) for c in pr["conic"])
        a = min(0.99, np.float64(pr["opacity"]) * 2.0 ** (-(A * (dx + b * dy) ** 2 + G * dy * dy)))
        want = np.float32(pr["color"][u] * a) if np.float32(a) >= np.float32(1 / 255) else 0.0
        assert img[y, x, u] == pytest.approx(want, abs=1e-7)
        hits += want > 0
    assert hits > 20


def test_reuse_quality_falls_with_cluster_size(tiny):
    # The qualitative trend of the paper's cluster-size study: PSNR against
    # the exact path drops as clusters grow.
    w, scene, cams, V = tiny
    d = DisplayParams(64, 36, 16, Rational(1, 6), Rational(23, 5))
    cams = pack_cameras(orbit_rig(16, 64, 36, 4.0, 30.0))
    V = oracle.view_map(d)
    sc = scene.subset(np.arange(0, 2000, 2))
    exact, _, _ = oracle.render_frame(sc, cams, d, V, 1)
    psnr = []
    for S in (2, 4, 8):
        r, _, _ = oracle.render_frame(sc, cams, d, V, S)
        mse = float(np.mean((r.astype(np.float64) - exact) ** 2))
        psnr.append(10 * math.log10(1.0 / max(mse, 1e-20)))
    assert psnr[0] > psnr[1] > psnr[2]


def test_near_threshold_flagging():
    # A splat whose alpha at a pixel centre sits on 1/255 is flagged.
    W, H, f, z, s = 8, 8, 40.0, 4.0, 0.2
    var = (f * s / z) ** 2 + 0.3
    r2 = 0.5                                          # pixel (4, 4) centre
    o = (1 / 255) / math.exp(-0.5 * r2 / var)
    sc = _scene([[0, 0, z]], [[math.log(s)] * 3], [o], [[1, 1, 1]])
    _, flags = _render(sc, _front_cam(W, H, f), _one_view_display(W, H))
    assert flags[4, 4, 0] & 1
