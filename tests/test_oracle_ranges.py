"""Pins for the oracle's host threading and for its near-threshold handling
(section 4.3 Eq. 10: alpha cutoff 1/255, clamp 0.99, stop when the
transmittance would fall below 1e-4).

* Threads: every parallel loop splits independent items, so the output of
  1, 3 and 8 threads must be bit-identical.
* Flags: a built-up stack whose T' lands just inside / just outside the
  float32 error band around 1e-4 is flagged (bit 1) / not flagged, and the
  stop itself falls where the closed form puts it.
* Admissible ranges: an independent float32 blend (written here in numpy,
  in two evaluation orders) must land inside [lo, hi] for every sample, and
  where the oracle flags nothing it must equal the oracle's value; stacks
  are built so that alphas sit near 1/255 and T' near 1e-4 on purpose.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import DisplayParams, Rational, Scene, get_workload
from workloads.cameras import Camera, orbit_rig, pack_cameras

F32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
C0 = 0.5 / math.sqrt(math.pi)


def _one_view(W, H):
    return DisplayParams(W, H, 1, Rational(0), Rational(3))


def _front_cam(W, H, f=40.0):
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f, W / 2, H / 2).packed()[None]


def _scene(means, log_scales, opac, colours, quats=None):
    m = len(means)
    sh = ((np.asarray(colours, np.float64) - 0.5) / C0).reshape(m, 1, 3)
    if quats is None:
        quats = [[1, 0, 0, 0]] * m
    return Scene(F32(means), F32(log_scales), F32(quats), F32(opac), F32(sh), 0)


# --------------------------------------------------------------------------
# threads
# --------------------------------------------------------------------------

def test_threads_are_bit_identical():
    w = get_workload("tiny")
    scene = w.make_scene()
    cams = pack_cameras(w.cameras())
    V = oracle.view_map(w.display)
    rng = np.random.default_rng(4)
    samples = np.sort(rng.choice(V.size, 3000, replace=False))
    runs = []
    for n in (1, 3, 8):
        with oracle.threads(n):
            assert oracle.get_threads() == n
            r = oracle.render_subpixels_ranged(scene, cams, w.display, V, 4, samples)
            img, fl, tf = oracle.render_view(scene, cams[5], 96, 54)
            pr = oracle.project(scene, cams[3], w.display.width, w.display.height)
        runs.append((r, img, fl, tf, pr))
    assert oracle.get_threads() == 1
    for r, img, fl, tf, pr in runs[1:]:
        for k in r:
            np.testing.assert_array_equal(r[k], runs[0][0][k])
        np.testing.assert_array_equal(img, runs[0][1])
        np.testing.assert_array_equal(fl, runs[0][2])
        np.testing.assert_array_equal(tf, runs[0][3])
        assert pr.tobytes() == runs[0][4].tobytes()
    # the plain entry point gives the main walk of the ranged one
    out, flags, tflag = oracle.render_subpixels(scene, cams, w.display, V, 4, samples)
    np.testing.assert_array_equal(out, runs[0][0]["out"])
    np.testing.assert_array_equal(flags, runs[0][0]["flags"])
    np.testing.assert_array_equal(tflag, runs[0][0]["tflag"])


# --------------------------------------------------------------------------
# the transmittance-stop flag (bit 1) on a constructed stack
# --------------------------------------------------------------------------

def _centre_stack(opacities, W=8, H=8, f=40.0):
    """Coincident flat splats whose means project exactly onto the centre of
    pixel (W/2, H/2): there E = 0, so alpha equals the opacity exactly.
    Colours differ per splat so every contribution is visible."""
    k = len(opacities)
    z = 4.0 + 0.1 * np.arange(k)
    # pixel centre (x + 0.5) at cx = W/2: X / Z * f = 0.5
    means = [[0.5 * zz / f, 0.5 * zz / f, zz] for zz in z]
    cols = [[0.1 + 0.8 * (i % 5) / 4.0, 0.9 - 0.2 * (i % 4), 0.3 + 0.1 * (i % 3)] for i in range(k)]
    sc = _scene(means, [[math.log(2.0)] * 3] * k, opacities, cols)
    pr = oracle.project(sc, _front_cam(W, H, f)[0], W, H)
    assert (pr["mean2d"] == np.float32(W / 2 + 0.5)).all()
    return sc, pr


def _stack_with_last_T(front, rel):
    """Opacities: `front`, then one splat whose alpha puts T' at
    1e-4 * (1 + rel) exactly in double arithmetic (if representable)."""
    a = [float(np.float32(v)) for v in front]
    T = 1.0
    for v in a:
        T = T * (1.0 - v)
    last = float(np.float32(1.0 - 1e-4 * (1.0 + rel) / T))
    return a + [last], T, T * (1.0 - last)


@pytest.mark.parametrize("rel,inside", [(1e-6, True), (-1e-6, True), (1e-3, False), (-1e-3, False)])
def test_transmittance_stop_flag_inside_and_outside(rel, inside):
    W = H = 8
    ops, T_before, Tn = _stack_with_last_T([0.9, 0.9, 0.9], rel)
    # float32 rounding of the last opacity moves T' by at most ~1e-6 relative
    assert abs(Tn / 1e-4 - 1 - rel) <= 2e-6
    sc, pr = _centre_stack(ops + [0.5])            # a fifth splat behind
    V = oracle.view_map(_one_view(W, H))
    p = ((H // 2) * W + W // 2) * 3 + 1
    r = oracle.render_subpixels_ranged(sc, _front_cam(W, H), _one_view(W, H), V, 1, [p])
    col = pr["color"][:, 1].astype(np.float64)
    a = np.array(ops + [0.5], np.float64)
    # closed form of Eq. 9-10 with the stop: contributions while T' >= 1e-4
    C, T = 0.0, 1.0
    for i in range(len(a)):
        Tn_i = T * (1.0 - a[i])
        if np.float32(Tn_i) < np.float32(1e-4):
            break
        C += col[i] * a[i] * T
        T = Tn_i
    assert r["out"][0] == pytest.approx(C, abs=1e-6)
    if inside:
        assert r["flags"][0] & 2
        assert r["tflag"][0] == pytest.approx(T_before, rel=1e-12)
        # both outcomes of the stop are admissible: the range spans them
        stop_val = sum(col[i] * a[i] * np.prod(1 - a[:i]) for i in range(3))
        go_on = stop_val + col[3] * a[3] * T_before   # the 5th would then stop (T < 1e-4 * 0.5)
        assert r["paths"][0] == 2
        assert r["lo"][0] == pytest.approx(min(stop_val, go_on), abs=1e-6)
        assert r["hi"][0] == pytest.approx(max(stop_val, go_on), abs=1e-6)
    else:
        assert r["flags"][0] == 0
        assert r["paths"][0] == 1 and r["lo"][0] == r["hi"][0] == r["out"][0]
    # rel > 0: the fourth splat is blended (T' >= 1e-4); rel < 0: it stops
    blended_fourth = C > sum(col[i] * a[i] * np.prod(1 - a[:i]) for i in range(3)) + 1e-9
    assert blended_fourth == (rel > 0)


def test_alpha_cutoff_flag_spans_both_outcomes():
    # one splat whose alpha at the centre pixel is 1/255 (E = 0): flagged,
    # and the range holds 0 (skipped) and c * alpha (blended)
    W = H = 8
    o = float(np.float32(1.0 / 255.0))
    sc, pr = _centre_stack([o])
    V = oracle.view_map(_one_view(W, H))
    p = ((H // 2) * W + W // 2) * 3
    r = oracle.render_subpixels_ranged(sc, _front_cam(W, H), _one_view(W, H), V, 1, [p])
    assert r["flags"][0] & 1 and r["paths"][0] == 2
    c = float(pr["color"][0, 0])
    assert r["lo"][0] == 0.0
    assert r["hi"][0] == pytest.approx(c * o, rel=1e-6)


def test_path_limit_is_reported():
    # eight splats each at alpha = 1/255 at the centre: 2^8 outcomes, more
    # than the 64-leaf limit; the range is marked incomplete (paths < 0)
    W = H = 8
    o = float(np.float32(1.0 / 255.0))
    sc, _ = _centre_stack([o] * 8)
    V = oracle.view_map(_one_view(W, H))
    p = ((H // 2) * W + W // 2) * 3
    r = oracle.render_subpixels_ranged(sc, _front_cam(W, H), _one_view(W, H), V, 1, [p])
    assert r["paths"][0] < 0
    assert r["lo"][0] <= r["out"][0] <= r["hi"][0]


# --------------------------------------------------------------------------
# an independent float32 blend lands inside the admissible range
# --------------------------------------------------------------------------

def _f32_blend(recs, order, px, py, u, fused):
    """Front-to-back blend of Eq. 9-10 evaluated in float32 from the float32
    records: alpha = o 2^-E with E = A'(dx + beta dy)^2 + G' dy^2, cutoff
    1/255 and stop 1e-4 decided in float32.  `fused` evaluates E and the
    colour update with one rounding each (as fused multiply-adds would),
    otherwise every operation rounds."""
    f = np.float32
    T, C = f(1.0), f(0.0)
    amin, tstop = f(1.0) / f(255.0), f(1e-4)
    for i in order:
        g = recs[i]
        if not g["valid_mean"]:
            continue
        dx = f(f(px) - g["mean2d"][0])
        dy = f(f(py) - g["mean2d"][1])
        A, b, G = g["conic"]
        if fused:
            w = f(np.float64(dx) + np.float64(b) * np.float64(dy))
            E = f(np.float64(A) * np.float64(w) * np.float64(w) + np.float64(G) * np.float64(dy) * np.float64(dy))
            a = f(np.float64(g["opacity"]) * np.exp2(-np.float64(E)))
        else:
            w = f(dx + f(b * dy))
            E = f(f(A * f(w * w)) + f(G * f(dy * dy)))
            a = f(g["opacity"] * np.exp2(-E, dtype=np.float32))
        a = min(a, f(0.99))
        if a < amin:
            continue
        Tn = f(T * f(f(1.0) - a))
        if Tn < tstop:
            break
        if fused:
            C = f(np.float64(C) + np.float64(g["color"][u]) * np.float64(f(a * T)))
        else:
            C = f(C + f(g["color"][u] * f(a * T)))
        T = Tn
    return float(C)


def _adversarial_stacks(seed, n_cases, W=6, H=6, f=30.0):
    """Stacks of 3..9 random anisotropic splats near the centre of a 6x6
    single-view panel whose opacities are chosen (from the projected
    records) so that at the centre pixel some alphas sit within a few 1e-6 of
    1/255 and the final T' within a few 1e-6 of 1e-4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cam = _front_cam(W, H, f)[0]
    cx = cy = W / 2 + 0.5                               # centre of pixel (3, 3)
    for _ in range(n_cases):
        k = int(rng.integers(3, 10))
        z = 3.0 + 0.05 * np.arange(k) + rng.uniform(0, 0.01, k)
        off = rng.uniform(-0.8, 0.8, (k, 2))            # pixels from the centre
        means = np.c_[(W / 2 + 0.5 + off[:, 0] - W / 2) * z / f, (H / 2 + 0.5 + off[:, 1] - H / 2) * z / f, z]
        ls = rng.uniform(-3.5, -2.0, (k, 3))
        q = rng.standard_normal((k, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        cols = rng.uniform(0.1, 1.0, (k, 3))
        opac = np.full(k, 0.5)
        sc = _scene(means, ls, opac, cols, quats=q)
        pr = oracle.project(sc, cam, W, H)
        dx = cx - pr["mean2d"][:, 0].astype(np.float64)
        dy = cy - pr["mean2d"][:, 1].astype(np.float64)
        A, b, G = (pr["conic"][:, c].astype(np.float64) for c in range(3))
        E = A * (dx + b * dy) ** 2 + G * dy ** 2
        kind = rng.integers(0, 3, k)                    # 0: near cutoff, 1: opaque, 2: random
        o = np.where(kind == 0, (1 / 255) * np.exp2(E) * (1 + rng.uniform(-4e-6, 4e-6, k)),
                     np.where(kind == 1, 0.9 * np.exp2(E), rng.uniform(0.05, 0.9, k)))
        o = np.clip(o, 1 / 255 * 1.0001, 0.999)
        # the last splat puts T' near 1e-4 when the stack is deep enough
        a = np.minimum(0.99, o * np.exp2(-E))
        T = np.prod(np.where(a >= 1 / 255, 1 - a, 1.0)[:-1])
        if 1e-4 / 0.99 < T < 1e-2:
            want = 1 - 1e-4 * (1 + rng.uniform(-4e-6, 4e-6)) / T
            o[-1] = min(0.999, want * np.exp2(E[-1]))
        yield Scene(sc.means, sc.log_scales, sc.quats, F32(o), sc.sh, 0), cam


def test_float32_blend_lies_in_the_admissible_range():
    W = H = 6
    disp = _one_view(W, H)
    V = oracle.view_map(disp)
    samples = np.arange(V.size)
    stats = {"flagged": 0, "outside_main": 0, "checked": 0}
    for sc, cam in _adversarial_stacks(11, 150):
        r = oracle.render_subpixels_ranged(sc, cam[None], disp, V, 1, samples)
        recs = oracle.project(sc, cam, W, H)
        order = sorted(range(sc.num_gaussians), key=lambda i: (recs[i]["depth"], i))
        order = [i for i in order if recs[i]["valid"]]
        assert (r["lo"] <= r["out"]).all() and (r["out"] <= r["hi"]).all()
        assert (r["paths"] > 0).all()
        plain = r["flags"] == 0
        assert (r["lo"][plain] == r["out"][plain]).all() and (r["hi"][plain] == r["out"][plain]).all()
        for s in samples:
            pix, u = divmod(int(s), 3)
            px, py = pix % W + 0.5, pix // W + 0.5
            for fused in (False, True):
                v = _f32_blend(recs, order, px, py, u, fused)
                assert r["lo"][s] - 2e-5 <= v <= r["hi"][s] + 2e-5, (s, v, r["lo"][s], r["hi"][s], r["flags"][s])
                if plain[s]:
                    assert abs(v - r["out"][s]) <= 2e-5
                elif abs(v - r["out"][s]) > 2e-5:
                    stats["outside_main"] += 1
                stats["checked"] += 1
        stats["flagged"] += int((~plain).sum())
    # the construction does exercise the branches: many flagged samples, and
    # float32 values that only the alternative outcomes explain
    assert stats["flagged"] >= 100, stats
    assert stats["outside_main"] >= 5, stats


# --------------------------------------------------------------------------
# a rotated anisotropic splat against the EWA Gaussian built independently
# --------------------------------------------------------------------------

def test_rotated_anisotropic_splat_closed_form():
    from scipy.spatial.transform import Rotation

    W, H = 64, 40
    cams = orbit_rig(5, W, H, 3.0, 40.0, 60.0, centre=(0.0, 0.0, 3.0))
    cam = cams[4]                                      # rotated by +20 degrees
    q = np.array([0.90, 0.12, -0.08, 0.42])
    q /= np.linalg.norm(q)
    mu = np.array([0.12, -0.05, 3.1])
    ls = np.array([-1.3, -3.4, -2.9])
    o, col = 0.93, [0.8, 0.35, 0.6]
    sc = _scene([mu], [ls], [o], [col], quats=[q])
    img, flags, _ = oracle.render_frame(sc, cam.packed()[None], _one_view(W, H), oracle.view_map(_one_view(W, H)), 1)
    # independent construction in float64 from the float32 parameters
    mu, ls, q, o = (sc.means[0].astype(np.float64), sc.log_scales[0].astype(np.float64),
                    sc.quats[0].astype(np.float64), float(sc.opacities[0]))
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Sig3 = Rq @ np.diag(np.exp(2 * ls)) @ Rq.T
    Rc, tc = cam.R.astype(np.float64), cam.t.astype(np.float64)
    X, Y, Z = Rc @ mu + tc
    fx, fy, cx, cy = (float(v) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    J = np.array([[fx / Z, 0.0, -fx * X / Z ** 2], [0.0, fy / Z, -fy * Y / Z ** 2]])
    Sig2 = J @ Rc @ Sig3 @ Rc.T @ J.T + 0.3 * np.eye(2)
    assert abs(X / Z) < 1.3 * (W / 2) / fx and abs(Y / Z) < 1.3 * (H / 2) / fy   # Jacobian clamp inactive
    m2 = np.array([fx * X / Z + cx, fy * Y / Z + cy])
    Qi = np.linalg.inv(Sig2)
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    d = np.stack([xs - m2[0], ys - m2[1]], -1)
    a = o * np.exp(-0.5 * np.einsum("...i,ij,...j->...", d, Qi, d))
    a = np.minimum(a, 0.99)
    c = np.array([float(sc.sh[0, 0, u]) * C0 + 0.5 for u in range(3)])
    want = np.where(a[..., None] >= 1 / 255, a[..., None] * c, 0.0)
    near = np.abs(a - 1 / 255) <= 1e-5 / 255
    ok = ~near[..., None].repeat(3, -1)
    np.testing.assert_allclose(img[ok], want[ok], rtol=0, atol=2e-6)
    # the splat is anisotropic and rotated: its ellipse axes are not the
    # pixel axes, and it covers a good part of the panel
    ev, evec = np.linalg.eigh(Sig2)
    assert ev[1] / ev[0] > 4 and abs(evec[0, 1]) > 0.2
    assert (want[..., 0] > 0).sum() > 100
