"""Pins for the gradient oracle (oracle/lfr_oracle_grad.c): the analytic
derivative of the subpixel renderer (section 4.3 Eq. 9-10, the reuse rule of
section 4.2, the projection of Eq. 4-6) checked against

* central finite differences of the oracle's own double-precision forward, on
  a scene built so that every discrete branch occurs (alpha clamp, colour
  clamp, Jacobian clamp, transmittance stop, background), for S = 1, 2, 3;
* closed forms for an isolated isotropic Gaussian on the optical axis (EWA
  covariance diag((f s / z)^2 + 0.3)) and for two stacked Gaussians;
* invariants: q . dL/dq = 0 (only q/|q| matters), dL/dq = 0 for isotropic
  scales, linearity in the output gradient, and agreement of the double
  forward with the float32-attribute oracle."""
import math

import numpy as np
import pytest

import oracle
from workloads import DisplayParams, Rational, Scene
from workloads.cameras import Camera, orbit_rig, pack_cameras

F32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
Y0 = 0.5 / math.sqrt(math.pi)


def _branchy_scene(seed=7):
    """~45 Gaussians in front of a 24x16 panel: a random field plus groups
    that trigger each discrete branch of the renderer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = 30
    means = np.c_[rng.uniform(-0.8, 0.8, m), rng.uniform(-0.5, 0.5, m), rng.uniform(3, 5, m)]
    ls = rng.normal(-1.8, 0.4, (m, 3))
    q = rng.standard_normal((m, 4))
    o = 1.0 / (1.0 + np.exp(-rng.normal(0, 1.5, m)))
    sh = rng.normal(0, 0.2, (m, 16, 3))
    sh[:, 0] = rng.uniform(0, 1, (m, 3))
    # an opaque stack in the centre: alpha clamp and transmittance stop
    k = 8
    st_means = np.c_[rng.uniform(-0.15, 0.15, k), rng.uniform(-0.1, 0.1, k), np.linspace(2.6, 3.4, k)]
    st_ls = np.full((k, 3), math.log(0.5)) + rng.normal(0, 0.1, (k, 3))
    st_q = rng.standard_normal((k, 4))
    st_o = np.full(k, 0.999)
    st_sh = rng.normal(0, 0.2, (k, 16, 3))
    st_sh[:, 0] = rng.uniform(0, 1, (k, 3))
    # negative DC on some channels: colour clamp at 0
    neg = np.zeros((4, 16, 3))
    neg[:, 0] = [[-3.0, 0.8, 0.5], [0.5, -3.0, 0.2], [0.9, 0.9, -3.0], [-3.0, -3.0, 0.9]]
    neg_means = np.c_[rng.uniform(-0.6, 0.6, 4), rng.uniform(-0.4, 0.4, 4), rng.uniform(3.5, 4.5, 4)]
    neg_ls = rng.normal(-1.5, 0.2, (4, 3))
    neg_q = rng.standard_normal((4, 4))
    neg_o = np.full(4, 0.6)
    # large Gaussians beyond 1.3 tan(fov/2) whose footprint reaches the panel
    jc_means = np.array([[3.6, 0.0, 4.0], [-3.5, 0.3, 4.2], [0.2, 2.6, 4.0]])
    jc_ls = np.full((3, 3), 0.0)
    jc_q = rng.standard_normal((3, 4))
    jc_o = np.full(3, 0.5)
    jc_sh = rng.normal(0, 0.2, (3, 16, 3))
    jc_sh[:, 0] = rng.uniform(0, 1, (3, 3))
    cat = lambda *a: np.concatenate(a, axis=0)
    qq = cat(q, st_q, neg_q, jc_q)
    qq /= np.linalg.norm(qq, axis=1, keepdims=True)
    return Scene(F32(cat(means, st_means, neg_means, jc_means)), F32(cat(ls, st_ls, neg_ls, jc_ls)), F32(qq),
                 F32(cat(o, st_o, neg_o, jc_o)), F32(cat(sh, st_sh, neg, jc_sh)), 3)


def _branchy_setup(S):
    W, H, N = 24, 16, 5
    disp = DisplayParams(W, H, N, Rational(1, 6), Rational(5, 2))
    cams = pack_cameras(orbit_rig(N, W, H, 4.0, 20.0, centre=(0, 0, 4.0)))
    return disp, cams, oracle.view_map(disp)


def test_branchy_scene_hits_every_branch():
    sc = _branchy_scene()
    disp, cams, V = _branchy_setup(1)
    W, H = disp.width, disp.height
    n = 3 * W * H
    # colour clamp and Jacobian clamp in the centre view
    pr = oracle.project(sc, cams[2], W, H)
    assert np.any((pr["valid"] == 1) & np.any(pr["color"] == 0.0, axis=1))
    lim = 1.3 * (0.5 * W) / cams[2][12]
    R, t = cams[2][:9].reshape(3, 3).astype(np.float64), cams[2][9:12].astype(np.float64)
    cam_pts = sc.means.astype(np.float64) @ R.T + t
    ux = cam_pts[:, 0] / cam_pts[:, 2]
    uy = cam_pts[:, 1] / cam_pts[:, 2]
    off = (np.abs(ux) > lim) | (np.abs(uy) > 1.3 * (0.5 * H) / cams[2][13])
    # ... and those Gaussians do reach the panel: removing them changes it
    img = oracle.render_frame(sc, cams, disp, V, 1)[0]
    keep = np.flatnonzero(~off)
    img2 = oracle.render_frame(sc.subset(keep), cams, disp, V, 1)[0]
    assert off.sum() >= 2 and np.abs(img - img2).max() > 1e-3
    # alpha clamp and transmittance stop, on the opaque stack: some subpixel
    # sees o 2^-E > 0.99, and some subpixel of view j has >= 5 stack members
    # with alpha >= 0.9 in view j, so T would fall below 0.1^4 = 1e-4 within
    # its first five passing Gaussians: the stop rule must cut its list
    st = np.arange(30, 38)
    a_max, most = 0.0, 0
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    for j in range(disp.num_views):
        mine = np.any(V == j, axis=2)
        count = np.zeros((H, W), dtype=int)
        for g in oracle.project(sc.subset(st), cams[j], W, H):
            if not g["valid"]:
                continue
            dx, dy = xs - g["mean2d"][0], ys - g["mean2d"][1]
            w = dx + g["conic"][1] * dy
            E = g["conic"][0] * w * w + g["conic"][2] * dy * dy
            a = g["opacity"] * np.exp2(-E)
            a_max = max(a_max, float(a.max()))
            count += a >= 0.9
        most = max(most, int(count[mine].max()))
    assert a_max > 0.99
    assert most >= 5


def _fd_check(sc, disp, cams, V, S, bg, samples, gout, rel_tol=1e-5):
    val, sig, g = oracle.grad_subpixels(sc, cams, disp, V, S, samples, gout, bg=bg, mode=0)
    report = {}
    for name in oracle.GRAD_NAMES:
        base = getattr(sc, name)
        flat = base.reshape(-1)
        gflat = g[name].reshape(-1)
        gmax = float(np.abs(gflat).max())
        worst, excluded, checked = 0.0, 0, 0
        for idx in range(flat.size):
            th = float(flat[idx])
            h = 1e-6 * max(1.0, abs(th))
            tp, tm = np.float32(th + h), np.float32(th - h)
            F, same = [], True
            for tv in (tp, tm):
                arr = base.copy()
                arr.reshape(-1)[idx] = tv
                kw = {k: getattr(sc, k) for k in oracle.GRAD_NAMES}
                kw[name] = arr
                v2, s2, _ = oracle.grad_subpixels(Scene(**kw, sh_degree=sc.sh_degree), cams, disp, V, S,
                                                  samples, bg=bg, mode=0, grads=False)
                same = same and np.array_equal(s2, sig)
                F.append(float(gout @ v2))
            if not same:       # a discrete decision changed inside [th - h, th + h]
                excluded += 1
                continue
            fd = (F[0] - F[1]) / (float(tp) - float(tm))
            err = abs(fd - gflat[idx]) / max(abs(gflat[idx]), 1e-3 * gmax, 1e-30)
            worst = max(worst, err)
            checked += 1
        report[name] = (checked, excluded, worst, gmax)
    for name, (checked, excluded, worst, gmax) in report.items():
        assert gmax > 0.0, name
        assert excluded <= 0.02 * (checked + excluded), (name, report)
        assert worst <= rel_tol, (name, report)
    return report


@pytest.mark.parametrize("S", [1, 2, 3])
def test_gradient_matches_central_differences(S):
    sc = _branchy_scene()
    disp, cams, V = _branchy_setup(S)
    n = 3 * disp.width * disp.height
    rng = np.random.Generator(np.random.PCG64(100 + S))
    gout = rng.standard_normal(n)
    _fd_check(sc, disp, cams, V, S, (0.2, 0.1, 0.3), np.arange(n), gout)


def _single_view(W=24, H=16):
    return DisplayParams(W, H, 1, Rational(0), Rational(3))


def _front_cam(W, H, f):
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f, W / 2, H / 2).packed()[None]


def _iso_scene(means, scales, opac, colours, deg=0):
    m = len(means)
    sh = np.zeros((m, (deg + 1) ** 2, 3))
    sh[:, 0] = (np.asarray(colours, np.float64) - 0.5) / Y0
    return Scene(F32(means), F32(np.log(np.asarray(scales, np.float64))[:, None].repeat(3, 1)),
                 F32([[1, 0, 0, 0]] * m), F32(opac), F32(sh), deg)


def test_isotropic_on_axis_closed_form():
    W, H, f, z, s, o = 24, 16, 40.0, 4.0, 0.15, 0.7
    col = [0.9, 0.4, 0.1]
    sc = _iso_scene([[0, 0, z]], [s], [o], [col])
    # the closed form takes the parameters as stored (float32)
    s, o = math.exp(float(sc.log_scales[0, 0])), float(sc.opacities[0])
    col = [float(sc.sh[0, 0, u]) * Y0 + 0.5 for u in range(3)]
    disp = _single_view(W, H)
    V = oracle.view_map(disp)
    var = (f * s / z) ** 2 + 0.3
    for px_off, u in ((1, 0), (2, 1), (3, 2)):
        x, y = W // 2 + px_off, H // 2
        p = (y * W + x) * 3 + u
        dx = px_off + 0.5
        dy = 0.5
        a = o * math.exp(-0.5 * (dx * dx + dy * dy) / var)
        I = col[u] * a
        _, _, g = oracle.grad_subpixels(sc, _front_cam(W, H, f), disp, V, 1, [p], [1.0])
        assert g["opacities"][0] == pytest.approx(col[u] * a / o, rel=1e-9)
        # log-scale (all three axes): d var / d log s_axis; x and y see the
        # camera-plane axes only, the depth axis does not enter Sigma2D on axis
        r2 = dx * dx + dy * dy
        dvar_total = 2 * (f * s / z) ** 2
        assert g["log_scales"][0].sum() == pytest.approx(I * 0.5 * r2 / var ** 2 * dvar_total, rel=1e-7)
        assert g["log_scales"][0][2] == pytest.approx(0.0, abs=1e-12)
        # mean: the 2D mean moves by f/z per unit of world x (y), and the
        # covariance has no first-order dependence on the mean on the axis
        assert g["means"][0][0] == pytest.approx(I * dx / var * f / z, rel=1e-7)
        assert g["means"][0][1] == pytest.approx(I * dy / var * f / z, rel=1e-7)
        # depth: var depends on z through (f s / z)^2
        assert g["means"][0][2] == pytest.approx(-I * 0.5 * r2 / var ** 2 * 2 * (f * s) ** 2 / z ** 3, rel=1e-7)
        # colour DC of the sample's channel only
        want = np.zeros(3)
        want[u] = Y0 * a
        np.testing.assert_allclose(g["sh"][0, 0], want, rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(g["quats"][0], 0.0, atol=1e-12)


def test_two_stacked_gaussians_closed_form():
    W, H, f = 24, 16, 40.0
    cols = [[0.8, 0.2, 0.3], [0.1, 0.7, 0.4]]
    sc = _iso_scene([[0, 0, 4], [0, 0, 8]], [0.2, 0.4], [0.6, 0.5], cols)
    sd = [math.exp(float(v)) for v in sc.log_scales[:, 0]]
    op = [float(v) for v in sc.opacities]
    cols = [[float(sc.sh[i, 0, u]) * Y0 + 0.5 for u in range(3)] for i in range(2)]
    disp = _single_view(W, H)
    V = oracle.view_map(disp)
    bg = (0.3, 0.6, 0.9)
    x, y, u = W // 2, H // 2 + 1, 1
    p = (y * W + x) * 3 + u
    dx, dy = 0.5, 1.5
    var = [(f * sd[0] / 4) ** 2 + 0.3, (f * sd[1] / 8) ** 2 + 0.3]
    e = [math.exp(-0.5 * (dx * dx + dy * dy) / v) for v in var]
    a1, a2 = op[0] * e[0], op[1] * e[1]
    c1, c2, b = cols[0][u], cols[1][u], float(np.float32(bg[u]))
    val, _, g = oracle.grad_subpixels(sc, _front_cam(W, H, f), disp, V, 1, [p], [1.0], bg=bg)
    assert val[0] == pytest.approx(c1 * a1 + c2 * a2 * (1 - a1) + b * (1 - a1) * (1 - a2), rel=1e-12)
    dI_da1 = c1 - c2 * a2 - b * (1 - a2)
    dI_da2 = c2 * (1 - a1) - b * (1 - a1)
    assert g["opacities"][0] == pytest.approx(dI_da1 * e[0], rel=1e-9)
    assert g["opacities"][1] == pytest.approx(dI_da2 * e[1], rel=1e-9)
    assert g["sh"][0, 0, u] == pytest.approx(Y0 * a1, rel=1e-9)
    assert g["sh"][1, 0, u] == pytest.approx(Y0 * a2 * (1 - a1), rel=1e-9)


def test_quaternion_gradient_is_orthogonal_to_q_and_zero_when_isotropic():
    sc = _branchy_scene()
    disp, cams, V = _branchy_setup(1)
    n = 3 * disp.width * disp.height
    gout = np.random.Generator(np.random.PCG64(3)).standard_normal(n)
    _, _, g = oracle.grad_subpixels(sc, cams, disp, V, 1, np.arange(n), gout)
    dots = np.einsum("ij,ij->i", g["quats"], sc.quats.astype(np.float64))
    assert np.abs(dots).max() <= 1e-9 * max(1.0, np.abs(g["quats"]).max())
    iso = Scene(sc.means, F32(np.repeat(sc.log_scales[:, :1], 3, axis=1)), sc.quats, sc.opacities, sc.sh, 3)
    _, _, gi = oracle.grad_subpixels(iso, cams, disp, V, 1, np.arange(n), gout)
    assert np.abs(gi["quats"]).max() <= 1e-9 * np.abs(gi["means"]).max()


def test_linear_in_output_gradient_and_additive_over_samples():
    sc = _branchy_scene()
    disp, cams, V = _branchy_setup(2)
    n = 3 * disp.width * disp.height
    rng = np.random.Generator(np.random.PCG64(5))
    g1, g2 = rng.standard_normal(n), rng.standard_normal(n)
    all_s = np.arange(n)
    _, _, ga = oracle.grad_subpixels(sc, cams, disp, V, 2, all_s, g1)
    _, _, gb = oracle.grad_subpixels(sc, cams, disp, V, 2, all_s, g2)
    _, _, gab = oracle.grad_subpixels(sc, cams, disp, V, 2, all_s, 2.0 * g1 - 0.5 * g2)
    half = all_s[: n // 2]
    _, _, gh1 = oracle.grad_subpixels(sc, cams, disp, V, 2, half, g1[: n // 2])
    _, _, gh2 = oracle.grad_subpixels(sc, cams, disp, V, 2, all_s[n // 2:], g1[n // 2:])
    for k in oracle.GRAD_NAMES:
        scale = np.abs(ga[k]).max() + np.abs(gb[k]).max()
        np.testing.assert_allclose(gab[k], 2.0 * ga[k] - 0.5 * gb[k], rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(gh1[k] + gh2[k], ga[k], rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("S", [1, 3])
def test_double_forward_matches_float_oracle(S):
    sc = _branchy_scene()
    disp, cams, V = _branchy_setup(S)
    n = 3 * disp.width * disp.height
    bg = (0.2, 0.1, 0.3)
    ref, flags, _ = oracle.render_subpixels(sc, cams, disp, V, S, np.arange(n), bg)
    for mode in (0, 1):
        val, _, _ = oracle.grad_subpixels(sc, cams, disp, V, S, np.arange(n), bg=bg, mode=mode, grads=False)
        ok = flags == 0
        # float32 attributes vs double attributes: a few float32 ulps per term
        assert np.abs(val[ok] - ref[ok]).max() <= 2e-5
        assert ok.mean() >= 0.99


def test_decision_modes_agree_on_generic_scene():
    sc = _branchy_scene()
    disp, cams, V = _branchy_setup(1)
    n = 3 * disp.width * disp.height
    gout = np.random.Generator(np.random.PCG64(9)).standard_normal(n)
    _, _, g0 = oracle.grad_subpixels(sc, cams, disp, V, 1, np.arange(n), gout, mode=0)
    _, _, g1 = oracle.grad_subpixels(sc, cams, disp, V, 1, np.arange(n), gout, mode=1)
    for k in oracle.GRAD_NAMES:
        rel = np.linalg.norm(g0[k] - g1[k]) / np.linalg.norm(g0[k])
        assert rel <= 1e-4, (k, rel)


def test_mse_gradient_on_the_500_gaussian_subset_matches_central_differences():
    """The differentiable configuration's loss on its finite-difference
    subset: 500 Gaussians drawn like the 200k-Gaussian display scene (SH3),
    64x36 panel, 45 views over 40 degrees, exact path; L = mean over the
    subpixels of (I - I*)^2 with I* rendered from the same scene with means +
    N(0, 0.01).  Central differences of L itself (double forward, decisions
    on the double values) at 16 sampled parameters of every group."""
    from workloads import perturb_means
    from workloads.configs import grad_subset

    sc, disp, rig = grad_subset()
    cams = pack_cameras(rig)
    V = oracle.view_map(disp)
    n = 3 * disp.width * disp.height
    samples = np.arange(n)
    target, _, _ = oracle.grad_subpixels(perturb_means(sc, seed=505, std=0.01), cams, disp, V, 1, samples,
                                         mode=0, grads=False)

    def loss(scene):
        v, s, _ = oracle.grad_subpixels(scene, cams, disp, V, 1, samples, mode=0, grads=False)
        return float(np.mean((v - target) ** 2)), s

    val, sig, g = oracle.grad_subpixels(sc, cams, disp, V, 1, samples, mode=0, grads=False)
    gout = 2.0 * (val - target) / n
    _, sig, g = oracle.grad_subpixels(sc, cams, disp, V, 1, samples, gout, mode=0)
    rng = np.random.Generator(np.random.PCG64(77))
    report = {}
    for name in oracle.GRAD_NAMES:
        base = getattr(sc, name)
        gflat = g[name].reshape(-1)
        gmax = float(np.abs(gflat).max())
        live = np.flatnonzero(np.abs(gflat) > 1e-3 * gmax)
        picks = rng.choice(live, min(16, live.size), replace=False)
        worst, excluded = 0.0, 0
        for idx in picks:
            th = float(base.reshape(-1)[idx])
            h = 1e-6 * max(1.0, abs(th))
            tp, tm = np.float32(th + h), np.float32(th - h)
            Ls, same = [], True
            for tv in (tp, tm):
                arr = base.copy()
                arr.reshape(-1)[idx] = tv
                kw = {k: getattr(sc, k) for k in oracle.GRAD_NAMES}
                kw[name] = arr
                L, s2 = loss(Scene(**kw, sh_degree=sc.sh_degree))
                same = same and np.array_equal(s2, sig)
                Ls.append(L)
            if not same:
                excluded += 1
                continue
            fd = (Ls[0] - Ls[1]) / (float(tp) - float(tm))
            worst = max(worst, abs(fd - gflat[idx]) / max(abs(gflat[idx]), 1e-3 * gmax))
        report[name] = (len(picks), excluded, worst)
    print("FD on the 500-Gaussian subset (checked, excluded, worst relative error):", report)
    for name, (checked, excluded, worst) in report.items():
        assert checked >= 8 and excluded <= 1, (name, report)
        assert worst <= 1e-5, (name, report)
