"""Pins for the oracle's projection (section 4.1 Eq. 4, section 4.2 Eq. 5-6).

The oracle stores the inverse 2D covariance in factored form
(A', beta, G'), E = A'(dx + beta dy)^2 + G' dy^2 = (log2 e / 2) d^T Sigma2D^-1 d.
These tests rebuild Sigma2D from that form and compare it with quantities
computed by independent routes: closed forms, a numerically differentiated
pinhole, scipy's rotation and spherical-harmonic routines, and Monte Carlo.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy import special

import oracle
from workloads import Scene
from workloads.cameras import Camera

HALF_LOG2E = 0.5 / math.log(2.0)


def _scene(means, log_scales, quats, opac, sh=None, degree=0):
    m = len(means)
    if sh is None:
        sh = np.zeros((m, (degree + 1) ** 2, 3))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means), f(log_scales), f(quats), f(opac), f(sh), degree)


def _cam(R=np.eye(3), t=(0, 0, 0), f=200.0, W=256, H=144):
    return Camera(np.asarray(R, np.float32), np.asarray(t, np.float32), f, f, W / 2, H / 2).packed()


def sigma2d_from_conic(conic):
    A = np.float64(conic[0]) / HALF_LOG2E
    b = np.float64(conic[1])
    G = np.float64(conic[2]) / HALF_LOG2E
    Q = np.array([[A, A * b], [A * b, A * b * b + G]])
    return np.linalg.inv(Q)


def test_on_axis_isotropic_closed_form():
    z0, s, f = 4.0, 0.05, 200.0
    sc = _scene([[0, 0, z0]], [[math.log(s)] * 3], [[1, 0, 0, 0]], [0.8])
    p = oracle.project(sc, _cam(f=f), 256, 144)[0]
    assert p["valid"] == 1 and p["valid_mean"] == 1
    np.testing.assert_allclose(p["mean2d"], [128.0, 72.0], rtol=0, atol=1e-5)
    assert p["depth"] == np.float32(z0)
    S2 = sigma2d_from_conic(p["conic"])
    want = (f * s / z0) ** 2 + 0.3
    np.testing.assert_allclose(S2, np.diag([want, want]), rtol=2e-6, atol=2e-6)
    # SH degree 0 with a zero DC coefficient -> colour 0.5
    np.testing.assert_allclose(p["color"], [0.5] * 3, atol=1e-7)


def _pinhole(Rc, tc, f, cx, cy, X):
    Y = Rc @ X + tc
    return np.array([f * Y[0] / Y[2] + cx, f * Y[1] / Y[2] + cy])


def _num_jacobian(Rc, tc, f, cx, cy, X, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_pinhole(Rc, tc, f, cx, cy, X + e) - _pinhole(Rc, tc, f, cx, cy, X - e)) / (2 * h)
    return J


@pytest.mark.parametrize("seed", range(6))
def test_ewa_against_numerical_jacobian_and_scipy_rotation(seed):
    rng = np.random.default_rng(seed)
    f, W, H = 300.0, 320, 240
    rot = Rotation.from_euler("xyz", rng.uniform(-0.15, 0.15, 3))
    Rc = rot.as_matrix().astype(np.float32).astype(np.float64)
    tc = rng.uniform(-0.5, 0.5, 3).astype(np.float32).astype(np.float64)
    mu = np.array([rng.uniform(-1, 1), rng.uniform(-0.7, 0.7), rng.uniform(3, 6)], np.float32)
    ls = rng.normal(-2.5, 0.5, 3).astype(np.float32)
    q = rng.standard_normal(4).astype(np.float32)
    sc = _scene([mu], [ls], [q], [0.9])
    cam = Camera(Rc.astype(np.float32), tc.astype(np.float32), f, f, W / 2, H / 2).packed()
    p = oracle.project(sc, cam, W, H)[0]
    assert p["valid"] == 1
    X = mu.astype(np.float64)
    Y = Rc @ X + tc                      # keep the Jacobian clamp inactive here
    assert abs(Y[0] / Y[2]) < 1.3 * (W / 2) / f and abs(Y[1] / Y[2]) < 1.3 * (H / 2) / f
    # 2D mean: the exact pinhole
    np.testing.assert_allclose(p["mean2d"], _pinhole(Rc, tc, f, W / 2, H / 2, X), rtol=0, atol=1e-4)
    # 3D covariance via scipy (scalar-last quaternion convention)
    qw, qx, qy, qz = q.astype(np.float64) / np.linalg.norm(q.astype(np.float64))
    Rq = Rotation.from_quat([qx, qy, qz, qw]).as_matrix()
    Sig = Rq @ np.diag(np.exp(2 * ls.astype(np.float64))) @ Rq.T
    J = _num_jacobian(Rc, tc, f, W / 2, H / 2, X)        # d pixel / d world
    want = J @ Sig @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(sigma2d_from_conic(p["conic"]), want, rtol=2e-5, atol=1e-6)
    # depth = camera-space z of the mean
    assert abs(float(p["depth"]) - (Rc @ X + tc)[2]) <= 1e-6 * abs(p["depth"])


def test_ewa_monte_carlo():
    # The EWA covariance is the covariance of projected samples for a small
    # Gaussian (first-order).  Checks semantics, not just algebra.
    rng = np.random.default_rng(3)
    f, W, H = 400.0, 400, 300
    mu = np.array([0.4, -0.3, 5.0], np.float32)
    ls = np.log(np.array([0.02, 0.05, 0.01], np.float32))
    q = np.array([0.9, 0.2, -0.3, 0.1], np.float32)
    sc = _scene([mu], [ls], [q], [0.9])
    p = oracle.project(sc, _cam(f=f, W=W, H=H), W, H)[0]
    qn = q.astype(np.float64) / np.linalg.norm(q)
    Rq = Rotation.from_quat([qn[1], qn[2], qn[3], qn[0]]).as_matrix()
    z = rng.standard_normal((400_000, 3)) * np.exp(ls.astype(np.float64))
    Xs = mu.astype(np.float64) + z @ Rq.T
    px = np.stack([f * Xs[:, 0] / Xs[:, 2] + W / 2, f * Xs[:, 1] / Xs[:, 2] + H / 2], 1)
    emp = np.cov(px.T) + 0.3 * np.eye(2)
    np.testing.assert_allclose(sigma2d_from_conic(p["conic"]), emp, rtol=2e-2, atol=2e-2)


def test_jacobian_clamp_off_screen():
    # A mean far outside the frustum uses the Jacobian at the clamped
    # direction x/z = 1.3 tan(fov_x/2) (the 3DGS convention).
    f, W, H = 200.0, 256, 144
    mu = np.array([3.0, 0.1, 2.0], np.float32)      # x/z = 1.5 > 1.3*0.64
    ls = np.log(np.full(3, 0.05, np.float32))
    sc = _scene([mu], [ls], [[1, 0, 0, 0]], [0.9])
    p = oracle.project(sc, _cam(f=f, W=W, H=H), W, H)[0]
    lim = 1.3 * (W / 2) / f
    Xc = np.array([lim * 2.0, 0.1, 2.0])           # the clamped point, same depth
    J = _num_jacobian(np.eye(3), np.zeros(3), f, W / 2, H / 2, Xc)
    want = J @ np.diag(np.full(3, 0.05 ** 2)) @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(sigma2d_from_conic(p["conic"]), want, rtol=1e-5)
    np.testing.assert_allclose(p["mean2d"], [f * 1.5 + W / 2, f * 0.05 + H / 2], atol=1e-4)


def _real_sh_scipy(l, m, d):
    """Real SH with the Condon-Shortley phase built from scipy's complex SH."""
    x, y, z = d
    polar = math.acos(max(-1.0, min(1.0, z)))
    az = math.atan2(y, x)
    if hasattr(special, "sph_harm_y"):
        Y = lambda mm: special.sph_harm_y(l, mm, polar, az)
    else:
        Y = lambda mm: special.sph_harm(mm, l, az, polar)
    if m == 0:
        return Y(0).real
    if m > 0:
        return math.sqrt(2.0) * Y(m).real
    return math.sqrt(2.0) * Y(-m).imag


def test_sh_basis_against_scipy():
    rng = np.random.default_rng(11)
    for _ in range(25):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(3, d)
        want = [_real_sh_scipy(l, m, d) for l in range(4) for m in range(-l, l + 1)]
        np.testing.assert_allclose(Y, want, rtol=1e-12, atol=1e-12)


def test_sh_basis_orthonormal():
    # Gauss-Legendre in cos(polar) x uniform azimuth integrates these exactly.
    xs, ws = np.polynomial.legendre.leggauss(12)
    phis = np.linspace(0, 2 * np.pi, 24, endpoint=False)
    G = np.zeros((16, 16))
    for z, w in zip(xs, ws):
        r = math.sqrt(1 - z * z)
        for ph in phis:
            Y = oracle.sh_basis(3, np.array([r * math.cos(ph), r * math.sin(ph), z]))
            G += w * (2 * np.pi / len(phis)) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_colour_uses_view_direction():
    # Put all SH energy in the l=1, m=1 band (-c1 * x) for the red channel:
    # two cameras on either side see opposite signs.
    sh = np.zeros((1, 16, 3))
    sh[0, 3, 0] = 0.4
    sc = _scene([[0, 0, 4]], [[-3, -3, -3]], [[1, 0, 0, 0]], [0.9], sh, 3)
    c1 = math.sqrt(3 / (4 * math.pi))
    for cam_x in (-1.0, 1.0):
        Rc = np.eye(3)
        tc = -Rc @ np.array([cam_x, 0, 0])
        p = oracle.project(sc, _cam(R=Rc, t=tc), 256, 144)[0]
        d = np.array([0 - cam_x, 0, 4.0])
        d /= np.linalg.norm(d)
        want = max(0.0, -c1 * d[0] * 0.4 + 0.5)
        assert abs(p["color"][0] - want) < 1e-7
        assert abs(p["color"][1] - 0.5) < 1e-7


def test_validity_rules():
    means = [[0, 0, 4], [0, 0, -4], [0, 0, 0.1], [0, 0, 4], [0, 0, 4], [np.nan, 0, 4]]
    opac = [0.5, 0.5, 0.5, 1.0 / 255.0 * 0.999, np.float32(1.0 / 255.0), 0.5]
    sc = _scene(means, [[-3] * 3] * 6, [[1, 0, 0, 0]] * 6, opac)
    p = oracle.project(sc, _cam(), 256, 144)
    assert p["valid"].tolist() == [1, 0, 0, 0, 1, 0]
    assert p["valid_mean"].tolist() == [1, 0, 0, 1, 1, 0]
