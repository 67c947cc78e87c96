"""CPU oracle for the subpixel-level light-field Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  A plain, slow C implementation (``lfr_oracle.c``)
of what the method computes, written from the paper, plus this ctypes
wrapper.  It is single-threaded unless :func:`set_threads` asks for more;
its parallel loops split independent items, so results are bit-identical for
any thread count.  It shares no code with the HIP library.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.

Functions and the passages they follow:

* :func:`view_map`        -- section 3.1, Eq. 1-3
* :func:`cluster_table`   -- appendix B.1
* :func:`remap`           -- section 4.3, Eq. 8
* :func:`project`         -- section 4.1 Eq. 4; section 4.2 Eq. 5-6
* :func:`render_subpixels`-- section 4.3 Eq. 9-10 with the reuse rule of 4.2
* :func:`render_subpixels_ranged` -- the same, plus the range of values a
  float32 renderer may reach when near-threshold decisions go either way
* :func:`render_view`     -- section 3.3 (standard full-frame blend)
* :func:`render_interlaced_fullframe` -- render every view, then sample the
  subpixel each view owns (the full-frame-then-interlace definition)
* :func:`grad_subpixels`  -- the same renderer in double precision and its
  analytic derivative (chain rule through Eq. 9-10, 4.2, Eq. 4-6)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("lfr_oracle.c", "lfr_oracle_grad.c")]
_DEPS = _SRCS + [os.path.join(_HERE, f) for f in ("lfr_oracle.h", "lfr_oracle_impl.h")]
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None

PROJ_DTYPE = np.dtype([
    ("mean2d", np.float32, 2), ("conic", np.float32, 3), ("depth", np.float32),
    ("color", np.float32, 3), ("opacity", np.float32), ("valid", np.int32),
    ("valid_mean", np.int32),
])
assert PROJ_DTYPE.itemsize == 48


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction) into ``_build/``."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _DEPS):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            P = ctypes.c_void_p
            i32, i64 = ctypes.c_int32, ctypes.c_int64
            lib.orc_view_map.argtypes = [i32, i32, i32, i64, i64, i64, i64, i64, i64, P]
            lib.orc_view_map.restype = ctypes.c_int
            lib.orc_cluster_table.argtypes = [i32, i32, P, P]
            lib.orc_cluster_table.restype = i32
            lib.orc_remap.argtypes = [i32, i32, i32, i32, P, P]
            lib.orc_remap.restype = ctypes.c_int
            lib.orc_project.argtypes = [i64, i32, P, P, P, P, P, P, i32, i32, P]
            lib.orc_project.restype = None
            lib.orc_sh_basis.argtypes = [i32, P, P]
            lib.orc_sh_basis.restype = None
            lib.orc_render_subpixels.argtypes = [i64, i32, P, P, P, P, P, P, i32, P, i32, i32, i32,
                                                 P, i64, P, P, P, P]
            lib.orc_render_subpixels.restype = ctypes.c_int
            lib.orc_render_subpixels_ex.argtypes = [i64, i32, P, P, P, P, P, P, i32, P, i32, i32, i32,
                                                    P, i64, P, P, P, P, P, P, P]
            lib.orc_render_subpixels_ex.restype = ctypes.c_int
            lib.orc_set_threads.argtypes = [i32]
            lib.orc_set_threads.restype = None
            lib.orc_get_threads.argtypes = []
            lib.orc_get_threads.restype = i32
            lib.orc_render_view.argtypes = [i64, i32, P, P, P, P, P, P, i32, i32, P, P, P, P]
            lib.orc_render_view.restype = None
            lib.orc_grad_subpixels.argtypes = [i64, i32, P, P, P, P, P, P, i32, P, i32, i32, i32, P,
                                               i64, P, P, i32, P, P, P, P, P, P, P]
            lib.orc_grad_subpixels.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def view_map(display) -> np.ndarray:
    """[H, W, 3] int32 view index of every subpixel (Eq. 1-3)."""
    d = display
    V = np.empty((d.height, d.width, 3), dtype=np.int32)
    rc = _load().orc_view_map(d.width, d.height, d.num_views, d.tan_slant.num, d.tan_slant.den,
                              d.pitch.num, d.pitch.den, d.offset.num, d.offset.den, _ptr(V))
    if rc != 0:
        raise ValueError("invalid display parameters")
    return V


def cluster_table(num_views: int, cluster_size: int):
    K = (num_views + cluster_size - 1) // cluster_size
    slots = np.empty((K, cluster_size), dtype=np.int32)
    rep = np.empty(K, dtype=np.int32)
    k = _load().orc_cluster_table(num_views, cluster_size, _ptr(slots), _ptr(rep))
    if k < 0:
        raise ValueError("invalid cluster arguments")
    return slots, rep


def remap(display, V=None) -> np.ndarray:
    d = display
    if V is None:
        V = view_map(d)
    V = np.ascontiguousarray(V, dtype=np.int32)
    psi = np.empty(3 * d.width * d.height, dtype=np.uint32)
    rc = _load().orc_remap(d.width, d.height, d.tile_w, d.tile_h, _ptr(V), _ptr(psi))
    if rc != 0:
        raise ValueError("invalid remap arguments")
    return psi


def _scene_args(scene):
    arrs = [_f32(a) for a in scene.arrays()]
    return arrs, [_ptr(a) for a in arrs]


def project(scene, cam_packed, width: int, height: int) -> np.ndarray:
    arrs, ptrs = _scene_args(scene)
    cam = _f32(cam_packed)
    out = np.empty(scene.num_gaussians, dtype=PROJ_DTYPE)
    _load().orc_project(scene.num_gaussians, scene.sh_degree, *ptrs, _ptr(cam), width, height,
                        _ptr(out))
    return out


def sh_basis(degree: int, direction) -> np.ndarray:
    d = np.ascontiguousarray(direction, dtype=np.float64)
    out = np.zeros(16, dtype=np.float64)
    _load().orc_sh_basis(degree, _ptr(d), _ptr(out))
    return out[: (degree + 1) ** 2]


def render_subpixels(scene, cams_packed, display, V, cluster_size, samples, bg=(0.0, 0.0, 0.0)):
    """Render the given panel-linear subpixels.  Returns (values, flags, tflag)."""
    arrs, ptrs = _scene_args(scene)
    cams = _f32(cams_packed).reshape(-1, 16)
    V = np.ascontiguousarray(V, dtype=np.int32)
    samples = np.ascontiguousarray(samples, dtype=np.int64)
    bgv = _f32(bg)
    n = samples.shape[0]
    out = np.empty(n, dtype=np.float32)
    flags = np.empty(n, dtype=np.int32)
    tflag = np.empty(n, dtype=np.float64)
    rc = _load().orc_render_subpixels(scene.num_gaussians, scene.sh_degree, *ptrs, _ptr(cams),
                                      cams.shape[0], _ptr(V), display.width, display.height,
                                      cluster_size, _ptr(bgv), n, _ptr(samples), _ptr(out),
                                      _ptr(flags), _ptr(tflag))
    if rc != 0:
        raise ValueError("invalid render arguments")
    return out, flags, tflag


def render_subpixels_ranged(scene, cams_packed, display, V, cluster_size, samples, bg=(0.0, 0.0, 0.0)):
    """:func:`render_subpixels` plus the admissible range of every sample.

    Returns a dict with ``out``, ``flags``, ``tflag`` (as render_subpixels),
    ``lo`` / ``hi`` (float32: the smallest and largest value over every way
    the flagged near-threshold decisions can go; equal to ``out`` when
    nothing is flagged) and ``paths`` (leaves explored; negative when the
    64-leaf limit cut some branch off, in which case the range is
    incomplete)."""
    arrs, ptrs = _scene_args(scene)
    cams = _f32(cams_packed).reshape(-1, 16)
    V = np.ascontiguousarray(V, dtype=np.int32)
    samples = np.ascontiguousarray(samples, dtype=np.int64)
    bgv = _f32(bg)
    n = samples.shape[0]
    r = {"out": np.empty(n, np.float32), "flags": np.empty(n, np.int32), "tflag": np.empty(n, np.float64),
         "lo": np.empty(n, np.float32), "hi": np.empty(n, np.float32), "paths": np.empty(n, np.int32)}
    rc = _load().orc_render_subpixels_ex(scene.num_gaussians, scene.sh_degree, *ptrs, _ptr(cams),
                                         cams.shape[0], _ptr(V), display.width, display.height,
                                         cluster_size, _ptr(bgv), n, _ptr(samples),
                                         *[_ptr(r[k]) for k in ("out", "flags", "tflag", "lo", "hi", "paths")])
    if rc != 0:
        raise ValueError("invalid render arguments")
    return r


def set_threads(n: int) -> int:
    """Host threads for the oracle's parallel loops; returns the previous count."""
    lib = _load()
    prev = lib.orc_get_threads()
    lib.orc_set_threads(int(n))
    return prev


def get_threads() -> int:
    return _load().orc_get_threads()


def host_threads() -> int:
    """The host threads a run may use: OMP_NUM_THREADS when set (the GPU
    hosts set it to the CPU share of one GPU), else the visible cores, at
    most 16."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class threads:
    """Context manager: run the oracle on n host threads inside the block."""

    def __init__(self, n: int | None = None):
        self.n = host_threads() if n is None else n
        self.prev = None

    def __enter__(self):
        self.prev = set_threads(self.n)
        return self

    def __exit__(self, *exc):
        set_threads(self.prev)
        return False


def render_frame(scene, cams_packed, display, V, cluster_size, bg=(0.0, 0.0, 0.0)):
    """Every subpixel of the panel, as an [H, W, 3] image (plus flags, tflag)."""
    n = 3 * display.width * display.height
    out, flags, tflag = render_subpixels(scene, cams_packed, display, V, cluster_size,
                                         np.arange(n, dtype=np.int64), bg)
    shp = (display.height, display.width, 3)
    return out.reshape(shp), flags.reshape(shp), tflag.reshape(shp)


def render_frame_ranged(scene, cams_packed, display, V, cluster_size, bg=(0.0, 0.0, 0.0)):
    """:func:`render_subpixels_ranged` over every subpixel; each entry of the
    returned dict has shape [H, W, 3]."""
    n = 3 * display.width * display.height
    r = render_subpixels_ranged(scene, cams_packed, display, V, cluster_size, np.arange(n, dtype=np.int64), bg)
    shp = (display.height, display.width, 3)
    return {k: v.reshape(shp) for k, v in r.items()}


def render_view(scene, cam_packed, width, height, bg=(0.0, 0.0, 0.0)):
    arrs, ptrs = _scene_args(scene)
    cam = _f32(cam_packed)
    bgv = _f32(bg)
    img = np.empty((height, width, 3), dtype=np.float32)
    flags = np.empty((height, width), dtype=np.int32)
    tflag = np.empty((height, width), dtype=np.float64)
    _load().orc_render_view(scene.num_gaussians, scene.sh_degree, *ptrs, _ptr(cam), width, height,
                            _ptr(bgv), _ptr(img), _ptr(flags), _ptr(tflag))
    return img, flags, tflag


def render_interlaced_fullframe(scene, cams_packed, display, V, bg=(0.0, 0.0, 0.0)):
    """Full-frame-then-interlace: render each referenced view, then take
    I_LF[y, x, u] = I_{V[y,x,u]}[y, x, u]."""
    cams = _f32(cams_packed).reshape(-1, 16)
    out = np.empty((display.height, display.width, 3), dtype=np.float32)
    for j in np.unique(V):
        img, _, _ = render_view(scene, cams[j], display.width, display.height, bg)
        mask = V == j
        out[mask] = img[mask]
    return out


GRAD_NAMES = ("means", "log_scales", "quats", "opacities", "sh")


def grad_subpixels(scene, cams_packed, display, V, cluster_size, samples, gout=None,
                   bg=(0.0, 0.0, 0.0), mode=1, grads=True):
    """Double-precision values of the given subpixels and, with ``grads``,
    the derivative of sum(gout * values) with respect to every scene
    parameter.  Returns (values [n] f64, signatures [n] u64, grads dict or
    None).  ``mode`` 1 takes the discrete decisions like
    :func:`render_subpixels`, 0 on the double values."""
    arrs, ptrs = _scene_args(scene)
    cams = _f32(cams_packed).reshape(-1, 16)
    V = np.ascontiguousarray(V, dtype=np.int32)
    samples = np.ascontiguousarray(samples, dtype=np.int64)
    n = samples.shape[0]
    bgv = _f32(bg)
    out = np.empty(n, dtype=np.float64)
    sig = np.empty(n, dtype=np.uint64)
    g = None
    gp = [None] * 5
    if grads:
        gv = np.ascontiguousarray(gout if gout is not None else np.ones(n), dtype=np.float64)
        if gv.shape != (n,):
            raise ValueError("gout must have one entry per sample")
        g = {k: np.empty(a.shape, dtype=np.float64) for k, a in zip(GRAD_NAMES, arrs)}
        gp = [_ptr(g[k]) for k in GRAD_NAMES]
    else:
        gv = None
    rc = _load().orc_grad_subpixels(scene.num_gaussians, scene.sh_degree, *ptrs, _ptr(cams), cams.shape[0],
                                    _ptr(V), display.width, display.height, cluster_size, _ptr(bgv), n,
                                    _ptr(samples), _ptr(gv), mode, _ptr(out), _ptr(sig), *gp)
    if rc != 0:
        raise ValueError("invalid gradient-oracle arguments")
    return out, sig, g
