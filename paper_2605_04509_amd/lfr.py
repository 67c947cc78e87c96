"""ctypes binding of liblfr (include/lfr.h).

The functions named ``lfr_*`` mirror the C entry points one to one and only
marshal arguments; every step of rendering runs in the HIP library.  The
small classes below (:class:`Context`, :class:`Display`, :func:`render`, ...)
wrap them for torch tensors: PyTorch supplies device memory and the stream,
nothing else.  Importing this module does not load the library; the first
call does, and raises if ``liblfr.so`` has not been built
(``python -m paper_2605_04509_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
import threading
from ctypes import POINTER, Structure, c_char_p, c_float, c_int32, c_int64, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblfr.so")

LFR_OK = 0
LFR_ERR_INVALID_ARG = -1
LFR_ERR_OUT_OF_MEMORY = -2
LFR_ERR_HIP = -3
LFR_ERR_CAPACITY = -4
LFR_ERR_UNSUPPORTED = -5

LFR_REMAP = 1
LFR_CULL_UNREFERENCED = 2
LFR_TIMING = 4
LFR_SAVE_FOR_BACKWARD = 8
LFR_COUNT_WORK = 16


class lfr_rational(Structure):
    _fields_ = [("num", c_int64), ("den", c_int64)]


class lfr_display_desc(Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("num_views", c_int32),
                ("tan_slant", lfr_rational), ("pitch", lfr_rational), ("offset", lfr_rational),
                ("tile_w", c_int32), ("tile_h", c_int32)]


class lfr_camera(Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float)]


class lfr_view_cone(Structure):
    _fields_ = [("orbit_center", c_float * 3), ("radius", c_float), ("span_deg", c_float),
                ("fov_x_deg", c_float), ("rig_offset", c_float * 3), ("num_views", c_int32),
                ("width", c_int32), ("height", c_int32)]


class lfr_scene(Structure):
    _fields_ = [("num_gaussians", c_int64), ("sh_degree", c_int32), ("reserved", c_int32),
                ("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacities", c_void_p), ("sh", c_void_p)]


class lfr_render_opts(Structure):
    _fields_ = [("cluster_size", c_int32), ("flags", c_uint32), ("background", c_float * 3),
                ("first_chunk", c_int32), ("fullframe_tile", c_int32)]


class lfr_stats(Structure):
    _fields_ = [("pairs", c_uint64), ("workspace_bytes", c_uint64),
                ("clusters", c_int32), ("views", c_int32), ("tasks", c_int32), ("chunks", c_int32),
                ("ms_project", c_float), ("ms_depth_sort", c_float), ("ms_keygen", c_float),
                ("ms_sort", c_float), ("ms_ranges", c_float), ("ms_blend", c_float),
                ("ms_total", c_float), ("evals", c_uint64), ("blended", c_uint64),
                ("ms_sort_scatter", c_float), ("sort_scatter_launches", c_int32), ("blend_launches", c_int32),
                ("ms_bwd_blend", c_float), ("ms_bwd_project", c_float), ("ms_bwd_total", c_float),
                ("batch_frames", c_int32), ("batch_unplanned", c_int32), ("batch_graphs", c_int32),
                ("batch_rerendered", c_int32), ("batch_groups", c_int32), ("wave_steps", c_uint64),
                ("wave_steps_live", c_uint64),
                ("saved_forward", c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class lfr_frame(Structure):
    _fields_ = [("display", c_void_p), ("scene", POINTER(lfr_scene)), ("host_cams", c_void_p),
                ("num_cams", c_int32), ("opts", lfr_render_opts), ("out_device", c_void_p)]


LFR_BATCH_GRAPH = 1
LFR_BATCH_TIGHT_PLANS = 2
LFR_BATCH_NO_MERGE = 4


class lfr_scene_grads(Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacities", c_void_p),
                ("sh", c_void_p)]


class lfr_tune_result(Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("cluster_size", c_int32), ("ms", c_float),
                ("pairs", c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lfr_proj_record(Structure):
    _fields_ = [("mean2d", c_float * 2), ("conic", c_float * 3), ("depth", c_float),
                ("color", c_float * 3), ("opacity", c_float), ("valid", c_int32),
                ("valid_mean", c_int32)]


assert ctypes.sizeof(lfr_proj_record) == 48

_P = c_void_p
_SIGS = {
    "lfr_context_create": (c_int32, [c_int32, c_void_p, POINTER(c_void_p)]),
    "lfr_context_destroy": (None, [c_void_p]),
    "lfr_context_set_stream": (c_int32, [c_void_p, c_void_p]),
    "lfr_context_set_limit": (c_int32, [c_void_p, c_uint64]),
    "lfr_context_trim": (c_int32, [c_void_p]),
    "lfr_get_stats": (c_int32, [c_void_p, POINTER(lfr_stats)]),
    "lfr_last_error": (c_char_p, [c_void_p]),
    "lfr_display_create": (c_int32, [c_void_p, POINTER(lfr_display_desc), POINTER(c_void_p)]),
    "lfr_display_create_from_map": (c_int32, [c_void_p, c_int32, c_int32, c_int32, _P, c_int32, c_int32,
                                              POINTER(c_void_p)]),
    "lfr_display_destroy": (None, [c_void_p]),
    "lfr_display_get_view_map": (c_int32, [c_void_p, _P]),
    "lfr_display_get_remap": (c_int32, [c_void_p, _P]),
    "lfr_display_referenced_views": (c_int32, [c_void_p, POINTER(c_int32), _P]),
    "lfr_make_view_cone": (c_int32, [POINTER(lfr_view_cone), _P]),
    "lfr_render": (c_int32, [c_void_p, c_void_p, POINTER(lfr_scene), _P, c_int32, POINTER(lfr_render_opts), _P]),
    "lfr_render_batch": (c_int32, [c_void_p, POINTER(lfr_frame), c_int32, c_uint32]),
    "lfr_render_backward": (c_int32, [c_void_p, c_uint64, c_void_p, POINTER(lfr_scene), _P,
                                      POINTER(lfr_scene_grads)]),
    "lfr_render_fullframe_interlace": (c_int32, [c_void_p, c_void_p, POINTER(lfr_scene), _P, c_int32,
                                                 POINTER(lfr_render_opts), c_int32, _P]),
    "lfr_project": (c_int32, [c_void_p, POINTER(lfr_scene), _P, c_int32, c_int32, _P]),
    "lfr_autotune": (c_int32, [c_void_p, POINTER(lfr_display_desc), POINTER(lfr_scene), _P, c_int32,
                               POINTER(lfr_render_opts), _P, c_int32, _P, c_int32, c_int32, _P,
                               POINTER(lfr_tune_result), POINTER(lfr_tune_result)]),
    "lfr_sort_pairs_u32": (c_int32, [c_void_p, _P, _P, c_int64, c_int32, c_int32]),
    "lfr_sort_pairs_u64": (c_int32, [c_void_p, _P, _P, c_int64, c_int32, c_int32]),
    "lfr_sort_pairs_u32_noalloc": (c_int32, [c_void_p, _P, _P, c_int64, c_int32, c_int32]),
}

_lib = None
_lock = threading.Lock()


def library():
    """Load liblfr.so (once).  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2605_04509_amd.build` (there is no fallback)")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def __getattr__(name):
    # lfr_* names resolve to the raw C functions
    if name in _SIGS:
        return getattr(library(), name)
    raise AttributeError(name)


class LfrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblfr error {code}: {msg}")
        self.code = code


def _check(rc, ctx=None):
    if rc != LFR_OK:
        msg = library().lfr_last_error(ctx).decode() if ctx else ""
        raise LfrError(rc, msg)


# ---------------------------------------------------------------------------
# torch-facing wrappers
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_device_f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float32")


class Context:
    """An lfr_context bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = c_void_p()
        _check(library().lfr_context_create(device, c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            lib = _lib
            if lib is not None:          # may already be gone at interpreter exit
                lib.lfr_context_destroy(self.handle)
            self.handle = None

    __del__ = close

    def set_limit(self, nbytes: int):
        _check(library().lfr_context_set_limit(self.handle, nbytes), self.handle)

    def trim(self):
        _check(library().lfr_context_trim(self.handle), self.handle)

    def stats(self) -> dict:
        s = lfr_stats()
        _check(library().lfr_get_stats(self.handle, ctypes.byref(s)), self.handle)
        return s.as_dict()

    def last_error(self) -> str:
        return library().lfr_last_error(self.handle).decode()


def _rat(r):
    return lfr_rational(int(r.num), int(r.den))


class Display:
    """V and Psi for one lenticular display, built on the device."""

    def __init__(self, ctx: Context, params=None, view_map=None, width=None, height=None,
                 num_views=None, tile=(16, 16)):
        import numpy as np
        h = c_void_p()
        if view_map is None:
            p = params
            desc = lfr_display_desc(p.width, p.height, p.num_views, _rat(p.tan_slant), _rat(p.pitch),
                                    _rat(p.offset), p.tile_w, p.tile_h)
            _check(library().lfr_display_create(ctx.handle, ctypes.byref(desc), ctypes.byref(h)), ctx.handle)
            self.width, self.height, self.num_views = p.width, p.height, p.num_views
            self.tile = (p.tile_w, p.tile_h)
        else:
            vm = np.ascontiguousarray(view_map, dtype=np.int32)
            _check(library().lfr_display_create_from_map(ctx.handle, width, height, num_views,
                                                         vm.ctypes.data_as(c_void_p), tile[0], tile[1],
                                                         ctypes.byref(h)), ctx.handle)
            self.width, self.height, self.num_views = width, height, num_views
            self.tile = tuple(tile)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib = _lib
            if lib is not None:
                lib.lfr_display_destroy(self.handle)
            self.handle = None

    __del__ = close

    def view_map(self):
        import numpy as np
        out = np.empty((self.height, self.width, 3), dtype=np.int32)
        _check(library().lfr_display_get_view_map(self.handle, out.ctypes.data_as(c_void_p)))
        return out

    def remap(self):
        import numpy as np
        out = np.empty(3 * self.width * self.height, dtype=np.uint32)
        _check(library().lfr_display_get_remap(self.handle, out.ctypes.data_as(c_void_p)))
        return out

    def referenced_views(self):
        import numpy as np
        n = c_int32()
        mask = np.empty(self.num_views, dtype=np.uint8)
        _check(library().lfr_display_referenced_views(self.handle, ctypes.byref(n),
                                                      mask.ctypes.data_as(c_void_p)))
        return int(n.value), mask.astype(bool)


class DeviceScene:
    """Scene arrays as contiguous float32 device tensors."""

    def __init__(self, means, log_scales, quats, opacities, sh, sh_degree: int):
        for t, n in ((means, "means"), (log_scales, "log_scales"), (quats, "quats"),
                     (opacities, "opacities"), (sh, "sh")):
            _require_device_f32(t, n)
        m = means.shape[0] if means.dim() else 0
        nb = (int(sh_degree) + 1) ** 2
        if not (0 <= int(sh_degree) <= 3):
            raise ValueError("sh_degree must be in [0, 3]")
        if (means.numel() != 3 * m or log_scales.numel() != 3 * m or quats.numel() != 4 * m
                or opacities.numel() != m or sh.numel() != nb * 3 * m):
            raise ValueError("scene arrays must be [M,3], [M,3], [M,4], [M], [M,(d+1)^2,3]")
        self.means, self.log_scales, self.quats, self.opacities, self.sh = means, log_scales, quats, opacities, sh
        self.sh_degree = int(sh_degree)

    @staticmethod
    def from_numpy(scene, device="cuda"):
        torch = _torch()
        f = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        return DeviceScene(f(scene.means), f(scene.log_scales), f(scene.quats), f(scene.opacities),
                           f(scene.sh), scene.sh_degree)

    @property
    def num_gaussians(self):
        return int(self.means.shape[0])

    def c_struct(self):
        return lfr_scene(self.num_gaussians, self.sh_degree, 0, self.means.data_ptr(), self.log_scales.data_ptr(),
                         self.quats.data_ptr(), self.opacities.data_ptr(), self.sh.data_ptr())


def cameras_array(cams_packed):
    """[N,16] float32 (R, t, fx, fy, cx, cy) -> ctypes array of lfr_camera."""
    import numpy as np
    a = np.ascontiguousarray(cams_packed, dtype=np.float32).reshape(-1, 16)
    arr = (lfr_camera * a.shape[0])()
    ctypes.memmove(arr, a.ctypes.data, a.nbytes)
    return arr


def make_view_cone(num_views, width, height, radius, span_deg, fov_x_deg=60.0, center=None, rig_offset=(0, 0, 0)):
    import numpy as np
    if center is None:
        center = (0.0, 0.0, radius)
    cone = lfr_view_cone((c_float * 3)(*center), radius, span_deg, fov_x_deg, (c_float * 3)(*rig_offset),
                         num_views, width, height)
    out = np.empty((num_views, 16), dtype=np.float32)
    _check(library().lfr_make_view_cone(ctypes.byref(cone), out.ctypes.data_as(c_void_p)))
    return out


def render(ctx: Context, display: Display, scene: DeviceScene, cams, cluster_size=1, remap=True, cull=True,
           timing=False, background=(0.0, 0.0, 0.0), out=None, count_work=False, first_chunk=0,
           save_for_backward=False):
    torch = _torch()
    if out is None:
        out = torch.empty((display.height, display.width, 3), dtype=torch.float32, device=scene.means.device)
    _require_device_f32(out, "out")
    flags = (LFR_REMAP if remap else 0) | (LFR_CULL_UNREFERENCED if cull else 0) | (LFR_TIMING if timing else 0)
    flags |= (LFR_COUNT_WORK if count_work else 0) | (LFR_SAVE_FOR_BACKWARD if save_for_backward else 0)
    opts = lfr_render_opts(cluster_size, flags, (c_float * 3)(*background), first_chunk, 0)
    ca = cams if isinstance(cams, ctypes.Array) else cameras_array(cams)
    sc = scene.c_struct()
    _check(library().lfr_render(ctx.handle, display.handle, ctypes.byref(sc), ca, len(ca), ctypes.byref(opts),
                                _ptr(out)), ctx.handle)
    return out


class Frame:
    """One frame of a batch: lfr_render's arguments."""

    def __init__(self, display: Display, scene: DeviceScene, cams, out, cluster_size=1, remap=True, cull=True,
                 background=(0.0, 0.0, 0.0), first_chunk=0):
        _require_device_f32(out, "out")
        if tuple(out.shape) != (display.height, display.width, 3):
            raise ValueError("out must be [H, W, 3] of the frame's display")
        self.display, self.scene, self.out = display, scene, out
        self.cams = cams if isinstance(cams, ctypes.Array) else cameras_array(cams)
        flags = (LFR_REMAP if remap else 0) | (LFR_CULL_UNREFERENCED if cull else 0)
        self.opts = lfr_render_opts(cluster_size, flags, (c_float * 3)(*background), first_chunk, 0)

    def set_cameras(self, cams):
        self.cams = cams if isinstance(cams, ctypes.Array) else cameras_array(cams)


def render_batch(ctx: Context, frames, graph=True, tight_plans=False, merge=True):
    """Render a list of :class:`Frame` with lfr_render_batch (one host
    synchronization at the end; planned groups replayed from hipGraphs with
    ``graph``; consecutive frames sharing display, scene and options merged
    into one render unless ``merge`` is False).  Returns the batch counters
    of lfr_stats."""
    n = len(frames)
    scenes = [f.scene.c_struct() for f in frames]          # kept alive for the call
    arr = (lfr_frame * max(n, 1))()
    for i, f in enumerate(frames):
        arr[i] = lfr_frame(f.display.handle.value, ctypes.pointer(scenes[i]), ctypes.addressof(f.cams), len(f.cams),
                           f.opts, f.out.data_ptr())
    flags = ((LFR_BATCH_GRAPH if graph else 0) | (LFR_BATCH_TIGHT_PLANS if tight_plans else 0)
             | (0 if merge else LFR_BATCH_NO_MERGE))
    _check(library().lfr_render_batch(ctx.handle, arr, n, flags), ctx.handle)
    st = ctx.stats()
    return {k: st[k] for k in ("batch_frames", "batch_unplanned", "batch_graphs", "batch_rerendered",
                               "batch_groups")}


GRAD_NAMES = ("means", "log_scales", "quats", "opacities", "sh")


def render_backward(ctx: Context, display: Display, scene: DeviceScene, grad_out, grads=None, saved_forward=0):
    """Gradients of the last ``render(..., save_for_backward=True)`` on
    ``ctx`` for the image gradient ``grad_out`` ([H, W, 3] float32 device).
    Returns a dict of tensors shaped like the scene arrays (``grads`` may
    supply them; every element is overwritten).  ``saved_forward``: the
    ``stats()["saved_forward"]`` id read after that render (0: whichever
    forward the context keeps); the library refuses an id it no longer
    keeps."""
    torch = _torch()
    _require_device_f32(grad_out, "grad_out")
    if tuple(grad_out.shape) != (display.height, display.width, 3):
        raise ValueError("grad_out must be [H, W, 3]")
    if grads is None:
        grads = {k: torch.empty_like(getattr(scene, k)) for k in GRAD_NAMES}
    for k in GRAD_NAMES:
        _require_device_f32(grads[k], f"grads[{k}]")
        if grads[k].shape != getattr(scene, k).shape:
            raise ValueError(f"grads[{k}] must have the shape of scene.{k}")
    g = lfr_scene_grads(*(grads[k].data_ptr() for k in GRAD_NAMES))
    sc = scene.c_struct()
    _check(library().lfr_render_backward(ctx.handle, int(saved_forward), display.handle, ctypes.byref(sc),
                                         _ptr(grad_out), ctypes.byref(g)), ctx.handle)
    return grads


def _autograd_function():
    torch = _torch()

    class RenderFunction(torch.autograd.Function):
        """Forward: lfr_render with LFR_SAVE_FOR_BACKWARD; backward:
        lfr_render_backward of that forward (its id is recorded).  The
        context must not render again before the backward runs: the library
        refuses with LFR_ERR_INVALID_ARG rather than return the gradients of
        another render."""

        @staticmethod
        def forward(fctx, means, log_scales, quats, opacities, sh, ctx, display, cams, sh_degree, cluster_size,
                    remap, cull, background):
            scene = DeviceScene(means.detach(), log_scales.detach(), quats.detach(), opacities.detach(),
                                sh.detach(), sh_degree)
            out = render(ctx, display, scene, cams, cluster_size=cluster_size, remap=remap, cull=cull,
                         background=background, save_for_backward=True)
            fctx.lfr = (ctx, display, scene, ctx.stats()["saved_forward"])
            return out

        @staticmethod
        def backward(fctx, grad_out):
            ctx, display, scene, saved = fctx.lfr
            g = render_backward(ctx, display, scene, grad_out.contiguous(), saved_forward=saved)
            return (g["means"], g["log_scales"], g["quats"], g["opacities"], g["sh"],
                    None, None, None, None, None, None, None, None)

    return RenderFunction


_render_fn = None


def render_differentiable(ctx: Context, display: Display, means, log_scales, quats, opacities, sh, sh_degree, cams,
                          cluster_size=1, remap=True, cull=True, background=(0.0, 0.0, 0.0)):
    """The interlaced image as a differentiable function of the scene
    tensors (torch.autograd): forward lfr_render, backward
    lfr_render_backward."""
    global _render_fn
    if _render_fn is None:
        _render_fn = _autograd_function()
    ca = cams if isinstance(cams, ctypes.Array) else cameras_array(cams)
    return _render_fn.apply(means.contiguous(), log_scales.contiguous(), quats.contiguous(), opacities.contiguous(),
                            sh.contiguous(), ctx, display, ca, int(sh_degree), int(cluster_size), bool(remap),
                            bool(cull), tuple(float(b) for b in background))


def render_fullframe_interlace(ctx: Context, display: Display, scene: DeviceScene, cams, view_batch=8, cull=True,
                               timing=False, background=(0.0, 0.0, 0.0), out=None, tile=16):
    torch = _torch()
    if out is None:
        out = torch.zeros((display.height, display.width, 3), dtype=torch.float32, device=scene.means.device)
    _require_device_f32(out, "out")
    flags = (LFR_CULL_UNREFERENCED if cull else 0) | (LFR_TIMING if timing else 0)
    opts = lfr_render_opts(1, flags, (c_float * 3)(*background), 0, tile)
    ca = cams if isinstance(cams, ctypes.Array) else cameras_array(cams)
    sc = scene.c_struct()
    _check(library().lfr_render_fullframe_interlace(ctx.handle, display.handle, ctypes.byref(sc), ca, len(ca),
                                                    ctypes.byref(opts), view_batch, _ptr(out)), ctx.handle)
    return out


DEFAULT_TILES = ((16, 16), (32, 16), (16, 32), (32, 32), (64, 32), (32, 64), (64, 64), (128, 64), (64, 128))


def autotune(ctx: Context, params, scene: DeviceScene, cams, cluster_sizes=(8,), tiles=DEFAULT_TILES, reps=3,
             remap=True, cull=True):
    """Fastest (tile shape, cluster size) for this scene/display (lfr_autotune).
    Returns (best, all_results) as dicts."""
    import numpy as np
    torch = _torch()
    p = params
    desc = lfr_display_desc(p.width, p.height, p.num_views, _rat(p.tan_slant), _rat(p.pitch), _rat(p.offset),
                            p.tile_w, p.tile_h)
    t = np.ascontiguousarray(np.asarray(tiles, dtype=np.int32).reshape(-1))
    sz = np.ascontiguousarray(np.asarray(cluster_sizes, dtype=np.int32))
    flags = (LFR_REMAP if remap else 0) | (LFR_CULL_UNREFERENCED if cull else 0)
    opts = lfr_render_opts(int(sz[0]), flags, (c_float * 3)(0, 0, 0), 0, 0)
    out = torch.empty((p.height, p.width, 3), dtype=torch.float32, device=scene.means.device)
    ca = cams if isinstance(cams, ctypes.Array) else cameras_array(cams)
    res = (lfr_tune_result * (len(t) // 2 * len(sz)))()
    best = lfr_tune_result()
    sc = scene.c_struct()
    _check(library().lfr_autotune(ctx.handle, ctypes.byref(desc), ctypes.byref(sc), ca, len(ca), ctypes.byref(opts),
                                  t.ctypes.data_as(c_void_p), len(t) // 2, sz.ctypes.data_as(c_void_p), len(sz),
                                  reps, _ptr(out), res, ctypes.byref(best)), ctx.handle)
    return best.as_dict(), [r.as_dict() for r in res]


def project(ctx: Context, scene: DeviceScene, cam_packed, width, height):
    """Device projection records for one camera -> [M] structured numpy array."""
    import numpy as np
    torch = _torch()
    M = scene.num_gaussians
    buf = torch.empty(max(M, 1) * 12, dtype=torch.int32, device=scene.means.device)
    ca = cameras_array(cam_packed)
    sc = scene.c_struct()
    _check(library().lfr_project(ctx.handle, ctypes.byref(sc), ca, width, height, _ptr(buf)), ctx.handle)
    torch.cuda.synchronize()
    raw = buf.cpu().numpy().tobytes()[: 48 * M]
    dt = np.dtype([("mean2d", np.float32, 2), ("conic", np.float32, 3), ("depth", np.float32),
                   ("color", np.float32, 3), ("opacity", np.float32), ("valid", np.int32),
                   ("valid_mean", np.int32)])
    return np.frombuffer(raw, dtype=dt).copy()


def sort_pairs(ctx: Context, keys, values, begin_bit=0, end_bit=None):
    """In-place stable radix sort of device (keys, values) on bits [begin, end)."""
    torch = _torch()
    n = keys.numel()
    if keys.dtype == torch.int32 or keys.dtype == torch.uint32:
        fn, kb = library().lfr_sort_pairs_u32, 32
    elif keys.dtype == torch.int64 or keys.dtype == torch.uint64:
        fn, kb = library().lfr_sort_pairs_u64, 64
    else:
        raise ValueError("keys must be 32- or 64-bit integers")
    end_bit = kb if end_bit is None else end_bit
    _check(fn(ctx.handle, _ptr(keys), _ptr(values), n, begin_bit, end_bit), ctx.handle)
    return keys, values


def sort_pairs_noalloc(ctx: Context, keys, values, begin_bit=0, end_bit=32):
    """lfr_sort_pairs_u32_noalloc: the 32-bit-key sort without any device
    allocation (fixed per-GPU scratch, n <= 2^22)."""
    torch = _torch()
    if keys.dtype not in (torch.int32, torch.uint32) or values.dtype not in (torch.int32, torch.uint32):
        raise ValueError("keys and values must be 32-bit integers")
    if values.numel() != keys.numel():
        raise ValueError("keys and values differ in length")
    _check(library().lfr_sort_pairs_u32_noalloc(ctx.handle, _ptr(keys), _ptr(values), keys.numel(), begin_bit,
                                                end_bit), ctx.handle)
    return keys, values
