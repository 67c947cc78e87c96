"""Host-side checks of liblfr that need no GPU: the shared library loads,
exports every entry point declared in include/lfr.h, and its host-only logic
(camera rig construction, argument validation) behaves."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2605_04509_amd import lfr
from workloads.cameras import orbit_rig, pack_cameras

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lfr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lfr_[a-z0-9_]+)\s*\(", src)))


def test_library_built():
    assert os.path.exists(lfr.LIB_PATH), "run python -m paper_2605_04509_amd.build"


def test_exports_every_declared_symbol():
    lib = lfr.library()
    declared = _declared()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lfr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lfr_[a-z0-9_]+)", out))
    assert set(declared) <= exported
    # and the binding covers exactly the declared surface
    assert set(lfr.exported_symbols()) == set(declared)


def test_make_view_cone_matches_rig_generator():
    for (n, W, H, R, span, off) in [(16, 256, 144, 4.0, 30.0, (0, 0, 0)), (45, 1920, 1080, 6.0, 40.0, (0.01, -0.02, 0.03)),
                                    (1, 64, 36, 3.0, 10.0, (0, 0, 0))]:
        got = lfr.make_view_cone(n, W, H, R, span, 60.0, rig_offset=off)
        want = pack_cameras(orbit_rig(n, W, H, R, span, 60.0, centre=(0, 0, R), rig_offset=off))
        np.testing.assert_allclose(got, want, rtol=2e-7, atol=2e-6)


def test_make_view_cone_rejects_bad_args():
    cone = lfr.lfr_view_cone((ctypes.c_float * 3)(0, 0, 4), 4.0, 30.0, 200.0, (ctypes.c_float * 3)(0, 0, 0), 4, 8, 8)
    out = np.empty((4, 16), np.float32)
    assert lfr.library().lfr_make_view_cone(ctypes.byref(cone), out.ctypes.data_as(ctypes.c_void_p)) == lfr.LFR_ERR_INVALID_ARG


def test_null_context_and_arguments_are_rejected():
    lib = lfr.library()
    assert lib.lfr_render(None, None, None, None, 0, None, None) == lfr.LFR_ERR_INVALID_ARG
    assert lib.lfr_get_stats(None, None) == lfr.LFR_ERR_INVALID_ARG
    assert lib.lfr_context_set_limit(None, 1) == lfr.LFR_ERR_INVALID_ARG
    assert lib.lfr_display_get_view_map(None, None) == lfr.LFR_ERR_INVALID_ARG
    assert lib.lfr_last_error(None) == b"context is NULL"


def test_context_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    rc = lfr.library().lfr_context_create(0, None, ctypes.byref(h))
    assert rc == lfr.LFR_ERR_INVALID_ARG and not h.value
