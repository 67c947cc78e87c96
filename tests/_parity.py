"""Comparison rules shared by the GPU parity tests.

Floating-point parity (exact and reuse paths) is |gpu - oracle| <= 2e-5 per
channel.  Subpixels the oracle flags as near a discrete threshold (an alpha
or a transmittance within four times its float32 error bound of 1/255 or
1e-4) may legitimately take the other branch in float32; for them the bound
is what the differing tail can contribute: 2 * T_flag * c_max + 2e-5, with
T_flag the oracle's transmittance at the first flagged event.  They are
counted and must stay rare.
"""
from __future__ import annotations

import numpy as np

TOL = 2e-5


def compare(gpu, ref, flags, tflag, cmax, max_flag_frac=5e-3, label=""):
    gpu = np.asarray(gpu, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    flags = np.asarray(flags).reshape(-1)
    tflag = np.asarray(tflag, np.float64).reshape(-1)
    err = np.abs(gpu - ref)
    flagged = flags != 0
    bound = np.where(flagged, 2.0 * tflag * cmax + TOL, TOL)
    bad = err > bound
    info = {
        "n": int(err.size),
        "max_err_unflagged": float(err[~flagged].max()) if (~flagged).any() else 0.0,
        "flagged": int(flagged.sum()),
        "bad": int(bad.sum()),
    }
    if bad.any():
        k = np.argsort(-(err - bound))[:8]
        raise AssertionError(f"{label}: {info}; worst idx {k.tolist()} gpu {gpu[k].tolist()} ref {ref[k].tolist()} "
                             f"flags {flags[k].tolist()}")
    assert flagged.mean() <= max_flag_frac, f"{label}: too many flagged subpixels {info}"
    return info


def colour_bound(scene) -> float:
    """An upper bound on any SH colour of the scene: 0.5 + sum_b max|Y_b| |h_b|,
    with |Y_b| <= 1.1 for bands <= 3 (the largest real SH value on the sphere
    is about 1.09 for l = 3)."""
    sh = np.abs(scene.sh.astype(np.float64))
    return float(0.5 + 1.1 * sh.sum(axis=1).max())
