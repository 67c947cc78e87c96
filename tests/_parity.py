"""Comparison rule shared by the GPU parity tests.

Floating-point parity (exact and reuse paths) is |gpu - oracle| <= 2e-5 per
channel.  A subpixel the oracle flags as near a discrete threshold (an alpha
within four times its float32 error bound of 1/255, or a transmittance T'
within four times its bound of 1e-4) may legitimately take the other branch
in float32.  For those the oracle follows both outcomes of every flagged
decision and returns the range [lo, hi] of the values the leaves reach
(oracle.render_subpixels_ranged); the GPU value must lie in
[lo - 2e-5, hi + 2e-5].  If the oracle had to cut the tree off (more than 64
leaves; reported as incomplete, which must stay rare) the bound is what the
differing tail can contribute at all: 2 * T_flag * c_max + 2e-5.  Flagged
subpixels are counted and must stay rare; the report gives their number and
the largest flagged deviation from the main value.
"""
from __future__ import annotations

import numpy as np

TOL = 2e-5


def compare(gpu, r, cmax=None, max_flag_frac=5e-3, label=""):
    """gpu: values of the samples; r: the dict of oracle.render_subpixels_ranged
    (or of oracle.render_frame_ranged, any shape)."""
    gpu = np.asarray(gpu, np.float64).reshape(-1)
    ref = np.asarray(r["out"], np.float64).reshape(-1)
    lo = np.asarray(r["lo"], np.float64).reshape(-1)
    hi = np.asarray(r["hi"], np.float64).reshape(-1)
    flags = np.asarray(r["flags"]).reshape(-1)
    paths = np.asarray(r["paths"]).reshape(-1)
    tflag = np.asarray(r["tflag"], np.float64).reshape(-1)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    err = np.abs(gpu - ref)
    flagged = flags != 0
    incomplete = paths < 0
    inside = (gpu >= lo - TOL) & (gpu <= hi + TOL)
    ok = err <= TOL
    ok |= flagged & ~incomplete & inside
    if incomplete.any():
        assert cmax is not None, f"{label}: incomplete ranges need a colour bound"
        ok |= incomplete & (err <= 2.0 * tflag * cmax + TOL)
    info = {
        "n": int(err.size),
        "max_err_unflagged": float(err[~flagged].max()) if (~flagged).any() else 0.0,
        "flagged": int(flagged.sum()),
        "flagged_alpha": int(((flags & 1) != 0).sum()),
        "flagged_stop": int(((flags & 2) != 0).sum()),
        "max_err_flagged": float(err[flagged].max()) if flagged.any() else 0.0,
        "incomplete": int(incomplete.sum()),
        "bad": int((~ok).sum()),
    }
    if not ok.all():
        k = np.flatnonzero(~ok)[:8]
        raise AssertionError(f"{label}: {info}; idx {k.tolist()} gpu {gpu[k].tolist()} ref {ref[k].tolist()} "
                             f"lo {lo[k].tolist()} hi {hi[k].tolist()} flags {flags[k].tolist()}")
    assert flagged.mean() <= max_flag_frac, f"{label}: too many flagged subpixels {info}"
    assert info["incomplete"] <= max(1, err.size // 2000), f"{label}: too many incomplete ranges {info}"
    return info


def colour_bound(scene) -> float:
    """An upper bound on any SH colour of the scene: 0.5 + sum_b max|Y_b| |h_b|,
    with |Y_b| <= 1.1 for bands <= 3 (the largest real SH value on the sphere
    is about 1.09 for l = 3)."""
    sh = np.abs(scene.sh.astype(np.float64))
    return float(0.5 + 1.1 * sh.sum(axis=1).max())
