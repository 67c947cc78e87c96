"""The named workloads (scene + display + view rig) used by tests and bench.

* ``tiny``     2,000 Gaussians (SH0), 16 views on a 30 degree arc, 256x144
               panel, slant 1/6, pitch 23/5.
* ``display``  200,000 Gaussians (SH3), 45 views over 40 degrees, 1920x1080,
               slant 1/6, pitch 5.
* ``outdoor``  3,000,000 Gaussians (clustered + far shell, SH3), 100 views
               over 50 degrees, 3840x2160, slant 1/5, pitch 31/5.
* ``landscape71`` the outdoor scene on the paper's landscape shape: 71 views
               over 53 degrees, 3840x2160, slant 3/17, pitch 123/20 (every view
               owns subpixels; reuse groups of 18 views).
* ``portrait63``   the outdoor scene on the paper's portrait shape: 63 views over
               53 degrees, 1440x2560, slant 3/17, pitch 57/10 (every view owns
               subpixels; reuse groups of 16 views).
* ``batched``  three outdoor-style scenes (0.5M / 1M / 3M) on 1080p/45-view,
               1440p/64-view and 4K/100-view panels, 16 jittered head poses
               each.
* ``grad``     the ``display`` workload for the differentiable path, plus a
               500-Gaussian 64x36 subset for finite-difference checks.

Orbit geometry (radius, centre), the scene details and the lens slant /
pitch of the two paper display shapes are this project's choices; the paper
gives only view counts, angular ranges, resolutions and reuse group sizes.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np

from .cameras import Camera, orbit_rig
from .displays import DisplayParams, Rational
from .scenes import Scene, mixture_scene, uniform_scene


@dataclasses.dataclass
class Workload:
    name: str
    display: DisplayParams
    make_scene: Callable[[], Scene]
    radius: float
    span_deg: float
    fov_x_deg: float = 60.0
    cluster_sizes: tuple = (1,)

    def cameras(self, rig_offset=(0.0, 0.0, 0.0)) -> list[Camera]:
        d = self.display
        return orbit_rig(d.num_views, d.width, d.height, self.radius, self.span_deg,
                         self.fov_x_deg, centre=(0.0, 0.0, self.radius), rig_offset=rig_offset)


def _tiny():
    return uniform_scene(1, 2000, 1.0, (2.0, 6.0), 0)


def _display():
    return uniform_scene(2, 200_000, 3.0, (3.0, 9.0), 3)


def _outdoor():
    return mixture_scene(3, 3_000_000, 3)


WORKLOADS = {
    "tiny": Workload("tiny", DisplayParams(256, 144, 16, Rational(1, 6), Rational(23, 5)),
                     _tiny, radius=4.0, span_deg=30.0, cluster_sizes=(1, 2, 4, 8)),
    "display": Workload("display", DisplayParams(1920, 1080, 45, Rational(1, 6), Rational(5, 1)),
                        _display, radius=6.0, span_deg=40.0, cluster_sizes=(1, 8)),
    "outdoor": Workload("outdoor", DisplayParams(3840, 2160, 100, Rational(1, 5), Rational(31, 5)),
                        _outdoor, radius=12.0, span_deg=50.0, cluster_sizes=(1, 2, 4, 8)),
    "landscape71": Workload("landscape71", DisplayParams(3840, 2160, 71, Rational(3, 17), Rational(123, 20)),
                            _outdoor, radius=12.0, span_deg=53.0, cluster_sizes=(1, 18)),
    "portrait63": Workload("portrait63", DisplayParams(1440, 2560, 63, Rational(3, 17), Rational(57, 10)),
                           _outdoor, radius=12.0, span_deg=53.0, cluster_sizes=(1, 16)),
}


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]


def batched_frames(num_poses: int = 16, seed: int = 4, scale: float = 1.0):
    """The serving-style batch: (scene seed, M, display, radius, span, offsets).

    Scene i sits on panel i; each scene is seen from ``num_poses`` head poses
    whose rig offsets are drawn U[-0.05, 0.05]^3 (scene units).
    ``scale`` shrinks the Gaussian counts for small test runs.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = [
        (41, int(500_000 * scale), DisplayParams(1920, 1080, 45, Rational(1, 6), Rational(5, 1)), 12.0, 50.0),
        (42, int(1_000_000 * scale), DisplayParams(2560, 1440, 64, Rational(1, 6), Rational(5, 1)), 12.0, 50.0),
        (43, int(3_000_000 * scale), DisplayParams(3840, 2160, 100, Rational(1, 5), Rational(31, 5)), 12.0, 50.0),
    ]
    out = []
    for seed_i, m, disp, radius, span in specs:
        offs = rng.uniform(-0.05, 0.05, (num_poses, 3))
        out.append((seed_i, m, disp, radius, span, offs))
    return out


def grad_subset():
    """500 Gaussians drawn like ``display`` (seed 55) on a 64x36 panel with
    45 views over 40 degrees (slant 1/6, pitch 5)."""
    scene = uniform_scene(55, 500, 3.0, (3.0, 9.0), 3)
    disp = DisplayParams(64, 36, 45, Rational(1, 6), Rational(5, 1))
    return scene, disp, orbit_rig(45, 64, 36, 6.0, 40.0, 60.0, centre=(0.0, 0.0, 6.0))
