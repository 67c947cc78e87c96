"""Camera rigs for the light-field views.

A camera is a pinhole with OpenCV axes (x right, y down, z forward):
world-to-camera rotation R (3x3, row-major), translation t, focal lengths
fx, fy and principal point cx, cy, all float32.  The views of a display are
placed on a horizontal arc around an orbit centre, all facing inward (the
paper only says the trajectories orbit the scene with inward-facing cameras;
the arc geometry below is this project's choice).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Camera:
    R: np.ndarray   # [3,3] float32 world->camera rotation
    t: np.ndarray   # [3]   float32 world->camera translation
    fx: float
    fy: float
    cx: float
    cy: float

    def packed(self) -> np.ndarray:
        """16 float32: R row-major (9), t (3), fx, fy, cx, cy."""
        out = np.empty(16, dtype=np.float32)
        out[0:9] = self.R.reshape(-1)
        out[9:12] = self.t
        out[12:16] = (self.fx, self.fy, self.cx, self.cy)
        return out


def orbit_rig(num_views: int, width: int, height: int, radius: float,
              span_deg: float, fov_x_deg: float = 60.0,
              centre=None, rig_offset=(0.0, 0.0, 0.0)) -> list[Camera]:
    """Views on an arc of ``span_deg`` degrees around ``centre``.

    View j sits at angle theta_j = -span/2 + span * j / (N - 1) (endpoints
    inclusive; a single view sits at theta = 0).  Its position is
    centre + radius * (sin theta, 0, -cos theta) + rig_offset, it looks along
    (-sin theta, 0, cos theta) with image-right (cos theta, 0, sin theta) and
    image-down (0, 1, 0).  Intrinsics: fx = fy = (W/2) / tan(fov_x/2),
    cx = W/2, cy = H/2.
    """
    if centre is None:
        centre = (0.0, 0.0, radius)
    c = np.asarray(centre, dtype=np.float64)
    off = np.asarray(rig_offset, dtype=np.float64)
    f = (0.5 * width) / math.tan(math.radians(fov_x_deg) * 0.5)
    cams = []
    for j in range(num_views):
        if num_views > 1:
            th = math.radians(-0.5 * span_deg + span_deg * j / (num_views - 1))
        else:
            th = 0.0
        pos = c + radius * np.array([math.sin(th), 0.0, -math.cos(th)]) + off
        right = np.array([math.cos(th), 0.0, math.sin(th)])
        down = np.array([0.0, 1.0, 0.0])
        fwd = np.array([-math.sin(th), 0.0, math.cos(th)])
        R = np.stack([right, down, fwd])
        t = -R @ pos
        cams.append(Camera(R.astype(np.float32), t.astype(np.float32),
                           float(np.float32(f)), float(np.float32(f)),
                           float(np.float32(0.5 * width)), float(np.float32(0.5 * height))))
    return cams


def pack_cameras(cams) -> np.ndarray:
    return np.ascontiguousarray(np.stack([c.packed() for c in cams]), dtype=np.float32)
