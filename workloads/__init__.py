"""Seeded synthetic workloads for the light-field rasterizer.

This package only *draws inputs*: Gaussian scenes, lenticular display
parameters and camera rigs.  It holds none of the rasterizer's arithmetic
(no projection, no blending, no view-index map), so the CPU oracle and the
HIP path can both consume its outputs without sharing any method code.

Every array is drawn from ``numpy.random.Generator(PCG64(seed))`` in a fixed
order (means, log-scales, quaternions, opacities, SH), so a seed fully
determines a workload.
"""
from .scenes import Scene, make_scene, uniform_scene, mixture_scene, perturb_means
from .displays import DisplayParams, Rational
from .cameras import Camera, orbit_rig
from .configs import WORKLOADS, Workload, get_workload

__all__ = [
    "Scene", "make_scene", "uniform_scene", "mixture_scene", "perturb_means",
    "DisplayParams", "Rational", "Camera", "orbit_rig",
    "WORKLOADS", "Workload", "get_workload",
]
