"""Seeded synthetic 3D Gaussian scenes.

A scene is the set G = {mu, Sigma(log-scale, quaternion), o, SH} of a 3DGS
model (paper section 3.3).  Arrays are float32, C-contiguous:

* ``means``       [M, 3]   world position
* ``log_scales``  [M, 3]   per-axis log standard deviation
* ``quats``       [M, 4]   rotation quaternion (w, x, y, z), unit norm
* ``opacities``   [M]      opacity o in (0, 1) (already activated)
* ``sh``          [M, B, 3] SH coefficients, B = (degree + 1)^2, band-major,
                            RGB innermost; ``sh[:, 0, :]`` is the DC term.

Draw order for every generator: means, log-scales, quaternions, opacities,
SH (DC then the higher bands).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def num_gaussians(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(
            np.ascontiguousarray(self.means[idx]),
            np.ascontiguousarray(self.log_scales[idx]),
            np.ascontiguousarray(self.quats[idx]),
            np.ascontiguousarray(self.opacities[idx]),
            np.ascontiguousarray(self.sh[idx]),
            self.sh_degree,
        )

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacities, self.sh)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _quats(rng, m):
    q = rng.standard_normal((m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _sh(rng, m, degree, dc_uniform=True, rest_std=0.2):
    nb = (degree + 1) ** 2
    sh = np.zeros((m, nb, 3), dtype=np.float64)
    sh[:, 0, :] = rng.uniform(0.0, 1.0, (m, 3)) if dc_uniform else rng.standard_normal((m, 3))
    if nb > 1:
        sh[:, 1:, :] = rng.normal(0.0, rest_std, (m, nb - 1, 3))
    return sh


def _pack(means, log_scales, quats, opac, sh, degree) -> Scene:
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means), f(log_scales), f(quats), f(opac), f(sh), int(degree))


def uniform_scene(seed: int, m: int, xy_range: float, z_range, degree: int,
                  log_scale_mean: float = -3.0, log_scale_std: float = 0.5,
                  sh_rest_std: float = 0.2) -> Scene:
    """Means uniform in a box, log-scales normal, opacity sigmoid(N(0,1))."""
    rng = _rng(seed)
    means = np.empty((m, 3))
    means[:, 0:2] = rng.uniform(-xy_range, xy_range, (m, 2))
    means[:, 2] = rng.uniform(z_range[0], z_range[1], m)
    log_scales = rng.normal(log_scale_mean, log_scale_std, (m, 3))
    quats = _quats(rng, m)
    opac = _sigmoid(rng.standard_normal(m))
    sh = _sh(rng, m, degree, rest_std=sh_rest_std)
    return _pack(means, log_scales, quats, opac, sh, degree)


def mixture_scene(seed: int, m: int, degree: int = 3, n_components: int = 64,
                  far_fraction: float = 0.10) -> Scene:
    """Outdoor-shaped scene: a clustered foreground plus a far shell.

    * (1 - far_fraction) of the means come from an equal-weight mixture of
      ``n_components`` isotropic Gaussians with centres uniform in
      [-8, 8] x [-3, 3] x [6, 18] and per-component std uniform in [0.3, 1.2];
    * the rest form a far shell: z ~ U[20, 60], x ~ U[-0.7z, 0.7z],
      y ~ U[-0.4z, 0.4z];
    * log-scales are heavy tailed: -3.5 + 0.5 * t(nu=3) per axis, clipped to
      [-8, -0.5];
    * opacity = sigmoid(N(0.5, 1.5)); SH: DC ~ U(0,1), other bands ~ N(0, 0.2).
    """
    rng = _rng(seed)
    n_far = int(round(m * far_fraction))
    n_mix = m - n_far
    centres = np.column_stack([
        rng.uniform(-8.0, 8.0, n_components),
        rng.uniform(-3.0, 3.0, n_components),
        rng.uniform(6.0, 18.0, n_components),
    ])
    sig = rng.uniform(0.3, 1.2, n_components)
    comp = rng.integers(0, n_components, n_mix)
    near = centres[comp] + sig[comp, None] * rng.standard_normal((n_mix, 3))
    z = rng.uniform(20.0, 60.0, n_far)
    far = np.column_stack([
        rng.uniform(-0.7, 0.7, n_far) * z,
        rng.uniform(-0.4, 0.4, n_far) * z,
        z,
    ])
    means = np.concatenate([near, far], axis=0)
    log_scales = np.clip(-3.5 + 0.5 * rng.standard_t(3.0, (m, 3)), -8.0, -0.5)
    quats = _quats(rng, m)
    opac = _sigmoid(rng.normal(0.5, 1.5, m))
    sh = _sh(rng, m, degree)
    return _pack(means, log_scales, quats, opac, sh, degree)


def make_scene(kind: str, seed: int, m: int, **kw) -> Scene:
    if kind == "uniform":
        return uniform_scene(seed, m, **kw)
    if kind == "mixture":
        return mixture_scene(seed, m, **kw)
    raise ValueError(f"unknown scene kind {kind!r}")


def perturb_means(scene: Scene, seed: int, std: float) -> Scene:
    """Copy of ``scene`` with means + N(0, std^2) (the target of the
    differentiable-path workload)."""
    rng = _rng(seed)
    means = scene.means.astype(np.float64) + rng.normal(0.0, std, scene.means.shape)
    return Scene(np.ascontiguousarray(means, dtype=np.float32), scene.log_scales.copy(),
                 scene.quats.copy(), scene.opacities.copy(), scene.sh.copy(), scene.sh_degree)
