"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module holds input synthesis only: random-ellipse phantoms, standard-normal
noise draws, angle masks and the named workload shapes. It contains none of the
reconstruction arithmetic (no projection, no solver), so both sides of every
parity test can take their inputs from here without sharing method code.

Conventions (the paper fixes a parallel-beam geometry, Section 1, but not these
details; they are stated readings):

* image of N x N unit pixels covering [-N/2, N/2]^2, pixel (iy, ix) has its
  centre at (ix - N/2 + 1/2, iy - N/2 + 1/2); flat index j = iy*N + ix;
* an ellipse (cx, cy, a, b, phi, rho) is given in coordinates normalised by
  N/2; a pixel gets the sum of rho over the ellipses that contain its centre;
* per ellipse the draws are, in this order: cx, cy ~ U[-0.6, 0.6],
  a, b ~ U[0.05, 0.4], phi ~ U[0, pi), rho ~ U[0.1, 1];
* measurement noise is drawn after the phantom from the same generator as
  standard normals; how it is scaled into the data is up to the consumer.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ellipse_params", "rasterize_ellipses", "phantom", "phantom_and_noise",
    "n_bins_for", "angle_mask", "Workload", "WORKLOADS", "mixed_batch_specs",
    "slice_rng",
]


def ellipse_params(rng: np.random.Generator, n_ellipses: int) -> np.ndarray:
    """Draw ``n_ellipses`` rows of (cx, cy, a, b, phi, rho) in the fixed order."""
    out = np.empty((n_ellipses, 6), dtype=np.float64)
    for e in range(n_ellipses):
        out[e, 0] = rng.uniform(-0.6, 0.6)
        out[e, 1] = rng.uniform(-0.6, 0.6)
        out[e, 2] = rng.uniform(0.05, 0.4)
        out[e, 3] = rng.uniform(0.05, 0.4)
        out[e, 4] = rng.uniform(0.0, math.pi)
        out[e, 5] = rng.uniform(0.1, 1.0)
    return out


def rasterize_ellipses(params: np.ndarray, n: int) -> np.ndarray:
    """Centre-point sampling of additive ellipses on an n x n grid (float64)."""
    h = 0.5 * n
    c = (np.arange(n, dtype=np.float64) - h + 0.5) / h
    yy, xx = np.meshgrid(c, c, indexing="ij")  # yy[iy, ix], xx[iy, ix]
    img = np.zeros((n, n), dtype=np.float64)
    for cx, cy, a, b, phi, rho in params:
        dx = xx - cx
        dy = yy - cy
        cp, sp = math.cos(phi), math.sin(phi)
        u = dx * cp + dy * sp
        v = -dx * sp + dy * cp
        inside = (u / a) ** 2 + (v / b) ** 2 <= 1.0
        img[inside] += rho
    return img


def slice_rng(seed: int, index: int | None = None) -> np.random.Generator:
    """Generator for a whole workload (index None) or for slice/instance ``index``."""
    if index is None:
        return np.random.default_rng(seed)
    return np.random.default_rng([seed, index])


def phantom(n: int, n_ellipses: int, seed: int = 0, index: int | None = None) -> np.ndarray:
    """Random-ellipse phantom, flattened row-major (length n*n, float64)."""
    rng = slice_rng(seed, index)
    return rasterize_ellipses(ellipse_params(rng, n_ellipses), n).reshape(-1)


def phantom_and_noise(n: int, n_ellipses: int, n_noise: int, seed: int = 0,
                      index: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Phantom and then ``n_noise`` standard normals from the same generator."""
    rng = slice_rng(seed, index)
    img = rasterize_ellipses(ellipse_params(rng, n_ellipses), n).reshape(-1)
    eps = rng.standard_normal(n_noise)
    return img, eps


def n_bins_for(n: int) -> int:
    """Smallest odd bin count covering the image diagonal: odd >= n*sqrt(2)."""
    nb = int(math.ceil(n * math.sqrt(2.0) - 1e-12))
    if nb % 2 == 0:
        nb += 1
    return nb


def angle_mask(n_angles: int, every: int = 1) -> np.ndarray:
    """Measured-angle flags: angle k is measured when k % every == 0."""
    m = np.zeros(n_angles, dtype=np.uint8)
    m[::every] = 1
    return m


@dataclass(frozen=True)
class Workload:
    """One named workload shape (sizes only; arrays are made on demand)."""
    name: str
    n: int
    n_angles: int
    n_bins: int
    every: int               # measured angles: k % every == 0
    n_ellipses: int
    noise: float             # relative noise level (times RMS of the clean data)
    alpha: float
    lam: float
    n_outer: int
    n_cg: int
    dtype: str               # "f32" or "f64"
    batch: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def mask(self) -> np.ndarray:
        return angle_mask(self.n_angles, self.every)

    @property
    def n_meas(self) -> int:
        return int(self.mask.sum())


# Shapes of the five workloads the library is measured and tested on.  Only the
# 64x64 case fixes the split-Bregman weights (alpha = 10, lambda = 1).  For the
# larger images the data are line integrals over hundreds of unit pixels, so
# alpha = 10 makes the data term outweigh the TV term by orders of magnitude:
# the iterates then fit the noise (error to the phantom grows from 0.33 to 0.92
# over 20 Bregman steps on the 512x512 case) and the trajectory amplifies a
# 1e-13 data perturbation by ~1e11.  alpha = 0.01, lambda = 1 balances the two
# terms at this data scale (error to the phantom 0.045 after 50 x 20) and keeps
# the solve well posed.
WORKLOADS = {
    "small_64_f64": Workload("small_64_f64", 64, 45, 91, 1, 5, 0.01, 10.0, 1.0, 20, 10, "f64"),
    "gpu_512_f32": Workload("gpu_512_f32", 512, 360, 725, 2, 10, 0.02, 0.01, 1.0, 50, 20, "f32"),
    "large_2048_f32": Workload("large_2048_f32", 2048, 90, 2897, 1, 30, 0.01, 0.01, 1.0, 30, 10, "f32"),
    "volume_64x1024_f32": Workload("volume_64x1024_f32", 1024, 360, 1449, 1, 10, 0.01, 0.01, 1.0,
                                   20, 10, "f32", batch=64),
    "grad_16x512_f32": Workload("grad_16x512_f32", 512, 120, 725, 1, 10, 0.01, 10.0, 0.0, 0, 10,
                                "f32", batch=16, extra={"tau": 0.1, "ckpt": 5}),
}


def small_batch_specs(count: int = 64, seed: int = 0) -> list[tuple[int, int]]:
    """(N, n_angles) of a batch of small instances, where launches rather
    than bandwidth bound a per-instance loop: N in {32, 64, 128}, angles in
    16..64."""
    rng = np.random.default_rng([seed, 2000])
    out = []
    for _ in range(count):
        n = int(rng.choice([32, 64, 128]))
        na = int(rng.integers(16, 65))
        out.append((n, na))
    return out


def mixed_batch_specs(count: int = 32, seed: int = 0) -> list[tuple[int, int]]:
    """(N, n_angles) of the uneven-size instances: N in {256,512,1024}, angles in 60..180."""
    rng = np.random.default_rng([seed, 1000])
    out = []
    for _ in range(count):
        n = int(rng.choice([256, 512, 1024]))
        na = int(rng.integers(60, 181))
        out.append((n, na))
    return out
