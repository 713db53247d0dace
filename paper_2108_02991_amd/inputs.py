"""Seeded synthetic inputs for the SPARKLING energy/gradient path.

This module only draws numbers: sample trajectories, target densities and
finite-difference directions.  It holds none of the method's arithmetic (no
kernel, no gradient, no projection), so both the HIP path and the FP64 CPU
oracle can be fed from the same bytes.

Layouts
  K    : float64 array of shape (3, p), rows x, y, z; sample i = c*Ns + n is
         sample n of shot c (shot-lexicographic order, Sec. "3D SPARKLING
         formulation").
  rho  : float64 array of length G**3, cell-centred grid over [-L, L]^3 with
         x fastest: voxel v = ix + G*(iy + G*iz) sits at
         (-L + (ix+1/2)*2L/G, -L + (iy+1/2)*2L/G, -L + (iz+1/2)*2L/G).
"""
from __future__ import annotations

import hashlib

import numpy as np


def voxel_axis(G: int, L: float) -> np.ndarray:
    """Cell-centre coordinates of one grid axis: -L + (i + 1/2) * (2L/G)."""
    i = np.arange(G, dtype=np.float64)
    return -L + (i + 0.5) * (2.0 * L / G)


def radial_density(G: int, L: float, C: float, D: float) -> np.ndarray:
    """Radially decaying target density with a flat centre, sampled on the grid.

    The law is the two-parameter density of Sec. "Choice of target sampling
    density": constant for |x| < C and (C/|x|)^D beyond.  Its normalising
    constant is replaced by a numerical normalisation of the grid weights to
    sum 1 (the printed constant is the 1-D one and is singular at D = 1).
    """
    ax = voxel_axis(G, L)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")  # x fastest in C order
    r = np.sqrt(x * x + y * y + z * z)
    w = np.ones_like(r)
    far = r > C
    w[far] = (C / r[far]) ** D
    w = w.reshape(-1)
    return w / w.sum()


def uniform_density(G: int) -> np.ndarray:
    return np.full(G ** 3, 1.0 / G ** 3)


def separable_density(G: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Random positive weights a[ix] b[iy] c[iz] on the G^3 grid (x fastest),
    normalised to sum 1: non-uniform in every axis yet cheap at very large G."""
    rng = np.random.default_rng(seed)
    a, b, c = (rng.uniform(0.5, 1.5, G) for _ in range(3))
    a, b, c = a / a.sum(), b / b.sum(), c / c.sum()
    out = np.multiply.outer(np.multiply.outer(c, b), a).astype(dtype, copy=False)
    return out.reshape(-1)


def radial_spokes(n_shots: int, n_samples: int, L: float, seed: int,
                  jitter: float = 0.0) -> np.ndarray:
    """Centre-out radial spokes with uniform random directions, optionally jittered.

    Sample n of shot c lies at radius L*n/(Ns-1) along a direction drawn
    uniformly on the sphere (normalised Gaussian triple).  With jitter J > 0,
    every sample except the first gets an independent U(-J, J)^3 offset
    (the init perturbation of Sec. "Initialization and Perturbation"), and
    the result is clamped to [-L, L]^3.  Sample 0 of every shot stays at the
    origin (+0.0), the echo-time point.
    """
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n_shots, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    radius = L * np.arange(n_samples, dtype=np.float64) / max(n_samples - 1, 1)
    pts = d[:, None, :] * radius[None, :, None]          # (Nc, Ns, 3)
    if jitter > 0.0:
        noise = rng.uniform(-jitter, jitter, size=(n_shots, n_samples, 3))
        noise[:, 0, :] = 0.0
        pts = pts + noise
    pts = np.clip(pts, -L, L)
    pts[:, 0, :] = 0.0
    return np.ascontiguousarray(pts.reshape(-1, 3).T)    # (3, p)


def uniform_points(p: int, L: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-L, L, size=(3, p))


def two_density_points(p_dense: int, p_sparse: int, L: float, seed: int) -> np.ndarray:
    """(3, p_dense + p_sparse) points uniform in [-L, L]^3: the first p_dense in
    the half x < 0, the rest in the half x >= 0 (a dense and a sparse region)."""
    rng = np.random.default_rng(seed)
    K = rng.uniform(-L, L, (3, p_dense + p_sparse))
    K[0, :p_dense] = -np.abs(K[0, :p_dense])
    K[0, p_dense:] = np.abs(K[0, p_dense:])
    return K


def rademacher(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=shape).astype(np.float64) * 2.0 - 1.0


def sample_targets(p: int, n: int, seed: int) -> np.ndarray:
    """n distinct target indices in [0, p), sorted, always including 0 and p-1."""
    rng = np.random.default_rng(seed)
    n = min(n, p)
    if n <= 2 or p <= 2:
        return np.unique(np.array([0, p - 1][:n], dtype=np.int64))
    inner = rng.choice(np.arange(1, p - 1), size=n - 2, replace=False)
    return np.unique(np.concatenate([[0, p - 1], inner])).astype(np.int64)


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
