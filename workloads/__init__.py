"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generators only: random points, values, sample index
sets and the fluorite lattice.  It contains none of the transform's
arithmetic, so both the CPU oracle side and the GPU side may use it.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` in float64.
FP32 runs use the same draws rounded to float32, and the oracle is evaluated
on exactly the values the GPU received.

Workloads (domain [-1/2, 1/2)^3, Section 1 of the paper):
  * ``c1``: N = 16^3, M = 4096 uniform points, complex values with
    re, im ~ N(0, 1)   (the precision experiment of Section 4);
  * ``c2``: N = 64^3, M = 2^20 uniform points;
  * ``c3``: N = 128^3, M = 2^23: half uniform, half in 64 Gaussian clusters
    (2^16 points each, per-dimension std 0.02, wrapped into the domain);
  * ``c4``: 256 independent transforms, M_b = floor(10^U(3,6)) points and a
    cubic bandwidth drawn from {32, 48, 64, 96} per transform;
  * fluorite lattice (Section 5): 4 Ca(2+) and 8 F(-) per cubic cell,
    Ca-F distance r0 = 1, Gaussian displacements.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def wrap_unit(x: np.ndarray) -> np.ndarray:
    """Map coordinates periodically into [-1/2, 1/2)."""
    y = x - np.floor(x + 0.5)
    y = np.where(y >= 0.5, y - 1.0, y)
    y = np.where(y < -0.5, y + 1.0, y)
    return y


def uniform_points(M: int, d: int, g: np.random.Generator) -> np.ndarray:
    """M points i.i.d. uniform in [-1/2, 1/2)^d, float64, shape (M, d)."""
    return g.random((M, d)) - 0.5


def complex_normal(M: int, g: np.random.Generator) -> np.ndarray:
    """M complex128 values with re, im ~ N(0, 1)."""
    re = g.standard_normal(M)
    im = g.standard_normal(M)
    return re + 1j * im


def clustered_points(M_uniform: int, n_clusters: int, per_cluster: int, std: float, d: int,
                     g: np.random.Generator) -> np.ndarray:
    """Uniform points followed by Gaussian clusters (centres uniform), wrapped."""
    u = uniform_points(M_uniform, d, g)
    centres = uniform_points(n_clusters, d, g)
    c = centres[:, None, :] + std * g.standard_normal((n_clusters, per_cluster, d))
    c = wrap_unit(c.reshape(-1, d))
    return np.concatenate([u, c], axis=0)


def sample_indices(total: int, count: int, g: np.random.Generator) -> np.ndarray:
    """``count`` distinct sorted int64 indices in [0, total)."""
    count = min(count, total)
    return np.sort(g.choice(total, size=count, replace=False)).astype(np.int64)


def c1(seed: int = 1):
    g = rng(seed)
    x = uniform_points(4096, 3, g)
    f = complex_normal(4096, g)
    return dict(N=(16, 16, 16), x=x, f=f)


def c2(seed: int = 2, M: int = 1 << 20):
    g = rng(seed)
    x = uniform_points(M, 3, g)
    f = complex_normal(M, g)
    fhat = complex_normal(64 ** 3, g).reshape(64, 64, 64)
    return dict(N=(64, 64, 64), x=x, f=f, fhat=fhat)


def c3(seed: int = 3, M: int = 1 << 23):
    g = rng(seed)
    half = M // 2
    per = half // 64
    x = clustered_points(half, 64, per, 0.02, 3, g)
    f = complex_normal(x.shape[0], g)
    return dict(N=(128, 128, 128), x=x, f=f)


C4_SIZES = (32, 48, 64, 96)


def c4_element(b: int):
    """Batch element b of the 256-transform workload (seed 4000 + b)."""
    g = rng(4000 + b)
    M = int(math.floor(10.0 ** g.uniform(3.0, 6.0)))
    Nb = int(C4_SIZES[int(g.integers(0, len(C4_SIZES)))])
    x = uniform_points(M, 3, g)
    f = complex_normal(M, g)
    return dict(N=(Nb, Nb, Nb), x=x, f=f)


def c4(B: int = 256):
    return [c4_element(b) for b in range(B)]


# ---------------------------------------------------------------------------
# Fluorite (CaF2) lattice, Section 5 of the paper.
FLUORITE_CA = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0]], dtype=np.float64) / 4.0
FLUORITE_F = np.array([[i, j, k] for i in (1, 3) for j in (1, 3) for k in (1, 3)],
                      dtype=np.float64) / 4.0


def fluorite(cells: int, displacement_std: float = 0.0, seed: int = 5):
    """Fluorite supercell of ``cells``^3 cubic unit cells.

    Unit length r0 = Ca-F distance = sqrt(3) l / 4, so the cell side is
    l = 4 / sqrt(3).  Returns (r, q, L_box): positions (n, 3) in [0, L_box)
    before displacement, charges +2 (Ca) / -1 (F), box side.
    Displacements are N(0, std^2) in units of r0.
    """
    l = 4.0 / math.sqrt(3.0)
    idx = np.stack(np.meshgrid(np.arange(cells), np.arange(cells), np.arange(cells),
                               indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    ca = (idx[:, None, :] + FLUORITE_CA[None, :, :]).reshape(-1, 3) * l
    fl = (idx[:, None, :] + FLUORITE_F[None, :, :]).reshape(-1, 3) * l
    r = np.concatenate([ca, fl], axis=0)
    q = np.concatenate([np.full(ca.shape[0], 2.0), np.full(fl.shape[0], -1.0)])
    if displacement_std > 0.0:
        r = r + displacement_std * rng(seed).standard_normal(r.shape)
    return r, q, cells * l


def to_unit_box(r: np.ndarray, L_box: float) -> np.ndarray:
    """Scale positions by the box side and wrap into [-1/2, 1/2)^3."""
    return wrap_unit(np.asarray(r, dtype=np.float64) / L_box)
