"""Seeded synthetic workloads (input generation only; no arithmetic of the method).

Both the GPU path and the CPU oracle are fed from the arrays drawn here, so the
two sides always see identical inputs.  Draw order per batch: every H first
(shape [B, d, d]), then the per-RVE scalars in the order listed.

Workloads (synthetic stand-ins for the paper's microstructures, which are images
and tessellations that are not available):
  * ``rve2d``   -- batch of 2D periodic RVEs n x n, circular inclusion of radius
                   r ~ U[r_lo, r_hi] at the cell centre, stiffness ratio 10,
                   F = I + H with H_ij ~ U[-h, h] (rejected if det F < 0.5);
  * ``rve3d``   -- uneven 3D batch, n ~ uniform{8, 12, 16}, spherical inclusion
                   with volume fraction f ~ U[0.05, 0.3] (r = (3f / 4 pi)^(1/3)),
                   stiffness ratio log-uniform in [2, 50], H_ij ~ U[-0.1, 0.1].
Material: matrix E = 1, nu = 0.3; inclusion E = ratio, same nu (the inclusion is
the stiffer phase).
"""
from dataclasses import dataclass

import numpy as np

E_MATRIX = 1.0
NU = 0.3


@dataclass
class RVEBatch:
    d: int
    n: np.ndarray          # [B] elements per edge
    F: np.ndarray          # [B, d, d]
    radius: np.ndarray     # [B] inclusion radius (unit cell)
    ratio: np.ndarray      # [B] inclusion / matrix Young's modulus
    seed: int


def draw_F(rng, B, d, h, det_min=0.5):
    """F = I + H, H_ij iid U[-h, h]; rows with det F < det_min are redrawn."""
    H = rng.uniform(-h, h, size=(B, d, d))
    F = np.eye(d)[None] + H
    bad = np.linalg.det(F) < det_min
    while bad.any():
        H2 = rng.uniform(-h, h, size=(int(bad.sum()), d, d))
        F[bad] = np.eye(d)[None] + H2
        bad = np.linalg.det(F) < det_min
    return F


def rve2d(B, n=32, h=0.15, r_lo=0.15, r_hi=0.35, ratio=10.0, seed=1001):
    rng = np.random.default_rng(seed)
    F = draw_F(rng, B, 2, h)
    r = rng.uniform(r_lo, r_hi, size=B)
    return RVEBatch(2, np.full(B, n, np.int32), F, r, np.full(B, float(ratio)), seed)


def rve3d(B, sizes=(8, 12, 16), h=0.1, f_lo=0.05, f_hi=0.3, ratio_lo=2.0, ratio_hi=50.0, seed=1002):
    rng = np.random.default_rng(seed)
    F = draw_F(rng, B, 3, h)
    n = rng.choice(np.asarray(sizes, np.int32), size=B)
    f = rng.uniform(f_lo, f_hi, size=B)
    ratio = np.exp(rng.uniform(np.log(ratio_lo), np.log(ratio_hi), size=B))
    r = (3.0 * f / (4.0 * np.pi)) ** (1.0 / 3.0)
    return RVEBatch(3, n.astype(np.int32), F, r, ratio, seed)


def fixed_radius_2d(B, n, r=0.25, h=0.15, ratio=10.0, seed=1003):
    """Same microstructure for every RVE (macro quadrature points of one material)."""
    rng = np.random.default_rng(seed)
    F = draw_F(rng, B, 2, h)
    return RVEBatch(2, np.full(B, n, np.int32), F, np.full(B, r), np.full(B, float(ratio)), seed)
