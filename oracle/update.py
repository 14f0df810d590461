"""Super-resolution volume update, FP64 numpy -- TEST INFRASTRUCTURE ONLY.

Paper Sec. II: registered patches are reintegrated into X by iterative
super-resolution with gradient descent; the cited reconstruction method adds
edge-preserving regularisation by anisotropic diffusion (Sec. I-A).  The paper
prints no formula or constants, so the update is a reading:

    X' = max(clamp_min, X + alpha * num/den * [den > den_eps]
                          + alpha * lambda * R(X))

with num = A^T(W p e), den = A^T(W p) and the regulariser
    R_i = sum_{d in N26} b_d * D_d / sqrt(1 + (D_d / delta)^2),
    D_d = X_{i+d} - X_i,  b_d = 1 / |d|  (voxel units),
neighbours outside the grid skipped.  With W p = 1 and lambda = 0 this is
SIRT (rows of A sum to one; column-sum preconditioning).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

OFFSETS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def _shifted(X: np.ndarray, d):
    """(X[i + d], inside) with d = (dz, dy, dx) and inside = neighbour in grid."""
    nz, ny, nx = X.shape
    out = np.zeros_like(X)
    ins = np.zeros(X.shape, dtype=bool)
    src = []
    dst = []
    for ax, (o, n) in enumerate(zip(d, (nz, ny, nx))):
        if o >= 0:
            dst.append(slice(0, n - o)); src.append(slice(o, n))
        else:
            dst.append(slice(-o, n)); src.append(slice(0, n + o))
    out[tuple(dst)] = X[tuple(src)]
    ins[tuple(dst)] = True
    return out, ins


def regulariser(X: np.ndarray, delta: float) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    R = np.zeros_like(X)
    for d in OFFSETS:
        nb, ins = _shifted(X, d)
        D = np.where(ins, nb - X, 0.0)
        b = 1.0 / math.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        R += b * D / np.sqrt(1.0 + (D / delta) ** 2)
    return R


def sr_update(X, num, den, alpha=1.0, lam=0.02, delta=150.0, clamp_min=0.0,
              den_eps=1e-6):
    X = np.asarray(X, dtype=np.float64)
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        step = np.where(den > den_eps, num / np.where(den > den_eps, den, 1.0), 0.0)
    out = X + alpha * step
    if lam != 0.0:
        out = out + alpha * lam * regulariser(X, delta)
    if clamp_min is not None:
        out = np.maximum(out, clamp_min)
    return out
