"""Error bars of the FP32 adjoint against the FP64 oracle.

The PSF weight of a sample j at voxel i is g_ij = (exp(-Q_ij/2) - exp(-k^2/2))
/ Z_j on Q_ij <= k^2 (shifted truncated Gaussian).  In FP32 the first term
carries a relative error of a few units of roundoff, so g_ij carries an
absolute error proportional to exp(-Q_ij/2) / Z_j = g_ij + exp(-k^2/2) / Z_j:
near the support edge the error stays at the size of exp(-k^2/2) / Z_j while
g_ij tends to 0 (cancellation).  Summed over the samples that reach voxel i,
the error of (A^T r)_i is bounded to first order by a few units of roundoff
times

    (A^T |r|)_i + exp(-k^2/2) (S^T (|r| / Z))_i,

S the support indicator.  The bar is rel times that sum; both parts come
from the oracle.
"""
import math

import numpy as np


def adjoint_bar(ctx, theta, r, rel=1e-5, k=3.0, voxels=None):
    """Per-voxel bar for an FP32 adjoint A^T r: over the whole grid, or over
    the listed flat voxel indices."""
    r = np.abs(np.asarray(r, np.float64).reshape(-1))
    if voxels is None:
        rabs = ctx.backproject(theta, r).reshape(-1)
        edge = ctx.backproject(theta, r, support=True).reshape(-1)
    else:
        rabs = ctx.backproject_voxels(theta, r, voxels)
        edge = ctx.backproject_voxels(theta, r, voxels, support=True)
    return rel * (rabs + math.exp(-0.5 * k * k) * edge)
