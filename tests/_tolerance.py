"""Error bars of the FP32 adjoint against the FP64 oracle.

The PSF weight of a sample j at voxel i is g_ij = (exp(-Q_ij/2) - exp(-k^2/2))
/ Z_j on Q_ij <= k^2 (shifted truncated Gaussian, Sec. III).  In FP32 the
first term carries a relative error of a few units of roundoff, so g_ij
carries an absolute error proportional to exp(-Q_ij/2) / Z_j, which near the
support edge is exp(-k^2/2) / Z_j even though g_ij itself tends to 0 there
(cancellation).  A voxel reached only by near-edge samples therefore cannot
be held to a bar relative to sum_j |r_j| g_ij alone; the bar adds one sample's
edge term exp(-k^2/2) max_j |r_j| / Z_j.
"""
import math

import numpy as np


def adjoint_bar(ctx, theta, r, rel=1e-5, k=3.0):
    """Per-voxel bar rel * ((A^T |r|)_i + exp(-k^2/2) max_j |r_j| / Z_j) for an
    FP32 adjoint A^T r, from the oracle only."""
    r = np.abs(np.asarray(r, np.float64).reshape(-1))
    rabs = ctx.backproject(theta, r).reshape(-1)
    _, Z, val = ctx.simulate(np.zeros(ctx.V), theta)
    edge = math.exp(-0.5 * k * k) * float(np.max(np.where(val, r / np.where(val, Z, 1.0), 0.0)))
    return rel * (rabs + edge)
