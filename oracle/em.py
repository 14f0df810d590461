"""EM-based outlier removal, FP64 numpy -- TEST INFRASTRUCTURE ONLY.

Paper Sec. II "EM-Based Outlier Removal":
  * inliers follow a zero-mean Gaussian G_sigma(e) of variance sigma^2, outliers
    a uniform density m = 1 / (max(e) - min(e))            (eq. for m);
  * the log-likelihood sum log P(e | sigma, c) is maximised   (eq. log P);
  * the inlier posterior of a pixel is
        p = G_sigma(e) c / (G_sigma(e) c + m (1 - c))         (eq. for p);
  * a patch potential is p_bar = sqrt(sum p^2 / N)           (eq. for p_bar);
  * each patch gets an inlier / outlier probability and is excluded when it
    is classified as an outlier.

Readings where the paper is silent (it defers the updates of c and sigma^2 to
the cited reconstruction method):
  * m uses the extremes over all valid samples, guarded by eps_m = 1e-6 *
    max|y|;
  * patch classification: a two-component 1D Gaussian mixture fitted to the
    potentials by EM (20 iterations) from a fixed start (split at the median;
    component means / standard deviations from each half, deviations floored
    at 1e-3; inlier mixing weight 0.9); the component with the larger mean is
    the inlier one; W_s = pi_s when pi_s >= 0.5, else 0;
  * M-step: sigma^2 = sum W p e^2 / sum W p (floored at (1e-4 max|y|)^2),
    c = sum W p / sum W with sum W = sum_s W_s N_s;
  * start of a cycle: sigma^2 = mean(e^2), c = 0.9.
"""
from __future__ import annotations

import math

import numpy as np

GMM_ITERS = 20
GMM_STD_FLOOR = 1e-3
GMM_INLIER_START = 0.9
C_START = 0.9


def outlier_density(e_valid: np.ndarray, y_abs_max: float) -> float:
    """m = 1 / max(max e - min e, eps_m)."""
    if e_valid.size == 0:
        return 1.0
    rng = float(np.max(e_valid) - np.min(e_valid))
    eps = 1e-6 * y_abs_max
    return 1.0 / max(rng, eps) if max(rng, eps) > 0 else 1.0


def inlier_density(e: np.ndarray, sigma2: float) -> np.ndarray:
    """Zero-mean Gaussian G_sigma(e)."""
    return np.exp(-e * e / (2.0 * sigma2)) / math.sqrt(2.0 * math.pi * sigma2)


def posterior(e: np.ndarray, sigma2: float, c: float, m: float) -> np.ndarray:
    """Inlier posterior p = G c / (G c + m (1 - c)); 0 where both vanish."""
    Gc = inlier_density(e, sigma2) * c
    den = Gc + m * (1.0 - c)
    with np.errstate(invalid="ignore", divide="ignore"):
        p = np.where(den > 0, Gc / np.where(den > 0, den, 1.0), 0.0)
    return p


def log_likelihood(e: np.ndarray, sigma2: float, c: float, m: float) -> float:
    """sum log(c G_sigma(e) + (1 - c) m) over the given residuals."""
    return float(np.sum(np.log(c * inlier_density(e, sigma2) + (1 - c) * m)))


def patch_potentials(p: np.ndarray, valid: np.ndarray,
                     patch_of_sample: np.ndarray, M: int):
    """(p_bar, N_s, sum p, sum p^2) per patch; p_bar = sqrt(sum p^2 / N_s)
    over the patch's valid samples, 0 when N_s = 0."""
    pv = np.where(valid, p, 0.0)
    n = np.bincount(patch_of_sample, weights=valid.astype(np.float64), minlength=M)
    s2 = np.bincount(patch_of_sample, weights=pv * pv, minlength=M)
    s1 = np.bincount(patch_of_sample, weights=pv, minlength=M)
    with np.errstate(invalid="ignore", divide="ignore"):
        pbar = np.where(n > 0, np.sqrt(s2 / np.where(n > 0, n, 1.0)), 0.0)
    return pbar, n, s1, s2


def _log_normal(v, mu, sd):
    return -0.5 * ((v - mu) / sd) ** 2 - math.log(sd) - 0.5 * math.log(2 * math.pi)


def patch_mixture(values: np.ndarray):
    """Fit the two-component mixture to the potentials; returns the inlier
    responsibility of every value and the final (mu, sd, weight) of both
    components, inlier component first."""
    v = np.asarray(values, dtype=np.float64)
    n = v.size
    if n == 0:
        return np.zeros(0), None
    if n == 1:
        return np.ones(1), None
    srt = np.sort(v)
    n_lo = n // 2
    lo, hi = srt[:n_lo], srt[n_lo:]
    mu = [float(lo.mean()), float(hi.mean())]
    sd = [max(float(lo.std()), GMM_STD_FLOOR), max(float(hi.std()), GMM_STD_FLOOR)]
    w1 = GMM_INLIER_START

    def resp(mu, sd, w1):
        l1 = math.log(w1) + _log_normal(v, mu[1], sd[1]) if w1 > 0 else np.full(n, -np.inf)
        l0 = math.log(1 - w1) + _log_normal(v, mu[0], sd[0]) if w1 < 1 else np.full(n, -np.inf)
        with np.errstate(over="ignore"):
            return 1.0 / (1.0 + np.exp(l0 - l1))

    for _ in range(GMM_ITERS):
        r1 = resp(mu, sd, w1)
        r0 = 1.0 - r1
        s1, s0 = r1.sum(), r0.sum()
        if s1 <= 0 or s0 <= 0:
            break
        w1 = s1 / n
        mu = [float((r0 * v).sum() / s0), float((r1 * v).sum() / s1)]
        sd = [max(math.sqrt(float((r0 * (v - mu[0]) ** 2).sum() / s0)), GMM_STD_FLOOR),
              max(math.sqrt(float((r1 * (v - mu[1]) ** 2).sum() / s1)), GMM_STD_FLOOR)]
    r1 = resp(mu, sd, w1)
    if mu[0] > mu[1]:
        r1 = 1.0 - r1
        mu, sd, w1 = mu[::-1], sd[::-1], 1 - w1
    return r1, ((mu[1], sd[1], w1), (mu[0], sd[0], 1 - w1))


def patch_weights(pbar: np.ndarray, n_s: np.ndarray, active=None):
    """W_s from the mixture posterior pi_s (W = pi if pi >= 0.5 else 0);
    patches with no valid sample, or inactive ones, get W = 0.
    Returns (W, pi)."""
    M = pbar.size
    use = n_s > 0
    if active is not None:
        use &= np.asarray(active, bool)
    pi = np.zeros(M)
    r, _ = patch_mixture(pbar[use])
    pi[use] = r
    W = np.where(use & (pi >= 0.5), pi, 0.0)
    return W, pi


def mstep(e, p, valid, W_sample, n_s, W, sigma2, c, y_abs_max):
    """sigma^2 = sum W p e^2 / sum W p (floored), c = sum W p / sum W."""
    wp = np.where(valid, W_sample * p, 0.0)
    swp = wp.sum()
    swpe2 = (wp * e * e).sum()
    sw = float((W * n_s).sum())
    floor = (1e-4 * y_abs_max) ** 2
    s2 = max(swpe2 / swp, floor) if swp > 0 else sigma2
    cc = swp / sw if sw > 0 else c
    return s2, cc


def init_state(e_valid: np.ndarray):
    """Start of a cycle: sigma^2 = mean(e^2), c = 0.9."""
    s2 = float(np.mean(e_valid * e_valid)) if e_valid.size else 1.0
    return s2, C_START
