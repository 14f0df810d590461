"""Pins for the oracle's EM outlier removal (paper Sec. II "EM-Based Outlier
Removal": inlier Gaussian G_sigma, uniform outlier density m, posterior p,
patch potential p_bar) and the patch inlier/outlier mixture.

Pinned against: closed-form values of the posterior, monotonicity,
recovery of a known Gaussian-plus-uniform mixture, the non-decreasing
log-likelihood of EM, and scikit-learn's GaussianMixture as an independent
implementation of the two-component mixture EM.
"""
import math

import numpy as np
import pytest

from oracle import em
from paper_1611_07289_amd import synth


def test_posterior_closed_form_and_monotone():
    sigma2, c, m = 25.0, 0.7, 1e-3
    G0 = 1.0 / math.sqrt(2 * math.pi * sigma2)
    assert em.posterior(np.array([0.0]), sigma2, c, m)[0] == pytest.approx(
        c * G0 / (c * G0 + m * (1 - c)), rel=1e-15)
    e = np.linspace(0, 60, 200)
    p = em.posterior(e, sigma2, c, m)
    assert np.all(np.diff(p) < 0)
    assert np.allclose(em.posterior(-e, sigma2, c, m), p)
    # p = 1/2 exactly where c G(e) = m (1 - c)
    e_half = math.sqrt(-2 * sigma2 * math.log(m * (1 - c) / c * math.sqrt(2 * math.pi * sigma2)))
    assert em.posterior(np.array([e_half]), sigma2, c, m)[0] == pytest.approx(0.5, abs=1e-12)


def test_outlier_density_is_inverse_range():
    e = np.array([-3.0, 5.0, 1.0])
    assert em.outlier_density(e, 100.0) == pytest.approx(1 / 8.0)
    assert em.outlier_density(np.zeros(4), 100.0) == pytest.approx(1 / 1e-4)


def _voxel_em(e, iters, sigma2, c):
    m = em.outlier_density(e, float(np.abs(e).max()))
    lls = []
    for _ in range(iters):
        lls.append(em.log_likelihood(e, sigma2, c, m))
        p = em.posterior(e, sigma2, c, m)
        ones = np.ones_like(e)
        sigma2, c = em.mstep(e, p, ones.astype(bool), ones, np.array([e.size]),
                             np.array([1.0]), sigma2, c, 0.0)
    return sigma2, c, lls


def test_mixture_recovery_gaussian_plus_uniform():
    e = synth.residual_mixture(1_000_000, seed=11, sigma=10.0, frac_in=0.8,
                               lo=-500.0, hi=500.0)
    s2, c, lls = _voxel_em(e, 200, sigma2=float(np.mean(e * e)), c=0.9)
    assert math.sqrt(s2) == pytest.approx(10.0, rel=0.01)
    assert c == pytest.approx(0.8, abs=0.005)
    # EM never decreases the log-likelihood of the data
    assert np.all(np.diff(lls) >= -1e-6 * np.abs(lls[:-1]))


def test_patch_potential():
    p = np.ones(12)
    valid = np.ones(12, bool)
    pos = np.repeat([0, 1, 2], 4)
    pbar, n, _, _ = em.patch_potentials(p, valid, pos, 4)
    assert np.allclose(pbar[:3], 1.0) and pbar[3] == 0 and n[3] == 0
    p = np.array([0.0, 1.0, 0.0, 1.0])
    pbar, n, _, _ = em.patch_potentials(p, np.ones(4, bool), np.zeros(4, int), 1)
    assert pbar[0] == pytest.approx(math.sqrt(0.5))
    # invalid samples do not count
    pbar, n, _, _ = em.patch_potentials(p, np.array([1, 1, 0, 0], bool), np.zeros(4, int), 1)
    assert n[0] == 2 and pbar[0] == pytest.approx(math.sqrt(0.5))


def test_patch_mixture_matches_sklearn_and_recovers_components():
    from sklearn.mixture import GaussianMixture
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(0.9, 0.03, 900), rng.normal(0.35, 0.08, 100)])
    rng.shuffle(v)
    r1, comps = em.patch_mixture(v)
    (mu1, sd1, w1), (mu0, sd0, w0) = comps
    assert mu1 == pytest.approx(0.9, abs=0.01) and mu0 == pytest.approx(0.35, abs=0.03)
    assert w1 == pytest.approx(0.9, abs=0.02)
    # the same start and iteration count in an independent implementation
    srt = np.sort(v)
    lo, hi = srt[:500], srt[500:]
    gm = GaussianMixture(2, covariance_type="full", max_iter=em.GMM_ITERS, tol=0.0,
                         reg_covar=0.0, weights_init=[0.1, 0.9],
                         means_init=[[lo.mean()], [hi.mean()]],
                         precisions_init=[[[1 / lo.var()]], [[1 / hi.var()]]])
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gm.fit(v[:, None])
    ref = gm.predict_proba(v[:, None])[:, int(np.argmax(gm.means_[:, 0]))]
    assert np.allclose(r1, ref, atol=1e-8)
    assert np.sort(gm.means_[:, 0]) == pytest.approx([mu0, mu1], rel=1e-8)
    # classification: W > 0 exactly for the high-potential cluster
    W, pi = em.patch_weights(v, np.ones_like(v))
    assert np.all((W > 0) == (v > 0.65))


def test_patch_weights_edge_cases():
    W, pi = em.patch_weights(np.array([0.8]), np.array([10.0]))
    assert W[0] == 1.0
    W, pi = em.patch_weights(np.array([0.8, 0.0]), np.array([10.0, 0.0]))
    assert W[1] == 0.0 and W[0] == 1.0


def _mixture_loglik(v, comps):
    (mu1, sd1, w1), (mu0, sd0, w0) = comps
    d1 = w1 * np.exp(-0.5 * ((v - mu1) / sd1) ** 2) / (sd1 * math.sqrt(2 * math.pi))
    d0 = w0 * np.exp(-0.5 * ((v - mu0) / sd0) ** 2) / (sd0 * math.sqrt(2 * math.pi))
    return float(np.sum(np.log(d1 + d0)))


def test_patch_mixture_log_likelihood_never_decreases(monkeypatch):
    """EM on the potentials' two-component mixture: the data log-likelihood
    after k iterations is non-decreasing in k (the mixture is refitted with
    k = 1 ... 20 iterations from the same start)."""
    rng = np.random.default_rng(8)
    v = np.concatenate([rng.normal(0.85, 0.05, 300), rng.normal(0.45, 0.12, 60),
                        rng.uniform(0.0, 1.0, 20)])
    rng.shuffle(v)
    lls = []
    for k in range(1, em.GMM_ITERS + 1):
        monkeypatch.setattr(em, "GMM_ITERS", k)
        _, comps = em.patch_mixture(v)
        lls.append(_mixture_loglik(v, comps))
    assert np.all(np.diff(lls) >= -1e-9 * np.abs(lls[:-1])), lls
    assert lls[-1] > lls[0]


def _weighted_case():
    """Three patches of different sizes with patch weights != 1 and per-sample
    posteriors, some samples invalid."""
    rng = np.random.default_rng(31)
    n = np.array([7, 5, 9])
    pos = np.repeat(np.arange(3), n)
    e = rng.normal(0, 12, pos.size)
    p = rng.uniform(0.05, 1.0, pos.size)
    valid = rng.uniform(size=pos.size) > 0.15
    W = np.array([0.6, 0.9, 0.75])
    n_s = np.bincount(pos, weights=valid.astype(float), minlength=3)
    return e, p, valid, pos, n_s, W


def test_mstep_is_the_weighted_complete_data_maximiser():
    """The M-step maximises the expected complete-data log-likelihood with
    every sample weighted by its patch weight,
      Q(sigma^2, c) = sum_j W_j [p_j log(c G_sigma(e_j)) + (1 - p_j) log((1 - c) m)],
    over several patches with W != 1 (checked by a numerical maximiser)."""
    from scipy.optimize import minimize
    e, p, valid, pos, n_s, W = _weighted_case()
    Wj = W[pos]
    s2, c = em.mstep(e, p, valid, Wj, n_s, W, 50.0, 0.5, 0.0)
    m = 1e-3
    ev, pv, wv = e[valid], p[valid], Wj[valid]

    def negQ(x):
        ls2, lc = x
        sig2, cc = math.exp(ls2), 1 / (1 + math.exp(-lc))
        logG = -ev * ev / (2 * sig2) - 0.5 * math.log(2 * math.pi * sig2)
        return -float(np.sum(wv * (pv * (math.log(cc) + logG) + (1 - pv) * math.log((1 - cc) * m))))

    res = minimize(negQ, x0=[math.log(100.0), 0.0], method="Nelder-Mead",
                   options=dict(xatol=1e-10, fatol=1e-12, maxiter=20000))
    s2_num, c_num = math.exp(res.x[0]), 1 / (1 + math.exp(-res.x[1]))
    assert s2 == pytest.approx(s2_num, rel=1e-6)
    assert c == pytest.approx(c_num, rel=1e-6)


def test_mstep_integer_patch_weight_is_replication():
    """A patch weight of 2 counts the patch twice: the M-step equals the one
    over the same data with that patch duplicated at weight 1."""
    e, p, valid, pos, n_s, _ = _weighted_case()
    W = np.array([2.0, 1.0, 1.0])
    s2a, ca = em.mstep(e, p, valid, W[pos], n_s, W, 50.0, 0.5, 0.0)
    sel = pos == 0
    e2 = np.concatenate([e, e[sel]]); p2 = np.concatenate([p, p[sel]])
    v2 = np.concatenate([valid, valid[sel]]); pos2 = np.concatenate([pos, np.full(sel.sum(), 3)])
    n2 = np.bincount(pos2, weights=v2.astype(float), minlength=4)
    W2 = np.ones(4)
    s2b, cb = em.mstep(e2, p2, v2, W2[pos2], n2, W2, 50.0, 0.5, 0.0)
    assert s2a == pytest.approx(s2b, rel=1e-14)
    assert ca == pytest.approx(cb, rel=1e-14)
