"""Pins for the oracle's sinc PSF (paper Sec. II, the PSF paragraph): the
sinc in-plane, evaluated by its Taylor series cut at a relative error, times
the slice profile through-plane.

Readings: the in-plane sinc is sin(pi t)/(pi t) with t = offset / in-plane
FWHM (its first zero at the FWHM), main lobe only (|t| < 1, where it is
positive and falls to 0 at the edge); the slice profile is a Gaussian of the
through-plane FWHM cut at k sigma and shifted to 0 there, as for the Gaussian
PSF.  Pinned by: numpy's sinc; a brute-force dense A over every voxel built
from numpy and scipy's rotation (rows, simulate and its transpose); rows
summing to one; the support lying in the box and the weights being
positive.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_1611_07289_amd import synth
from tests._problems import brute_problem


def test_taylor_sinc_matches_numpy():
    R = np.linspace(-math.pi, math.pi, 4001)
    got = np.array([oracle.sinc_taylor(r) for r in R])
    assert np.max(np.abs(got - np.sinc(R / math.pi))) < 1e-14
    assert oracle.sinc_taylor(0.0) == 1.0
    assert abs(oracle.sinc_taylor(math.pi)) < 1e-15


def _dense_A_sinc(P, k=3.0):
    """Dense A of the sinc PSF from scratch: numpy over every voxel."""
    g = P.grid
    ii, jj, kk = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.arange(g.nz), indexing="ij")
    vidx = ((kk * g.ny + jj) * g.nx + ii).reshape(-1)
    vw = np.stack([ii, jj, kk, np.ones_like(ii)], -1).reshape(-1, 4) @ g.vox2world.T
    A = np.zeros((P.N, g.n_voxels))
    valid = np.zeros(P.N, bool)
    tab = P.patches.table()
    off = P.patches.sample_off
    for s in range(P.M):
        st, sl, x0, y0, w, h = tab[s]
        S = P.stacks[st]
        Lp, op = S.pix2world[:, :3], S.pix2world[:, 3]
        E = Lp / np.linalg.norm(Lp, axis=0)
        fw = np.asarray(S.fwhm_mm, float)
        sig_n = fw[2] / (2 * math.sqrt(2 * math.log(2)))
        R = Rotation.from_euler("xyz", P.theta_true[s, :3]).as_matrix()
        c = Lp @ [x0 + (w - 1) / 2, y0 + (h - 1) / 2, sl] + op
        F = R @ E
        for l in range(w * h):
            u, v = x0 + l % w, y0 + l // w
            x = R @ (Lp @ [u, v, sl] + op - c) + c + P.theta_true[s, 3:]
            xv = np.linalg.solve(g.vox2world[:, :3], x - g.vox2world[:, 3])
            inside = np.all(xv >= -0.5) and np.all(xv < np.array([g.nx, g.ny, g.nz]) - 0.5)
            d = (vw - x) @ F
            tu, tv, qn = d[:, 0] / fw[0], d[:, 1] / fw[1], (d[:, 2] / sig_n) ** 2
            sup = (np.abs(tu) < 1) & (np.abs(tv) < 1) & (qn <= k * k)
            gh = np.where(sup, np.sinc(tu) * np.sinc(tv) * (np.exp(-qn / 2) - math.exp(-k * k / 2)), 0.0)
            Z = gh.sum()
            j = off[s] + l
            if inside and Z > 0:
                valid[j] = True
                A[j, vidx] = gh / Z
    return A, valid


@pytest.fixture(scope="module")
def brute_sinc():
    P = brute_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches, psf="sinc")
    A, valid = _dense_A_sinc(P)
    return P, ctx, A, valid


def test_bruteforce_dense_sinc_A_equals_oracle_rows(brute_sinc):
    P, ctx, A, valid = brute_sinc
    _, _, val = ctx.simulate(np.zeros(P.grid.n_voxels), P.theta_true)
    assert np.array_equal(val, valid)
    assert valid.sum() > 0.6 * P.N and (~valid).sum() > 0
    for j in range(P.N):
        idx, w = ctx.sample_row(P.theta_true, j)
        row = np.zeros(P.grid.n_voxels)
        row[idx] = w
        assert np.allclose(row, A[j], rtol=1e-12, atol=1e-15), j
    x = np.random.default_rng(1).normal(size=P.grid.n_voxels)
    r = np.random.default_rng(2).normal(size=P.N)
    yh, _, _ = ctx.simulate(x, P.theta_true)
    assert np.allclose(yh, A @ x, rtol=1e-12, atol=1e-12)
    bp = ctx.backproject(P.theta_true, r).reshape(-1)
    assert np.allclose(bp, A.T @ r, rtol=1e-12, atol=1e-12)
    vox = np.random.default_rng(3).choice(P.grid.n_voxels, 40, replace=False)
    assert np.allclose(ctx.backproject_voxels(P.theta_true, r, vox), bp[vox], rtol=1e-12, atol=1e-14)


def test_sinc_rows_sum_to_one_and_weights_positive(brute_sinc):
    P, ctx, A, valid = brute_sinc
    yh, Z, val = ctx.simulate(np.full(P.grid.n_voxels, 321.0), P.theta_true)
    assert np.allclose(yh[val], 321.0, rtol=1e-13)
    for j in np.nonzero(val)[0][::29]:
        _, w = ctx.sample_row(P.theta_true, j)
        assert abs(w.sum() - 1.0) < 1e-12 and np.all(w >= 0)
    # the sinc support differs from the Gaussian one (a box, not an ellipsoid)
    ctx_g = oracle.Ctx(P.grid, P.stacks, P.patches)
    j = int(np.nonzero(val)[0][0])
    assert not np.array_equal(ctx.sample_row(P.theta_true, j)[0], ctx_g.sample_row(P.theta_true, j)[0])
    with pytest.raises(NotImplementedError):
        ctx.register(np.zeros(P.grid.n_voxels), np.zeros(P.N), P.theta_true, gradient="analytic")


def test_sinc_registration_recovers_known_motion():
    """Central-difference registration with the sinc PSF: the truth is a fixed
    point and perturbed motion is recovered on a textured phantom."""
    from scipy.ndimage import gaussian_filter
    P = synth.tiny_problem()
    X = gaussian_filter(np.random.default_rng(5).uniform(0, 1000, (32, 32, 32)), 1.5)
    X = (X - X.min()) / (X.max() - X.min()) * 1000.0
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches, psf="sinc")
    y, _, _ = ctx.simulate(X, P.theta_true)
    th_t, n_t = ctx.register(X, y, P.theta_true)
    assert np.allclose(th_t, P.theta_true, atol=1e-6) and np.allclose(n_t, 1.0)
    th0 = P.theta_true + synth.random_motion(P.M, 3.0, 1.0, 99)
    th, ncc = ctx.register(X, y, th0)
    dtr = np.abs(th[:, 3:] - P.theta_true[:, 3:]).max(1)
    drot = np.degrees(np.abs(th[:, :3] - P.theta_true[:, :3])).max(1)
    dtr0 = np.abs(th0[:, 3:] - P.theta_true[:, 3:]).max(1)
    assert np.median(dtr) < 0.03 and np.median(dtr) < 0.1 * np.median(dtr0)
    assert np.median(drot) < 0.35
    assert np.mean(ncc > 0.999) > 0.8
