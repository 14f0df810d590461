"""Pins for the SR volume update and its edge-preserving regulariser.

The paper reintegrates registered patches by gradient-descent super-resolution
(Sec. II) with anisotropic-diffusion regularisation from the cited method
(Sec. I-A).  Pinned by: antisymmetric fluxes (the regulariser conserves the
sum), zero response to constants and interior linear ramps, bounded flux across
a large step, and the textbook special case: with W p = 1 and lambda = 0 the
update is SIRT, whose fixed point solves the least-squares normal equations
(checked against numpy.linalg.lstsq on a dense A).
"""
import numpy as np
import pytest

import oracle
from oracle import recon
from oracle.update import regulariser, sr_update
from tests._problems import brute_problem


def test_regulariser_conserves_sum_and_kills_constants_and_ramps():
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1000, size=(9, 10, 11))
    R = regulariser(X, 150.0)
    assert abs(R.sum()) < 1e-9 * np.abs(R).sum()
    assert np.all(regulariser(np.full((6, 6, 6), 7.0), 150.0) == 0)
    z, y, x = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    ramp = 3.0 * x - 2.0 * y + 5.0 * z
    Rr = regulariser(ramp, 150.0)
    assert np.allclose(Rr[1:-1, 1:-1, 1:-1], 0.0, atol=1e-10)
    assert np.abs(Rr).max() > 1.0  # borders are not balanced (Neumann)


def test_regulariser_edge_flux_bounded():
    X = np.zeros((5, 5, 5))
    X[:, :, 3:] = 1e6  # a step far above delta
    delta = 150.0
    R = regulariser(X, delta)
    # each neighbour flux is bounded by b_d * delta (9 neighbours across)
    b = np.array([1.0] + [1 / np.sqrt(2)] * 4 + [1 / np.sqrt(3)] * 4)
    assert R[2, 2, 2] <= b.sum() * delta + 1e-9
    assert R[2, 2, 2] > 0.9 * b.sum() * delta


def test_update_formula_and_clamp():
    X = np.array([[[1.0, 2.0], [3.0, 4.0]]])
    num = np.array([[[1.0, -10.0], [0.5, 0.0]]])
    den = np.array([[[2.0, 1.0], [0.0, 1.0]]])
    out = sr_update(X, num, den, alpha=1.0, lam=0.0)
    assert np.allclose(out, [[[1.5, 0.0], [3.0, 4.0]]])


def test_sirt_fixed_point_solves_least_squares():
    """With W p = 1 and lambda = 0 the update is SIRT: the least-squares
    solution of the normal equations is its fixed point, and from X_0 the
    data residual falls monotonically towards the least-squares residual."""
    P = brute_problem(seed=3)
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    th = P.theta_true
    A = np.zeros((P.N, P.grid.n_voxels))
    for j in range(P.N):
        idx, w = ctx.sample_row(th, j)
        A[j, idx] = w
    yh0, _, valid = ctx.simulate(np.asarray(P.x_true, np.float64), th)
    y = yh0 + np.random.default_rng(4).normal(0, 20.0, P.N)
    y = np.where(valid, y, 0.0)
    den = ctx.backproject(th, np.ones(P.N)).reshape(-1)
    cols = A.any(axis=0)
    Av = A[valid][:, cols]
    ref, *_ = np.linalg.lstsq(Av, y[valid], rcond=None)
    res_ref = np.linalg.norm(Av @ ref - y[valid])

    def step(X):
        yh, _, _ = ctx.simulate(X, th)
        num = ctx.backproject(th, np.where(valid, y - yh, 0.0)).reshape(-1)
        return sr_update(X, num, den, alpha=1.0, lam=0.0, clamp_min=None)

    Xs = np.zeros(P.grid.n_voxels)
    Xs[cols] = ref
    assert np.allclose(step(Xs)[cols], ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())
    X = recon.initial_volume(ctx, y, th).reshape(-1)
    res = [np.linalg.norm(Av @ X[cols] - y[valid])]
    for _ in range(400):
        X = step(X)
        res.append(np.linalg.norm(Av @ X[cols] - y[valid]))
    assert np.all(np.diff(res) <= 1e-9 * res[0])
    assert res[-1] >= res_ref * (1 - 1e-9)
    assert (res[-1] - res_ref) < 0.1 * (res[0] - res_ref)


def test_psnr_hand_computed():
    """PSNR = 10 log10(I_max^2 / MSE) (Sec. IV-A, base-10 logarithm read):
    errors of +-10 on every voxel of a truth whose maximum is 1000 give
    MSE = 100 and exactly 40 dB; a mask restricts the mean; zero error is
    infinite."""
    import math
    from oracle import recon
    T = np.array([[0.0, 1000.0], [500.0, 250.0]])
    X = T + np.array([[10.0, -10.0], [10.0, -10.0]])
    assert recon.psnr(X, T) == pytest.approx(40.0, abs=1e-12)
    X2 = T + np.array([[0.0, 20.0], [0.0, 0.0]])
    m = np.array([[False, True], [True, False]])
    # masked MSE = (400 + 0) / 2 = 200
    assert recon.psnr(X2, T, m) == pytest.approx(10 * math.log10(1e6 / 200), abs=1e-12)
    assert recon.psnr(T, T) == float("inf")
