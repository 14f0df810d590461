"""Pins for the oracle's geometry, PSF weights and forward model.

The observation model x_i = W_i y + n_i with W_i = D B T_i (paper Sec. I,
eq. (1)) is pinned by properties fixed by the mathematics, not by re-typing
the oracle's formula:
  * rotation matrices against an independent library (scipy), orthonormality;
  * every valid row of A sums to one (normalisation reading);
  * a constant volume simulates to that constant (partition of unity);
  * a brute-force dense A, evaluated by numpy over *all* voxels with
    scipy's rotation, equals the oracle's bounding-box rows;
  * a vanishing PSF reduces simulation to nearest-voxel sampling;
  * integer-voxel translations commute with the forward model.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_1611_07289_amd import synth
from tests._problems import brute_problem, tiny


def test_rotation_matches_scipy_extrinsic_xyz():
    rng = np.random.default_rng(0)
    for _ in range(20):
        th = rng.uniform(-math.pi, math.pi, size=3)
        R = oracle.rotation(th)
        ref = Rotation.from_euler("xyz", th).as_matrix()  # = Rz Ry Rx
        assert np.allclose(R, ref, atol=1e-14)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
    assert np.allclose(oracle.rotation([0, 0, 0]), np.eye(3))
    # a quarter turn about z takes x to y
    assert np.allclose(oracle.rotation([0, 0, math.pi / 2]) @ [1, 0, 0], [0, 1, 0])


def _dense_A(P: synth.Problem, k=3.0):
    """Dense A from scratch: numpy over every voxel of the grid."""
    g = P.grid
    ii, jj, kk = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.arange(g.nz),
                             indexing="ij")
    # flat voxel order X[(k*ny + j)*nx + i]
    vidx = (kk * g.ny + jj) * g.nx + ii
    vw = np.stack([ii, jj, kk, np.ones_like(ii)], -1).reshape(-1, 4) @ g.vox2world.T
    vidx = vidx.reshape(-1)
    A = np.zeros((P.N, g.n_voxels))
    valid = np.zeros(P.N, bool)
    tab = P.patches.table()
    off = P.patches.sample_off
    lo = -0.5
    for s in range(P.M):
        st, sl, x0, y0, w, h = tab[s]
        S = P.stacks[st]
        Lp, op = S.pix2world[:, :3], S.pix2world[:, 3]
        E = Lp / np.linalg.norm(Lp, axis=0)
        sig = S.fwhm_mm / (2 * math.sqrt(2 * math.log(2)))
        R = Rotation.from_euler("xyz", P.theta_true[s, :3]).as_matrix()
        c = Lp @ [x0 + (w - 1) / 2, y0 + (h - 1) / 2, sl] + op
        F = R @ E
        for l in range(w * h):
            u, v = x0 + l % w, y0 + l // w
            x = R @ (Lp @ [u, v, sl] + op - c) + c + P.theta_true[s, 3:]
            xv = np.linalg.solve(g.vox2world[:, :3], x - g.vox2world[:, 3])
            inside = np.all(xv >= lo) and np.all(xv < np.array([g.nx, g.ny, g.nz]) - 0.5)
            d = (vw - x) @ F
            Q = ((d / sig) ** 2).sum(1)
            gh = np.where(Q <= k * k, np.exp(-Q / 2) - math.exp(-k * k / 2), 0.0)
            Z = gh.sum()
            j = off[s] + l
            if inside and Z > 0:
                valid[j] = True
                A[j, vidx] = gh / Z
    return A, valid


@pytest.fixture(scope="module")
def brute():
    P = brute_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    return P, ctx


def test_bruteforce_dense_A_equals_oracle_rows(brute):
    P, ctx = brute
    A, valid = _dense_A(P)
    _, _, val = ctx.simulate(np.zeros(P.grid.n_voxels), P.theta_true)
    assert np.array_equal(val, valid)
    assert valid.sum() > 0.6 * P.N and (~valid).sum() > 0  # both cases occur
    nnz = 0
    for j in range(P.N):
        idx, w = ctx.sample_row(P.theta_true, j)
        row = np.zeros(P.grid.n_voxels)
        row[idx] = w
        assert np.allclose(row, A[j], rtol=1e-12, atol=1e-15), j
        nnz += idx.size
    # the same dense matrix reproduces simulate and its transpose backproject
    x = np.random.default_rng(1).normal(size=P.grid.n_voxels)
    r = np.random.default_rng(2).normal(size=P.N)
    yh, _, _ = ctx.simulate(x, P.theta_true)
    assert np.allclose(yh, A @ x, rtol=1e-12, atol=1e-12)
    bp = ctx.backproject(P.theta_true, r).reshape(-1)
    assert np.allclose(bp, A.T @ r, rtol=1e-12, atol=1e-12)
    assert nnz > 0


def test_support_backprojection_is_the_indicator_transpose(brute):
    """The support form of the adjoint (1/Z_j on every support voxel, used
    for the FP32 error bars) equals S^T (r / Z) with S the support pattern of
    the brute-force dense matrix; the per-voxel form agrees with the full one."""
    P, ctx = brute
    A, valid = _dense_A(P)
    _, Z, val = ctx.simulate(np.zeros(P.grid.n_voxels), P.theta_true)
    r = np.random.default_rng(4).normal(size=P.N)
    rz = np.where(val, r / np.where(val, Z, 1.0), 0.0)
    ref = (A > 0).T.astype(np.float64) @ rz
    got = ctx.backproject(P.theta_true, r, support=True).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14)
    vox = np.random.default_rng(5).choice(P.grid.n_voxels, 40, replace=False)
    gv = ctx.backproject_voxels(P.theta_true, r, vox, support=True)
    assert np.allclose(gv, got[vox], rtol=1e-12, atol=1e-14)


def test_rows_sum_to_one_and_constant_volume(brute):
    P, ctx = brute
    yh, Z, val = ctx.simulate(np.full(P.grid.n_voxels, 321.0), P.theta_true)
    assert np.allclose(yh[val], 321.0, rtol=1e-13)
    assert np.all(yh[~val] == 0)
    for j in np.nonzero(val)[0][::37]:
        _, w = ctx.sample_row(P.theta_true, j)
        assert abs(w.sum() - 1.0) < 1e-12


def test_tiny_support_size_and_weights_positive():
    P = tiny()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    sizes = []
    for j in range(0, P.N, 997):
        idx, w = ctx.sample_row(P.theta_true, j)
        if idx.size:
            assert np.all(w >= 0)
            sizes.append(idx.size)
    # FWHM (1,1,4) mm, k = 3: ellipsoid volume 4/3 pi k^3 sigma^3 ~ 34.6 voxels
    assert 25 < np.mean(sizes) < 45


def test_narrow_psf_is_nearest_voxel_sampling():
    """With a PSF much narrower than a voxel only the nearest voxel is in the
    support, so simulation samples the volume at the moved pixel centre."""
    g = synth.iso_grid(11)
    x = np.random.default_rng(3).uniform(0, 1, size=(11, 11, 11))
    c = synth.grid_center(g)
    st = synth.make_stack(c, *synth.orthogonal_frames()[1], 11, 11, 5, (1, 1), 2.0,
                          (0.05, 0.05, 0.05))
    P = synth.square_patches([st], 5, 5)
    ctx = oracle.Ctx(g, [st], P)
    th = np.zeros((P.M, 6))
    th[:, 3:] = [1.0, 0.0, -2.0]  # integer translation keeps centres on voxels
    yh, _, val = ctx.simulate(x, th)
    off = P.sample_off
    L, o = st.pix2world[:, :3], st.pix2world[:, 3]
    checked = 0
    for s in range(P.M):
        for l in range(P.w[s] * P.h[s]):
            u, v = P.x0[s] + l % P.w[s], P.y0[s] + l // P.w[s]
            pos = L @ [u, v, P.slice[s]] + o + th[s, 3:]
            i, j, k = np.rint(pos).astype(int)
            jj = off[s] + l
            if 0 <= i < 11 and 0 <= j < 11 and 0 <= k < 11:
                assert val[jj] and yh[jj] == pytest.approx(x[k, j, i], rel=1e-12)
                checked += 1
            else:
                assert not val[jj]
    assert checked > 100


def test_integer_translation_equivariance():
    P = tiny()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    X = np.asarray(P.x_true, np.float64)
    shift = np.array([2, -1, 3])  # voxels (x, y, z), 1 mm voxels
    Xs = np.zeros_like(X)
    # Xs(i + shift) = X(i)
    src = tuple(slice(max(0, -s), X.shape[a] - max(0, s)) for a, s in
                enumerate(shift[::-1]))
    dst = tuple(slice(max(0, s), X.shape[a] - max(0, -s)) for a, s in
                enumerate(shift[::-1]))
    Xs[dst] = X[src]
    th2 = P.theta_true.copy()
    th2[:, 3:] += shift
    y1, _, v1 = ctx.simulate(X, P.theta_true)
    y2, _, v2 = ctx.simulate(Xs, th2)
    # compare samples whose support stays well inside both grids
    rng = np.random.default_rng(5)
    js = rng.choice(np.nonzero(v1 & v2)[0], 300, replace=False)
    ok = 0
    for j in js:
        i1, _ = ctx.sample_row(P.theta_true, j)
        i2, _ = ctx.sample_row(th2, j)
        if i1.size != i2.size:
            continue  # support clipped by a border in one of them
        assert y2[j] == pytest.approx(y1[j], rel=1e-10, abs=1e-9)
        ok += 1
    assert ok > 100


def test_cheap_validity_equals_simulate_validity(brute):
    """The oracle's validity shortcut (nearest-voxel weight, else the full Z)
    reports exactly what simulate reports, with a mask and inactive patches."""
    for P, ctx in (brute, (tiny(), oracle.Ctx(tiny().grid, tiny().stacks, tiny().patches))):
        rng = np.random.default_rng(6)
        mask = (rng.uniform(size=P.N) > 0.1).astype(np.uint8)
        active = (rng.uniform(size=P.M) > 0.2).astype(np.uint8)
        for m, a in ((None, None), (mask, active)):
            _, _, v = ctx.simulate(np.zeros(P.grid.n_voxels), P.theta_true, m, a)
            assert np.array_equal(ctx.valid(P.theta_true, m, a), v)
