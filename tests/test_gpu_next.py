"""Rows beyond the SR hot path, built on its calls, against the oracle.

  * rigidity / uncertainty maps (sample posteriors and patch potentials
    integrated into the volume with the reconstruction's PSF, normalised by
    A^T 1): voxel-wise against the oracle's ratio of the same back-projections,
    within (bar_num + |map| bar_den) / den + 1e-6 |map| -- the adjoint bars
    of tests/_tolerance.py carried through the division.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402  (CPU import is fine; GPU use is gated by the marker)

import oracle
from oracle import recon
from paper_1611_07289_amd import driver, pvr, synth
from tests._gpu import sr_loop
from tests._tolerance import adjoint_bar


def test_uncertainty_maps_match_oracle():
    P = synth.tiny_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    th32 = np.asarray(P.theta_true, np.float32).astype(np.float64)
    rng = np.random.default_rng(21)
    p = rng.uniform(0, 1, size=P.N).astype(np.float32)
    pbar = rng.uniform(0, 1, size=P.M).astype(np.float32)
    plan = pvr.Plan.from_problems([P])
    plan.build(torch.from_numpy(np.asarray(P.theta_true, np.float32)).cuda())
    buf = driver.Buffers(plan)
    mp, mb = driver.uncertainty_maps(plan, torch.from_numpy(p).cuda(), torch.from_numpy(pbar).cuda(), buf)
    torch.cuda.synchronize()
    den = ctx.backproject(th32, np.ones(P.N)).reshape(-1)
    bar_d = adjoint_bar(ctx, th32, np.ones(P.N))
    for got, r, name in ((mp, p.astype(np.float64), "p"),
                         (mb, pbar.astype(np.float64)[ctx.patch_of_sample], "pbar")):
        ref = recon.initial_volume(ctx, r, th32).reshape(-1)
        bar_n = adjoint_bar(ctx, th32, r)
        g = got.cpu().numpy().astype(np.float64)
        # the den > 1e-6 decision is taken on FP32 sums on the GPU: voxels
        # whose den lies within its bar of the threshold may go either way
        near = np.abs(den - 1e-6) <= bar_d
        ok = (den > 1e-6) & ~near
        allowed = (bar_n[ok] + np.abs(ref[ok]) * bar_d[ok]) / den[ok] + 1e-6 * np.abs(ref[ok])
        worst = float((np.abs(g[ok] - ref[ok]) / allowed).max())
        print(f"[gpu] uncertainty map {name}: worst error / bar {worst:.2e}")
        assert worst <= 1.0
        assert np.all(g[(den <= 1e-6) & ~near] == 0)
        assert np.all((g >= 0) & (g <= 1 + 1e-5))


@pytest.mark.parametrize("scale", [0, 1])
def test_multiscale_active_set_sr_matches_oracle(scale):
    """Multi-scale patches: one plan holds the patches of two sizes (8 and 16
    pixels on a 32^3 problem); a build with the active mask of one scale runs
    SR iterations from that scale's patches only, against the oracle run with
    the same active set."""
    P, sc = synth.multiscale_problem(seed_cfg=7, n=32, slices=8, sizes=(8, 16))
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    th32 = np.asarray(P.theta_true, np.float32).astype(np.float64)
    yc, _, _ = ctx.simulate(P.x_true, th32)
    y = synth.corrupt(yc, P.patches, P.outlier_patch, 0.01, P.seed_base + 3, P.seed_base + 5)
    active = (sc == scale).astype(np.uint8)
    # oracle: initial volume and 3 SR iterations on the active patches
    X0 = recon.initial_volume(ctx, y, th32, active=active)
    X = X0
    state = recon.EMState()
    pis, Ws = [], []
    for _ in range(3):
        X, state, diag = recon.sr_iteration(ctx, X, y, th32, state, recon.SRParams(), active=active)
        pis.append(diag["pi"]); Ws.append(diag["W"])
    near = sum(int(np.sum(np.abs(pi - 0.5) < 1e-3)) for pi in pis)
    # GPU through the driver
    plan = pvr.Plan.from_problems([P])
    plan.build(torch.from_numpy(np.asarray(P.theta_true, np.float32)).cuda(),
               active=torch.from_numpy(active).cuda())
    buf = driver.Buffers(plan)
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    Xg = driver.initial_volume(plan, yd, buf)
    driver.sr_iterations(plan, Xg, yd, buf, 3)
    torch.cuda.synchronize()
    g = Xg.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - X.reshape(-1)) / np.linalg.norm(X)
    print(f"[gpu] multiscale scale {scale} ({int(active.sum())} of {P.M} patches): "
          f"3 SR iterations rel-L2 {rel:.2e}, near-threshold {near}")
    if near:
        # a posterior within rounding of the 0.5 threshold: the same three
        # iterations from the oracle's X_0 with the oracle's patch weights
        Xf, _ = sr_loop(plan, X0, y, 3, fix_w_list=Ws)
        rel = np.linalg.norm(Xf.reshape(-1) - X.reshape(-1)) / np.linalg.norm(X)
        print(f"[gpu] multiscale scale {scale}: with the oracle's W, rel-L2 {rel:.2e}")
    assert rel <= 1e-4
    # inactive patches take no part: their samples carry weight 0
    W = buf.W.cpu().numpy()
    assert np.all(W[active == 0] == 0)
