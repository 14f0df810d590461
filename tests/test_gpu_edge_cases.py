"""Edge cases of the hot path against the FP64 oracle, on one plan built to
contain them:

  * a ragged grid (37 x 29 x 23: partial bricks and sub-bricks on every
    axis) with anisotropic spacing (1, 1.2, 0.9) and a rotated, shifted
    voxel-to-world map;
  * two stacks (one along the grid, one oblique at 25 deg, anisotropic
    pixels and thickness), and a third placed 100 mm away, outside the
    volume;
  * patches of 1 x 1 pixel, ragged sizes (17 x 5, 3 x 29), whole slices (the
    largest a slice allows, partly outside the volume) and one whole slice of
    the outside stack (every sample invalid).

Checked: every simulated sample (and validity) and every voxel of the
adjoint against the oracle, the adjoint identity, five SR iterations (patch
weights pinned to the oracle's where a posterior sits on the 0.5 threshold)
to 1e-4 relative L2, and a registration pass in which the patch without
valid samples and the 1 x 1 patch (flat) keep their motion and every other
patch reaches the oracle's NCC (the oracle's NCC at the GPU's motion, within
1e-4)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from oracle import recon
from paper_1611_07289_amd import pvr, synth
from tests._tolerance import adjoint_bar
from tests.test_gpu_parity import _gpu_sr_loop, dev, host

OUTSIDE = 6  # index of the patch of the stack outside the volume


def _problem():
    from scipy.ndimage import gaussian_filter
    R = synth.axis_rotation(np.array([1.0, 2.0, 3.0]), 0.3)
    v2w = np.zeros((3, 4))
    v2w[:, :3] = R @ np.diag([1.0, 1.2, 0.9])
    v2w[:, 3] = [5.0, -3.0, 2.0]
    g = synth.Grid(37, 29, 23, v2w)
    c = synth.grid_center(g)
    fr = synth.orthogonal_frames([25.0])
    e1, e2, n = (R @ np.asarray(v, float) for v in fr[0])
    stacks = [
        synth.make_stack(c, e1, e2, n, 40, 36, 10, (1.0, 1.0), 2.5, (1.0, 1.0, 2.5)),
        synth.make_stack(c, *fr[3], 33, 41, 12, (0.9, 1.1), 2.0, (0.9, 1.1, 2.0)),
        synth.make_stack(c + np.array([100.0, 0.0, 0.0]), *fr[0], 12, 12, 3, (1.0, 1.0), 2.0,
                         (1.0, 1.0, 2.0)),
    ]
    rows = [  # stack, slice, x0, y0, w, h
        (0, 5, 20, 18, 1, 1),
        (0, 5, 3, 4, 17, 5),
        (0, 4, 30, 2, 3, 29),
        (0, 6, 0, 0, 40, 36),
        (1, 6, 0, 0, 33, 41),
        (1, 0, 5, 7, 20, 20),
        (2, 1, 0, 0, 12, 12),
    ]
    t = np.asarray(rows, np.int32)
    P = synth.Patches(t[:, 0], t[:, 1], t[:, 2], t[:, 3], t[:, 4], t[:, 5])
    rng = np.random.default_rng(41)
    x = gaussian_filter(rng.uniform(0, 1000, (g.nz, g.ny, g.nx)), 1.2).astype(np.float32)
    th = synth.random_motion(P.M, 4.0, 1.5, 42)
    return synth.Problem("edge", g, stacks, P, x, th, np.zeros(P.M, bool), 4200, 0.01, 0.0)


@pytest.fixture(scope="module")
def edge():
    P = _problem()
    print(f"[gpu] edge cases: grid 37x29x23, M={P.M}, N={P.N}", flush=True)
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    plan = pvr.Plan.from_problems([P])
    plan.build(dev(P.theta_true, torch.float32))
    th32 = np.asarray(P.theta_true, np.float32).astype(np.float64)
    yo, Z, val = ctx.simulate(P.x_true, th32)
    return dict(P=P, ctx=ctx, plan=plan, th32=th32, y=yo, val=val)


def test_edge_simulate_every_sample(edge):
    P, plan, yo, val = edge["P"], edge["plan"], edge["y"], edge["val"]
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(dev(P.x_true.reshape(-1)), y_sim=ys)
    g = host(ys)
    one = torch.ones(plan.V, device="cuda")
    v1 = torch.empty_like(ys)
    plan.simulate(one, y_sim=v1)
    assert np.array_equal(host(v1) > 0.5, val)
    off = P.patches.sample_off
    assert not val[off[OUTSIDE]:off[OUTSIDE + 1]].any()
    assert 0 < val.mean() < 1  # some samples of the whole slices fall outside
    scale = np.maximum(np.abs(yo), 1e-3 * np.abs(yo).max())
    worst = float((np.abs(g - yo) / scale).max())
    print(f"[gpu] edge simulate: {val.sum()} valid of {P.N}, worst {worst:.2e}", flush=True)
    assert worst <= 1e-5


def test_edge_backproject_every_voxel_and_adjoint_identity(edge):
    P, ctx, plan, th32 = edge["P"], edge["ctx"], edge["plan"], edge["th32"]
    rng = np.random.default_rng(43)
    r = rng.normal(size=P.N).astype(np.float32)
    p = rng.uniform(0, 1, size=P.N).astype(np.float32)
    w = rng.uniform(0.2, 1.0, size=P.M).astype(np.float32)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    den = torch.empty_like(num)
    plan.backproject(dev(r), dev(p), dev(w), num, den)
    n1, d1 = host(num), host(den)
    ws = w.astype(np.float64)[ctx.patch_of_sample]
    ro = ctx.backproject(th32, ws * p * r).reshape(-1)
    do = ctx.backproject(th32, ws * p).reshape(-1)
    en = float((np.abs(n1 - ro) / (adjoint_bar(ctx, th32, ws * p * r) + 1e-30)).max())
    ed = float((np.abs(d1 - do) / (adjoint_bar(ctx, th32, ws * p) + 1e-30)).max())
    print(f"[gpu] edge backproject: {int(np.sum(do > 0))} covered voxels of {P.grid.n_voxels}, "
          f"worst / bar num {en:.2e} den {ed:.2e}", flush=True)
    assert en <= 1.0 and ed <= 1.0
    x = dev(rng.normal(size=plan.V).astype(np.float32))
    rr = dev(rng.normal(size=plan.N).astype(np.float32))
    Ax = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(x, y_sim=Ax)
    ATr = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    plan.backproject(rr, num=ATr)
    lhs = float((Ax.double() * rr.double()).sum())
    rhs = float((x.double() * ATr.double()).sum())
    scale = float((Ax.double().abs() * rr.double().abs()).sum())
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_edge_sr_iterations_match_oracle(edge):
    P, ctx, plan, th32 = edge["P"], edge["ctx"], edge["plan"], edge["th32"]
    y = (edge["y"] + np.random.default_rng(44).normal(0, 5.0, P.N)).astype(np.float32)
    y = np.where(edge["val"], y, 0.0).astype(np.float32)
    X0 = recon.initial_volume(ctx, y, th32)
    X = X0.copy()
    state = recon.EMState()
    Ws, pis = [], []
    for it in range(5):
        X, state, diag = recon.sr_iteration(ctx, X, y, th32, state, recon.SRParams())
        Ws.append(diag["W"])
        pis.append(diag["pi"])
    assert all(W[OUTSIDE] == 0 for W in Ws)
    near = sum(int(np.sum(np.abs(pi - 0.5) < 1e-3)) for pi in pis)
    Xg, Wg = _gpu_sr_loop(plan, X0, y, 5, pvr.SRParams.make(), fix_w_list=Ws if near else None)
    assert all(W[OUTSIDE] == 0 for W in Wg)
    rel = np.linalg.norm(Xg.reshape(-1) - X.reshape(-1)) / np.linalg.norm(X)
    print(f"[gpu] edge: 5 SR iterations rel-L2 {rel:.2e} (near-threshold {near})", flush=True)
    assert rel <= 1e-4


def test_edge_registration_keeps_patches_without_signal(edge):
    P, ctx, plan, th32 = edge["P"], edge["ctx"], edge["plan"], edge["th32"]
    y = edge["y"].astype(np.float32)
    th0 = (th32 + synth.random_motion(P.M, 2.0, 0.5, 45)).astype(np.float32)
    tt = dev(th0)
    ncc = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    ymax = float(np.abs(y).max())
    plan.build(dev(th0))
    plan.register(dev(P.x_true.reshape(-1)), dev(y), tt, ncc,
                  params=pvr.RegParams.make(min_std=0.01 * ymax, exact=True))
    thg = host(tt)
    plan.build(dev(th32.astype(np.float32)))
    assert np.array_equal(thg[OUTSIDE], th0[OUTSIDE])  # no valid sample
    assert np.array_equal(thg[0], th0[0])              # 1 x 1: no spread to correlate
    n0 = ctx.ncc(P.x_true, y, th0.astype(np.float64))
    assert np.all(host(ncc) >= n0 - 1e-5)
    tho, nco = ctx.register(P.x_true, y, th0.astype(np.float64), min_std=0.01 * ymax,
                            gradient="analytic")
    d = np.abs(thg.astype(np.float64) - tho)
    same = (d[:, :3].max(1) < math.radians(0.25)) & (d[:, 3:].max(1) < 0.1)
    ncg = ctx.ncc(P.x_true, y, thg.astype(np.float64))
    print(f"[gpu] edge registration: agreement with the oracle {same.mean():.3f}; NCC gpu "
          f"{np.round(ncg, 5)} oracle {np.round(nco, 5)}", flush=True)
    # every patch ends at least as well aligned as the oracle leaves it
    assert np.all(ncg >= nco - 1e-4)
