"""Edge cases of the hot path against the FP64 oracle: a ragged anisotropic
grid (37 x 29 x 23 voxels of 1.0 x 1.25 x 1.5 mm, so every brick axis ends in
a partial brick), an axial and an oblique stack, and patches of degenerate
shapes -- 1 x 1, a 1-pixel column strip, 13 x 7, a whole slice -- plus a
patch moved wholly out of the volume (every sample invalid), patches on the
first and last slices and a corner patch reaching outside the volume.  Checked: validity exactly,
simulation 1e-5, the adjoint within its bar, robust weights (the empty patch
takes no part), three SR iterations rel-L2 1e-4, NCC at fixed motion (0 for
the empty patch), and a build with every patch inactive (empty adjoint, the
update leaves the data term at 0)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from oracle import recon
from paper_1611_07289_amd import pvr, synth
from tests._tolerance import adjoint_bar
from tests.test_gpu_parity import _gpu_sr_loop, dev, host, sample_close


@pytest.fixture(scope="module")
def edge():
    print("[gpu] edge cases: ragged anisotropic grid, degenerate patches", flush=True)
    v2w = np.zeros((3, 4))
    v2w[0, 0], v2w[1, 1], v2w[2, 2] = 1.0, 1.25, 1.5
    v2w[:, 3] = (-3.0, 2.0, 5.0)
    g = synth.Grid(37, 29, 23, v2w)
    c = synth.grid_center(g)
    ex, ey, ez = np.eye(3)
    R = synth.axis_rotation(ex + 0.3 * ey, math.radians(25.0))
    stacks = [synth.make_stack(c, ex, ey, ez, 40, 30, 11, (1.0, 1.0), 3.0, (1.2, 1.2, 3.0)),
              synth.make_stack(c, R @ ex, R @ ey, R @ ez, 36, 36, 9, (1.1, 1.1), 3.5, (1.3, 1.3, 3.5))]
    rows = [  # stack, slice, x0, y0, w, h
        (0, 5, 10, 12, 1, 1),
        (0, 5, 20, 0, 1, 30),
        (0, 4, 3, 9, 13, 7),
        (0, 6, 0, 0, 40, 30),
        (0, 0, 5, 5, 16, 16),     # first slice
        (0, 10, 8, 8, 16, 16),    # last slice
        (0, 7, 8, 8, 16, 16),     # moved out of the volume below
        (1, 4, 0, 0, 36, 36),
        (1, 2, 11, 4, 13, 7),
        (1, 6, 30, 30, 6, 6),     # corner: partly outside the volume
        (1, 8, 2, 20, 1, 1),
    ]
    rows += [(s, k, x0, y0, 12, 12) for s in (0, 1) for k in range(1, 9, 2)
             for (x0, y0) in ((4, 4), (14, 10))]
    cols = np.asarray(rows, np.int32)
    pat = synth.Patches(*[cols[:, i].copy() for i in range(6)])
    th = synth.random_motion(pat.M, 6.0, 2.0, 901)
    th[6, 3:] = (0.0, 0.0, 200.0)  # every sample of patch 6 leaves the volume
    th32 = th.astype(np.float32).astype(np.float64)
    X = synth.phantom_ellipsoids(37, 902)[:23, :29, :37].astype(np.float32).copy()
    ctx = oracle.Ctx(g, stacks, pat)
    yc, _, val = ctx.simulate(X, th32)
    out = np.zeros(pat.M, bool)
    out[pat.M - 3] = True
    y = synth.corrupt(yc, pat, out, 0.01, 903, 904)
    plan = pvr.Plan([g], [stacks], [pat])
    plan.build(dev(th32.astype(np.float32)))
    torch.cuda.synchronize()
    off = pat.sample_off
    assert not val[off[6]:off[7]].any(), "patch 6 should be wholly invalid"
    assert 0 < val[off[9]:off[10]].mean() < 1, "patch 9 should reach outside the volume"
    return dict(g=g, stacks=stacks, pat=pat, th32=th32, X=X, ctx=ctx, y=y, val=val, plan=plan)


def test_edge_validity_and_simulation(edge):
    ctx, plan, X, th32, val = edge["ctx"], edge["plan"], edge["X"], edge["th32"], edge["val"]
    one = torch.ones(plan.V, dtype=torch.float32, device="cuda")
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(one, y_sim=ys)
    g1 = host(ys)
    assert np.array_equal(g1 > 0.5, val)
    assert np.allclose(g1[val], 1.0, atol=2e-6)
    plan.simulate(dev(X.reshape(-1)), y_sim=ys)
    g = host(ys)
    yo, _, _ = ctx.simulate(X, th32)
    assert np.all(g[~val] == 0)
    worst, _ = sample_close(g[val], yo[val])
    assert worst <= 1e-5


def test_edge_adjoint(edge):
    ctx, plan, th32 = edge["ctx"], edge["plan"], edge["th32"]
    rng = np.random.default_rng(5)
    r = rng.normal(size=plan.N).astype(np.float32)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    den = torch.empty_like(num)
    plan.backproject(dev(r), None, None, num, den)
    ro = ctx.backproject(th32, r.astype(np.float64)).reshape(-1)
    err = np.abs(host(num) - ro) / (adjoint_bar(ctx, th32, r) + 1e-30)
    assert err.max() <= 1.0
    do = ctx.backproject(th32, np.ones(plan.N)).reshape(-1)
    errd = np.abs(host(den) - do) / (adjoint_bar(ctx, th32, np.ones(plan.N)) + 1e-30)
    assert errd.max() <= 1.0


def test_edge_robust_weights_sr_and_ncc(edge):
    ctx, plan, th32, y, X, pat = edge["ctx"], edge["plan"], edge["th32"], edge["y"], edge["X"], edge["pat"]
    X0 = recon.initial_volume(ctx, y, th32)
    Xo = X0.copy()
    state = recon.EMState()
    Ws, pis = [], []
    for _ in range(3):
        Xo, state, diag = recon.sr_iteration(ctx, Xo, y, th32, state, recon.SRParams())
        Ws.append(diag["W"]); pis.append(diag["pi"])
    assert all(w[6] == 0 for w in Ws)  # the empty patch takes no part
    near = sum(int(np.sum(np.abs(pi - 0.5) < 1e-3)) for pi in pis)
    Xg, Wg = _gpu_sr_loop(plan, X0, y, 3, pvr.SRParams.make(), fix_w_list=Ws if near else None)
    assert all(w[6] == 0 for w in Wg)
    rel = np.linalg.norm(Xg.reshape(-1) - Xo.reshape(-1)) / np.linalg.norm(Xo)
    print(f"[gpu] edge cases: 3 SR iterations rel-L2 {rel:.2e}, near-threshold {near}")
    assert rel <= 1e-4
    ncc = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.register(dev(X.reshape(-1)), dev(y), dev(th32.astype(np.float32)), ncc,
                  params=pvr.RegParams.make(max_iter=0))
    no = ctx.ncc(X, y, th32)
    ng = host(ncc)
    assert ng[6] == 0 and no[6] == 0
    assert np.abs(ng - no).max() <= 1e-5


def test_edge_all_patches_inactive(edge):
    plan, th32, X = edge["plan"], edge["th32"], edge["X"]
    act = torch.zeros(plan.M, dtype=torch.uint8, device="cuda")
    plan.build(dev(th32.astype(np.float32)), active=act)
    e = torch.ones(plan.N, dtype=torch.float32, device="cuda")
    num = torch.full((plan.V,), 7.0, dtype=torch.float32, device="cuda")
    den = torch.full_like(num, 7.0)
    plan.backproject(e, None, None, num, den)
    assert float(num.abs().max()) == 0.0 and float(den.abs().max()) == 0.0
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(dev(X.reshape(-1)), y_sim=ys)
    assert float(ys.abs().max()) == 0.0
    Xd = dev(X.reshape(-1))
    Xn = torch.empty_like(Xd)
    plan.sr_update(Xd, num, den, Xn, pvr.SRParams.make(lam=0.0))
    assert torch.equal(Xn, Xd)
    plan.build(dev(th32.astype(np.float32)))
    plan.check()


def test_non_finite_motion_makes_a_patch_invalid(edge):
    """A patch whose motion is NaN or infinite has no valid sample: it
    simulates to 0, takes no part in the adjoint, and the other patches are
    unaffected (compared with the same build where that patch is inactive)."""
    plan, th32, X, pat = edge["plan"], edge["th32"], edge["X"], edge["pat"]
    rng = np.random.default_rng(9)
    r = dev(rng.normal(size=plan.N).astype(np.float32))
    off = pat.sample_off
    outs = []
    for bad in (float("nan"), float("inf")):
        th = th32.astype(np.float32).copy()
        th[2, 1] = bad
        th[4, 4] = -bad if bad == bad else bad
        plan.build(dev(th))
        ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
        plan.simulate(dev(X.reshape(-1)), y_sim=ys)
        num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
        den = torch.empty_like(num)
        plan.backproject(r, None, None, num, den)
        outs.append((host(ys).copy(), host(num).copy(), host(den).copy()))
    act = np.ones(pat.M, np.uint8)
    act[[2, 4]] = 0
    plan.build(dev(th32.astype(np.float32)), active=dev(act))
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(dev(X.reshape(-1)), y_sim=ys)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    den = torch.empty_like(num)
    plan.backproject(r, None, None, num, den)
    ref = (host(ys), host(num), host(den))
    for y_b, n_b, d_b in outs:
        assert np.all(y_b[off[2]:off[3]] == 0) and np.all(y_b[off[4]:off[5]] == 0)
        assert np.array_equal(y_b, ref[0])
        assert np.array_equal(n_b, ref[1]) and np.array_equal(d_b, ref[2])
    plan.build(dev(th32.astype(np.float32)))
    plan.check()
