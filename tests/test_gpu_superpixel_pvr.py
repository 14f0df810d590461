"""The hot path on superpixel patches (paper Sec. II "Patch Extraction"):
patches are the dilated superpixels' boxes with the pixels outside the
dilated superpixel masked out, through the plan's per-sample mask.

Inputs come from the oracle alone: the tiny 32^3 case's 24 slices are
simulated whole by the oracle, clustered by the oracle's SLIC (a = 8) and cut
into dilated superpixel patches (gamma = 3) by the oracle.  The GPU plan and
the oracle then run on the same patches, masks and motion: validity (the mask
included) exactly, simulated samples to 1e-5, the masked adjoint within the
bar of tests/_tolerance.py, NCC at fixed motion to 1e-5, and five SR
iterations to relative L2 1e-4."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from oracle import recon
from oracle import slic as oslic
from paper_1611_07289_amd import pvr, synth
from tests._tolerance import adjoint_bar
from tests.test_gpu_parity import _gpu_sr_loop, dev, host, sample_close

A, GAMMA = 8, 3


@pytest.fixture(scope="module")
def sp():
    print("[gpu] tiny32 superpixel patches: oracle slices, SLIC and packing", flush=True)
    P = synth.tiny_problem()
    whole = synth.square_patches(P.stacks, 32, 32)
    ctx_w = oracle.Ctx(P.grid, P.stacks, whole)
    th_w = synth.random_motion(whole.M, 3.0, 1.0, 71)
    imgs, _, _ = ctx_w.simulate(P.x_true, th_w)
    imgs = imgs.reshape(whole.M, 32, 32)
    cols = {k: [] for k in ("stack", "slice", "x0", "y0", "w", "h")}
    masks = []
    for i in range(whole.M):
        lab, _ = oslic.slic(imgs[i], A, 40.0, 5.0, iters=5)
        for (x0, y0, w, h, m) in oslic.superpixel_patches(lab, GAMMA):
            for k, v in zip(("stack", "slice", "x0", "y0", "w", "h"),
                            (whole.stack[i], whole.slice[i], x0, y0, w, h)):
                cols[k].append(v)
            masks.append(m.reshape(-1))
    pat = synth.Patches(*[np.asarray(cols[k], np.int32) for k in ("stack", "slice", "x0", "y0", "w", "h")])
    mask = np.concatenate(masks).astype(np.uint8)
    # each patch takes its slice's motion about its own centre: use the slice's
    # parameters plus a small per-patch offset (any motion will do here)
    slice_of = np.array([np.nonzero((whole.stack == s) & (whole.slice == k))[0][0]
                         for s, k in zip(pat.stack, pat.slice)])
    th = th_w[slice_of] + synth.random_motion(pat.M, 1.0, 0.5, 72)
    th32 = th.astype(np.float32).astype(np.float64)
    ctx = oracle.Ctx(P.grid, P.stacks, pat)
    y = np.concatenate([imgs[slice_of[s]][pat.y0[s]:pat.y0[s] + pat.h[s],
                                          pat.x0[s]:pat.x0[s] + pat.w[s]].reshape(-1)
                        for s in range(pat.M)]).astype(np.float32)
    plan = pvr.Plan([P.grid], [P.stacks], [pat])
    md = dev(mask)
    plan.build(dev(th32.astype(np.float32)), mask=md)
    torch.cuda.synchronize()
    assert 0.05 < 1 - mask.mean() < 0.9, "the masks should switch a real share of samples off"
    return dict(P=P, ctx=ctx, plan=plan, th32=th32, mask=mask, md=md, y=y)


def test_masked_validity_and_simulation(sp):
    P, ctx, plan, th32, mask = sp["P"], sp["ctx"], sp["plan"], sp["th32"], sp["mask"]
    yo, _, val = ctx.simulate(P.x_true, th32, mask=mask)
    assert not np.any(val & (mask == 0))
    one = torch.ones(plan.V, dtype=torch.float32, device="cuda")
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(one, y_sim=ys)
    assert np.array_equal(host(ys) > 0.5, val)
    plan.simulate(dev(P.x_true), y_sim=ys)
    g = host(ys)
    assert np.all(g[~val] == 0)
    worst, _ = sample_close(g[val], yo[val])
    assert worst <= 1e-5


def test_masked_adjoint(sp):
    P, ctx, plan, th32, mask = sp["P"], sp["ctx"], sp["plan"], sp["th32"], sp["mask"]
    rng = np.random.default_rng(3)
    r = rng.normal(size=plan.N).astype(np.float32)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    den = torch.empty_like(num)
    plan.backproject(dev(r), None, None, num, den)
    ro = ctx.backproject(th32, r.astype(np.float64), mask=mask).reshape(-1)
    r_in = r.astype(np.float64) * (mask != 0)
    err = np.abs(host(num) - ro) / (adjoint_bar(ctx, th32, r_in) + 1e-30)
    assert err.max() <= 1.0
    do = ctx.backproject(th32, np.ones(plan.N), mask=mask).reshape(-1)
    errd = np.abs(host(den) - do) / (adjoint_bar(ctx, th32, (mask != 0).astype(np.float64)) + 1e-30)
    assert errd.max() <= 1.0


def test_masked_ncc_and_sr_iterations(sp):
    P, ctx, plan, th32, mask, y = sp["P"], sp["ctx"], sp["plan"], sp["th32"], sp["mask"], sp["y"]
    ncc = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    tt = dev(th32.astype(np.float32))
    plan.register(dev(P.x_true), dev(y), tt, ncc, params=pvr.RegParams.make(max_iter=0))
    no = ctx.ncc(P.x_true, y.astype(np.float64), th32, mask=mask)
    assert np.abs(host(ncc) - no).max() <= 1e-5
    X0 = recon.initial_volume(ctx, y.astype(np.float64), th32, mask)
    X = X0.copy()
    state = recon.EMState()
    Ws, pis = [], []
    for _ in range(5):
        X, state, diag = recon.sr_iteration(ctx, X, y.astype(np.float64), th32, state,
                                            recon.SRParams(), mask)
        Ws.append(diag["W"]); pis.append(diag["pi"])
    # patches whose posterior sits at the 0.5 threshold may classify either
    # way in FP32: then the oracle's weights are imposed on both sides
    near = sum(int(np.sum(np.abs(pi - 0.5) < 1e-3)) for pi in pis)
    Xg, Wg = _gpu_sr_loop(plan, X0, y, 5, pvr.SRParams.make(), fix_w_list=Ws if near else None)
    rel = np.linalg.norm(Xg.reshape(-1) - X.reshape(-1)) / np.linalg.norm(X)
    print(f"[gpu] superpixel patches: 5 SR iterations rel-L2 {rel:.2e}, near-threshold {near}")
    assert rel <= 1e-4


@pytest.mark.parametrize("scale", [0, 1])
def test_multiscale_superpixels_active_set(scale):
    """Multi-scale superpixels: the oracle's superpixel patches of two sizes
    (a = 8 and a = 12) in one plan with their masks; a build with one size's
    active set runs three SR iterations from that size's patches only,
    against the oracle with the same mask and active set."""
    from paper_1611_07289_amd import driver
    P = synth.tiny_problem()
    whole = synth.square_patches(P.stacks, 32, 32)
    ctx_w = oracle.Ctx(P.grid, P.stacks, whole)
    th_w = synth.random_motion(whole.M, 3.0, 1.0, 81)
    imgs = ctx_w.simulate(P.x_true, th_w)[0].reshape(whole.M, 32, 32)
    cols = {k: [] for k in ("stack", "slice", "x0", "y0", "w", "h")}
    masks, sc, owner = [], [], []
    for si, (a, gam) in enumerate([(8, 3), (12, 5)]):
        for i in range(whole.M):
            lab, _ = oslic.slic(imgs[i], a, 40.0, 5.0, iters=4)
            for (x0, y0, w, h, m) in oslic.superpixel_patches(lab, gam):
                for k, v in zip(("stack", "slice", "x0", "y0", "w", "h"),
                                (whole.stack[i], whole.slice[i], x0, y0, w, h)):
                    cols[k].append(v)
                masks.append(m.reshape(-1)); sc.append(si); owner.append(i)
    pat = synth.Patches(*[np.asarray(cols[k], np.int32) for k in ("stack", "slice", "x0", "y0", "w", "h")])
    mask = np.concatenate(masks).astype(np.uint8)
    sc, owner = np.asarray(sc), np.asarray(owner)
    th32 = (th_w[owner] + synth.random_motion(pat.M, 1.0, 0.5, 82)).astype(np.float32).astype(np.float64)
    y = np.concatenate([imgs[owner[s]][pat.y0[s]:pat.y0[s] + pat.h[s],
                                       pat.x0[s]:pat.x0[s] + pat.w[s]].reshape(-1)
                        for s in range(pat.M)])
    active = (sc == scale).astype(np.uint8)
    ctx = oracle.Ctx(P.grid, P.stacks, pat)
    X0 = recon.initial_volume(ctx, y, th32, mask, active)
    X = X0
    state = recon.EMState()
    pis, Ws = [], []
    for _ in range(3):
        X, state, diag = recon.sr_iteration(ctx, X, y, th32, state, recon.SRParams(), mask, active)
        pis.append(diag["pi"]); Ws.append(diag["W"])
    near = sum(int(np.sum(np.abs(pi - 0.5) < 1e-3)) for pi in pis)
    plan = pvr.Plan([P.grid], [P.stacks], [pat])
    plan.build(dev(th32.astype(np.float32)), active=dev(active), mask=dev(mask))
    buf = driver.Buffers(plan)
    yd = dev(y.astype(np.float32))
    Xg = driver.initial_volume(plan, yd, buf)
    driver.sr_iterations(plan, Xg, yd, buf, 3)
    g = host(Xg).astype(np.float64)
    rel = np.linalg.norm(g - X.reshape(-1)) / np.linalg.norm(X)
    print(f"[gpu] multi-scale superpixels, scale {scale} ({int(active.sum())} of {pat.M} patches): "
          f"3 SR iterations rel-L2 {rel:.2e}, near-threshold {near}")
    if near:
        # a posterior within rounding of the 0.5 threshold: the same three
        # iterations from the oracle's X_0 with the oracle's patch weights
        Xf, _ = _gpu_sr_loop(plan, X0, y, 3, pvr.SRParams.make(), fix_w_list=Ws)
        rel = np.linalg.norm(Xf.reshape(-1) - X.reshape(-1)) / np.linalg.norm(X)
        print(f"[gpu] multi-scale superpixels, scale {scale}: with the oracle's W, rel-L2 {rel:.2e}")
    assert rel <= 1e-4
    assert np.all(host(buf.W)[active == 0] == 0)


@pytest.mark.parametrize("gradient", ["fd", "exact"])
def test_masked_registration_matches_oracle(sp, gradient):
    """Registration of the superpixel patches (masked samples excluded from
    the NCC) from perturbed motion: the same outcome as the oracle's."""
    import math
    P, ctx, plan, th32, mask, y = sp["P"], sp["ctx"], sp["plan"], sp["th32"], sp["mask"], sp["y"]
    from scipy.ndimage import gaussian_filter
    X = gaussian_filter(np.random.default_rng(5).uniform(0, 1000, (32, 32, 32)), 1.5)
    X = ((X - X.min()) / (X.max() - X.min()) * 1000.0).astype(np.float32)
    yt = ctx.simulate(X, th32, mask=mask)[0].astype(np.float32)
    th0 = (th32 + synth.random_motion(len(th32), 3.0, 1.0, 99)).astype(np.float32)
    tho, nco = ctx.register(X, yt, th0.astype(np.float64), mask=mask,
                            gradient="analytic" if gradient == "exact" else "fd")
    plan.build(dev(th0), mask=sp["md"])
    tt = dev(th0)
    ncc = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.register(dev(X), dev(yt), tt, ncc, params=pvr.RegParams.make(exact=gradient == "exact"))
    thg, ncg = host(tt).astype(np.float64), host(ncc)
    n0 = ctx.ncc(X, yt, th0.astype(np.float64), mask=mask)
    assert np.all(ncg >= n0 - 1e-5)
    drot_g = np.degrees(np.abs(thg[:, :3] - th32[:, :3])).max(1)
    drot_o = np.degrees(np.abs(tho[:, :3] - th32[:, :3])).max(1)
    dtr_g = np.abs(thg[:, 3:] - th32[:, 3:]).max(1)
    dtr_o = np.abs(tho[:, 3:] - th32[:, 3:]).max(1)
    same = (np.abs(thg - tho)[:, :3].max(1) < math.radians(0.25)) & (np.abs(thg - tho)[:, 3:].max(1) < 0.1)
    print(f"[gpu] masked reg ({gradient}): median rot err gpu {np.median(drot_g):.3f} ora "
          f"{np.median(drot_o):.3f}; trans gpu {np.median(dtr_g):.4f} ora {np.median(dtr_o):.4f}; "
          f"agreement {same.mean():.3f}")
    assert same.mean() >= 0.95
    assert np.median(drot_g) <= max(0.35, 1.25 * np.median(drot_o))
    assert np.median(dtr_g) <= max(0.03, 1.25 * np.median(dtr_o))
    assert np.mean(ncg > 0.999) >= np.mean(nco > 0.999) - 0.05
    plan.build(dev(th32.astype(np.float32)), mask=sp["md"])
