"""Parity at full size: the 256^3 four-stack uterus workload (11 760 patches
of 64 x 64, 48.2 M samples) in the launch configuration the benchmark times,
against the FP64 oracle on sampled outputs it computes one by one, plus
properties that hold at any size.

  * simulate: 4 000 random samples and every sample of three whole patches,
    |y_gpu - y_ora| <= 1e-5 max(|y_ora|, 1e-3 max|y_ora|), validity exact;
  * back-projection (with per-sample p and patch weights W): 300 voxels
    (random, plus voxels around the volume centre where many patches overlap)
    within the bar of tests/_tolerance.py;
  * adjoint identity <A x, r> = <x, A^T r> in FP32 relative to
    sum |A x| |r| <= 1e-5; A 1 = 1 on valid samples; bitwise repeatable
    back-projection;
  * robust weights on seeded residuals at full size against the oracle's
    E-step, potentials, patch classification and M-step;
  * the volume update on two 34^3 crops (one at the volume corner, one inside)
    against the oracle, interior voxels of each crop;
  * registration (either gradient) of 24 sampled patches from perturbed
    motion, observations simulated by the oracle: the oracle's outcome on
    >= 95 % of them, no NCC lowered, the other patches untouched.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402  (CPU import is fine; GPU use is gated by the marker)

import oracle
from oracle import recon
from oracle.update import sr_update as ora_update
from paper_1611_07289_amd import pvr, synth
from tests._tolerance import adjoint_bar


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def full():
    print("[gpu] uterus256: generating and building", flush=True)
    P = synth.full_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    plan = pvr.Plan.from_problems([P])
    th32 = np.asarray(P.theta_true, np.float32).astype(np.float64)
    plan.build(dev(P.theta_true, torch.float32))
    torch.cuda.synchronize()
    print(f"[gpu] uterus256: N={plan.N} M={plan.M}", flush=True)
    return dict(P=P, ctx=ctx, plan=plan, th32=th32)


def test_full_simulate_sampled_matches_oracle(full):
    P, ctx, plan, th32 = full["P"], full["ctx"], full["plan"], full["th32"]
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(dev(P.x_true.reshape(-1)), y_sim=ys)
    g = host(ys)
    rng = np.random.default_rng(11)
    off = P.patches.sample_off
    whole = [np.arange(off[s], off[s + 1]) for s in rng.choice(P.M, 3, replace=False)]
    js = np.unique(np.concatenate([rng.choice(plan.N, 4000, replace=False)] + whole))
    yo, _, val = ctx.simulate(P.x_true, th32, samples=js)
    assert np.array_equal(g[js] != 0, val & (yo != 0))
    scale = np.maximum(np.abs(yo), 1e-3 * np.abs(yo).max())
    worst = float((np.abs(g[js] - yo) / scale).max())
    print(f"[gpu] full-size simulate: {js.size} samples, worst rel err {worst:.2e}")
    assert worst <= 1e-5


def test_full_normalisation_and_adjoint_identity(full):
    plan, ctx = full["plan"], full["ctx"]
    one = torch.ones(plan.V, dtype=torch.float32, device="cuda")
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(one, y_sim=ys)
    v = ys > 0.5
    assert torch.all(torch.abs(ys[v] - 1) <= 2e-6)
    assert torch.all(ys[~v] == 0)
    assert np.array_equal(host(v), ctx.valid(full["th32"])), "validity differs from the oracle"
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.rand(plan.V, generator=g, device="cuda")
    r = torch.randn(plan.N, generator=g, device="cuda")
    Ax = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(x, y_sim=Ax)
    ATr = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    plan.backproject(r, num=ATr)
    lhs = float(torch.dot(Ax.double(), r.double()))
    rhs = float(torch.dot(x.double(), ATr.double()))
    scale = float(torch.dot(Ax.double().abs(), r.double().abs()))
    print(f"[gpu] full-size adjoint identity: |lhs - rhs| / scale = {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_full_backproject_sampled_matches_oracle(full):
    P, ctx, plan, th32 = full["P"], full["ctx"], full["plan"], full["th32"]
    rng = np.random.default_rng(12)
    r = rng.normal(size=plan.N).astype(np.float32)
    p = rng.uniform(0, 1, size=plan.N).astype(np.float32)
    w = rng.uniform(0.2, 1.0, size=plan.M).astype(np.float32)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    den = torch.empty_like(num)
    plan.backproject(dev(r), dev(p), dev(w), num, den)
    n1, d1 = host(num).copy(), host(den).copy()
    plan.backproject(dev(r), dev(p), dev(w), num, den)
    assert np.array_equal(host(num), n1) and np.array_equal(host(den), d1), "not bitwise repeatable"
    # voxels: random over the grid, and a block around the volume centre
    # (dense overlap of patches and stacks)
    n = P.grid.nx
    vox = list(rng.choice(plan.V, 200, replace=False))
    c = np.array([n // 2, n // 2, n // 2])
    for d in rng.integers(-5, 6, size=(100, 3)):
        i, j, k = c + d
        vox.append((k * n + j) * n + i)
    vox = np.unique(np.asarray(vox, np.int64))
    ws = w.astype(np.float64)[ctx.patch_of_sample]
    rr = ws * p * r
    ro = ctx.backproject_voxels(th32, rr, vox)
    bar = adjoint_bar(ctx, th32, rr, voxels=vox)
    do = ctx.backproject_voxels(th32, ws * p, vox)
    bard = adjoint_bar(ctx, th32, ws * p, voxels=vox)
    en = float((np.abs(n1[vox] - ro) / (bar + 1e-30)).max())
    ed = float((np.abs(d1[vox] - do) / (bard + 1e-30)).max())
    covered = int(np.sum(do > 0))
    print(f"[gpu] full-size backproject: {vox.size} voxels ({covered} covered), worst error / bar "
          f"num {en:.2e} den {ed:.2e}")
    assert covered > vox.size // 2
    assert en <= 1.0 and ed <= 1.0


def test_full_robust_weights_match_oracle(full):
    """Seeded residuals shaped like the workload's (1 % noise on inlier
    patches, 10 % outlier patches with uniform residuals), through the same
    kernels at full size."""
    P, ctx, plan, th32 = full["P"], full["ctx"], full["plan"], full["th32"]
    val = ctx.valid(th32)
    rng = np.random.default_rng(13)
    y = rng.uniform(0, 1000, size=plan.N).astype(np.float32)
    e = rng.normal(0, 10.0, size=plan.N)
    out = rng.uniform(size=plan.M) < 0.10
    so = out[ctx.patch_of_sample]
    e[so] = rng.uniform(-500, 500, size=int(so.sum()))
    e = np.where(val, e, 0.0).astype(np.float32)
    emg = plan.em_state()
    pg = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    pbg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    Wg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.robust_weights(dev(e), dev(y), emg, pg, pbg, Wg, flags=pvr.PVR_EM_INIT)
    st = pvr.Plan.read_em(emg)[0]
    p, pbar, W, pi, new, diag = recon.robust_weights(e.astype(np.float64), y.astype(np.float64),
                                                     val, recon.EMState(), ctx.patch_of_sample,
                                                     P.M)
    assert st.m == pytest.approx(diag["m"], rel=1e-6)
    worst_p = float(np.abs(host(pg) - p).max())
    assert worst_p <= 1e-5, worst_p
    assert np.allclose(host(pbg), pbar, rtol=1e-5, atol=1e-6)
    near = np.abs(pi - 0.5) < 1e-3
    Wh = host(Wg)
    assert np.array_equal((Wh > 0)[~near], (W > 0)[~near])
    assert np.allclose(Wh[~near], W[~near], rtol=1e-4, atol=1e-5)
    assert st.sigma2 == pytest.approx(new.sigma2, rel=1e-5)
    assert st.c == pytest.approx(new.c, rel=1e-5)
    print(f"[gpu] full-size EM: p worst {worst_p:.1e}; excluded {st.n_excluded} of {P.M} "
          f"(oracle {diag['excluded']}, planted {int(out.sum())}); sigma2 {st.sigma2:.3f}")
    assert abs(st.n_excluded - diag["excluded"]) <= int(near.sum())


def test_full_sr_update_matches_oracle_on_crops(full):
    plan = full["plan"]
    n = full["P"].grid.nx
    rng = np.random.default_rng(14)
    shape = (n, n, n)
    X = rng.uniform(0, 1000, size=shape).astype(np.float32)
    num = rng.normal(0, 50, size=shape).astype(np.float32)
    den = rng.uniform(0, 2, size=shape).astype(np.float32)
    den[den < 0.2] = 0
    Xo = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    plan.sr_update(dev(X.reshape(-1)), dev(num.reshape(-1)), dev(den.reshape(-1)), Xo,
                   pvr.SRParams.make())
    g = host(Xo).reshape(shape)
    for lo in (0, 100):
        sl = slice(lo, lo + 34)
        ref = ora_update(X[sl, sl, sl], num[sl, sl, sl], den[sl, sl, sl])
        # crop faces that are not volume faces lack their outer neighbours
        a = 0 if lo == 0 else 1
        inner = (slice(a, 33),) * 3
        got = g[sl, sl, sl][inner]
        err = np.abs(got - ref[inner]) / np.maximum(np.abs(ref[inner]), 1.0)
        print(f"[gpu] full-size update, crop at {lo}: worst rel err {err.max():.2e}")
        assert err.max() <= 1e-5


@pytest.mark.parametrize("gradient", ["fd", "exact"])
def test_full_registration_sampled(full, gradient):
    """Registration at full size on 24 sampled patches (the others are not
    registered): observations simulated by the oracle for those patches,
    motion perturbed by <= 3 deg, <= 1 mm; the GPU reaches the oracle's
    outcome (within 0.25 deg and 0.1 mm) on >= 95 % of them and never lowers
    a patch's NCC."""
    import math
    P, ctx, plan, th32 = full["P"], full["ctx"], full["plan"], full["th32"]
    rng = np.random.default_rng(21)
    # patches holding phantom structure
    cand = np.nonzero(np.arange(P.M) % 7 == 3)[0]
    pick = rng.choice(cand, 24, replace=False)
    off = P.patches.sample_off
    samples = np.concatenate([np.arange(off[s], off[s + 1]) for s in pick])
    X = P.x_true.astype(np.float32)
    ys, _, _ = ctx.simulate(X, th32, samples=samples)
    y = np.zeros(P.N, np.float32)
    y[samples] = ys
    reg = np.zeros(P.M, np.uint8)
    reg[pick] = 1
    th0 = th32.copy()
    th0[pick] += synth.random_motion(len(pick), 3.0, 1.0, 22)
    th0 = th0.astype(np.float32)
    ymax = float(np.abs(ys).max())
    tho, nco = ctx.register(X, y, th0.astype(np.float64), reg=reg, min_std=0.01 * ymax,
                            gradient="analytic" if gradient == "exact" else "fd")
    plan.build(dev(th0))
    tt = dev(th0)
    ncc = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.register(dev(X.reshape(-1)), dev(y), tt, ncc, reg=dev(reg),
                  params=pvr.RegParams.make(min_std=0.01 * ymax, exact=gradient == "exact"))
    thg, ncg = host(tt).astype(np.float64), host(ncc)
    plan.build(dev(th32.astype(np.float32)))
    n0 = ctx.ncc(X, y, th0.astype(np.float64))
    assert np.all(ncg[pick] >= n0[pick] - 1e-5)
    others = np.setdiff1d(np.arange(P.M), pick)
    assert np.array_equal(thg[others], th0[others].astype(np.float64))
    d = np.abs(thg[pick] - tho[pick])
    same = (d[:, :3].max(1) < math.radians(0.25)) & (d[:, 3:].max(1) < 0.1)
    err_g = np.abs(thg[pick, 3:] - th32[pick, 3:]).max(1)
    err_o = np.abs(tho[pick, 3:] - th32[pick, 3:]).max(1)
    print(f"[gpu] full-size registration ({gradient}), 24 patches: agreement {same.mean():.3f}; "
          f"median translation error gpu {np.median(err_g):.4f} ora {np.median(err_o):.4f}")
    assert same.mean() >= 0.95
    assert np.median(err_g) <= max(0.03, 1.25 * np.median(err_o))


def test_full_gradient_registration_sampled(full):
    """Joint registration through the differentiable forward model
    (driver.register_gradient) at full size, with only 24 sampled patches
    active (observations simulated by the oracle for them, motion perturbed by
    <= 3 deg, <= 1 mm), against the oracle's per-patch ascent with the exact
    gradient: agreement within 0.25 deg and 0.1 mm on >= 95 % of them."""
    import math
    from paper_1611_07289_amd import driver
    P, ctx, plan, th32 = full["P"], full["ctx"], full["plan"], full["th32"]
    rng = np.random.default_rng(23)
    cand = np.nonzero(np.arange(P.M) % 7 == 3)[0]
    pick = rng.choice(cand, 24, replace=False)
    off = P.patches.sample_off
    samples = np.concatenate([np.arange(off[s], off[s + 1]) for s in pick])
    X = P.x_true.astype(np.float32)
    ys, _, _ = ctx.simulate(X, th32, samples=samples)
    y = np.zeros(P.N, np.float32)
    y[samples] = ys
    reg = np.zeros(P.M, np.uint8)
    reg[pick] = 1
    th0 = th32.copy()
    th0[pick] += synth.random_motion(len(pick), 3.0, 1.0, 24)
    th0 = th0.astype(np.float32)
    ymax = float(np.abs(ys).max())
    tho, _ = ctx.register(X, y, th0.astype(np.float64), reg=reg, min_std=0.01 * ymax,
                          gradient="analytic", max_iter=40)
    th = dev(th0)
    ncc = driver.register_gradient(plan, dev(X.reshape(-1)), dev(y), th, iters=40,
                                   min_std=0.01 * ymax, active=dev(reg))
    thg, ncg = host(th).astype(np.float64), host(ncc)
    plan.build(dev(th32.astype(np.float32)))
    n0 = ctx.ncc(X, y, th0.astype(np.float64))
    assert np.all(ncg[pick] >= n0[pick] - 1e-5)
    others = np.setdiff1d(np.arange(P.M), pick)
    assert np.array_equal(thg[others], th0[others].astype(np.float64))
    d = np.abs(thg[pick] - tho[pick])
    same = (d[:, :3].max(1) < math.radians(0.25)) & (d[:, 3:].max(1) < 0.1)
    print(f"[gpu] full-size joint gradient registration, 24 patches: agreement {same.mean():.3f}",
          flush=True)
    assert same.mean() >= 0.95
