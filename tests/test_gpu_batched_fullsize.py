"""The batched form at its own sizes: 8 independent reconstructions of 96^3 to
192^3 voxels with 3-6 stacks each (3 orthogonal + seeded obliques) and
square patches of 32, 64 or 128 pixels (stride half the size) per stack, all
in one plan, in the launch configuration the batched benchmark runs; per
problem against the FP64 oracle on sampled outputs, plus properties that
hold at any size.

  * simulate: per problem 1 000 random samples and every sample of two whole
    patches, |y_gpu - y_ora| <= 1e-5 max(|y_ora|, 1e-3 max|y_ora|);
  * back-projection with per-sample p and patch weights: per problem 60
    voxels (random, plus around the problem's centre) within the adjoint bar
    of tests/_tolerance.py, num and den;
  * A 1 = 1 on valid samples, validity exact per problem, and the adjoint
    identity <A x, r> = <x, A^T r> per problem to 1e-5 of sum |A x| |r|;
  * robust weights on seeded residuals (1 % noise, 10 % outlier patches with
    uniform residuals): per problem E-step, potentials, patch classification
    and M-step against the oracle's;
  * a graph of two SR iterations over the whole batch, replayed twice,
    reproduces the eager iterations bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from oracle import recon
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
def batch8():
    print("[gpu] batched 8 x 96..192^3: generating and building", flush=True)
    probs = synth.batched_problems()
    plan = pvr.Plan.from_problems(probs)
    th = np.concatenate([P.theta_true for P in probs]).astype(np.float32)
    plan.build(dev(th))
    m0 = np.concatenate([[0], np.cumsum([P.M for P in probs])])
    ctxs = [oracle.Ctx(P.grid, P.stacks, P.patches) for P in probs]
    th64 = [P.theta_true.astype(np.float32).astype(np.float64) for P in probs]
    print(f"[gpu] batched: N={plan.N} M={plan.M} V={plan.V}; sizes "
          f"{[P.grid.nx for P in probs]}, stacks {[len(P.stacks) for P in probs]}, patch sizes "
          f"{[sorted(set(P.patches.w.tolist())) for P in probs]}", flush=True)
    return dict(probs=probs, plan=plan, m0=m0, ctxs=ctxs, th64=th64)


def _samples(b, d):
    plan, m0 = d["plan"], d["m0"]
    return int(plan.sample_off[m0[b]]), int(plan.sample_off[m0[b + 1]])


def _voxels(b, d):
    plan = d["plan"]
    return int(plan.vol_off[b]), int(plan.vol_off[b + 1])


def test_batched_simulate_sampled(batch8):
    probs, plan = batch8["probs"], batch8["plan"]
    X = dev(np.concatenate([P.x_true.reshape(-1) for P in probs]))
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(X, y_sim=ys)
    g = host(ys)
    rng = np.random.default_rng(31)
    for b, P in enumerate(probs):
        a, z = _samples(b, batch8)
        off = P.patches.sample_off
        whole = [np.arange(off[s], off[s + 1]) for s in rng.choice(P.M, 2, replace=False)]
        js = np.unique(np.concatenate([rng.choice(z - a, 1000, replace=False)] + whole))
        yo, _, val = batch8["ctxs"][b].simulate(P.x_true, batch8["th64"][b], samples=js)
        gb = g[a:z][js]
        assert np.array_equal(gb != 0, val & (yo != 0)), b
        scale = np.maximum(np.abs(yo), 1e-3 * np.abs(yo).max())
        worst = float((np.abs(gb - yo) / scale).max())
        print(f"[gpu] batched problem {b} ({P.grid.nx}^3): simulate {js.size} samples, worst "
              f"{worst:.2e}", flush=True)
        assert worst <= 1e-5, b


def test_batched_backproject_sampled(batch8):
    probs, plan = batch8["probs"], batch8["plan"]
    rng = np.random.default_rng(32)
    r = rng.normal(size=plan.N).astype(np.float32)
    p = rng.uniform(0, 1, size=plan.N).astype(np.float32)
    w = rng.uniform(0.2, 1.0, size=plan.M).astype(np.float32)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    den = torch.empty_like(num)
    plan.backproject(dev(r), dev(p), dev(w), num, den)
    n1, d1 = host(num), host(den)
    for b, P in enumerate(probs):
        ctx, th = batch8["ctxs"][b], batch8["th64"][b]
        a, z = _samples(b, batch8)
        va, vz = _voxels(b, batch8)
        m0 = batch8["m0"][b]
        n = P.grid.nx
        vox = list(rng.choice(vz - va, 40, replace=False))
        c = np.array([n // 2] * 3)
        for dd in rng.integers(-4, 5, size=(20, 3)):
            i, j, k = c + dd
            vox.append((k * n + j) * n + i)
        vox = np.unique(np.asarray(vox, np.int64))
        ws = w[m0:m0 + P.M].astype(np.float64)[ctx.patch_of_sample]
        pb = p[a:z].astype(np.float64)
        rr = ws * pb * r[a:z]
        ro = ctx.backproject_voxels(th, rr, vox)
        bar = adjoint_bar(ctx, th, rr, voxels=vox)
        do = ctx.backproject_voxels(th, ws * pb, vox)
        bard = adjoint_bar(ctx, th, ws * pb, voxels=vox)
        en = float((np.abs(n1[va:vz][vox] - ro) / (bar + 1e-30)).max())
        ed = float((np.abs(d1[va:vz][vox] - do) / (bard + 1e-30)).max())
        print(f"[gpu] batched problem {b}: backproject {vox.size} voxels "
              f"({int(np.sum(do > 0))} covered), worst / bar num {en:.2e} den {ed:.2e}",
              flush=True)
        assert int(np.sum(do > 0)) > vox.size // 2
        assert en <= 1.0 and ed <= 1.0, b


def test_batched_normalisation_validity_and_adjoint_identity(batch8):
    probs, plan = batch8["probs"], batch8["plan"]
    one = torch.ones(plan.V, dtype=torch.float32, device="cuda")
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(one, y_sim=ys)
    v = ys > 0.5
    assert torch.all(torch.abs(ys[v] - 1) <= 2e-6)
    assert torch.all(ys[~v] == 0)
    vh = host(v)
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.rand(plan.V, generator=g, device="cuda")
    r = torch.randn(plan.N, generator=g, device="cuda")
    Ax = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(x, y_sim=Ax)
    ATr = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    plan.backproject(r, num=ATr)
    Axh, rh, xh, ATrh = (host(t).astype(np.float64) for t in (Ax, r, x, ATr))
    for b, P in enumerate(probs):
        a, z = _samples(b, batch8)
        va, vz = _voxels(b, batch8)
        assert np.array_equal(vh[a:z], batch8["ctxs"][b].valid(batch8["th64"][b])), b
        lhs = float(Axh[a:z] @ rh[a:z])
        rhs = float(xh[va:vz] @ ATrh[va:vz])
        scale = float(np.abs(Axh[a:z]) @ np.abs(rh[a:z]))
        print(f"[gpu] batched problem {b}: adjoint identity {abs(lhs - rhs) / scale:.2e}",
              flush=True)
        assert abs(lhs - rhs) <= 1e-5 * scale, b


def test_batched_robust_weights_per_problem(batch8):
    probs, plan = batch8["probs"], batch8["plan"]
    rng = np.random.default_rng(33)
    y = rng.uniform(0, 1000, size=plan.N).astype(np.float32)
    e = np.zeros(plan.N)
    vals = []
    for b, P in enumerate(probs):
        a, z = _samples(b, batch8)
        val = batch8["ctxs"][b].valid(batch8["th64"][b])
        eb = rng.normal(0, 10.0, size=z - a)
        out = rng.uniform(size=P.M) < 0.10
        so = out[batch8["ctxs"][b].patch_of_sample]
        eb[so] = rng.uniform(-500, 500, size=int(so.sum()))
        e[a:z] = np.where(val, eb, 0.0)
        vals.append(val)
    e = e.astype(np.float32)
    emg = plan.em_state()
    pg = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    pbg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    Wg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.robust_weights(dev(e), dev(y), emg, pg, pbg, Wg, flags=pvr.PVR_EM_INIT)
    sts = pvr.Plan.read_em(emg)
    ph, pbh, Wh = host(pg), host(pbg), host(Wg)
    for b, P in enumerate(probs):
        a, z = _samples(b, batch8)
        m0 = batch8["m0"][b]
        p, pbar, W, pi, new, diag = recon.robust_weights(
            e[a:z].astype(np.float64), y[a:z].astype(np.float64), vals[b], recon.EMState(),
            batch8["ctxs"][b].patch_of_sample, P.M)
        st = sts[b]
        assert st.m == pytest.approx(diag["m"], rel=1e-6)
        assert float(np.abs(ph[a:z] - p).max()) <= 1e-5, b
        assert np.allclose(pbh[m0:m0 + P.M], pbar, rtol=1e-5, atol=1e-6)
        near = np.abs(pi - 0.5) < 1e-3
        Wb = Wh[m0:m0 + P.M]
        assert np.array_equal((Wb > 0)[~near], (W > 0)[~near]), b
        assert np.allclose(Wb[~near], W[~near], rtol=1e-4, atol=1e-5)
        assert st.sigma2 == pytest.approx(new.sigma2, rel=1e-5)
        assert st.c == pytest.approx(new.c, rel=1e-5)
        print(f"[gpu] batched problem {b}: EM excluded {st.n_excluded} of {P.M} (oracle "
              f"{diag['excluded']})", flush=True)
        assert abs(st.n_excluded - diag["excluded"]) <= int(near.sum())


def test_batched_graph_replays_equal_eager(batch8):
    from paper_1611_07289_amd.batch import GraphedSR
    from tests.test_gpu_batched import Eager
    probs, plan = batch8["probs"], batch8["plan"]
    X0 = dev(np.concatenate([P.x_true.reshape(-1) for P in probs]) * 0.9)
    yc = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(X0 / 0.9, y_sim=yc)
    y = yc * 1.01 + 1.0
    ref = Eager(plan, X0.clone(), y)
    ref.step(init=True)
    snaps = []
    for k in range(2):
        ref.step()
        ref.step()
        snaps.append(ref.X.clone())
    torch.cuda.synchronize()
    gs = GraphedSR(plan, y, X0.clone())
    gs.start()
    gs.capture()
    for k in range(2):
        gs.replay_pairs(1)
        torch.cuda.synchronize()
        assert torch.equal(gs.X, snaps[k]), f"replay {k} differs from eager"
    print("[gpu] batched: graph replays equal eager iterations bit for bit", flush=True)
