"""Batched form: several independent reconstructions (different grid sizes,
stack counts and patch sizes) in one plan, against the oracle run problem by
problem, and the graph-captured SR iteration against eager execution.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402  (CPU import is fine; GPU use is gated by the marker)

import oracle
from oracle import recon
from paper_1611_07289_amd import pvr, synth

from tests._tolerance import adjoint_bar


@pytest.fixture(scope="module")
def batch():
    print("[gpu] batched problems (3 x 24..40^3)", flush=True)
    probs = synth.batched_problems(seed_cfg=3, count=3, n_range=(24, 40), sizes=(8, 16, 32))
    plan = pvr.Plan.from_problems(probs)
    th = np.concatenate([P.theta_true for P in probs]).astype(np.float32)
    plan.build(torch.from_numpy(th).cuda())
    ctxs, ys, th64 = [], [], []
    for b, P in enumerate(probs):
        ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
        t64 = P.theta_true.astype(np.float32).astype(np.float64)
        yc, _, _ = ctx.simulate(P.x_true, t64)
        ys.append(synth.corrupt(yc, P.patches, P.outlier_patch, 0.01, P.seed_base + 3,
                                P.seed_base + 5))
        ctxs.append(ctx)
        th64.append(t64)
    return dict(probs=probs, plan=plan, ctxs=ctxs, ys=ys, th64=th64)


def _split(plan, probs, arr, kind):
    out = []
    for b in range(len(probs)):
        if kind == "s":
            m0 = sum(P.M for P in probs[:b]); m1 = m0 + probs[b].M
            out.append(arr[plan.sample_off[m0]:plan.sample_off[m1]])
        else:
            out.append(arr[plan.vol_off[b]:plan.vol_off[b + 1]])
    return out


def test_batched_simulate_and_backproject_match_oracle(batch):
    probs, plan, ctxs = batch["probs"], batch["plan"], batch["ctxs"]
    X = torch.from_numpy(np.concatenate([P.x_true.reshape(-1) for P in probs])).cuda()
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(X, y_sim=ys)
    r = np.random.default_rng(0).normal(size=plan.N).astype(np.float32)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    plan.backproject(torch.from_numpy(r).cuda(), num=num)
    torch.cuda.synchronize()
    for b, (P, ctx) in enumerate(zip(probs, ctxs)):
        yo, _, _ = ctx.simulate(P.x_true, batch["th64"][b])
        yg = _split(plan, probs, ys.cpu().numpy(), "s")[b]
        scale = np.maximum(np.abs(yo), 1e-3 * np.abs(yo).max())
        assert (np.abs(yg - yo) / scale).max() <= 1e-5, b
        rb = _split(plan, probs, r, "s")[b].astype(np.float64)
        bo = ctx.backproject(batch["th64"][b], rb).reshape(-1)
        bar = adjoint_bar(ctx, batch["th64"][b], rb)
        bg = _split(plan, probs, num.cpu().numpy(), "v")[b]
        worst = (np.abs(bg - bo) / (bar + 1e-30)).max()
        print(f"[gpu] problem {b}: backproject worst error / bar {worst:.2e}")
        assert worst <= 1.0, b


class Eager:
    """Plain eager SR iterations keeping one EM state."""

    def __init__(self, plan, X, y):
        f32 = dict(dtype=torch.float32, device="cuda")
        self.plan, self.X, self.y = plan, X, y
        self.e = torch.empty(plan.N, **f32); self.p = torch.empty(plan.N, **f32)
        self.pb = torch.empty(plan.M, **f32); self.W = torch.empty(plan.M, **f32)
        self.num = torch.empty(plan.V, **f32); self.den = torch.empty(plan.V, **f32)
        self.Xn = torch.empty_like(X)
        self.em = plan.em_state()
        self.prm = pvr.SRParams.make()

    def step(self, init=False):
        pl = self.plan
        pl.simulate(self.X, y_obs=self.y, resid=self.e)
        pl.robust_weights(self.e, self.y, self.em, self.p, self.pb, self.W,
                          pvr.PVR_EM_INIT if init else 0)
        pl.backproject(self.e, self.p, self.W, self.num, self.den)
        pl.sr_update(self.X, self.num, self.den, self.Xn, self.prm)
        self.X, self.Xn = self.Xn, self.X


def test_batched_sr_iterations_match_oracle_per_problem(batch):
    probs, plan, ctxs, ys = batch["probs"], batch["plan"], batch["ctxs"], batch["ys"]
    X0s = [recon.initial_volume(ctx, y, t) for ctx, y, t in zip(ctxs, ys, batch["th64"])]
    X = torch.from_numpy(np.concatenate([x.reshape(-1) for x in X0s]).astype(np.float32)).cuda()
    y = torch.from_numpy(np.concatenate(ys)).cuda()
    run = Eager(plan, X, y)
    for it in range(4):
        run.step(init=(it == 0))
    Xg = run.X.cpu().numpy()
    for b, (ctx, yb, t) in enumerate(zip(ctxs, ys, batch["th64"])):
        Xo = X0s[b]
        st = recon.EMState()
        for it in range(4):
            Xo, st, diag = recon.sr_iteration(ctx, Xo, yb, t, st, recon.SRParams())
        xg = Xg[plan.vol_off[b]:plan.vol_off[b + 1]]
        rel = np.linalg.norm(xg - Xo.reshape(-1)) / np.linalg.norm(Xo)
        print(f"[gpu] batched problem {b} ({probs[b].name}): 4 SR iterations rel-L2 {rel:.2e}")
        assert rel <= 1e-4


def test_graph_replays_equal_eager(batch):
    """A graph of two SR iterations over the whole batch, replayed three
    times with other GPU work in between, reproduces eager execution bit for
    bit after every replay."""
    from paper_1611_07289_amd.batch import GraphedSR
    probs, plan, ys = batch["probs"], batch["plan"], batch["ys"]
    y = torch.from_numpy(np.concatenate(ys)).cuda()
    X0 = torch.from_numpy(np.concatenate([P.x_true.reshape(-1) for P in probs]) * 0.9).cuda()
    ref = Eager(plan, X0.clone(), y)
    ref.step(init=True)
    snaps = []
    for k in range(3):
        ref.step()
        ref.step()
        snaps.append(ref.X.clone())
    torch.cuda.synchronize()
    gs = GraphedSR(plan, y, X0.clone())
    gs.start()
    gs.capture()
    for k in range(3):
        gs.replay_pairs(1)
        torch.cuda.synchronize()
        busy = (gs.X * 2.0).sum() + torch.randn(1000, device="cuda").sum()  # eager work
        torch.cuda.synchronize()
        assert torch.equal(gs.X, snaps[k]), f"replay {k} differs from eager"
        del busy


def test_launch_shapes_change_no_result(batch):
    """The autotuner's knobs reorder workgroups only: every XCD granule of
    the forward walk and of the adjoint gives bit-identical outputs; the
    LDS-staged forward tiles agree with the walk within the per-sample bar;
    the tuner applies its choice and reports every candidate's time."""
    from paper_1611_07289_amd import autotune
    probs, plan = batch["probs"], batch["plan"]
    X = torch.from_numpy(np.concatenate([P.x_true.reshape(-1) for P in probs])).cuda()
    r = torch.from_numpy(np.random.default_rng(3).normal(size=plan.N).astype(np.float32)).cuda()
    p = torch.rand(plan.N, device="cuda")
    W = torch.rand(plan.M, device="cuda")

    def outputs():
        ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
        plan.simulate(X, y_sim=ys)
        num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
        den = torch.empty_like(num)
        plan.backproject(r, p, W, num, den)
        torch.cuda.synchronize()
        return ys.clone(), num.clone(), den.clone()

    plan.set_tiles(0, 0)
    plan.set_granules(1, 64)
    ref = outputs()
    for gs, gb in ((2, 1), (16, 4), (4, 32), (4, 256), (8, 1024)):
        plan.set_granules(gs, gb)
        got = outputs()
        assert all(torch.equal(a, b) for a, b in zip(got, ref)), (gs, gb)
    plan.set_granules(1, 64)
    plan.set_tiles(16, 16)
    ys_t = outputs()[0]
    scale = torch.clamp(ref[0].abs(), min=1e-3 * float(ref[0].abs().max()))
    assert float(((ys_t - ref[0]).abs() / scale).max()) <= 1e-5
    res = autotune.tune(plan, X, r, reps=2, cache=None)
    assert set(res["forward_ms"]) == {autotune._name(c) for c in autotune.FORWARD}
    assert set(res["adjoint_ms"]) == {str(g) for g in autotune.ADJOINT}
    print(f"[gpu] autotune: forward {res['forward']}, adjoint granule {res['adjoint_granule']}")
    got = outputs()
    assert torch.equal(got[1], ref[1]) and torch.equal(got[2], ref[2])
    plan.set_tiles(0, 0)
    plan.set_granules(1, 64)
