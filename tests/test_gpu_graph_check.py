"""The library's own graph capture of SR iterations (pvr_sr_graph_*) and the
numeric fault flags (pvr_check), on the tiny 32^3 case.

A graph of three SR iterations replays the eager calls bit for bit (odd
count: the volume ends in X_alt), twice in a row; after a rebuild of the plan
the launch is refused on the host.  A NaN planted in the volume raises the
update's flag, and a simulation from it the residual flag; pvr_check clears
what it reports."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from paper_1611_07289_amd import pvr, synth


class Bufs:
    def __init__(self, plan):
        f = dict(dtype=torch.float32, device="cuda")
        self.e = torch.empty(plan.N, **f)
        self.p = torch.empty(plan.N, **f)
        self.pbar = torch.empty(plan.M, **f)
        self.W = torch.empty(plan.M, **f)
        self.num = torch.empty(plan.V, **f)
        self.den = torch.empty(plan.V, **f)
        self.em = plan.em_state()


def _iter(plan, b, src, dst, y, flags):
    plan.simulate(src, y_obs=y, resid=b.e)
    plan.robust_weights(b.e, y, b.em, b.p, b.pbar, b.W, flags | pvr.PVR_EM_RESID_FRESH)
    plan.backproject(b.e, b.p, b.W, b.num, b.den)
    plan.sr_update(src, b.num, b.den, dst)


@pytest.fixture(scope="module")
def tiny():
    print("[gpu] tiny32: graph capture and fault flags", flush=True)
    P = synth.tiny_problem()
    plan = pvr.Plan.from_problems([P])
    th = torch.from_numpy(P.theta_true.astype(np.float32)).cuda()
    plan.build(th)
    Xt = torch.from_numpy(P.x_true.reshape(-1).astype(np.float32)).cuda()
    y = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(Xt, y_sim=y)
    y = torch.from_numpy(synth.corrupt(y.cpu().numpy(), P.patches, P.outlier_patch, 0.01, 3, 5)).cuda()
    return P, plan, th, Xt, y


def test_graph_of_three_iterations_equals_eager_and_is_refused_after_rebuild(tiny):
    P, plan, th, Xt, y = tiny
    X0 = Xt * 0.9
    # eager reference: one INIT iteration, then three
    r = Bufs(plan)
    a, b = X0.clone(), torch.empty_like(X0)
    _iter(plan, r, a, b, y, pvr.PVR_EM_INIT)
    start, em_after_init = b.clone(), r.em.clone()
    refs = []
    cur = start.clone()
    nxt = torch.empty_like(cur)
    for _ in range(2):  # two launches of three iterations
        for _ in range(3):
            _iter(plan, r, cur, nxt, y, 0)
            cur, nxt = nxt, cur
        refs.append(cur.clone())
    g_b = Bufs(plan)
    g_b.em.copy_(em_after_init)
    # the graph reads X first and leaves an odd count's result in X_alt: copy
    # it back before the next launch
    X, Xa = start.clone(), torch.empty_like(start)
    g = pvr.SRGraph(plan, X, Xa, y, g_b.e, g_b.p, g_b.pbar, g_b.W, g_b.num, g_b.den, g_b.em,
                    iters=3)
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(Xa, refs[0])
    X.copy_(Xa)
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(Xa, refs[1])
    plan.check()  # finite throughout
    plan.build(th)
    with pytest.raises(pvr.PvrError) as ei:
        g.launch()
    assert ei.value.status == 1 and "capture again" in str(ei.value)
    g.close()
    # a fresh capture works again
    g2 = pvr.SRGraph(plan, X, Xa, y, g_b.e, g_b.p, g_b.pbar, g_b.W, g_b.num, g_b.den, g_b.em,
                     iters=2)
    g2.launch()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(X).all())
    g2.close()


def test_check_reports_and_clears_non_finite_values(tiny):
    P, plan, th, Xt, y = tiny
    plan.build(th)
    b = Bufs(plan)
    X = Xt.clone()
    Xn = torch.empty_like(X)
    _iter(plan, b, X, Xn, y, pvr.PVR_EM_INIT)
    plan.check()
    X[1234] = float("nan")
    plan.sr_update(X, b.num, b.den, Xn)
    with pytest.raises(pvr.PvrError) as ei:
        plan.check()
    assert ei.value.status == 5 and "updated volume" in str(ei.value)
    plan.check()  # cleared
    plan.simulate(X, y_obs=y, resid=b.e)
    plan.robust_weights(b.e, y, b.em, b.p, b.pbar, b.W, pvr.PVR_EM_INIT | pvr.PVR_EM_RESID_FRESH)
    with pytest.raises(pvr.PvrError) as ei:
        plan.check()
    assert "residual statistics" in str(ei.value)
    plan.check()


def test_adjoint_preparation_beside_the_classification(tiny):
    """PVR_EM_PREP_ADJOINT: the back-projection that follows gives the same
    bits as without the flag; a simulation in between cancels the prepared
    inputs (the back-projection then prepares them itself)."""
    P, plan, th, Xt, y = tiny
    plan.build(th)
    X = Xt * 0.9

    def run(flags, resimulate=False):
        b = Bufs(plan)
        plan.simulate(X, y_obs=y, resid=b.e)
        plan.robust_weights(b.e, y, b.em, b.p, b.pbar, b.W, flags)
        if resimulate:
            plan.simulate(X * 1.05, y_obs=y, resid=b.e)
        plan.backproject(b.e, b.p, b.W, b.num, b.den)
        torch.cuda.synchronize()
        return b.num.clone(), b.den.clone()

    base = pvr.PVR_EM_INIT | pvr.PVR_EM_RESID_FRESH
    n0, d0 = run(base)
    n1, d1 = run(base | pvr.PVR_EM_PREP_ADJOINT)
    assert torch.equal(n0, n1) and torch.equal(d0, d1)
    n2, d2 = run(base, resimulate=True)
    n3, d3 = run(base | pvr.PVR_EM_PREP_ADJOINT, resimulate=True)
    assert torch.equal(n2, n3) and torch.equal(d2, d3)
    assert not torch.equal(n2, n0)
