"""Degenerate inputs of the robust weights and the registration against the
oracle, on the tiny 32^3 case: residuals all zero (max e = min e, so the
outlier density m takes its guard and sigma^2 its floor), and observations
without structure (every patch flat: registration keeps the motion, NCC 0).
Nothing non-finite is flagged."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from oracle import recon
from paper_1611_07289_amd import pvr, synth
from tests.test_gpu_parity import dev, host


@pytest.fixture(scope="module")
def tiny():
    print("[gpu] tiny32: degenerate EM and registration inputs", flush=True)
    P = synth.tiny_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    plan = pvr.Plan.from_problems([P])
    th32 = P.theta_true.astype(np.float32)
    plan.build(dev(th32))
    _, _, val = ctx.simulate(P.x_true, th32.astype(np.float64))
    return P, ctx, plan, th32, val


def test_zero_residuals(tiny):
    P, ctx, plan, th32, val = tiny
    e = np.zeros(P.N, np.float32)
    y = np.where(val, 500.0, 0.0).astype(np.float32)
    emg = plan.em_state()
    pg = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    pbg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    Wg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.robust_weights(dev(e), dev(y), emg, pg, pbg, Wg, flags=pvr.PVR_EM_INIT)
    st = pvr.Plan.read_em(emg)[0]
    p, pbar, W, pi, new, diag = recon.robust_weights(e.astype(np.float64), y.astype(np.float64),
                                                     val, recon.EMState(), ctx.patch_of_sample,
                                                     P.M)
    assert np.isfinite(st.m) and st.m == pytest.approx(diag["m"], rel=1e-6)
    assert np.isfinite(st.sigma2) and st.sigma2 == pytest.approx(new.sigma2, rel=1e-5)
    assert st.c == pytest.approx(new.c, rel=1e-5)
    assert np.abs(host(pg) - p).max() <= 1e-5
    assert np.allclose(host(pbg), pbar, rtol=1e-5, atol=1e-6)
    assert np.array_equal(host(Wg) > 0, W > 0)
    plan.check()


def test_flat_observations_keep_the_motion(tiny):
    P, ctx, plan, th32, val = tiny
    y = np.full(P.N, 100.0, np.float32)
    th0 = th32 + np.float32(0.01)
    tt = dev(th0)
    ncc = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.register(dev(P.x_true), dev(y), tt, ncc, params=pvr.RegParams.make(min_std=1.0))
    assert np.array_equal(host(tt), th0)
    assert np.all(host(ncc) == 0)
    tho, nco = ctx.register(P.x_true, y.astype(np.float64), th0.astype(np.float64), min_std=1.0)
    assert np.array_equal(tho, th0.astype(np.float64)) and np.all(nco == 0)
    plan.check()
