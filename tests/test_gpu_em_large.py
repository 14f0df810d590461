"""The patch classification of a problem with more patches than its LDS copy
holds (12 288): the potentials then live in the plan's scratch array.  The
tiny 32^3 case cut into 8x8 patches with stride 1 (15 000 patches, 960 000
samples); robust weights from the initial volume's residuals against the
oracle, to the bars of the 216-patch case."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from oracle import recon
from paper_1611_07289_amd import pvr, synth
from tests.test_gpu_parity import dev, host


def test_robust_weights_beyond_the_lds_copy():
    print("[gpu] tiny32 with 15 000 patches: robust weights", flush=True)
    P = synth.tiny_problem()
    pat = synth.square_patches(P.stacks, 8, 1)
    assert pat.M > 12288
    th = synth.random_motion(pat.M, 3.0, 1.0, 55)
    th32 = th.astype(np.float32).astype(np.float64)
    ctx = oracle.Ctx(P.grid, P.stacks, pat)
    yc, _, val = ctx.simulate(P.x_true, th32)
    out = synth.choose_outliers(pat.M, 0.10, 56)
    y = synth.corrupt(yc, pat, out, 0.01, 57, 58)
    X0 = recon.initial_volume(ctx, y, th32)
    yh, _, val = ctx.simulate(X0, th32)
    e = np.where(val, y - yh, 0.0).astype(np.float32)
    plan = pvr.Plan([P.grid], [P.stacks], [pat])
    plan.build(dev(th32.astype(np.float32)))
    emg = plan.em_state()
    pg = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    pbg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    Wg = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    plan.robust_weights(dev(e), dev(y), emg, pg, pbg, Wg, flags=pvr.PVR_EM_INIT)
    st = pvr.Plan.read_em(emg)[0]
    p, pbar, W, pi, new, diag = recon.robust_weights(e.astype(np.float64), y.astype(np.float64),
                                                     val, recon.EMState(), ctx.patch_of_sample,
                                                     pat.M)
    assert np.abs(host(pg) - p).max() <= 1e-5
    assert np.allclose(host(pbg), pbar, rtol=1e-5, atol=1e-6)
    near = np.abs(pi - 0.5) < 1e-3
    Wh = host(Wg)
    assert np.array_equal((Wh > 0)[~near], (W > 0)[~near])
    assert np.allclose(Wh[~near], W[~near], rtol=1e-4, atol=1e-5)
    assert st.sigma2 == pytest.approx(new.sigma2, rel=1e-5)
    assert st.c == pytest.approx(new.c, rel=1e-5)
    assert 0 < st.n_excluded < pat.M
    print(f"[gpu] 15 000 patches: excluded {st.n_excluded}, near-threshold {int(near.sum())}")
