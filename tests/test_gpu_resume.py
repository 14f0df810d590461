"""Checkpoint and resume of the reconstruction driver: the state between two
cycles is (X, theta, next cycle) because EM restarts every cycle, so three
cycles equal two cycles, a save and load through .npz, and one more cycle --
bit for bit, the kernels being deterministic.  The per-cycle JSON lines carry
the cycle's statistics."""
import io
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from paper_1611_07289_amd import driver, pvr, synth


def test_two_cycles_save_load_one_equals_three(tmp_path):
    print("[gpu] tiny32: resume after a checkpoint", flush=True)
    P = synth.tiny_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    yc, _, _ = ctx.simulate(P.x_true, P.theta_true)
    y = torch.from_numpy(synth.corrupt(yc, P.patches, P.outlier_patch, 0.01, 3, 5)).cuda()
    plan = pvr.Plan.from_problems([P])
    rp = pvr.RegParams.make(min_std=0.01 * float(y.abs().max()), exact=True, max_iter=10)
    th0 = torch.from_numpy((P.theta_true + synth.random_motion(P.M, 3.0, 1.0, 8)).astype(np.float32)).cuda()

    log = io.StringIO()
    th_a = th0.clone()
    Xa, th_a, _ = driver.reconstruct(plan, y, th_a, cycles=3, n_sr=4, reg_params=rp,
                                     on_cycle=driver.json_lines(log))
    lines = [json.loads(l) for l in log.getvalue().splitlines()]
    assert [r["cycle"] for r in lines] == [0, 1, 2]
    assert all(r["sigma2"][0] > 0 and 0 < r["c"][0] <= 1 and r["mean_ncc"] is not None for r in lines)

    th_b = th0.clone()
    Xb, th_b, _ = driver.reconstruct(plan, y, th_b, cycles=2, n_sr=4, reg_params=rp)
    f = str(tmp_path / "state.npz")
    driver.save_checkpoint(f, Xb, th_b, 2)
    X2, th2, nxt = driver.load_checkpoint(f)
    assert nxt == 2
    Xc, th_c, _ = driver.reconstruct(plan, y, th2, cycles=1, n_sr=4, reg_params=rp, X0=X2,
                                     first_cycle=nxt)
    torch.cuda.synchronize()
    assert torch.equal(th_c, th_a)
    assert torch.equal(Xc, Xa)
