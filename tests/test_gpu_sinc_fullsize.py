"""The sinc PSF at full size: the 256^3 four-stack uterus workload (11 760
patches of 64 x 64) in the launch configuration the sinc256 benchmark times,
against the FP64 oracle with the same PSF on sampled outputs: 3 000 random
samples and one whole patch of the forward pass (1e-5 relative), 150 voxels
of the adjoint (bar of tests/_tolerance.py), the FP32 adjoint identity."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import oracle
from paper_1611_07289_amd import pvr, synth
from tests._tolerance import adjoint_bar
from tests.test_gpu_fullsize import dev, host


def test_sinc_full_size_matches_oracle():
    print("[gpu] uterus256 sinc: generating and building", flush=True)
    P = synth.full_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches, psf="sinc")
    plan = pvr.Plan.from_problems([P])
    plan.set_psf(pvr.PVR_PSF_SINC)
    plan.build(dev(P.theta_true, torch.float32))
    th32 = np.asarray(P.theta_true, np.float32).astype(np.float64)
    ys = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(dev(P.x_true.reshape(-1)), y_sim=ys)
    g = host(ys)
    rng = np.random.default_rng(31)
    off = P.patches.sample_off
    s0 = int(rng.integers(P.M))
    js = np.unique(np.concatenate([rng.choice(plan.N, 3000, replace=False),
                                   np.arange(off[s0], off[s0 + 1])]))
    yo, _, val = ctx.simulate(P.x_true, th32, samples=js)
    assert np.array_equal(g[js] != 0, val & (yo != 0))
    scale = np.maximum(np.abs(yo), 1e-3 * np.abs(yo).max())
    worst = float((np.abs(g[js] - yo) / scale).max())
    print(f"[gpu] sinc full-size simulate: {js.size} samples, worst rel err {worst:.2e}")
    assert worst <= 1e-5
    r = rng.normal(size=plan.N).astype(np.float32)
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    plan.backproject(dev(r), num=num)
    n = P.grid.nx
    vox = list(rng.choice(plan.V, 100, replace=False))
    for d in rng.integers(-5, 6, size=(50, 3)):
        i, j, k = np.array([n // 2] * 3) + d
        vox.append((k * n + j) * n + i)
    vox = np.unique(np.asarray(vox, np.int64))
    rr = r.astype(np.float64)
    ro = ctx.backproject_voxels(th32, rr, vox)
    bar = adjoint_bar(ctx, th32, rr, voxels=vox)
    err = float((np.abs(host(num)[vox] - ro) / (bar + 1e-30)).max())
    print(f"[gpu] sinc full-size backproject: {vox.size} voxels, worst error / bar {err:.2e}")
    assert err <= 1.0
    x = torch.rand(plan.V, device="cuda")
    Ax = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    plan.simulate(x, y_sim=Ax)
    rd = dev(r)
    lhs = float(torch.dot(Ax.double(), rd.double()))
    rhs = float(torch.dot(x.double(), num.double()))
    assert abs(lhs - rhs) <= 1e-5 * float(torch.dot(Ax.double().abs(), rd.double().abs()))
