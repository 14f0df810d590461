"""What the learned registration initialiser gains in a whole reconstruction
(not part of the paper's method; the paper's registration, Sec. II "Patch to
Volume Registration", is the baseline).

The 256^3 uterus workload (4 stacks of 256 x 256 x 60 slices, 64 x 64
patches stride 32: 11 760 patches, enough to fill the GPU with registration
workgroups), reconstructed from zero motion: 3 cycles of [registration, 10 SR
iterations], exact-gradient registration.  The network is trained first on
300 000 forward-model pairs of a phantom of another seed (not timed).  Three
runs:
  plain        full optimiser budget (step0 1, 40 trial steps);
  plain_tight  tight budget (step0 0.25, 5 trial steps), no network;
  learned      the network's prediction refined with the tight budget; where
               the patch's NCC after the prediction stays below 0.3 the
               plain registration takes over with the full budget from the
               motion before the prediction.
Asserted: learned reaches the plain run's PSNR within 0.1 dB in less wall
time, and beats the tight-budget control by at least 0.3 dB (the network's
own contribution at equal optimiser budget)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from paper_1611_07289_amd import driver, learned, pvr, synth


def test_learned_init_gain_over_plain_registration():
    print("[gpu] learned PVR: 256^3 workload", flush=True)
    P = synth.full_problem()
    dev = torch.device("cuda")
    plan = pvr.Plan.from_problems([P])
    th = torch.from_numpy(P.theta_true.astype(np.float32)).to(dev)
    Xtrue = torch.from_numpy(P.x_true.reshape(-1)).to(dev)
    plan.build(th)
    yc = torch.empty(plan.N, device=dev)
    plan.simulate(Xtrue, y_sim=yc)
    y = torch.from_numpy(synth.corrupt(yc.cpu().numpy(), P.patches, P.outlier_patch,
                                       P.noise_frac, P.seed_base + 3, P.seed_base + 5)).to(dev)
    ymax = float(y.abs().max())
    print("[gpu] learned PVR: training", flush=True)
    Xtr = torch.from_numpy(synth.phantom_uterus(256, 8700, 8701).reshape(-1)).to(dev)
    net = learned.Net(seed=5005)
    learned.train(net, plan, [Xtr], n_pairs=300_000, batch=256, lr=1e-3, seed=8800)
    init_fn = learned.init_fn_factory(net)
    full = pvr.RegParams.make(min_std=0.01 * ymax, exact=True)
    tight = pvr.RegParams.make(step0=0.25, max_iter=5, min_std=0.01 * ymax, exact=True)

    def run(rp, init=None):
        th0 = torch.zeros(plan.M, 6, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, _, hist = driver.reconstruct(plan, y, th0, cycles=3, n_sr=10, reg_params=rp,
                                        init_fn=init, fallback_tau=0.3 if init else None,
                                        fallback_params=full)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, driver.psnr(X, Xtrue, plan), hist

    run(tight)  # warm-up
    res = {}
    for name, rp, init in (("plain", full, None), ("plain_tight", tight, None),
                           ("learned", tight, init_fn)):
        res[name] = run(rp, init)
        print(f"[gpu] learned PVR: {name} {res[name][0]:.3f} s, PSNR {res[name][1]:.2f} dB"
              + (f", fallback {res[name][2]['fallback']}" if init else ""), flush=True)
    t_p, ps_p, _ = res["plain"]
    t_t, ps_t, _ = res["plain_tight"]
    t_l, ps_l, _ = res["learned"]
    assert ps_l >= ps_p - 0.1
    assert t_l < t_p
    assert ps_l >= ps_t + 0.3
