"""The cycle's sample mask and active set survive the learned initialiser and
the joint gradient registration: both rebuild the plan several times, and
each build must take the mask (arbitrarily shaped patches inside their boxes,
paper Sec. II "Patch Extraction") and the active set (multi-scale cycles), or
the registration that follows would see every sample of every box.

A 96^3 phantom with 4 stacks of 96 x 96 x 24 and 64 x 64 patches (stride 32,
the learned initialiser's input size), a seeded mask dropping 30 % of the
samples and every third patch inactive.  Checked after the initialiser (just
before the registration reads the plan), after the cycle, and after the
joint registration: a unit volume simulates to 0 on every masked sample and
every sample of an inactive patch, and to 1 on most of the others."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from paper_1611_07289_amd import driver, learned, pvr, synth


def test_mask_and_active_set_survive_initialiser_and_joint_registration():
    P = synth.full_problem(seed_cfg=9, n=96, slices=24, a=64)
    print(f"[gpu] mask/active: M={P.M} N={P.N}", flush=True)
    dev = torch.device("cuda")
    plan = pvr.Plan.from_problems([P])
    th = torch.from_numpy(P.theta_true.astype(np.float32)).to(dev)
    Xt = torch.from_numpy(P.x_true.reshape(-1)).to(dev)
    plan.build(th)
    y = torch.empty(plan.N, device=dev)
    plan.simulate(Xt, y_sim=y)
    rng = np.random.default_rng(3)
    mask = (rng.uniform(size=P.N) > 0.3).astype(np.uint8)
    act = (np.arange(P.M) % 3 != 0).astype(np.uint8)
    off_samples = np.repeat(act == 0, np.diff(P.patches.sample_off))
    md, ad = torch.from_numpy(mask).to(dev), torch.from_numpy(act).to(dev)
    ones = torch.ones(plan.V, device=dev)

    def check(tag):
        ys = torch.empty(plan.N, device=dev)
        plan.simulate(ones, y_sim=ys)
        v = (ys > 0.5).cpu().numpy()
        assert not v[mask == 0].any(), tag
        assert not v[off_samples].any(), tag
        kept = v[(mask == 1) & ~off_samples].mean()
        print(f"[gpu] mask/active {tag}: {kept:.3f} of the kept samples valid", flush=True)
        assert kept > 0.5, tag

    base = learned.init_fn_factory(learned.Net(seed=5))
    calls = []

    def init(plan_, X, y_, theta, active=None, mask=None):
        out = base(plan_, X, y_, theta, active=active, mask=mask)
        check("after the initialiser")
        calls.append(1)
        return out

    th0 = th + torch.from_numpy(synth.random_motion(P.M, 2.0, 1.0, 4).astype(np.float32)).to(dev)
    driver.reconstruct(plan, y, th0.clone(), cycles=1, n_sr=2, init_fn=init, active_schedule=[ad],
                       sample_mask=md, fallback_tau=0.3)
    assert calls
    check("after the cycle")
    th1 = th0.clone()
    driver.register_gradient(plan, Xt, y, th1, iters=3, active=ad, mask=md)
    check("after the joint registration")
    # inactive patches keep their motion
    assert torch.equal(th1[torch.from_numpy(act == 0).to(dev)], th0[torch.from_numpy(act == 0).to(dev)])
