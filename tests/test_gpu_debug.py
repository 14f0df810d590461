"""Debug mode (pvr_set_debug / PVR_DEBUG): the core entry points reject a
non-finite input element (or a negative patch weight) by array and index
before launching anything, leave the results of valid calls unchanged, and
let bad values through when the mode is off (the device fault flags of
pvr_check cover that case)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from paper_1611_07289_amd import pvr, synth


def test_debug_mode_rejects_bad_inputs_by_name_and_index():
    P = synth.tiny_problem()
    dev = torch.device("cuda")
    plan = pvr.Plan.from_problems([P])
    th = torch.from_numpy(P.theta_true.astype(np.float32)).to(dev)
    X = torch.from_numpy(P.x_true.reshape(-1).astype(np.float32)).to(dev)
    was = pvr.get_debug()
    try:
        pvr.set_debug(False)
        plan.build(th)
        y0 = torch.empty(plan.N, device=dev)
        plan.simulate(X, y_sim=y0)
        pvr.set_debug(True)
        assert pvr.get_debug()
        plan.build(th)
        y1 = torch.empty(plan.N, device=dev)
        plan.simulate(X, y_sim=y1)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1)  # the checks change no result

        def rejected(fn, what):
            with pytest.raises(pvr.PvrError) as ei:
                fn()
            assert ei.value.status == pvr.PVR_EINVAL
            assert what in str(ei.value), str(ei.value)
            print(f"[gpu] debug mode: {ei.value}", flush=True)

        tb = th.clone()
        tb[5, 2] = math.nan
        rejected(lambda: plan.build(tb), "theta[32]")
        Xb = X.clone()
        Xb[1234] = math.inf
        rejected(lambda: plan.simulate(Xb, y_sim=y1), "X[1234]")
        e = y0.clone()
        w = torch.ones(plan.M, device=dev)
        w[7] = -0.5
        rejected(lambda: plan.backproject(e, None, w), "patch_w[7]")
        eb = e.clone()
        eb[99] = math.nan
        rejected(lambda: plan.backproject(eb), "e[99]")
        num = torch.zeros(plan.V, device=dev)
        den = torch.ones(plan.V, device=dev)
        den[3] = math.nan
        rejected(lambda: plan.sr_update(X, num, den, torch.empty_like(X)), "den[3]")
        em = plan.em_state()
        rejected(lambda: plan.robust_weights(eb, y0, em, patch_w=torch.empty_like(w)), "resid[99]")
        yb = y0.clone()
        yb[10] = -math.inf
        rejected(lambda: plan.register(X, yb, th.clone()), "y_obs[10]")
        # the plan is unharmed: a valid call still gives the same result
        y2 = torch.empty(plan.N, device=dev)
        plan.simulate(X, y_sim=y2)
        torch.cuda.synchronize()
        assert torch.equal(y0, y2)
        # with the mode off the same bad input goes through
        pvr.set_debug(False)
        plan.simulate(Xb, y_sim=y2)
        torch.cuda.synchronize()
    finally:
        pvr.set_debug(was)
