"""Stream ordering of the registration call, which forks work onto the plan's
second stream: pvr_register_patches registers the patches that read the
volume's y-fastest copy there, beside the others, and joins it back before
returning.  Work queued on the caller's stream right after the call must see
every result: here a copy taken on a fresh (default-priority) stream right
after the call, with no device-wide synchronisation in between, equals the
final values, for patches of both layouts (the 32^3 workload's sagittal
stack runs its rows along voxel y)."""
import numpy as np
import pytest
import torch

from paper_1611_07289_amd import pvr, synth
from tests._gpu import dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("exact", [False, True])
def test_registration_results_are_ordered_on_the_call_stream(exact):
    P = synth.tiny_problem()
    print(f"[gpu] stream ordering of registration (exact={exact}), M={P.M}", flush=True)
    th0 = (P.theta_true + synth.random_motion(P.M, 3.0, 1.0, 7)).astype(np.float32)
    plan = pvr.Plan.from_problems([P])
    # observations simulated at the true motion, registration from th0
    plan.build(dev(P.theta_true, torch.float32))
    X = dev(P.x_true.reshape(-1).astype(np.float32))
    y = torch.empty(plan.N, device="cuda")
    plan.simulate(X, y_sim=y)
    plan.build(dev(th0))
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tt = dev(th0)
        ncc = torch.zeros(plan.M, dtype=torch.float32, device="cuda")
        s.wait_stream(torch.cuda.default_stream())
        plan.register(X, y, tt, ncc, params=pvr.RegParams.make(exact=exact))
        snap_t = tt.clone()
        snap_n = ncc.clone()
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(snap_t, tt)
    assert torch.equal(snap_n, ncc)
    # both layouts did work: patches of every stack moved
    moved = (tt.cpu().numpy() != th0).any(1)
    for st in range(len(P.stacks)):
        assert moved[P.patches.stack == st].any(), st
