"""Learned initialiser kernels (BF16 MFMA convolutions, head, Adam) against
the FP64 reference on BF16-rounded inputs, and training on pairs from the
forward model.

Tolerance: relative L2 error per layer output / gradient <= 1e-2 (BF16
operands and BF16 stored outputs, FP32 accumulation).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402  (CPU import is fine; GPU use is gated by the marker)

from oracle import cnn as ocnn
from paper_1611_07289_amd import learned, pvr, synth


def _bf(a):
    """BF16 rounding (round to nearest even), returned as float64."""
    t = torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16)
    return t.float().double().numpy()


def _dev(a, dtype=torch.bfloat16):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dtype).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("cin,cout,s", learned.LAYERS[:4] + [(64, 64, 1)])
def test_conv_layer_matches_reference(cin, cout, s):
    L = pvr.load()
    rng = np.random.default_rng(cin * 100 + cout + s)
    B, H, W = 3, 16, 12
    x = _bf(rng.normal(size=(B, H, W, cin)))
    w = _bf(rng.normal(size=(cout, 3, 3, cin)) * math.sqrt(2.0 / (9 * cin)))
    b = rng.normal(size=cout).astype(np.float32) * 0.1
    Ho, Wo = (H - 1) // s + 1, (W - 1) // s + 1
    xd, wd, bd = _dev(x), _dev(w), torch.from_numpy(b).cuda()
    out = torch.empty(B * Ho * Wo * cout, dtype=torch.bfloat16, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    pvr._check(L.pvr_cnn_conv_fwd(xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), out.data_ptr(),
                                  B, H, W, cin, cout, s, 1, st))
    ref = ocnn.conv_fwd(x, w, b.astype(np.float64), s)
    got = out.float().cpu().numpy().reshape(ref.shape)
    e_f = _rel(got, ref)
    # gradients with the GPU's own ReLU mask
    g = _bf(rng.normal(size=ref.shape))
    gd = _dev(g)
    mask = (got > 0).astype(np.float64)
    gx_r, gw_r, gb_r = ocnn.conv_grads(x, w, b.astype(np.float64), s, g, out_mask=mask)
    wt = torch.from_numpy(np.ascontiguousarray(w.transpose(1, 2, 3, 0)).astype(np.float32)).to(
        torch.bfloat16).cuda()
    dw = torch.empty(cout * 9 * cin, device="cuda")
    db = torch.empty(cout, device="cuda")
    scr = torch.empty(L.pvr_cnn_wgrad_scratch(B, H, W, cin, cout, s) // 4 + 16, device="cuda")
    pvr._check(L.pvr_cnn_conv_wgrad(gd.data_ptr(), out.data_ptr(), xd.data_ptr(), scr.data_ptr(),
                                    dw.data_ptr(), db.data_ptr(), B, H, W, cin, cout, s, st))
    e_w = _rel(dw.cpu().numpy(), gw_r.reshape(-1))
    e_b = _rel(db.cpu().numpy(), gb_r)
    msg = f"[gpu] conv {cin}->{cout} s{s}: fwd {e_f:.1e} dw {e_w:.1e} db {e_b:.1e}"
    if cin >= 16:
        gin = torch.empty(B * H * W * cin, dtype=torch.bfloat16, device="cuda")
        pvr._check(L.pvr_cnn_conv_dgrad(gd.data_ptr(), out.data_ptr(), wt.data_ptr(),
                                        gin.data_ptr(), B, H, W, cin, cout, s, st))
        e_x = _rel(gin.float().cpu().numpy().reshape(gx_r.shape), gx_r)
        msg += f" dx {e_x:.1e}"
        assert e_x <= 1e-2
    torch.cuda.synchronize()
    print(msg)
    assert e_f <= 1e-2 and e_w <= 1e-2 and e_b <= 1e-2


def test_head_matches_reference():
    L = pvr.load()
    rng = np.random.default_rng(9)
    B, hw = 5, 64
    act = _bf(np.abs(rng.normal(size=(B, hw, 64))))
    wfc = rng.normal(size=(hw, 64, 6)).astype(np.float32) * 0.02
    bfc = rng.normal(size=6).astype(np.float32)
    tgt = rng.normal(size=(B, 6)).astype(np.float32)
    lw = np.array([1, 1, 1, 2, 2, 2], np.float32)
    pred_r, loss_r, ga_r, gw_r, gb_r = ocnn.head(act, wfc, bfc, tgt, lw)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    ad = _dev(act)
    pred = torch.empty(B * 6, device="cuda")
    loss = torch.empty(1, device="cuda")
    gact = torch.empty(B * hw * 64, dtype=torch.bfloat16, device="cuda")
    dwfc = torch.empty(hw * 64 * 6, device="cuda")
    dbfc = torch.empty(6, device="cuda")
    scr = torch.empty(L.pvr_cnn_head_scratch(B) // 4 + 16, device="cuda")
    tw, tb, tt, tl = t(wfc), t(bfc), t(tgt), t(lw)
    pvr._check(L.pvr_cnn_head(ad.data_ptr(), B, hw, tw.data_ptr(), tb.data_ptr(), tt.data_ptr(),
                              tl.data_ptr(), pred.data_ptr(), loss.data_ptr(), gact.data_ptr(),
                              dwfc.data_ptr(), dbfc.data_ptr(), scr.data_ptr(),
                              torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert _rel(pred.cpu().numpy(), pred_r.reshape(-1)) <= 1e-5
    assert float(loss) == pytest.approx(loss_r, rel=1e-5)
    assert _rel(dwfc.cpu().numpy(), gw_r.reshape(-1)) <= 1e-5
    assert _rel(dbfc.cpu().numpy(), gb_r) <= 1e-5
    assert _rel(gact.float().cpu().numpy(), ga_r.reshape(-1)) <= 1e-2


@pytest.fixture(scope="module")
def small():
    print("[gpu] 96^3 problem with 64x64 patches", flush=True)
    P = synth.full_problem(seed_cfg=5, n=96, slices=24, a=64)
    plan = pvr.Plan.from_problems([P])
    X = torch.from_numpy(P.x_true.reshape(-1)).cuda()
    return P, plan, X


def _heldout_rel_mse(net, plan, X):
    """Per-component mean squared error of the prediction over held-out
    offsets, relative to the targets' mean square (1 = no better than
    predicting no correction)."""
    dev = X.device
    ref = torch.from_numpy(synth.random_motion(plan.M, 10, 5, 9001).astype(np.float32)).to(dev)
    off = torch.from_numpy(synth.random_motion(plan.M, 10, 5, 9002).astype(np.float32)).to(dev)
    y_obs, y_sim = learned.make_pairs(plan, X, ref, off, 0.01 * float(X.max()), 9003)
    tgt = plan.motion_frame(off)
    B = 128
    se = torch.zeros(6, device=dev, dtype=torch.float64)
    ms = torch.zeros(6, device=dev, dtype=torch.float64)
    for b0 in range(0, plan.M - B + 1, B):
        ids = torch.arange(b0, b0 + B, dtype=torch.int32, device=dev)
        pred = net.predict(plan, y_obs, y_sim, ids, B).double()
        t = tgt[b0:b0 + B].double()
        se += ((t - pred) ** 2).sum(0)
        ms += (t ** 2).sum(0)
    return (se / ms).cpu().numpy()


def test_training_reduces_loss_and_prediction_helps(small):
    """Training on forward-model pairs lowers the loss, and on held-out
    offsets the prediction recovers the in-plane components of the offset
    (translation along u and v, rotation about the slice normal), which a
    single observed / simulated pair determines.  The out-of-plane
    components are reported only: from one pair the sign of a through-plane
    shift is ambiguous."""
    P, plan, X = small
    net = learned.Net(seed=7)
    before = _heldout_rel_mse(net, plan, X)
    res = learned.train(net, plan, [X], n_pairs=300_000, batch=128, lr=1e-3, seed=600)
    losses = [l for _, l in res["loss"]]
    after = _heldout_rel_mse(net, plan, X)
    print(f"[gpu] training: {res['pairs']} pairs in {res['seconds']:.1f} s; batch loss "
          f"{losses[0]:.3f} -> {np.mean(losses[-5:]):.3f} (mean of the last 5 logs)")
    print(f"[gpu] held-out relative MSE (rot u, rot v, rot n, t u, t v, t n): before "
          f"{np.round(before, 3)}, after {np.round(after, 3)}")
    assert np.mean(losses[-5:]) < 0.7 * losses[0]
    assert np.all(after[2:5] < 0.6)
    assert after.mean() < 0.8
