"""The learned initialiser's convolution kernels at the sizes training and
inference run them: batch 256 on the network's 64 x 64 input, every layer at
its own input size (64, 32, 16 and 8 pixels square), forward, weight gradient
and data gradient against the FP64 reference on the same BF16 inputs.  At
these sizes the kernels take their multi-tile persistent loops and the weight
gradient its two-level reduction (more than 256 partial rows per layer).

Tolerance as for the small cases: relative L2 <= 1e-2 per tensor (BF16
operands and BF16 stored outputs, FP32 accumulation).  Element-wise, the
forward output within one BF16 rounding of the reference (2^-8 of its
magnitude, plus 1e-3 of the tensor's RMS for the FP32 accumulation), and the
FP32 bias gradient within 1e-4 of the largest reference entry."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from oracle import cnn as ocnn
from paper_1611_07289_amd import learned, pvr

B = 256


def _bf(a):
    t = torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16)
    return t.float().double().numpy()


def _dev(a, dtype=torch.bfloat16):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dtype).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def _sizes():
    h, out = learned.SIDE, []
    for cin, cout, s in learned.LAYERS:
        out.append((cin, cout, s, h))
        h = (h - 1) // s + 1
    return out


@pytest.mark.parametrize("cin,cout,s,H", _sizes())
def test_conv_layer_at_training_size(cin, cout, s, H):
    W = H
    print(f"[gpu] conv {cin}->{cout} s{s} at {B}x{H}x{W}", flush=True)
    L = pvr.load()
    rng = np.random.default_rng(1000 + cin * 7 + cout + s + H)
    # post-ReLU-like inputs for the inner layers, signed for the first
    x = rng.normal(size=(B, H, W, cin))
    if cin > 2:
        x = np.maximum(x, 0)
    x = _bf(x)
    w = _bf(rng.normal(size=(cout, 3, 3, cin)) * math.sqrt(2.0 / (9 * cin)))
    b = rng.normal(size=cout).astype(np.float32) * 0.1
    Ho, Wo = (H - 1) // s + 1, (W - 1) // s + 1
    xd, wd, bd = _dev(x), _dev(w), torch.from_numpy(b).cuda()
    out = torch.empty(B * Ho * Wo * cout, dtype=torch.bfloat16, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    pvr._check(L.pvr_cnn_conv_fwd(xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), out.data_ptr(),
                                  B, H, W, cin, cout, s, 1, st))
    g = _bf(rng.normal(size=(B, Ho, Wo, cout)))
    gd = _dev(g)
    scr = torch.empty(L.pvr_cnn_wgrad_scratch(B, H, W, cin, cout, s) // 4 + 16, device="cuda")
    dw = torch.empty(cout * 9 * cin, device="cuda")
    db = torch.empty(cout, device="cuda")
    pvr._check(L.pvr_cnn_conv_wgrad(gd.data_ptr(), out.data_ptr(), xd.data_ptr(), scr.data_ptr(),
                                    dw.data_ptr(), db.data_ptr(), B, H, W, cin, cout, s, st))
    gin = None
    if cin >= 16:
        wt = torch.from_numpy(np.ascontiguousarray(w.transpose(1, 2, 3, 0)).astype(np.float32)).to(
            torch.bfloat16).cuda()
        gin = torch.empty(B * H * W * cin, dtype=torch.bfloat16, device="cuda")
        pvr._check(L.pvr_cnn_conv_dgrad(gd.data_ptr(), out.data_ptr(), wt.data_ptr(),
                                        gin.data_ptr(), B, H, W, cin, cout, s, st))
    torch.cuda.synchronize()
    got = out.float().cpu().numpy().reshape(B, Ho, Wo, cout)
    ref = ocnn.conv_fwd(x, w, b.astype(np.float64), s)
    e_f = _rel(got, ref)
    rms = float(np.sqrt(np.mean(ref ** 2)))
    # worst element error in units of its bar 2^-8 |ref| + 1e-3 RMS
    worst_f = float((np.abs(got - ref) / (2.0 ** -8 * np.abs(ref) + 1e-3 * rms)).max())
    mask = (got > 0).astype(np.float64)  # the GPU's own ReLU mask
    gx_r, gw_r, gb_r = ocnn.conv_grads(x, w, b.astype(np.float64), s, g, out_mask=mask)
    e_w = _rel(dw.cpu().numpy(), gw_r.reshape(-1))
    e_b = _rel(db.cpu().numpy(), gb_r)
    worst_b = float(np.abs(db.cpu().numpy() - gb_r).max()) / float(np.abs(gb_r).max())
    msg = (f"[gpu] conv {cin}->{cout} s{s} {B}x{H}x{W}: fwd {e_f:.1e} (worst {worst_f:.2f} of "
           f"its bar) dw {e_w:.1e} db {e_b:.1e} (worst {worst_b:.1e} of max)")
    if gin is not None:
        e_x = _rel(gin.float().cpu().numpy().reshape(gx_r.shape), gx_r)
        msg += f" dx {e_x:.1e}"
        assert e_x <= 1e-2
    print(msg, flush=True)
    assert e_f <= 1e-2 and e_w <= 1e-2 and e_b <= 1e-2
    assert worst_f <= 1.0 and worst_b <= 1e-4
