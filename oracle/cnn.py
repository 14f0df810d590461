"""FP64 CPU reference of the learned initialiser's layers -- TEST
INFRASTRUCTURE ONLY.

3x3 convolution (padding 1, stride s, bias, ReLU) on NHWC tensors through
torch.nn.functional.conv2d in float64, its gradients through autograd, and
the head (fully connected layer from the whole last feature map, weighted
squared loss).
Weights are [Cout][3][3][Cin].  Pinned against a brute-force loop and finite
differences in tests/test_oracle_cnn.py.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float64))


def conv_fwd(x, w, b, stride, relu=True):
    """x [B][H][W][Cin], w [Cout][3][3][Cin], b [Cout] -> [B][Ho][Wo][Cout]."""
    X = _t(x).permute(0, 3, 1, 2)
    Wt = _t(w).permute(0, 3, 1, 2)
    y = F.conv2d(X, Wt, _t(b), stride=stride, padding=1)
    if relu:
        y = torch.relu(y)
    return y.permute(0, 2, 3, 1).numpy()


def conv_grads(x, w, b, stride, gout, out_mask=None):
    """Gradients of sum(gout * relu(conv(x))) with respect to x, w, b.
    out_mask, if given, replaces the ReLU derivative (so that the mask of a
    BF16 forward output can be imposed)."""
    X = _t(x).permute(0, 3, 1, 2).requires_grad_(True)
    Wt = _t(w).permute(0, 3, 1, 2).requires_grad_(True)
    bb = _t(b).requires_grad_(True)
    pre = F.conv2d(X, Wt, bb, stride=stride, padding=1)
    mask = (pre > 0).double() if out_mask is None else _t(out_mask).permute(0, 3, 1, 2)
    g = _t(gout).permute(0, 3, 1, 2) * mask
    (pre * g).sum().backward()
    return (X.grad.permute(0, 2, 3, 1).numpy(), Wt.grad.permute(0, 2, 3, 1).numpy(),
            bb.grad.numpy())


def head(act, wfc, bfc, target=None, loss_w=None):
    """act [B][hw][64], wfc [hw][64][6]; pred[b] = sum_{q,c} act[b,q,c]
    wfc[q,c] + bfc; with a target, the loss sum_b sum_k w_k (pred - target)^2
    / (2B) and its gradients (wfc's in its own shape)."""
    A = _t(act).requires_grad_(True)
    Wf = _t(wfc).requires_grad_(True)
    bf = _t(bfc).requires_grad_(True)
    B = A.shape[0]
    pred = A.reshape(B, -1) @ Wf.reshape(-1, 6) + bf
    if target is None:
        return pred.detach().numpy()
    loss = ((pred - _t(target)) ** 2 * _t(loss_w)).sum() / (2 * B)
    loss.backward()
    return (pred.detach().numpy(), float(loss), A.grad.numpy(), Wf.grad.numpy(), bf.grad.numpy())


def brute_conv(x, w, b, stride):
    """Plain loop definition of the same convolution (no library), for pins."""
    B, H, W, Ci = x.shape
    Co = w.shape[0]
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    y = np.zeros((B, Ho, Wo, Co))
    for n in range(B):
        for oy in range(Ho):
            for ox in range(Wo):
                for co in range(Co):
                    s = b[co]
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = oy * stride + ky - 1, ox * stride + kx - 1
                            if 0 <= iy < H and 0 <= ix < W:
                                s += float(np.dot(w[co, ky, kx], x[n, iy, ix]))
                    y[n, oy, ox, co] = s
    return y
