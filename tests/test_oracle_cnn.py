"""Pins for the FP64 reference of the initialiser's layers: the library
convolution equals a plain loop, and its autograd gradients equal central
finite differences."""
import numpy as np
import pytest

from oracle import cnn


def test_conv_matches_loop_definition():
    rng = np.random.default_rng(0)
    for stride in (1, 2):
        x = rng.normal(size=(2, 7, 6, 3))
        w = rng.normal(size=(4, 3, 3, 3))
        b = rng.normal(size=4)
        ref = cnn.brute_conv(x, w, b, stride)
        got = cnn.conv_fwd(x, w, b, stride, relu=False)
        assert np.allclose(got, ref, atol=1e-12)
        assert np.allclose(cnn.conv_fwd(x, w, b, stride), np.maximum(ref, 0), atol=1e-12)


def test_conv_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 5, 5, 2))
    w = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=3) + 0.5
    g = rng.normal(size=(1, 3, 3, 3))
    gx, gw, gb = cnn.conv_grads(x, w, b, 2, g)
    f = lambda x_, w_, b_: float((cnn.conv_fwd(x_, w_, b_, 2) * g).sum())
    h = 1e-6
    for idx in [(0, 1, 2, 0), (0, 4, 4, 1), (0, 0, 3, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h; xm[idx] -= h
        assert gx[idx] == pytest.approx((f(xp, w, b) - f(xm, w, b)) / (2 * h), rel=1e-5, abs=1e-7)
    for idx in [(0, 1, 1, 0), (2, 0, 2, 1)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h; wm[idx] -= h
        assert gw[idx] == pytest.approx((f(x, wp, b) - f(x, wm, b)) / (2 * h), rel=1e-5, abs=1e-7)
    bp, bm = b.copy(), b.copy()
    bp[1] += h; bm[1] -= h
    assert gb[1] == pytest.approx((f(x, w, bp) - f(x, w, bm)) / (2 * h), rel=1e-5, abs=1e-7)


def test_head_gradients():
    """Prediction against a plain loop; loss and every gradient against
    central differences of the loss (the loss is quadratic in each argument,
    so central differences are exact up to rounding)."""
    rng = np.random.default_rng(2)
    B, hw = 3, 4
    act = rng.normal(size=(B, hw, 64))
    wfc, bfc = rng.normal(size=(hw, 64, 6)), rng.normal(size=6)
    tgt, lw = rng.normal(size=(B, 6)), np.array([1, 2, 1, 1, 0.5, 1.0])
    pred, loss, ga, gw, gb = cnn.head(act, wfc, bfc, tgt, lw)
    ref = np.zeros((B, 6))
    for b in range(B):
        for k in range(6):
            ref[b, k] = bfc[k] + sum(act[b, q, c] * wfc[q, c, k] for q in range(hw) for c in range(64))
    assert np.allclose(pred, ref, rtol=1e-12, atol=1e-12)
    assert loss == pytest.approx(sum(lw[k] * (ref[b, k] - tgt[b, k]) ** 2
                                     for b in range(B) for k in range(6)) / (2 * B))

    def L(a=act, w=wfc, bb=bfc):
        return cnn.head(a, w, bb, tgt, lw)[1]

    h = 1e-3
    for idx in [(0, 0, 0), (2, 3, 63), (1, 2, 17)]:
        ap, am = act.copy(), act.copy()
        ap[idx] += h; am[idx] -= h
        assert ga[idx] == pytest.approx((L(a=ap) - L(a=am)) / (2 * h), rel=1e-7, abs=1e-10)
    for idx in [(0, 0, 0), (3, 63, 5), (1, 30, 2)]:
        wp, wm = wfc.copy(), wfc.copy()
        wp[idx] += h; wm[idx] -= h
        assert gw[idx] == pytest.approx((L(w=wp) - L(w=wm)) / (2 * h), rel=1e-7, abs=1e-10)
    for k in range(6):
        bp, bm = bfc.copy(), bfc.copy()
        bp[k] += h; bm[k] -= h
        assert gb[k] == pytest.approx((L(bb=bp) - L(bb=bm)) / (2 * h), rel=1e-7, abs=1e-10)
