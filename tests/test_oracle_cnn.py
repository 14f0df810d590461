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
    rng = np.random.default_rng(2)
    act = rng.normal(size=(3, 4, 64))
    wfc, bfc = rng.normal(size=(64, 6)), rng.normal(size=6)
    tgt, lw = rng.normal(size=(3, 6)), np.array([1, 2, 1, 1, 0.5, 1.0])
    pred, loss, ga, gw, gb = cnn.head(act, wfc, bfc, tgt, lw)
    assert np.allclose(pred, act.mean(1) @ wfc + bfc)
    assert loss == pytest.approx(((pred - tgt) ** 2 * lw).sum() / 6)
    d = (pred - tgt) * lw / 3
    assert np.allclose(gb, d.sum(0))
    assert np.allclose(gw, act.mean(1).T @ d)
    assert np.allclose(ga, np.repeat((d @ wfc.T)[:, None, :] / 4, 4, axis=1))
