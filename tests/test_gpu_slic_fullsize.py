"""SLIC superpixel patches at the benchmark's size: the 240 observed slices of
the 256^3 uterus workload's four stacks of 256 x 256 x 60, step a = 32 (64
centres per slice), 10 iterations, dilation gamma = 19 (60 % of a), in the
launch configuration the benchmark times.  Checked on sampled slices: the
GPU's final labels are a valid assignment of its final centres (the oracle's
FP64 distances, near-ties aside); the full oracle run from the same slice
agrees on >= 98 % of the pixels; sampled patches' boxes, masks and samples
are bit-exact against the oracle's dilation of the GPU's labels."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from oracle import slic as oslic
from paper_1611_07289_amd import superpixel as sp
from paper_1611_07289_amd import synth
from tests.test_gpu_slic import _check_assignment

A, GAMMA, T0, TMIN, ITERS = 32, 19, 40.0, 5.0, 10


def test_fullsize_slic_sampled():
    print("[gpu] slic full size: 240 x 256 x 256, a=32, gamma=19", flush=True)
    I = synth.slice_images(240, 256, 256, seed=977, n=256)
    Ig = torch.from_numpy(I).cuda()
    lab, C = sp.slic(Ig, A, T0, TMIN, ITERS)
    B = sp.boxes(lab, C, A, GAMMA).cpu().numpy()
    tab = sp.patch_table(B)
    y, m = sp.pack(Ig, lab, GAMMA, tab)
    lab, C = lab.cpu().numpy(), C.cpu().numpy()
    y, m = y.cpu().numpy(), m.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(tab[:, 4].astype(np.int64) * tab[:, 5])])
    rng = np.random.default_rng(5)
    for i in rng.choice(240, 3, replace=False):
        img = I[i].astype(np.float64)
        _check_assignment(img, C[i].astype(np.float64), lab[i], A)
        lab_o, _ = oslic.slic(img, A, T0, TMIN, ITERS)
        assert (lab_o == lab[i]).mean() >= 0.98
    for s in rng.choice(tab.shape[0], 8, replace=False):
        i, k, x0, y0, w, h = (int(v) for v in tab[s])
        mk = lab[i] == k
        ys, xs = np.nonzero(mk)
        # the dilation within a crop reaching gamma past the superpixel equals
        # the dilation of the whole slice there
        cy0, cy1 = max(0, ys.min() - GAMMA), min(256, ys.max() + GAMMA + 1)
        cx0, cx1 = max(0, xs.min() - GAMMA), min(256, xs.max() + GAMMA + 1)
        d = oslic.dilate(mk[cy0:cy1, cx0:cx1], GAMMA)
        yy, xx = np.nonzero(d)
        assert (x0, y0, w, h) == (cx0 + xx.min(), cy0 + yy.min(), xx.max() - xx.min() + 1,
                                  yy.max() - yy.min() + 1)
        ref = d[yy.min():yy.max() + 1, xx.min():xx.max() + 1]
        seg = slice(off[s], off[s + 1])
        assert np.array_equal(m[seg].reshape(h, w).astype(bool), ref)
        assert np.array_equal(y[seg].reshape(h, w), I[i, y0:y0 + h, x0:x0 + w])
