"""pvr_slic_pack_noalloc (the packing without a workspace, for callers that
cannot allocate device memory) through the C ABI against pvr_slic_pack with
its caller workspace: samples and masks bit-exact, on two calls in a row, the
second with a smaller input (fewer images and patches, another dilation), so
that the second call's table overwrites only part of the first call's
entries in the library-resident array.  The size limit is checked on the
host."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from paper_1611_07289_amd import pvr
from paper_1611_07289_amd import superpixel as sp
from paper_1611_07289_amd import synth

A = 12


def _case(n_img, h, w, gamma, seed):
    I = torch.from_numpy(synth.slice_images(n_img, h, w, seed=seed)).cuda()
    lab, C = sp.slic(I, A, 40.0, 5.0, iters=4)
    tab = sp.patch_table(sp.boxes(lab, C, A, gamma).cpu().numpy())
    return I, lab, tab


@pytest.mark.parametrize("first,second", [((6, 61, 53, 5, 901), (2, 40, 33, 2, 902))])
def test_noalloc_pack_matches_workspace_pack(first, second):
    for n_img, h, w, gamma, seed in (first, second):
        print(f"[gpu] no-alloc pack: {n_img} images {h}x{w}, gamma {gamma}", flush=True)
        I, lab, tab = _case(n_img, h, w, gamma, seed)
        assert tab.shape[0] > 0
        y_ws, m_ws = sp.pack(I, lab, gamma, tab)
        y_na, m_na = sp.pack(I, lab, gamma, tab, noalloc=True)
        torch.cuda.synchronize()
        assert y_ws.shape == y_na.shape and m_ws.shape == m_na.shape
        assert torch.equal(y_ws, y_na)
        assert torch.equal(m_ws, m_na)
        print(f"[gpu] no-alloc pack: {tab.shape[0]} patches, {y_ws.numel()} samples identical",
              flush=True)


def test_noalloc_pack_rejects_too_many_patches():
    L = pvr.load()
    fake = ctypes.c_void_p(64)  # never dereferenced: the size check comes first
    M = pvr.PVR_SLIC_PACK_NOALLOC_MAX + 1
    tab = np.zeros((M, 6), np.int32)
    st = L.pvr_slic_pack_noalloc(fake, fake, 1, 8, 8, 1, M, tab.ctypes.data, fake, fake, None)
    assert st == pvr.PVR_ESHAPE and "at most" in L.pvr_last_error().decode()
