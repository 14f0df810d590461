"""Host-side checks of the superpixel entry points (no GPU): the centre count,
argument validation before any device call, and the ordering of the pack
table built from the boxes."""
import ctypes

import numpy as np

from oracle import slic
from paper_1611_07289_amd import pvr, superpixel


def test_centre_count():
    L = pvr.load()
    assert L.pvr_slic_centres(256, 256, 32) == 64
    assert L.pvr_slic_centres(61, 53, 12) == 6 * 5
    assert L.pvr_slic_centres(5, 7, 100) == 1
    assert L.pvr_slic_centres(0, 7, 3) == 0 and L.pvr_slic_centres(5, 7, 0) == 0


def test_invalid_arguments_rejected_on_host():
    L = pvr.load()
    fake = ctypes.c_void_p(64)  # never dereferenced: every case fails first
    assert L.pvr_slic_init(None, 1, 8, 8, 4, 1.0, fake, None) == 1
    assert L.pvr_slic_init(fake, 1, 8, 8, 0, 1.0, fake, None) == 1
    assert L.pvr_slic_assign(fake, 1, 8, 8, (1 << 20) + 1, fake, fake, fake, None) == 1
    assert L.pvr_slic_update(fake, 1, 1, (1 << 21), 4, fake, 0.0, fake, None) == 2
    assert L.pvr_slic_assign(fake, 0, 8, 8, 4, fake, fake, fake, None) == 1
    assert L.pvr_slic_assign(fake, 70000, 8, 8, 4, fake, fake, fake, None) == 2
    assert L.pvr_slic_assign(fake, 40000, 256, 256, 4, fake, fake, fake, None) == 2
    assert L.pvr_slic_update(fake, 1, 8, 8, 4, None, 0.0, fake, None) == 1
    assert L.pvr_slic(fake, 1, 8, 8, 4, 1.0, 1.0, -1, fake, fake, fake, None) == 1
    assert L.pvr_slic_boxes(fake, 1, 8, 8, 4, fake, -1, fake, None) == 1
    big = 1 << 20  # workspace bytes claimed by the fake pointer
    tab = np.array([[0, 0, 4, 4, 5, 4]], np.int32)  # x0 + w = 9 > 8
    st = L.pvr_slic_pack(fake, fake, 1, 8, 8, 2, 1, tab.ctypes.data, fake, big, fake, fake, None)
    assert st == 2 and "leaves its image" in L.pvr_last_error().decode()
    tab = np.array([[1, 0, 0, 0, 4, 4]], np.int32)  # image 1 of 1
    assert L.pvr_slic_pack(fake, fake, 1, 8, 8, 2, 1, tab.ctypes.data, fake, big, fake, fake,
                           None) == 2
    tab = np.array([[0, 0, 0, 0, 300, 300]], np.int32)  # 90 000 pixels
    st = L.pvr_slic_pack(fake, fake, 1, 512, 512, 2, 1, tab.ctypes.data, fake, big, fake, fake,
                         None)
    assert st == 2 and "at most 65536" in L.pvr_last_error().decode()
    assert L.pvr_slic_pack(fake, fake, 1, 8, 8, -1, 1, tab.ctypes.data, fake, big, fake, fake,
                           None) == 1
    assert L.pvr_slic_pack(fake, fake, 1, 8, 8, 1, 0, tab.ctypes.data, None, 0, None, None,
                           None) == 0
    # the staged descriptor table needs its workspace
    tab = np.array([[0, 0, 0, 0, 4, 4]] * 3, np.int32)
    need = L.pvr_slic_pack_workspace(3)
    assert need >= 3 * 28 and L.pvr_slic_pack_workspace(0) == 0
    st = L.pvr_slic_pack(fake, fake, 1, 8, 8, 1, 3, tab.ctypes.data, fake, need - 1, fake, fake,
                         None)
    assert st == 2 and "workspace" in L.pvr_last_error().decode()
    assert L.pvr_slic_pack(fake, fake, 1, 8, 8, 1, 3, tab.ctypes.data, None, need, fake, fake,
                           None) == 1


def test_pack_table_follows_the_oracle_patch_order():
    # boxes of two label images written from the oracle's patches; empty
    # superpixels (labels 1 and 5 of image 0) carry zero boxes and drop out
    rng = np.random.default_rng(4)
    labs = [rng.integers(0, 6, size=(20, 24)), rng.integers(0, 6, size=(20, 24))]
    labs[0][labs[0] == 1] = 0
    labs[0][labs[0] == 5] = 2
    B = np.zeros((2, 6, 4), np.int32)
    expect = []
    for i, lab in enumerate(labs):
        ks = [k for k in range(6) if (lab == k).any()]
        for k, (x0, y0, w, h, _) in zip(ks, slic.superpixel_patches(lab, 2)):
            B[i, k] = (x0, y0, w, h)
            expect.append((i, k, x0, y0, w, h))
    assert np.array_equal(superpixel.patch_table(B), np.array(expect, np.int32))


def test_misaligned_device_pointers_rejected_on_host():
    L = pvr.load()
    a, odd = ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 2)
    assert L.pvr_sr_update(None, odd, a, a, None, a, None) == 1
    assert "4-byte aligned" in L.pvr_last_error().decode()
    assert L.pvr_simulate_f64(None, ctypes.c_void_p(4096 + 4), None, None, None, None) == 1
    assert "8-byte aligned" in L.pvr_last_error().decode()
    assert L.pvr_slic_init(a, 1, 8, 8, 4, 1.0, ctypes.c_void_p(4096 + 8), None) == 1
    assert "centres is not 16-byte aligned" in L.pvr_last_error().decode()
    assert L.pvr_cnn_conv_fwd(ctypes.c_void_p(4096 + 8), a, a, a, 1, 8, 8, 32, 32, 1, 1, None) == 1
    assert "16-byte aligned" in L.pvr_last_error().decode()
