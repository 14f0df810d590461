"""Pins for the oracle's SLIC superpixels and superpixel patches (paper
Sec. II "Patch Extraction", eq. D and the dilation y_s (+) b).  Pinned by:
with an overwhelming compactness the labels are the Voronoi cells of the grid
(the a x a cells themselves); a piecewise-constant image whose blocks are the
cells is recovered exactly at low compactness; every labelled pixel lies in
its centre's window and takes the least D^2 among the windows covering it
(brute force over every centre); the iteration settles; the dilation equals scipy's binary dilation with the square element,
and the patch masks cover every pixel of the slice."""
import numpy as np
from scipy import ndimage

from oracle import slic


def test_huge_compactness_gives_the_grid_cells():
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 1, size=(32, 40))
    lab, C = slic.slic(img, 8, 1e6, 1e6, iters=3)
    ys, xs = np.mgrid[0:32, 0:40]
    assert np.array_equal(lab, (ys // 8) * 5 + xs // 8)


def test_piecewise_constant_blocks_are_recovered():
    ys, xs = np.mgrid[0:48, 0:48]
    cell = (ys // 16) * 3 + xs // 16
    img = (cell * 37 % 9) * 100.0 + 50.0
    lab, C = slic.slic(img, 16, 1.0, 1e-3, iters=5)
    assert np.array_equal(lab, cell)
    assert np.allclose(C[:, 2], [img[cell == k].mean() for k in range(9)])


def test_assignment_is_the_windowed_argmin_and_centres_are_means():
    rng = np.random.default_rng(1)
    img = ndimage.gaussian_filter(rng.uniform(0, 1000, size=(40, 36)), 2.0)
    lab, C = slic.slic(img, 10, 50.0, 1.0, iters=6)
    h, w = img.shape
    for y in range(0, h, 3):
        for x in range(0, w, 3):
            d2 = [(img[y, x] - c[2]) ** 2 + ((x - c[0]) ** 2 + (y - c[1]) ** 2) / 100.0 * c[3] ** 2
                  if abs(x - c[0]) <= 10 and abs(y - c[1]) <= 10 else np.inf for c in C]
            k = int(np.argmin(d2)) if np.isfinite(min(d2)) else -1
            assert lab[y, x] == k
    assert (lab >= 0).all()
    # the iteration settles: after enough rounds an update moves no centre
    # by more than a small fraction of a pixel
    lab, C = slic.slic(img, 10, 50.0, 1.0, iters=40)
    C2 = slic.update(img, lab, C, 1.0)
    assert np.abs(C2[:, :2] - C[:, :2]).max() < 0.25


def test_dilation_and_patch_masks_cover_the_slice():
    rng = np.random.default_rng(2)
    m = rng.uniform(size=(30, 30)) > 0.97
    for g in (0, 1, 3):
        ref = ndimage.binary_dilation(m, structure=np.ones((2 * g + 1, 2 * g + 1)), iterations=1) if g else m
        assert np.array_equal(slic.dilate(m, g), ref)
    img = ndimage.gaussian_filter(rng.uniform(0, 1000, size=(48, 48)), 2.0)
    lab, _ = slic.slic(img, 12, 50.0, 1.0, iters=4)
    cover = np.zeros(img.shape, int)
    for x0, y0, w, h, mk in slic.superpixel_patches(lab, 3):
        assert mk.shape == (h, w) and mk.any()
        cover[y0:y0 + h, x0:x0 + w] += mk
    assert (cover >= 1).all()
