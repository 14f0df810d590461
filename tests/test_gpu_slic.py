"""SLIC superpixels and superpixel patches through the C ABI against the FP64
oracle (paper Sec. II "Patch Extraction", eq. D and the dilation by gamma).

Cases: 6 ragged images (61 x 53, step 12: 6 x 5 cells, the last row and
column of cells cut short).  Initial centres are bit-exact.  One assignment
from common centres agrees everywhere except at near-ties of D^2 (FP32 on the
GPU, FP64 in the oracle; a disagreement is accepted only when the oracle's
two distances differ by less than 1e-5 relative).  One update from common
labels agrees to 1e-5.  Ten full iterations agree on >= 99 % of the pixels,
and the GPU's final labels are a valid assignment of its own final centres.
Boxes, masks and packed samples are integer / copy work: bit-exact against
the oracle on the GPU's labels.  Edge cases: a step larger than the image,
a constant image (pure spatial distance, exact ties), gamma = 0."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

from oracle import slic as oslic
from paper_1611_07289_amd import superpixel as sp
from paper_1611_07289_amd import synth

A, T0, TMIN = 12, 40.0, 5.0


@pytest.fixture(scope="module")
def imgs():
    print("[gpu] slic: 6 ragged 61x53 images, step 12", flush=True)
    I = synth.slice_images(6, 61, 53, seed=811)
    return I, torch.from_numpy(I).cuda()


def _d2(img, C, lab, a):
    """FP64 D^2 of every pixel to the centre of its label (inf for -1)."""
    h, w = img.shape
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    c = C[np.maximum(lab, 0)]
    d = (img - c[..., 2]) ** 2 + ((xs - c[..., 0]) ** 2 + (ys - c[..., 1]) ** 2) / (a * a) * c[..., 3] ** 2
    return np.where(lab >= 0, d, np.inf)


def _check_assignment(img, C, lab_gpu, a, max_frac=1e-3):
    """lab_gpu is an assignment of centres C (float64 copies of the FP32
    centres) up to FP32 near-ties."""
    lab_o, best = oslic.assign(img, C, a)
    diff = lab_gpu != lab_o
    assert diff.mean() <= max_frac, diff.mean()
    if diff.any():
        assert (lab_gpu[diff] >= 0).all() and (lab_o[diff] >= 0).all()
        dg = _d2(img, C, lab_gpu, a)[diff]
        do = best[diff]
        assert np.all(np.abs(dg - do) <= 1e-5 * np.maximum(do, 1.0)), np.abs(dg - do).max()
        h, w = img.shape
        ys, xs = np.nonzero(diff)
        cg = C[lab_gpu[diff]]
        assert np.all(np.abs(xs - cg[:, 0]) <= a) and np.all(np.abs(ys - cg[:, 1]) <= a)
    return diff.mean()


def test_init_is_bit_exact(imgs):
    I, Ig = imgs
    C = sp.init(Ig, A, T0).cpu().numpy()
    for i in range(I.shape[0]):
        ref = oslic.init_centres(I[i].astype(np.float64), A, T0)
        assert np.array_equal(C[i].astype(np.float64), ref)


def test_one_assignment_matches_oracle(imgs):
    I, Ig = imgs
    # common centres: two oracle iterations from the grid, rounded to FP32
    Cs = []
    for i in range(I.shape[0]):
        img = I[i].astype(np.float64)
        C = oslic.init_centres(img, A, T0)
        for _ in range(2):
            C = oslic.update(img, oslic.assign(img, C, A)[0], C, TMIN)
        Cs.append(C.astype(np.float32))
    Cg = torch.from_numpy(np.stack(Cs)).cuda()
    lab = sp.assign(Ig, Cg, A).cpu().numpy()
    for i in range(I.shape[0]):
        _check_assignment(I[i].astype(np.float64), Cs[i].astype(np.float64), lab[i], A)


def test_one_update_matches_oracle(imgs):
    I, Ig = imgs
    C0 = sp.init(Ig, A, T0)
    lab = sp.assign(Ig, C0, A)
    C1 = sp.update(Ig, lab, C0.clone(), A, TMIN).cpu().numpy()
    labn, C0n = lab.cpu().numpy(), C0.cpu().numpy()
    for i in range(I.shape[0]):
        ref = oslic.update(I[i].astype(np.float64), labn[i], C0n[i].astype(np.float64), TMIN)
        assert np.allclose(C1[i][:, :2], ref[:, :2], rtol=0, atol=1e-4)
        assert np.allclose(C1[i][:, 2:], ref[:, 2:], rtol=1e-5, atol=1e-3)
        empty = np.array([not (labn[i] == k).any() for k in range(ref.shape[0])])
        assert np.array_equal(C1[i][empty], C0n[i][empty])


def test_full_slic_matches_oracle_and_is_valid(imgs):
    I, Ig = imgs
    lab, C = sp.slic(Ig, A, T0, TMIN, iters=10)
    lab, C = lab.cpu().numpy(), C.cpu().numpy()
    agree = []
    for i in range(I.shape[0]):
        img = I[i].astype(np.float64)
        lab_o, C_o = oslic.slic(img, A, T0, TMIN, iters=10)
        agree.append((lab[i] == lab_o).mean())
        _check_assignment(img, C[i].astype(np.float64), lab[i], A)
    assert min(agree) >= 0.99, agree


@pytest.mark.parametrize("gamma", [0, 3, 7])
def test_boxes_masks_and_samples_bit_exact(imgs, gamma):
    I, Ig = imgs
    lab, C = sp.slic(Ig, A, T0, TMIN, iters=4)
    B = sp.boxes(lab, C, A, gamma).cpu().numpy()
    tab = sp.patch_table(B)
    y, m = sp.pack(Ig, lab, gamma, tab)
    y, m, labn = y.cpu().numpy(), m.cpu().numpy(), lab.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(tab[:, 4].astype(np.int64) * tab[:, 5])])
    s = 0
    for i in range(I.shape[0]):
        ref = oslic.superpixel_patches(labn[i], gamma)
        ks = [k for k in range(C.shape[1]) if (labn[i] == k).any()]
        assert len(ref) == len(ks) == int((tab[:, 0] == i).sum())
        for k, (x0, y0, w, h, mk) in zip(ks, ref):
            assert tuple(tab[s]) == (i, k, x0, y0, w, h)
            seg = slice(off[s], off[s + 1])
            assert np.array_equal(m[seg].reshape(h, w).astype(bool), mk)
            assert np.array_equal(y[seg].reshape(h, w), I[i, y0:y0 + h, x0:x0 + w])
            s += 1
        empty = [k for k in range(C.shape[1]) if k not in ks]
        assert np.all(B[i, empty] == 0)


def test_step_larger_than_the_image():
    I = synth.slice_images(2, 9, 7, seed=5)
    Ig = torch.from_numpy(I).cuda()
    lab, C = sp.slic(Ig, 16, T0, TMIN, iters=3)
    assert C.shape[1] == 1 and bool((lab == 0).all())
    B = sp.boxes(lab, C, 16, 2).cpu().numpy()
    assert B.reshape(-1, 4).tolist() == [[0, 0, 7, 9], [0, 0, 7, 9]]


def test_constant_image_is_the_voronoi_of_the_grid_with_exact_ties():
    I = np.full((2, 30, 41), 300.0, np.float32)
    Ig = torch.from_numpy(I).cuda()
    C0 = sp.init(Ig, 8, T0)
    lab = sp.assign(Ig, C0, 8).cpu().numpy()
    for i in range(2):
        ref, _ = oslic.assign(I[i].astype(np.float64), C0[i].cpu().numpy().astype(np.float64), 8)
        assert np.array_equal(lab[i], ref)
    C1 = sp.update(Ig, torch.from_numpy(lab).cuda(), C0.clone(), 8, TMIN).cpu().numpy()
    assert np.all(C1[..., 3] == TMIN) and np.all(C1[..., 2] == 300.0)


def test_assignment_with_centres_far_from_their_cells(imgs):
    # centres scattered anywhere over the image (several cells from their
    # own): the gather widens its search by the largest such distance
    I, Ig = imgs
    rng = np.random.default_rng(17)
    K = sp.n_centres(61, 53, A)
    Cs = np.zeros((I.shape[0], K, 4), np.float32)
    Cs[..., 0] = rng.uniform(0, 52, (I.shape[0], K))
    Cs[..., 1] = rng.uniform(0, 60, (I.shape[0], K))
    Cs[..., 2] = rng.uniform(0, 1000, (I.shape[0], K))
    Cs[..., 3] = rng.uniform(5, 300, (I.shape[0], K))
    Cs[0, :3, :2] = [[52.0, 60.0], [0.0, 0.0], [26.5, 30.25]]
    lab = sp.assign(Ig, torch.from_numpy(Cs).cuda(), A).cpu().numpy()
    for i in range(I.shape[0]):
        _check_assignment(I[i].astype(np.float64), Cs[i].astype(np.float64), lab[i], A)


def test_centres_off_the_image_take_no_pixels(imgs):
    # centres at NaN, at +-1e30 and far outside the image: their windows miss
    # every pixel, so they take none and the update leaves them as they were;
    # the remaining centres assign as usual
    I, Ig = imgs
    C = sp.init(Ig, A, T0)
    bad = torch.tensor([[float("nan"), 3.0, 100.0, 40.0], [1e30, -1e30, 100.0, 40.0],
                        [-500.0, 700.0, 100.0, 40.0]], device="cuda")
    C[:, :3] = bad
    lab = sp.assign(Ig, C, A)
    ln = lab.cpu().numpy()
    assert not np.isin(ln, [0, 1, 2]).any()
    C2 = sp.update(Ig, lab, C.clone(), A, TMIN).cpu().numpy()
    Cn = C.cpu().numpy()
    assert np.array_equal(C2[:, :3], Cn[:, :3], equal_nan=True)
    Cg = Cn.astype(np.float64)
    for i in range(I.shape[0]):
        _check_assignment(I[i].astype(np.float64), np.where(np.isnan(Cg[i]), 1e9, Cg[i]), ln[i], A)
    B = sp.boxes(lab, C, A, 3).cpu().numpy()
    assert np.all(B[:, :3] == 0)
