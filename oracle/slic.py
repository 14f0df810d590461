"""SLIC superpixels and superpixel patches, FP64 numpy -- TEST INFRASTRUCTURE
ONLY (tests, the smoke check and the benchmark's CPU leg; the product never
imports it).

Paper Sec. II "Patch Extraction": instead of square patches, every slice is
cut into superpixels by simple linear iterative clustering with the distance
    D = sqrt(d_c^2 + (d_s / a)^2 t^2)
(d_c intensity, d_s spatial Euclidean distance, a the initial grid step, t a
compactness that adapts per superpixel), and each superpixel is dilated by
gamma pixels with a flat structuring element before it becomes a patch.

Readings (the paper gives the distance only):
  * centres start on the a x a grid, one per cell (K_x = ceil(w/a) by
    K_y = ceil(h/a) cells), at the cell's middle pixel position with the
    intensity of the nearest pixel and t = t0;
  * a pixel may join a centre whose 2a x 2a window covers it
    (|x - c_x| <= a and |y - c_y| <= a), the one of least D^2, ties to the
    lower index; a pixel no window covers gets no label (-1);
  * update: every centre becomes the mean (x, y, intensity) of its pixels
    (unchanged when it has none), and its t the largest intensity distance
    |I_p - I_centre| over its pixels at the new mean, at least t_min
    (the SLICO rule, read into the paper's form of D);
  * `iters` assignment + update rounds, then a final assignment;
  * no connectivity post-processing;
  * dilation by gamma pixels with a square (2 gamma + 1)^2 element (the 2D
    counterpart of the 26-neighbourhood the paper names); the patch is the
    dilated superpixel's bounding box in its slice, its samples the box's
    pixels, of which those outside the dilated superpixel are masked out.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np


def grid_shape(h: int, w: int, a: int) -> Tuple[int, int]:
    return (h + a - 1) // a, (w + a - 1) // a


def init_centres(img: np.ndarray, a: int, t0: float) -> np.ndarray:
    """[K][4] (x, y, intensity, t) for one h x w image, cells in row-major order."""
    h, w = img.shape
    ky, kx = grid_shape(h, w, a)
    C = np.zeros((ky * kx, 4))
    for j in range(ky):
        for i in range(kx):
            x = 0.5 * (i * a + min(w, (i + 1) * a) - 1)
            y = 0.5 * (j * a + min(h, (j + 1) * a) - 1)
            C[j * kx + i] = (x, y, img[int(math.floor(y + 0.5)), int(math.floor(x + 0.5))], t0)
    return C


def assign(img: np.ndarray, C: np.ndarray, a: int) -> Tuple[np.ndarray, np.ndarray]:
    """(labels [h][w] int, D^2 of the label or inf): every centre is tried
    against every pixel, with the window test."""
    h, w = img.shape
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    best = np.full((h, w), np.inf)
    lab = np.full((h, w), -1, dtype=np.int64)
    for k in range(C.shape[0]):
        cx, cy, ci, t = C[k]
        inwin = (np.abs(xs - cx) <= a) & (np.abs(ys - cy) <= a)
        d2 = (img - ci) ** 2 + ((xs - cx) ** 2 + (ys - cy) ** 2) / (a * a) * t * t
        take = inwin & (d2 < best)
        best = np.where(take, d2, best)
        lab = np.where(take, k, lab)
    return lab, best


def update(img: np.ndarray, lab: np.ndarray, C: np.ndarray, t_min: float) -> np.ndarray:
    h, w = img.shape
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    Cn = C.copy()
    for k in range(C.shape[0]):
        m = lab == k
        n = int(m.sum())
        if n == 0:
            continue
        mx, my, mi = xs[m].mean(), ys[m].mean(), img[m].mean()
        Cn[k, :3] = (mx, my, mi)
        Cn[k, 3] = max(float(np.abs(img[m] - mi).max()), t_min)
    return Cn


def slic(img: np.ndarray, a: int, t0: float, t_min: float, iters: int = 10):
    """(labels, centres) of one image."""
    img = np.asarray(img, np.float64)
    C = init_centres(img, a, t0)
    for _ in range(iters):
        lab, _ = assign(img, C, a)
        C = update(img, lab, C, t_min)
    lab, _ = assign(img, C, a)
    return lab, C


def dilate(mask: np.ndarray, gamma: int) -> np.ndarray:
    """Dilation by the square (2 gamma + 1)^2 element, written out as the
    union of shifted copies."""
    h, w = mask.shape
    out = np.zeros_like(mask, dtype=bool)
    for dy in range(-gamma, gamma + 1):
        for dx in range(-gamma, gamma + 1):
            ys0, ys1 = max(0, dy), min(h, h + dy)
            xs0, xs1 = max(0, dx), min(w, w + dx)
            out[ys0:ys1, xs0:xs1] |= mask[ys0 - dy:ys1 - dy, xs0 - dx:xs1 - dx]
    return out


def superpixel_patches(labels: np.ndarray, gamma: int) -> List[Tuple[int, int, int, int, np.ndarray]]:
    """(x0, y0, w, h, mask [h][w] bool) of every non-empty superpixel of one
    image, in label order."""
    out = []
    for k in range(int(labels.max()) + 1):
        m = labels == k
        if not m.any():
            continue
        d = dilate(m, gamma)
        yy, xx = np.nonzero(d)
        y0, y1, x0, x1 = yy.min(), yy.max(), xx.min(), xx.max()
        out.append((int(x0), int(y0), int(x1 - x0 + 1), int(y1 - y0 + 1),
                    d[y0:y1 + 1, x0:x1 + 1].copy()))
    return out
