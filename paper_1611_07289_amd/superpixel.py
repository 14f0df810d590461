"""Superpixel patches (paper Sec. II, "Patch Extraction"): every observed
slice is clustered by SLIC with the paper's adaptive-compactness distance, and
each superpixel, dilated by gamma pixels, becomes one patch.  A patch is the
dilated superpixel's bounding box in its slice; the box's pixels outside the
dilated superpixel are switched off through the plan's sample mask, so they
are neither simulated, registered against nor reintegrated.

Every step runs in libpvr.so (pvr_slic*, include/pvr_slic.h); this module
marshals arguments and turns the boxes into the plan's patch table.
"""
from __future__ import annotations

import numpy as np

from . import pvr


def n_centres(h: int, w: int, a: int) -> int:
    return int(pvr.load().pvr_slic_centres(int(h), int(w), int(a)))


def _img(img):
    import torch
    if img.dtype != torch.float32 or not img.is_cuda or img.dim() != 3:
        raise ValueError("images must be a float32 CUDA tensor [n_img][h][w]")
    return img.contiguous()


def init(img, a: int, t0: float):
    import torch
    img = _img(img)
    n, h, w = img.shape
    C = torch.empty(n, n_centres(h, w, a), 4, dtype=torch.float32, device=img.device)
    pvr._check(pvr.load().pvr_slic_init(img.data_ptr(), n, h, w, int(a), float(t0),
                                        C.data_ptr(), pvr._stream()))
    return C


def assign(img, C, a: int, scratch=None):
    import torch
    img = _img(img)
    n, h, w = img.shape
    lab = torch.empty(n, h, w, dtype=torch.int32, device=img.device)
    if scratch is None:
        scratch = torch.empty(n, dtype=torch.int64, device=img.device)
    pvr._check(pvr.load().pvr_slic_assign(img.data_ptr(), n, h, w, int(a), C.data_ptr(),
                                          scratch.data_ptr(), lab.data_ptr(), pvr._stream()))
    return lab


def update(img, lab, C, a: int, t_min: float):
    """In place on C."""
    img = _img(img)
    n, h, w = img.shape
    pvr._check(pvr.load().pvr_slic_update(img.data_ptr(), n, h, w, int(a), lab.data_ptr(),
                                          float(t_min), C.data_ptr(), pvr._stream()))
    return C


def slic(img, a: int, t0: float, t_min: float, iters: int = 10):
    """(labels int32 [n][h][w], centres float32 [n][K][4])."""
    import torch
    img = _img(img)
    n, h, w = img.shape
    C = torch.empty(n, n_centres(h, w, a), 4, dtype=torch.float32, device=img.device)
    lab = torch.empty(n, h, w, dtype=torch.int32, device=img.device)
    scratch = torch.empty(n, dtype=torch.int64, device=img.device)
    pvr._check(pvr.load().pvr_slic(img.data_ptr(), n, h, w, int(a), float(t0), float(t_min),
                                   int(iters), scratch.data_ptr(), C.data_ptr(), lab.data_ptr(),
                                   pvr._stream()))
    return lab, C


def boxes(lab, C, a: int, gamma: int):
    """int32 [n][K][4] (x0, y0, w, h) of the dilated superpixels (device)."""
    import torch
    n, h, w = lab.shape
    B = torch.empty(n, C.shape[1], 4, dtype=torch.int32, device=lab.device)
    pvr._check(pvr.load().pvr_slic_boxes(lab.data_ptr(), n, h, w, int(a), C.data_ptr(),
                                         int(gamma), B.data_ptr(), pvr._stream()))
    return B


def pack(img, lab, gamma: int, table: np.ndarray, noalloc: bool = False):
    """(y float32 [N], mask uint8 [N]) of the patches table int32 [M][6] =
    (image, label, x0, y0, w, h), patch after patch, row-major inside each.
    noalloc: use pvr_slic_pack_noalloc (no workspace; at most
    PVR_SLIC_PACK_NOALLOC_MAX patches)."""
    import torch
    img = _img(img)
    n, h, w = img.shape
    tab = np.ascontiguousarray(table, dtype=np.int32)
    N = int((tab[:, 4].astype(np.int64) * tab[:, 5]).sum())
    y = torch.empty(max(N, 1), dtype=torch.float32, device=img.device)
    m = torch.empty(max(N, 1), dtype=torch.uint8, device=img.device)
    L = pvr.load()
    if noalloc:
        pvr._check(L.pvr_slic_pack_noalloc(img.data_ptr(), lab.data_ptr(), n, h, w, int(gamma),
                                           tab.shape[0], tab.ctypes.data, y.data_ptr(),
                                           m.data_ptr(), pvr._stream()))
        return y[:N], m[:N]
    nbytes = int(L.pvr_slic_pack_workspace(tab.shape[0]))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=img.device)
    pvr._check(L.pvr_slic_pack(img.data_ptr(), lab.data_ptr(), n, h, w, int(gamma),
                               tab.shape[0], tab.ctypes.data, ws.data_ptr(), nbytes,
                               y.data_ptr(), m.data_ptr(), pvr._stream()))
    return y[:N], m[:N]


def patch_table(B: np.ndarray) -> np.ndarray:
    """Pack table int32 [M][6] = (image, label, x0, y0, w, h) of the
    non-empty superpixels, image by image in label order."""
    B = np.asarray(B).reshape(B.shape[0], -1, 4)
    im, k = np.nonzero(B[:, :, 2] > 0)
    bx = B[im, k]
    return np.column_stack([im, k, bx]).astype(np.int32)


def superpixel_patches(img, a: int, gamma: int, t0: float, t_min: float, iters: int,
                       image_stack_slice: np.ndarray):
    """SLIC, dilation and packing of n observed slices img [n][h][w].
    image_stack_slice int [n][2]: the (stack, slice) of every image.
    Returns (patch columns dict for synth.Patches, y [N], mask [N], pack
    table [M][6], labels, centres)."""
    lab, C = slic(img, a, t0, t_min, iters)
    B = boxes(lab, C, a, gamma).cpu().numpy()
    tab = patch_table(B)
    y, m = pack(img, lab, gamma, tab)
    iss = np.asarray(image_stack_slice, np.int32).reshape(-1, 2)
    cols = {"stack": iss[tab[:, 0], 0], "slice": iss[tab[:, 0], 1], "x0": tab[:, 2],
            "y0": tab[:, 3], "w": tab[:, 4], "h": tab[:, 5]}
    return cols, y, m, tab, lab, C


def main():
    """Times the superpixel patch extraction (SLIC, boxes, packing) on seeded
    synthetic slices of the benchmark's shape: python -m
    paper_1611_07289_amd.superpixel [--repeat R] [--a A] [--gamma G]."""
    import argparse
    import json
    import sys
    import time

    import torch

    from . import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--slices", type=int, default=240)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--a", type=int, default=32)
    ap.add_argument("--gamma", type=int, default=19)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--repeat", type=int, default=5)
    args = ap.parse_args()
    n = args.size
    img = torch.from_numpy(synth.slice_images(args.slices, n, n, seed=977, n=n)).cuda()
    iss = np.stack([np.zeros(args.slices), np.arange(args.slices)], 1).astype(np.int32)
    superpixel_patches(img, args.a, args.gamma, 40.0, 5.0, args.iters, iss)  # warm-up
    ms = []
    for _ in range(args.repeat):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cols, y, m, tab, lab, C = superpixel_patches(img, args.a, args.gamma, 40.0, 5.0,
                                                     args.iters, iss)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        print(f"[superpixel] extraction {ms[-1]:.2f} ms", file=sys.stderr, flush=True)
    print(json.dumps({"slices": args.slices, "size": n, "a": args.a, "gamma": args.gamma,
                      "iters": args.iters, "patches": int(tab.shape[0]), "samples": int(y.numel()),
                      "samples_in_patches": int(m.sum()), "ms": ms, "ms_median": float(np.median(ms))}))


if __name__ == "__main__":
    main()
