"""Seeded synthetic inputs for patch-to-volume reconstruction (PVR).

This module only *synthesises inputs*: phantom volumes, acquisition geometry
(grids, stacks of slices, square patches), per-patch rigid motion draws and
corruption (noise, outlier patches).  It contains none of the method's own
arithmetic (PSF weights, simulation, back-projection, EM, update,
registration): the forward model lives in the HIP library and, separately,
in the FP64 oracle.  Both consume what this module produces.

Geometry conventions (shared input format, see the C header):
  * a volume grid is (nx, ny, nz) voxels with a 3x4 row-major affine
    ``vox2world`` mapping voxel index (i, j, k) to world millimetres;
    X is stored as X[(k*ny + j)*nx + i];
  * a stack is (nx, ny, nslices) pixels with a 3x4 affine ``pix2world``
    mapping (u, v, slice) to world mm; its three columns are mutually
    orthogonal (in-plane axes scaled by the pixel spacing, slice normal
    scaled by the slice spacing);
  * a square patch (size a, stride omega; paper Sec. II "Patch Extraction")
    is (stack, slice, x0, y0, w, h); its samples are packed patch-major and
    row-major inside the patch;
  * per-patch motion theta = (rx, ry, rz [rad], tx, ty, tz [mm]).

Random draws follow fixed seeds so that every consumer sees the same data.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


# ----------------------------------------------------------------------------
# descriptors
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    vox2world: np.ndarray  # (3, 4) float64

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Stack:
    nx: int
    ny: int
    nslices: int
    pix2world: np.ndarray  # (3, 4) float64, orthogonal columns
    fwhm_mm: np.ndarray    # (3,) PSF FWHM along in-plane x, in-plane y, normal
    problem: int = 0


@dataclasses.dataclass
class Patches:
    """Structure-of-arrays patch table (int32) plus sample offsets (int64)."""
    stack: np.ndarray
    slice: np.ndarray
    x0: np.ndarray
    y0: np.ndarray
    w: np.ndarray
    h: np.ndarray

    @property
    def M(self) -> int:
        return int(self.stack.shape[0])

    @property
    def sample_off(self) -> np.ndarray:
        n = (self.w.astype(np.int64) * self.h.astype(np.int64))
        off = np.zeros(self.M + 1, dtype=np.int64)
        np.cumsum(n, out=off[1:])
        return off

    @property
    def n_samples(self) -> int:
        return int(np.sum(self.w.astype(np.int64) * self.h.astype(np.int64)))

    def table(self) -> np.ndarray:
        """(M, 6) int32 rows (stack, slice, x0, y0, w, h)."""
        return np.stack([self.stack, self.slice, self.x0, self.y0, self.w,
                         self.h], axis=1).astype(np.int32)

    @staticmethod
    def concat(parts: Sequence["Patches"], stack_base: Sequence[int]) -> "Patches":
        f = lambda name, add: np.concatenate(
            [getattr(p, name) + (b if add else 0) for p, b in zip(parts, stack_base)]
        ).astype(np.int32)
        return Patches(f("stack", True), f("slice", False), f("x0", False),
                       f("y0", False), f("w", False), f("h", False))


@dataclasses.dataclass
class Problem:
    """One reconstruction: grid, stacks, patches, truth and observations."""
    name: str
    grid: Grid
    stacks: List[Stack]
    patches: Patches
    x_true: np.ndarray                 # (nz, ny, nx) float32
    theta_true: np.ndarray             # (M, 6) float64
    outlier_patch: np.ndarray          # (M,) bool
    seed_base: int
    noise_frac: float = 0.01
    outlier_frac: float = 0.0
    y_obs: Optional[np.ndarray] = None  # (N,) float32, filled by corrupt()

    @property
    def M(self) -> int:
        return self.patches.M

    @property
    def N(self) -> int:
        return self.patches.n_samples


# ----------------------------------------------------------------------------
# small geometry helpers used to *place* things (not the method)
# ----------------------------------------------------------------------------
def axis_rotation(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation matrix about a unit axis (Rodrigues' formula)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def euler_zyx_from_matrix(R: np.ndarray) -> np.ndarray:
    """Angles (rx, ry, rz) with R = Rz(rz) @ Ry(ry) @ Rx(rx)."""
    ry = math.asin(max(-1.0, min(1.0, -R[2, 0])))
    rx = math.atan2(R[2, 1], R[2, 2])
    rz = math.atan2(R[1, 0], R[0, 0])
    return np.array([rx, ry, rz])


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def iso_grid(n: int, spacing: float = 1.0) -> Grid:
    v2w = np.zeros((3, 4))
    v2w[0, 0] = v2w[1, 1] = v2w[2, 2] = spacing
    return Grid(n, n, n, v2w)


def grid_center(g: Grid) -> np.ndarray:
    c = np.array([(g.nx - 1) / 2, (g.ny - 1) / 2, (g.nz - 1) / 2, 1.0])
    return g.vox2world @ c


def make_stack(center: np.ndarray, e1, e2, n, nx: int, ny: int, ns: int,
               spacing=(1.0, 1.0), thickness: float = 1.0,
               fwhm=(1.0, 1.0, 1.0), problem: int = 0) -> Stack:
    """Stack of ns slices centred on ``center`` with unit axes e1, e2, n."""
    e1 = np.asarray(e1, float); e2 = np.asarray(e2, float); n = np.asarray(n, float)
    A = np.stack([e1 * spacing[0], e2 * spacing[1], n * thickness], axis=1)
    o = center - A @ np.array([(nx - 1) / 2, (ny - 1) / 2, (ns - 1) / 2])
    P = np.concatenate([A, o[:, None]], axis=1)
    return Stack(nx, ny, ns, P, np.asarray(fwhm, float), problem)


def orthogonal_frames(oblique_deg: Sequence[float] = ()):
    """(e1, e2, n) for axial, coronal, sagittal, then axial frames rotated
    about x by each requested oblique angle."""
    ex, ey, ez = np.eye(3)
    frames = [(ex, ey, ez), (ex, ez, -ey), (ey, ez, ex)]
    for deg in oblique_deg:
        R = axis_rotation(ex, math.radians(deg))
        frames.append((R @ ex, R @ ey, R @ ez))
    return frames


def square_patches(stacks: Sequence[Stack], a: int, stride: int,
                   stack_base: int = 0) -> Patches:
    """Overlapping a x a patches with stride omega on every slice (paper
    Sec. II "Patch Extraction").  A patch size larger than the slice is
    clamped to the slice; positions cover the slice from its first pixel."""
    cols = {k: [] for k in ("stack", "slice", "x0", "y0", "w", "h")}
    for si, st in enumerate(stacks):
        ax = min(a, st.nx); ay = min(a, st.ny)
        sx = max(1, min(stride, ax)); sy = max(1, min(stride, ay))
        xs = list(range(0, st.nx - ax + 1, sx))
        ys = list(range(0, st.ny - ay + 1, sy))
        for k in range(st.nslices):
            for y0 in ys:
                for x0 in xs:
                    cols["stack"].append(si + stack_base); cols["slice"].append(k)
                    cols["x0"].append(x0); cols["y0"].append(y0)
                    cols["w"].append(ax); cols["h"].append(ay)
    return Patches(*[np.asarray(cols[k], dtype=np.int32) for k in
                     ("stack", "slice", "x0", "y0", "w", "h")])


# ----------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------
def _paint_ellipsoid(vol: np.ndarray, center, semi, R, value) -> None:
    nz, ny, nx = vol.shape
    r = float(np.max(semi)) + 1.0
    lo = [max(0, int(math.floor(center[a] - r))) for a in range(3)]
    hi = [min(s, int(math.ceil(center[a] + r)) + 1)
          for a, s in zip(range(3), (nx, ny, nz))]
    if any(h <= l for l, h in zip(lo, hi)):
        return
    z, y, x = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]),
                          np.arange(lo[0], hi[0]), indexing="ij")
    d = np.stack([x - center[0], y - center[1], z - center[2]], axis=-1)
    loc = d @ R  # coordinates in the ellipsoid frame (columns of R = axes)
    q = ((loc / np.asarray(semi)) ** 2).sum(axis=-1)
    sub = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    sub[q <= 1.0] = value


def phantom_ellipsoids(n: int, seed: int, n_ell: int = 3,
                       values=(200.0, 600.0, 1000.0), semi_range=(4.0, 10.0),
                       blur_sigma: float = 1.0) -> np.ndarray:
    """Tiny phantom: ellipsoids with semi-axes U[semi_range] voxels, random
    orientation, centres in the inner 50 % of the cube, painted in order,
    then a Gaussian blur (sigma in voxels)."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    vol = np.zeros((n, n, n), dtype=np.float64)
    for e in range(n_ell):
        semi = rng.uniform(*semi_range, size=3)
        R = random_rotation(rng)
        c = rng.uniform(0.25 * (n - 1), 0.75 * (n - 1), size=3)
        _paint_ellipsoid(vol, c, semi, R, values[e % len(values)])
    if blur_sigma > 0:
        vol = gaussian_filter(vol, blur_sigma, mode="constant")
    return vol.astype(np.float32)


def _bspline_basis(t: np.ndarray) -> np.ndarray:
    """Uniform cubic B-spline weights for fractional t, shape (len(t), 4)."""
    t = np.asarray(t)
    return np.stack([(1 - t) ** 3 / 6,
                     (3 * t ** 3 - 6 * t ** 2 + 4) / 6,
                     (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6,
                     t ** 3 / 6], axis=-1)


def bspline_displacement(n: int, spacing_vox: float, max_amp: float,
                         seed: int) -> np.ndarray:
    """Smooth displacement field (3, n, n, n) in voxels: one cubic B-spline
    with control spacing ``spacing_vox`` and coefficients U[-1, 1], rescaled so
    that the largest displacement magnitude equals ``max_amp``."""
    rng = np.random.default_rng(seed)
    nc = int(math.ceil((n - 1) / spacing_vox)) + 4
    coef = rng.uniform(-1, 1, size=(3, nc, nc, nc))
    pos = np.arange(n) / spacing_vox
    i0 = np.floor(pos).astype(int)
    B = np.zeros((n, nc))
    w = _bspline_basis(pos - i0)
    for a in range(4):
        B[np.arange(n), i0 + a] += w[:, a]
    # separable tensor product: axes of coef are (comp, cz, cy, cx)
    u = np.einsum("zc,ncyx->nzyx", B, coef, optimize=True)
    u = np.einsum("yc,nzcx->nzyx", B, u, optimize=True)
    u = np.einsum("xc,nzyc->nzyx", B, u, optimize=True)
    mag = np.sqrt((u ** 2).sum(axis=0)).max()
    return (u * (max_amp / mag)).astype(np.float32)


def phantom_uterus(n: int, seed_phantom: int, seed_deform: int,
                   voxel_mm: float = 1.0, deform_spacing_mm: float = 20.0,
                   deform_amp_mm: float = 4.0) -> np.ndarray:
    """Whole-uterus-like phantom: a large ellipsoid (intensity 400) holding
    4-6 nested seeded ellipsoids (200 / 600 / 1000), lightly blurred, then
    warped by a smooth B-spline displacement (backward warp, trilinear)."""
    from scipy.ndimage import gaussian_filter, map_coordinates
    rng = np.random.default_rng(seed_phantom)
    vol = np.zeros((n, n, n), dtype=np.float32)
    scale = n / 256.0 / voxel_mm
    c0 = np.full(3, (n - 1) / 2)
    semi_u = np.array([110.0, 90.0, 80.0]) * scale
    Ru = axis_rotation(rng.normal(size=3), math.radians(rng.uniform(0, 20)))
    _paint_ellipsoid(vol, c0, semi_u, Ru, 400.0)
    k = int(rng.integers(4, 7))
    vals = [200.0, 600.0, 1000.0]
    for e in range(k):
        semi = rng.uniform(12, 40, size=3) * scale
        # centre inside the uterus, leaving room for the ellipsoid
        while True:
            d = rng.uniform(-1, 1, size=3)
            if (d ** 2).sum() <= 1:
                break
        c = c0 + Ru @ (d * np.maximum(semi_u - semi.max(), 0) * 0.8)
        _paint_ellipsoid(vol, c, semi, random_rotation(rng), vals[e % 3])
    vol = gaussian_filter(vol, 1.0, mode="constant").astype(np.float32)
    if deform_amp_mm > 0:
        u = bspline_displacement(n, deform_spacing_mm / voxel_mm,
                                 deform_amp_mm / voxel_mm, seed_deform)
        zz, yy, xx = np.meshgrid(np.arange(n, dtype=np.float32),
                                 np.arange(n, dtype=np.float32),
                                 np.arange(n, dtype=np.float32), indexing="ij")
        coords = np.stack([zz - u[2], yy - u[1], xx - u[0]])
        del zz, yy, xx, u
        vol = map_coordinates(vol, coords, order=1, mode="constant",
                              cval=0.0).astype(np.float32)
    return vol


# ----------------------------------------------------------------------------
# motion and corruption draws
# ----------------------------------------------------------------------------
def random_motion(M: int, max_rot_deg: float, max_trans: float,
                  seed: int) -> np.ndarray:
    """Per-patch rigid motion: rotation axis uniform on the sphere, angle
    U[0, max]; translation uniform in the ball of radius max (rejection).
    Returned as (rx, ry, rz [rad], tx, ty, tz) with R = Rz Ry Rx."""
    rng = np.random.default_rng(seed)
    th = np.zeros((M, 6))
    for s in range(M):
        ax = rng.normal(size=3)
        ang = math.radians(rng.uniform(0.0, max_rot_deg))
        th[s, :3] = euler_zyx_from_matrix(axis_rotation(ax, ang))
        while True:
            t = rng.uniform(-1, 1, size=3)
            if (t ** 2).sum() <= 1:
                break
        th[s, 3:] = t * max_trans
    return th


def random_motion_batch(M: int, max_rot_deg: float, max_trans: float,
                        seed: int) -> np.ndarray:
    """The distribution of random_motion, drawn for all patches at once (a
    different random stream; used for the learned initialiser's training
    pairs, where thousands of draws per second are needed)."""
    rng = np.random.default_rng(seed)
    ax = rng.normal(size=(M, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    ang = np.radians(rng.uniform(0.0, max_rot_deg, size=M))
    K = np.zeros((M, 3, 3))
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -ax[:, 2], ax[:, 1], -ax[:, 0]
    K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = ax[:, 2], -ax[:, 1], ax[:, 0]
    R = (np.eye(3)[None] + np.sin(ang)[:, None, None] * K
         + (1 - np.cos(ang))[:, None, None] * (K @ K))
    th = np.zeros((M, 6))
    th[:, 1] = np.arcsin(np.clip(-R[:, 2, 0], -1.0, 1.0))
    th[:, 0] = np.arctan2(R[:, 2, 1], R[:, 2, 2])
    th[:, 2] = np.arctan2(R[:, 1, 0], R[:, 0, 0])
    t = np.zeros((M, 3))
    todo = np.arange(M)
    while todo.size:
        c = rng.uniform(-1, 1, size=(todo.size, 3))
        ok = (c ** 2).sum(axis=1) <= 1
        t[todo[ok]] = c[ok]
        todo = todo[~ok]
    th[:, 3:] = t * max_trans
    return th


def choose_outliers(M: int, frac: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    k = int(round(frac * M))
    mask = np.zeros(M, dtype=bool)
    if k:
        mask[rng.choice(M, size=k, replace=False)] = True
    return mask


def corrupt(y_clean: np.ndarray, patches: Patches, outlier_patch: np.ndarray,
            noise_frac: float, seed_noise: int, seed_values: int) -> np.ndarray:
    """Gaussian noise with sigma = noise_frac * max clean sample, and outlier
    patches replaced by i.i.d. U[0, max clean sample] pixels."""
    y = np.asarray(y_clean, dtype=np.float64)
    ymax = float(np.max(y)) if y.size else 0.0
    rng_n = np.random.default_rng(seed_noise)
    out = y + rng_n.normal(scale=noise_frac * ymax, size=y.shape)
    rng_v = np.random.default_rng(seed_values)
    off = patches.sample_off
    for s in np.nonzero(outlier_patch)[0]:
        a, b = off[s], off[s + 1]
        out[a:b] = rng_v.uniform(0.0, ymax, size=b - a)
    return out.astype(np.float32)


# ----------------------------------------------------------------------------
# named workloads (the configurations the library is exercised on)
# ----------------------------------------------------------------------------
def tiny_problem(seed_cfg: int = 1) -> Problem:
    """32^3 phantom of 3 ellipsoids (200/600/1000), sigma-1 blur; 3 orthogonal
    stacks of 32x32x8 at slice thickness 4; PSF FWHM (1, 1, 4) voxels;
    16x16 patches stride 8 (M = 216, N = 55 296); motion <= 5 deg, <= 2 vox;
    1 % noise; 5 % outlier patches."""
    base = 1000 * seed_cfg
    n = 32
    g = iso_grid(n)
    x = phantom_ellipsoids(n, base + 0)
    c = grid_center(g)
    stacks = [make_stack(c, *fr, n, n, 8, (1, 1), 4.0, (1.0, 1.0, 4.0))
              for fr in orthogonal_frames()]
    P = square_patches(stacks, 16, 8)
    th = random_motion(P.M, 5.0, 2.0, base + 2)
    out = choose_outliers(P.M, 0.05, base + 4)
    return Problem("tiny32", g, stacks, P, x, th, out, base, 0.01, 0.05)


def full_problem(seed_cfg: int = 2, n: int = 256, slices: int = 60,
                 a: int = 64) -> Problem:
    """256^3 whole-uterus phantom at 1 mm with a B-spline warp; 4 stacks of
    256x256x60 at 1x1x4 mm (3 orthogonal + 1 oblique at 30 deg about x);
    PSF FWHM (1, 1, 4) mm; 64x64 patches stride 32 (M = 11 760);
    motion <= 10 deg, <= 5 mm; 1 % noise; 10 % outlier patches."""
    base = 1000 * seed_cfg
    g = iso_grid(n)
    x = phantom_uterus(n, base + 0, base + 1)
    c = grid_center(g)
    stacks = [make_stack(c, *fr, n, n, slices, (1, 1), 4.0, (1.0, 1.0, 4.0))
              for fr in orthogonal_frames([30.0])]
    P = square_patches(stacks, a, a // 2)
    th = random_motion(P.M, 10.0, 5.0, base + 2)
    out = choose_outliers(P.M, 0.10, base + 4)
    return Problem("uterus256", g, stacks, P, x, th, out, base, 0.01, 0.10)


def concat_patches(parts: Sequence[Patches]) -> Patches:
    return Patches(*[np.concatenate([getattr(p, k) for p in parts]).astype(np.int32)
                     for k in ("stack", "slice", "x0", "y0", "w", "h")])


def multiscale_problem(seed_cfg: int = 6, n: int = 96, slices: int = 24,
                       sizes=(32, 64)):
    """Multi-scale patches (paper Sec. II, eq. Y_i): the uterus phantom at n^3
    with 4 stacks of n x n x slices (3 orthogonal + 1 oblique), and square
    patches of every size a in `sizes` with stride a/2 on every slice, all in
    one table; returns (problem, scale index per patch).  Each patch has its
    own motion (<= 10 deg, <= 5 mm); 10 % outlier patches."""
    base = 1000 * seed_cfg
    g = iso_grid(n)
    x = phantom_uterus(n, base + 0, base + 1)
    c = grid_center(g)
    stacks = [make_stack(c, *fr, n, n, slices, (1, 1), 4.0, (1.0, 1.0, 4.0))
              for fr in orthogonal_frames([30.0])]
    parts = [square_patches(stacks, a, max(1, a // 2)) for a in sizes]
    P = concat_patches(parts)
    scale = np.concatenate([np.full(p.M, i, np.int32) for i, p in enumerate(parts)])
    th = random_motion(P.M, 10.0, 5.0, base + 2)
    out = choose_outliers(P.M, 0.10, base + 4)
    name = f"multiscale{n}_" + "_".join(str(a) for a in sizes)
    return Problem(name, g, stacks, P, x, th, out, base, 0.01, 0.10), scale


def diff_problem(seed_cfg: int = 4) -> Problem:
    """48^3 phantom; 3 orthogonal stacks of 48x48x12 (thickness 4);
    24x24 patches stride 12 (M = 324, N = 186 624)."""
    base = 1000 * seed_cfg
    n = 48
    g = iso_grid(n)
    x = phantom_ellipsoids(n, base + 0, semi_range=(6.0, 15.0))
    c = grid_center(g)
    stacks = [make_stack(c, *fr, n, n, 12, (1, 1), 4.0, (1.0, 1.0, 4.0))
              for fr in orthogonal_frames()]
    P = square_patches(stacks, 24, 12)
    th = random_motion(P.M, 5.0, 2.0, base + 2)
    out = np.zeros(P.M, dtype=bool)
    return Problem("diff48", g, stacks, P, x, th, out, base, 0.0, 0.0)


def batched_problems(seed_cfg: int = 3, count: int = 8,
                     n_range=(96, 192), sizes=(32, 64, 128)) -> List[Problem]:
    """Independent reconstructions: volume n^3 with n ~ U{n_range}; 3-6
    stacks (3 orthogonal + seeded obliques) of n x n x ceil(n/4) slices at
    thickness 4; patch size per stack ~ U{sizes} (clamped to the slice),
    stride a/2; motion <= 10 deg, <= 5 mm; 10 % outliers."""
    base = 1000 * seed_cfg
    rng = np.random.default_rng(base + 7)
    probs = []
    for b in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        ns = int(rng.integers(3, 7))
        obl = list(rng.uniform(15, 60, size=ns - 3))
        g = iso_grid(n)
        x = phantom_uterus(n, base + 100 * b, base + 100 * b + 1)
        c = grid_center(g)
        stacks = [make_stack(c, *fr, n, n, int(math.ceil(n / 4)), (1, 1), 4.0,
                             (1.0, 1.0, 4.0), problem=b)
                  for fr in orthogonal_frames(obl)]
        parts = []
        for si, st in enumerate(stacks):
            a = int(rng.choice(list(sizes)))
            parts.append(square_patches([st], a, a // 2, stack_base=si))
        P = Patches.concat(parts, [0] * len(parts))
        th = random_motion(P.M, 10.0, 5.0, base + 100 * b + 2)
        out = choose_outliers(P.M, 0.10, base + 100 * b + 4)
        probs.append(Problem(f"batch{b}_{n}", g, stacks, P, x, th, out,
                             base + 100 * b, 0.01, 0.10))
    return probs


def random_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0,
                 dtype=np.float32) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape).astype(dtype)


def residual_mixture(n: int, seed: int, sigma: float = 10.0, frac_in: float = 0.8,
                     lo: float = -500.0, hi: float = 500.0) -> np.ndarray:
    """Samples from frac_in * N(0, sigma^2) + (1 - frac_in) * U[lo, hi]."""
    rng = np.random.default_rng(seed)
    inl = rng.random(n) < frac_in
    e = np.where(inl, rng.normal(0.0, sigma, size=n), rng.uniform(lo, hi, size=n))
    return e


def slice_images(n_img: int, h: int, w: int, seed: int, n: int = 64,
                 noise: float = 0.01) -> np.ndarray:
    """float32 [n_img][h][w] test images for superpixel clustering: axial
    slices of a uterus phantom of n^3 voxels (evenly spaced through its middle
    half, cropped or zero-padded to h x w) plus Gaussian noise of `noise`
    times the phantom maximum."""
    V = phantom_uterus(n, seed, seed + 1)
    rng = np.random.default_rng(seed + 2)
    zs = np.linspace(n // 4, 3 * n // 4, n_img).astype(int)
    out = np.zeros((n_img, h, w), np.float32)
    hh, ww = min(h, n), min(w, n)
    out[:, :hh, :ww] = V[zs, :hh, :ww]
    out += rng.normal(0.0, noise * float(V.max()), out.shape).astype(np.float32)
    return out
