"""The plan's caller-owned workspace, on the host (no GPU): plan creation
makes no HIP call, the workspace size follows the flags, and the capacity of
the adjoint's brick -> patch index, bounded at creation, holds for any
motion.

The index lists a brick (8^3 voxels) or sub-brick (4^3) for a patch when the
brick's voxel-centre box meets each of the three slabs of the patch's
pixel-frame PSF support box (a separating-axis test on the patch's axes).
Here that test is evaluated by brute force over every brick of the grid for
many random rigid motions (any rotation, translations up to 20 mm) with the
larger in-plane reach of the two PSFs, and the largest count is compared
with the capacity the library reserved for a one-patch plan."""
import ctypes
import math

import numpy as np

from paper_1611_07289_amd import pvr, synth


def _create(grid, stacks, patches, k=3.0):
    L = pvr.load()
    g, s, p = pvr.make_descriptors([grid], [stacks], [patches])
    h = ctypes.c_void_p()
    st = L.pvr_plan_create(ctypes.addressof(g), len(g), ctypes.addressof(s), len(s),
                           ctypes.addressof(p), len(p), k, ctypes.byref(h))
    assert st == 0, L.pvr_last_error().decode()
    return h


def _info(h):
    out = pvr.PlanSizes()
    assert pvr.load().pvr_plan_info(h, ctypes.byref(out)) == 0
    return out


def _ws(h, flags):
    n = ctypes.c_size_t()
    st = pvr.load().pvr_plan_workspace_size(h, flags, ctypes.byref(n))
    return st, int(n.value)


def test_create_is_host_only_and_sizes_the_workspace():
    P = synth.tiny_problem()
    L = pvr.load()
    h = _create(P.grid, P.stacks, P.patches)
    try:
        info = _info(h)
        assert info.device_bytes == 0 and info.n_bin_pairs == 0
        assert info.bin_capacity > 0 and info.sub_capacity > 0
        st, plain = _ws(h, 0)
        assert st == 0
        st, wide = _ws(h, pvr.PVR_WS_F64)
        assert st == 0
        N = P.patches.n_samples
        # FP64 normalisers (8 B) and adjoint inputs (16 B) per sample
        assert 24 * N <= wide - plain <= 24 * N + 1024
        # the per-sample arrays alone: 1/Z (4), mask (1), adjoint inputs (8)
        assert plain >= 13 * N + 4 * (info.sub_capacity + info.bin_capacity)
        assert _ws(h, 2)[0] == pvr.PVR_EINVAL
        # nothing runs without a workspace
        theta = np.zeros((P.M, 6), np.float32)
        assert L.pvr_plan_build(h, theta.ctypes.data, None, None, None) == pvr.PVR_EINVAL
        assert "workspace" in L.pvr_last_error().decode()
        assert L.pvr_plan_inv_z(h) is None
    finally:
        L.pvr_plan_destroy(h)


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _listed(grid, stack, row, R, t, e, k=3.0):
    """Bricks of edge e whose voxel-centre box meets the three support slabs
    of the patch `row` = (stack, slice, x0, y0, w, h) moved by (R, t) about
    its centre."""
    V, tv = grid.vox2world[:, :3], grid.vox2world[:, 3]
    A, a = stack.pix2world[:, :3], stack.pix2world[:, 3]
    _, sl, x0, y0, w, h = [int(v) for v in row]
    sp = np.linalg.norm(A, axis=0)
    sig = np.asarray(stack.fwhm_mm, float) / (2 * math.sqrt(2 * math.log(2)))
    reach = [max(k * sig[0], stack.fwhm_mm[0]) / sp[0], max(k * sig[1], stack.fwhm_mm[1]) / sp[1],
             k * sig[2] / sp[2]]
    lo_s = np.array([x0 - reach[0], y0 - reach[1], sl - reach[2]])
    hi_s = np.array([x0 + w - 1 + reach[0], y0 + h - 1 + reach[1], sl + reach[2]])
    c = A @ np.array([x0 + (w - 1) / 2, y0 + (h - 1) / 2, sl]) + a
    # voxel -> unmoved pixel coordinates: A^-1 (R^T (V v + tv - c - t) + c - a)
    Ai = np.linalg.inv(A)
    Gl = Ai @ R.T @ V
    go = Ai @ (R.T @ (tv - c - t) + c - a)
    nb = [(grid.nx + 7) // 8 * (8 // e), (grid.ny + 7) // 8 * (8 // e),
          (grid.nz + 7) // 8 * (8 // e)]
    ii = np.stack(np.meshgrid(*[np.arange(n) * e for n in nb], indexing="ij"), -1).reshape(-1, 3)
    lo = ii @ Gl.T + go
    span = np.abs(Gl) @ np.full(3, e - 1.0)
    mn = lo + np.minimum(Gl * (e - 1), 0).sum(1)
    mx = mn + span
    ok = np.all((mx >= lo_s) & (mn <= hi_s), axis=1)
    return int(ok.sum())


def _check_case(grid, stack, row, n_motion, seed):
    patches = synth.Patches(*[np.array([v], np.int32) for v in row])
    patches.stack[:] = 0
    h = _create(grid, [stack], patches)
    try:
        info = _info(h)
    finally:
        pvr.load().pvr_plan_destroy(h)
    rng = np.random.default_rng(seed)
    most_b = most_s = 0
    for _ in range(n_motion):
        R = _rotation(rng)
        t = rng.uniform(-20, 20, 3)
        most_b = max(most_b, _listed(grid, stack, row, R, t, 8))
        most_s = max(most_s, _listed(grid, stack, row, R, t, 4))
    print(f"bricks: most listed {most_b}, capacity {info.bin_capacity}; "
          f"sub-bricks: most listed {most_s}, capacity {info.sub_capacity}")
    assert 0 < most_b <= info.bin_capacity
    assert 0 < most_s <= info.sub_capacity
    # and the bound is not vacuous: within a small factor of what is reached
    assert info.sub_capacity <= 12 * most_s
    return most_b, most_s


def test_index_capacity_bounds_every_motion_tiny():
    P = synth.tiny_problem()
    tab = P.patches.table()
    for s in range(3):  # one patch from each orthogonal stack
        row = tab[np.nonzero(tab[:, 0] == s)[0][len(tab) // 6]]
        _check_case(P.grid, P.stacks[s], row, 150, 10 + s)


def test_index_capacity_bounds_every_motion_uterus_patch():
    # a 64 x 64 patch of the oblique stack of a 96^3 grid with the uterus
    # workload's stack geometry (1 x 1 x 4 mm, FWHM 1, 1, 4 mm)
    g = synth.iso_grid(96)
    c = synth.grid_center(g)
    st = [synth.make_stack(c, *fr, 96, 96, 24, (1, 1), 4.0, (1.0, 1.0, 4.0))
          for fr in synth.orthogonal_frames([30.0])][3]
    _check_case(g, st, np.array([0, 12, 16, 16, 64, 64], np.int32), 60, 3)


def test_index_capacity_bounds_every_motion_anisotropic_grid():
    # sheared, anisotropic voxels (1 x 1.5 x 2 mm with a skew) and a
    # rectangular patch of a thin-slice stack
    g = synth.Grid(40, 36, 30, np.array([[1.0, 0.2, 0.0, -3.0],
                                         [0.0, 1.5, 0.1, 2.0],
                                         [0.0, 0.0, 2.0, 1.0]]))
    c = synth.grid_center(g)
    e1 = np.array([1.0, 1.0, 0.0]) / math.sqrt(2)
    e2 = np.array([-1.0, 1.0, 1.0]) / math.sqrt(3)
    n = np.cross(e1, e2)
    st = synth.make_stack(c, e1, e2, n, 48, 40, 10, (0.8, 0.9), 2.5, (1.2, 0.9, 2.5))
    _check_case(g, st, np.array([0, 4, 3, 5, 30, 18], np.int32), 80, 7)
