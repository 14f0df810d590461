"""FP64 CPU oracle for PVR (arXiv 1611.07289) -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never does, and the two share no code: the only common inputs are the arrays
produced by the seeded generator.

Layout:
  pvr_oracle.c   geometry, PSF, simulate, back-projection, NCC, registration
  em.py          voxel EM (E-step, outlier density, M-step), patch potentials
                 and the patch inlier/outlier mixture
  update.py      edge-preserving regulariser and the SR volume update
  recon.py       the SR iteration and the reconstruction cycle driver
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pvr_oracle.c")
_LIB = os.path.join(_HERE, "libpvr_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-D_GNU_SOURCE", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    """The oracle library: the in-tree build, or the file PVR_ORACLE_LIB names
    (a sanitizer build of the same source, in the tests)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PVR_ORACLE_LIB")
        if not path:
            path = build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.ora_ctx_create.restype = P
        L.ora_ctx_create.argtypes = [P, P, ctypes.c_int, P, P, P, ctypes.c_int,
                                     P, ctypes.c_double]
        L.ora_ctx_free.argtypes = [P]
        L.ora_n_samples.restype = i64
        L.ora_n_samples.argtypes = [P]
        L.ora_rotation.argtypes = [P, P]
        L.ora_simulate.argtypes = [P, P, P, P, P, i64, P, P, P, P]
        L.ora_sample_row.restype = ctypes.c_int
        L.ora_sample_row.argtypes = [P, P, i64, P, P, ctypes.c_int]
        L.ora_backproject.argtypes = [P, P, P, P, P, P]
        L.ora_backproject_voxels.argtypes = [P, P, P, P, P, i64, P, P]
        L.ora_support_backproject.argtypes = [P, P, P, P, P, P]
        L.ora_valid.argtypes = [P, P, P, P, P]
        L.ora_support_backproject_voxels.argtypes = [P, P, P, P, P, i64, P, P]
        L.ora_ncc.argtypes = [P, P, P, P, P, P]
        L.ora_register.argtypes = [P, P, P, P, P, P, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, P]
        L.ora_ncc_grad.argtypes = [P, P, P, P, P, P, P]
        L.ora_set_psf.argtypes = [P, ctypes.c_int]
        L.ora_sinc_taylor.restype = ctypes.c_double
        L.ora_sinc_taylor.argtypes = [ctypes.c_double]
        L.ora_ncc_patch.restype = ctypes.c_double
        L.ora_ncc_patch.argtypes = [P, ctypes.c_int, P, P, P, P]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_num_threads.argtypes = [ctypes.c_int]
        L.ora_set_num_threads.restype = None
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a) -> Optional[np.ndarray]:
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def rotation(th) -> np.ndarray:
    """R = Rz Ry Rx for (rx, ry, rz) in radians."""
    th = _f64(th)
    R = np.zeros(9)
    lib().ora_rotation(_p(th), _p(R))
    return R.reshape(3, 3)


def sinc_taylor(R: float) -> float:
    """sin(R)/R by the oracle's Taylor series (|R| <= pi)."""
    return float(lib().ora_sinc_taylor(float(R)))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    lib().ora_set_num_threads(int(n))


class Ctx:
    """One reconstruction problem (grid, stacks, patches, PSF cut-off k).

    ``grid`` needs nx, ny, nz, vox2world (3x4); each stack needs nx, ny,
    nslices, pix2world (3x4), fwhm_mm (3); ``patches`` needs table() ->
    (M, 6) int rows (stack, slice, x0, y0, w, h) with stack indices local to
    this problem."""

    PSF_KINDS = {"gaussian": 0, "sinc": 1}

    def __init__(self, grid, stacks, patches, k: float = 3.0,
                 stack_base: int = 0, psf: str = "gaussian"):
        self.dims = np.array([grid.nx, grid.ny, grid.nz], dtype=np.int32)
        self.v2w = _f64(grid.vox2world).reshape(12).copy()
        self.sdims = np.array([[s.nx, s.ny, s.nslices] for s in stacks],
                              dtype=np.int32).reshape(-1)
        self.p2w = _f64(np.stack([s.pix2world for s in stacks])).reshape(-1).copy()
        self.fwhm = _f64(np.stack([s.fwhm_mm for s in stacks])).reshape(-1).copy()
        tab = np.ascontiguousarray(patches.table(), dtype=np.int32).copy()
        tab[:, 0] -= stack_base
        self.pat = tab.reshape(-1).copy()
        self.M = tab.shape[0]
        self.k = float(k)
        self.V = int(grid.nx) * int(grid.ny) * int(grid.nz)
        self.shape = (int(grid.nz), int(grid.ny), int(grid.nx))
        n = tab[:, 4].astype(np.int64) * tab[:, 5]
        self.off = np.zeros(self.M + 1, dtype=np.int64)
        np.cumsum(n, out=self.off[1:])
        self._h = lib().ora_ctx_create(_p(self.dims), _p(self.v2w), len(stacks),
                                       _p(self.sdims), _p(self.p2w),
                                       _p(self.fwhm), self.M, _p(self.pat),
                                       self.k)
        self.N = int(lib().ora_n_samples(self._h))
        self.patch_of_sample = np.repeat(np.arange(self.M), n)
        if psf not in self.PSF_KINDS:
            raise ValueError(f"psf must be one of {sorted(self.PSF_KINDS)}, not {psf!r}")
        self.psf = psf
        lib().ora_set_psf(self._h, self.PSF_KINDS[psf])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:  # the module may be torn down at exit
            lib().ora_ctx_free(h)
            self._h = None

    # -- forward model ------------------------------------------------------
    def simulate(self, X, theta, mask=None, active=None, samples=None):
        """(y_hat, Z, valid) for all samples or the listed sample indices."""
        X = _f64(X).reshape(-1)
        th = _f64(theta).reshape(-1)
        lst = None if samples is None else np.ascontiguousarray(samples, np.int64)
        n = self.N if lst is None else lst.size
        yh = np.zeros(n); Z = np.zeros(n); val = np.zeros(n, np.uint8)
        m = _u8(mask); a = _u8(active)
        lib().ora_simulate(self._h, _p(X), _p(th), _p(m), _p(a),
                           0 if lst is None else lst.size, _p(lst), _p(yh),
                           _p(Z), _p(val))
        return yh, Z, val.astype(bool)

    def valid(self, theta, mask=None, active=None):
        """Validity of every sample (as simulate reports it), cheaply."""
        th = _f64(theta).reshape(-1)
        out = np.zeros(self.N, np.uint8)
        lib().ora_valid(self._h, _p(th), _p(_u8(mask)), _p(_u8(active)), _p(out))
        return out.astype(bool)

    def sample_row(self, theta, j: int, cap: int = 4096):
        th = _f64(theta).reshape(-1)
        idx = np.zeros(cap, np.int64); w = np.zeros(cap)
        n = lib().ora_sample_row(self._h, _p(th), int(j), _p(idx), _p(w), cap)
        if n < 0:
            raise RuntimeError("row capacity too small")
        return idx[:n].copy(), w[:n].copy()

    def backproject(self, theta, r, mask=None, active=None, support=False):
        """A^T r over the whole grid, shape (nz, ny, nx).  support=True
        replaces every weight psi_ji by 1/Z_j on the support."""
        th = _f64(theta).reshape(-1)
        r = _f64(r).reshape(-1)
        out = np.zeros(self.V)
        m = _u8(mask); a = _u8(active)
        f = lib().ora_support_backproject if support else lib().ora_backproject
        f(self._h, _p(th), _p(m), _p(a), _p(r), _p(out))
        return out.reshape(self.shape)

    def backproject_voxels(self, theta, r, voxels, mask=None, active=None, support=False):
        """(A^T r)_i for the listed flat voxel indices, one at a time
        (support=True: as in backproject)."""
        th = _f64(theta).reshape(-1)
        r = _f64(r).reshape(-1)
        vox = np.ascontiguousarray(voxels, np.int64)
        out = np.zeros(vox.size)
        m = _u8(mask); a = _u8(active)
        f = lib().ora_support_backproject_voxels if support else lib().ora_backproject_voxels
        f(self._h, _p(th), _p(m), _p(a), _p(r), vox.size, _p(vox), _p(out))
        return out

    # -- registration -----------------------------------------------------------
    def ncc(self, X, y, theta, mask=None):
        X = _f64(X).reshape(-1); y = _f64(y).reshape(-1)
        th = _f64(theta).reshape(-1)
        out = np.zeros(self.M)
        lib().ora_ncc(self._h, _p(X), _p(y), _p(th), _p(_u8(mask)), _p(out))
        return out

    def ncc_grad(self, X, y, theta, mask=None):
        """Per-patch NCC and its exact gradient with respect to the six
        motion parameters: (ncc (M,), grad (M, 6))."""
        if self.psf != "gaussian":
            raise NotImplementedError("the exact NCC gradient is written for the Gaussian PSF")
        X = _f64(X).reshape(-1); y = _f64(y).reshape(-1)
        th = _f64(theta).reshape(-1)
        out = np.zeros(self.M)
        g = np.zeros(6 * self.M)
        lib().ora_ncc_grad(self._h, _p(X), _p(y), _p(th), _p(_u8(mask)), _p(out), _p(g))
        return out, g.reshape(-1, 6)

    def register(self, X, y, theta, mask=None, reg=None, step0=1.0,
                 step_min=0.01, fd_h=0.05, max_iter=40, min_std=0.0,
                 gradient: str = "fd"):
        """Returns (theta_out (M, 6), ncc (M,)); theta is not modified.
        gradient: "fd" (central differences with step fd_h) or "analytic"."""
        if gradient not in ("fd", "analytic"):
            raise ValueError(f"gradient must be 'fd' or 'analytic', not {gradient!r}")
        if gradient == "analytic" and self.psf != "gaussian":
            raise NotImplementedError("the exact NCC gradient is written for the Gaussian PSF")
        X = _f64(X).reshape(-1); y = _f64(y).reshape(-1)
        th = _f64(theta).reshape(-1).copy()
        out = np.zeros(self.M)
        lib().ora_register(self._h, _p(X), _p(y), _p(th), _p(_u8(mask)),
                           _p(_u8(reg)), float(step0), float(step_min),
                           float(fd_h), int(max_iter), float(min_std),
                           1 if gradient == "analytic" else 0, _p(out))
        return th.reshape(-1, 6), out
