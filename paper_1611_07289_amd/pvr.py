"""ctypes binding of libpvr.so (the HIP library declared in include/pvr.h).

Argument marshalling only: every step runs in the library's kernels.  PyTorch
supplies device memory (``tensor.data_ptr()``) and the current HIP stream.
The library must be built (``python -m paper_1611_07289_amd.build``); a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpvr.so")

PVR_OK, PVR_EINVAL, PVR_ESHAPE, PVR_ENOMEM, PVR_EHIP, PVR_ENUMERIC, PVR_EUNSUPPORTED = range(7)
PVR_KERNEL_SIMULATE = 0
PVR_KERNEL_BACKPROJECT = 1
PVR_KERNEL_REGISTER = 2
PVR_EM_INIT = 1
PVR_EM_FIX_W = 2
PVR_EM_RESID_FRESH = 4
PVR_EM_PREP_ADJOINT = 8
PVR_REG_GRAD_FD = 0
PVR_REG_GRAD_EXACT = 1
PVR_PSF_GAUSSIAN = 0
PVR_PSF_SINC = 1
PVR_WS_F64 = 1
PVR_SLIC_PACK_NOALLOC_MAX = 65536

_STATUS = {0: "PVR_OK", 1: "PVR_EINVAL", 2: "PVR_ESHAPE", 3: "PVR_ENOMEM",
           4: "PVR_EHIP", 5: "PVR_ENUMERIC", 6: "PVR_EUNSUPPORTED"}


class PvrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("vox2world", ctypes.c_double * 12)]


class Stack(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nslices", ctypes.c_int32), ("pix2world", ctypes.c_double * 12),
                ("fwhm_mm", ctypes.c_double * 3)]


class Patch(ctypes.Structure):
    _fields_ = [("stack", ctypes.c_int32), ("slice", ctypes.c_int32), ("x0", ctypes.c_int32),
                ("y0", ctypes.c_int32), ("w", ctypes.c_int32), ("h", ctypes.c_int32)]


class PlanSizes(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_voxels", ctypes.c_int64),
                ("n_patches", ctypes.c_int32), ("n_problems", ctypes.c_int32),
                ("n_stacks", ctypes.c_int32), ("n_bricks", ctypes.c_int32),
                ("n_bin_pairs", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("bin_capacity", ctypes.c_int64), ("sub_capacity", ctypes.c_int64)]


class EMState(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_double), ("c", ctypes.c_double), ("m", ctypes.c_double),
                ("y_abs_max", ctypes.c_double), ("sum_wp", ctypes.c_double),
                ("sum_wpe2", ctypes.c_double), ("sum_w", ctypes.c_double),
                ("n_used", ctypes.c_int32), ("n_excluded", ctypes.c_int32),
                ("started", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class SRParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("lambda_", ctypes.c_float), ("delta", ctypes.c_float),
                ("clamp_min", ctypes.c_float), ("den_eps", ctypes.c_float),
                ("use_clamp", ctypes.c_int32)]

    @staticmethod
    def make(alpha=1.0, lam=0.02, delta=150.0, clamp_min=0.0, den_eps=1e-6, use_clamp=True):
        return SRParams(alpha, lam, delta, clamp_min, den_eps, 1 if use_clamp else 0)


class RegParams(ctypes.Structure):
    _fields_ = [("step0", ctypes.c_double), ("step_min", ctypes.c_double),
                ("fd_h", ctypes.c_double), ("min_std", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("gradient", ctypes.c_int32)]

    @staticmethod
    def make(step0=1.0, step_min=0.01, fd_h=0.05, min_std=0.0, max_iter=40, exact=False):
        """exact: the exact NCC gradient instead of central differences."""
        return RegParams(step0, step_min, fd_h, min_std, max_iter,
                         PVR_REG_GRAD_EXACT if exact else PVR_REG_GRAD_FD)


EXPORTS = ["pvr_last_error", "pvr_version", "pvr_plan_create", "pvr_plan_destroy",
           "pvr_plan_workspace_size", "pvr_plan_attach", "pvr_plan_reg_stats",
           "pvr_plan_set_granules",
           "pvr_motion_frame", "pvr_motion_step",
           "pvr_motion_accept", "pvr_motion_init_step", "pvr_motion_fallback", "pvr_motion_live",
           "pvr_plan_info", "pvr_plan_offsets", "pvr_plan_build", "pvr_plan_build_f64",
           "pvr_plan_inv_z", "pvr_simulate", "pvr_simulate_f64", "pvr_backproject",
           "pvr_backproject_f64", "pvr_robust_weights", "pvr_sr_update",
           "pvr_register_patches", "pvr_simulate_grad_theta", "pvr_simulate_grad_theta_f64",
           "pvr_ncc_grad", "pvr_plan_set_tiles", "pvr_plan_set_timing", "pvr_plan_kernel_time",
           "pvr_plan_set_psf",
           "pvr_cnn_conv_fwd", "pvr_cnn_conv_dgrad",
           "pvr_cnn_wgrad_scratch", "pvr_cnn_conv_wgrad", "pvr_cnn_pack_pairs",
           "pvr_cnn_head_scratch", "pvr_cnn_head", "pvr_cnn_adam",
           "pvr_slic_centres", "pvr_slic_init", "pvr_slic_assign", "pvr_slic_update", "pvr_slic",
           "pvr_slic_boxes", "pvr_slic_pack", "pvr_slic_pack_workspace", "pvr_slic_pack_noalloc",
           "pvr_check", "pvr_set_debug", "pvr_get_debug", "pvr_sr_graph_create",
           "pvr_sr_graph_launch", "pvr_sr_graph_destroy"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpvr.so and declare its signatures (no GPU call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpvr.so not built at {path}; run "
                           "python -m paper_1611_07289_amd.build")
    L = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.pvr_last_error.restype = ctypes.c_char_p
    L.pvr_version.restype = ctypes.c_char_p
    L.pvr_plan_create.argtypes = [P, i32, P, i32, P, i32, ctypes.c_double, P]
    L.pvr_plan_destroy.argtypes = [P]
    L.pvr_plan_destroy.restype = None
    L.pvr_plan_info.argtypes = [P, P]
    L.pvr_plan_workspace_size.argtypes = [P, i32, P]
    L.pvr_plan_attach.argtypes = [P, P, ctypes.c_size_t, i32, P]
    L.pvr_plan_reg_stats.argtypes = [P, P, P]
    L.pvr_plan_set_granules.argtypes = [P, i32, i32]
    f32_ = ctypes.c_float
    L.pvr_motion_frame.argtypes = [P, P, i32, P, P, P]
    L.pvr_motion_step.argtypes = [P, P, P, P, f32_, P, P]
    L.pvr_motion_accept.argtypes = [P, P, P, P, P, P, f32_, f32_, P, P]
    L.pvr_motion_init_step.argtypes = [P, P, f32_, ctypes.c_double, P, P]
    L.pvr_motion_fallback.argtypes = [P, P, f32_, P, P, P, P, P, P, P]
    L.pvr_motion_live.argtypes = [P, P, f32_, P, P, P]
    L.pvr_plan_offsets.argtypes = [P, P, P]
    L.pvr_plan_build.argtypes = [P, P, P, P, P]
    L.pvr_plan_build_f64.argtypes = [P, P, P, P, P]
    L.pvr_plan_inv_z.argtypes = [P]
    L.pvr_plan_inv_z.restype = P
    L.pvr_simulate.argtypes = [P, P, P, P, P, P]
    L.pvr_simulate_f64.argtypes = [P, P, P, P, P, P]
    L.pvr_backproject.argtypes = [P, P, P, P, P, P, P]
    L.pvr_backproject_f64.argtypes = [P, P, P, P, P, P, P]
    L.pvr_robust_weights.argtypes = [P, P, P, P, P, P, P, i32, P]
    L.pvr_sr_update.argtypes = [P, P, P, P, P, P, P]
    L.pvr_register_patches.argtypes = [P, P, P, P, P, P, P, P]
    L.pvr_simulate_grad_theta.argtypes = [P, P, P, P, P]
    L.pvr_simulate_grad_theta_f64.argtypes = [P, P, P, P, P]
    L.pvr_ncc_grad.argtypes = [P, P, P, P, P, P]
    L.pvr_plan_set_tiles.argtypes = [P, i32, i32, P]
    L.pvr_plan_set_psf.argtypes = [P, i32]
    L.pvr_plan_set_timing.argtypes = [P, i32]
    L.pvr_plan_kernel_time.argtypes = [P, i32, P, P]
    L.pvr_cnn_conv_fwd.argtypes = [P, P, P, P, i32, i32, i32, i32, i32, i32, i32, P]
    L.pvr_cnn_conv_dgrad.argtypes = [P, P, P, P, i32, i32, i32, i32, i32, i32, P]
    L.pvr_cnn_wgrad_scratch.argtypes = [i32, i32, i32, i32, i32, i32]
    L.pvr_cnn_wgrad_scratch.restype = i64
    L.pvr_cnn_conv_wgrad.argtypes = [P, P, P, P, P, P, i32, i32, i32, i32, i32, i32, P]
    L.pvr_cnn_pack_pairs.argtypes = [P, P, i32, P, P, P, P]
    L.pvr_cnn_head_scratch.argtypes = [i32]
    L.pvr_cnn_head_scratch.restype = i64
    L.pvr_cnn_head.argtypes = [P, i32, i32, P, P, P, P, P, P, P, P, P, P, P]
    L.pvr_cnn_adam.argtypes = [P, P, P, P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, i32, P, P, i32, i32, P]
    f32 = ctypes.c_float
    L.pvr_slic_centres.argtypes = [i32, i32, i32]
    L.pvr_slic_centres.restype = i64
    L.pvr_slic_init.argtypes = [P, i32, i32, i32, i32, f32, P, P]
    L.pvr_slic_assign.argtypes = [P, i32, i32, i32, i32, P, P, P, P]
    L.pvr_slic_update.argtypes = [P, i32, i32, i32, i32, P, f32, P, P]
    L.pvr_slic.argtypes = [P, i32, i32, i32, i32, f32, f32, i32, P, P, P, P]
    L.pvr_slic_boxes.argtypes = [P, i32, i32, i32, i32, P, i32, P, P]
    L.pvr_slic_pack.argtypes = [P, P, i32, i32, i32, i32, i32, P, P, ctypes.c_size_t, P, P, P]
    L.pvr_slic_pack_noalloc.argtypes = [P, P, i32, i32, i32, i32, i32, P, P, P, P]
    L.pvr_slic_pack_workspace.argtypes = [i32]
    L.pvr_slic_pack_workspace.restype = ctypes.c_size_t
    L.pvr_check.argtypes = [P, P]
    L.pvr_set_debug.argtypes = [i32]
    L.pvr_get_debug.argtypes = []
    L.pvr_get_debug.restype = i32
    L.pvr_sr_graph_create.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, i32, P, P]
    L.pvr_sr_graph_launch.argtypes = [P, P]
    L.pvr_sr_graph_destroy.argtypes = [P]
    L.pvr_sr_graph_destroy.restype = None
    for name in EXPORTS:
        if name not in ("pvr_last_error", "pvr_version", "pvr_plan_destroy", "pvr_plan_inv_z",
                        "pvr_cnn_wgrad_scratch", "pvr_cnn_head_scratch", "pvr_slic_centres",
                        "pvr_sr_graph_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def set_debug(on: bool = True):
    """Switch the library's debug mode (pvr_set_debug): the core calls then
    check their input arrays on the device and reject the first non-finite
    value (or negative patch weight) with PvrError(PVR_EINVAL)."""
    _check(load().pvr_set_debug(1 if on else 0))


def get_debug() -> bool:
    return bool(load().pvr_get_debug())


def _check(st: int):
    if st != 0:
        raise PvrError(st, load().pvr_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def make_descriptors(grids: Sequence, stacks_per_problem: Sequence[Sequence],
                     patches_per_problem: Sequence):
    """ctypes arrays from generator descriptors (one list of stacks and one
    patch table per problem; patch stack indices local to their problem)."""
    P = len(grids)
    g_arr = (Grid * P)()
    for b, g in enumerate(grids):
        g_arr[b].nx, g_arr[b].ny, g_arr[b].nz = int(g.nx), int(g.ny), int(g.nz)
        g_arr[b].vox2world[:] = [float(v) for v in np.asarray(g.vox2world, float).reshape(12)]
    st_list, pa_rows = [], []
    for b, (stacks, patches) in enumerate(zip(stacks_per_problem, patches_per_problem)):
        base = len(st_list)
        for s in stacks:
            st_list.append((b, s))
        tab = np.asarray(patches.table(), dtype=np.int64)
        tab = tab.copy()
        tab[:, 0] += base
        pa_rows.append(tab)
    s_arr = (Stack * len(st_list))()
    for i, (b, s) in enumerate(st_list):
        s_arr[i].problem = b
        s_arr[i].nx, s_arr[i].ny, s_arr[i].nslices = int(s.nx), int(s.ny), int(s.nslices)
        s_arr[i].pix2world[:] = [float(v) for v in np.asarray(s.pix2world, float).reshape(12)]
        s_arr[i].fwhm_mm[:] = [float(v) for v in np.asarray(s.fwhm_mm, float).reshape(3)]
    tab = np.concatenate(pa_rows).astype(np.int32)
    p_arr = (Patch * tab.shape[0]).from_buffer_copy(np.ascontiguousarray(tab).tobytes())
    return g_arr, s_arr, p_arr


class Plan:
    """A plan over one or more independent reconstructions."""

    def __init__(self, grids, stacks_per_problem, patches_per_problem, cutoff_k: float = 3.0,
                 f64: bool = False):
        """f64: give the workspace room for the FP64 calls (PVR_WS_F64)."""
        L = load()
        self._g, self._s, self._p = make_descriptors(grids, stacks_per_problem,
                                                     patches_per_problem)
        h = ctypes.c_void_p()
        _check(L.pvr_plan_create(ctypes.addressof(self._g), len(self._g),
                                 ctypes.addressof(self._s), len(self._s),
                                 ctypes.addressof(self._p), len(self._p),
                                 float(cutoff_k), ctypes.byref(h)))
        self.h = h
        info = self.info()
        self.N = int(info.n_samples)
        self.V = int(info.n_voxels)
        self.M = int(info.n_patches)
        self.P = int(info.n_problems)
        so = np.zeros(self.M + 1, np.int64)
        vo = np.zeros(self.P + 1, np.int64)
        _check(L.pvr_plan_offsets(self.h, so.ctypes.data, vo.ctypes.data))
        self.sample_off = so
        self.vol_off = vo
        self.workspace = None
        self.attach(f64)

    def attach(self, f64: bool = False):
        """Allocate the plan's device workspace with torch (the library
        allocates no device memory) and hand it to the plan; the plan then
        counts as unbuilt."""
        import torch
        L = load()
        flags = PVR_WS_F64 if f64 else 0
        n = ctypes.c_size_t()
        _check(L.pvr_plan_workspace_size(self.h, flags, ctypes.byref(n)))
        ws = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device="cuda")
        _check(L.pvr_plan_attach(self.h, ws.data_ptr(), ws.numel(), flags, _stream()))
        self.workspace = ws  # held as long as the plan uses it
        self.f64 = f64

    @classmethod
    def from_problems(cls, problems, cutoff_k: float = 3.0, f64: bool = False):
        return cls([p.grid for p in problems], [p.stacks for p in problems],
                   [p.patches for p in problems], cutoff_k, f64)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().pvr_plan_destroy(self.h)  # synchronises before the workspace goes
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> PlanSizes:
        out = PlanSizes()
        _check(load().pvr_plan_info(self.h, ctypes.byref(out)))
        return out

    # -- calls --------------------------------------------------------------------
    def build(self, theta, active=None, mask=None):
        import torch
        f = load().pvr_plan_build_f64 if theta.dtype == torch.float64 else load().pvr_plan_build
        _check(f(self.h, _ptr(theta), _ptr(active), _ptr(mask), _stream()))
        self.build_id = getattr(self, "build_id", 0) + 1

    def check(self):
        """Raises PvrError(PVR_ENUMERIC) when a kernel has flagged non-finite
        values since the last check (synchronises the current stream)."""
        _check(load().pvr_check(self.h, _stream()))

    def set_timing(self, on: bool = True):
        _check(load().pvr_plan_set_timing(self.h, 1 if on else 0))

    def kernel_time(self, kernel: int):
        """(summed ms, launches) of the timed kernel since the last read
        (kernel: PVR_KERNEL_SIMULATE or PVR_KERNEL_BACKPROJECT)."""
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _check(load().pvr_plan_kernel_time(self.h, int(kernel), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def set_psf(self, kind: int):
        """PVR_PSF_GAUSSIAN or PVR_PSF_SINC; takes effect at the next build."""
        _check(load().pvr_plan_set_psf(self.h, int(kind)))
        self.psf = int(kind)

    def set_tiles(self, tile_w: int, tile_h: int):
        _check(load().pvr_plan_set_tiles(self.h, int(tile_w), int(tile_h), _stream()))
        self.tiles = (int(tile_w), int(tile_h))

    def inv_z(self):
        """Device pointer of the per-sample inverse normalisers (float [N])."""
        return load().pvr_plan_inv_z(self.h)

    def simulate(self, X, y_obs=None, y_sim=None, resid=None):
        import torch
        f = load().pvr_simulate_f64 if X.dtype == torch.float64 else load().pvr_simulate
        _check(f(self.h, _ptr(X), _ptr(y_obs), _ptr(y_sim), _ptr(resid), _stream()))

    def backproject(self, e, p=None, patch_w=None, num=None, den=None):
        import torch
        f = load().pvr_backproject_f64 if e.dtype == torch.float64 else load().pvr_backproject
        _check(f(self.h, _ptr(e), _ptr(p), _ptr(patch_w), _ptr(num), _ptr(den), _stream()))

    def robust_weights(self, resid, y_obs, em, p=None, pbar=None, patch_w=None, flags=0):
        _check(load().pvr_robust_weights(self.h, _ptr(resid), _ptr(y_obs), _ptr(em), _ptr(p),
                                         _ptr(pbar), _ptr(patch_w), int(flags), _stream()))

    def sr_update(self, X, num, den, X_out, params: Optional[SRParams] = None):
        prm = params or SRParams.make()
        _check(load().pvr_sr_update(self.h, _ptr(X), _ptr(num), _ptr(den), ctypes.byref(prm),
                                    _ptr(X_out), _stream()))

    def register(self, X, y_obs, theta, ncc=None, reg=None, params: Optional[RegParams] = None):
        prm = params or RegParams.make()
        _check(load().pvr_register_patches(self.h, _ptr(X), _ptr(y_obs), _ptr(theta), _ptr(ncc),
                                           _ptr(reg), ctypes.byref(prm), _stream()))

    def set_granules(self, sim: int, bp: int):
        """XCD granules of the forward work list and the adjoint bricks."""
        _check(load().pvr_plan_set_granules(self.h, int(sim), int(bp)))

    def reg_stats(self):
        """Registration work since the previous read: dict of NCC evaluations
        and valid samples walked, plain and with the exact gradient."""
        v = (ctypes.c_int64 * 4)()
        _check(load().pvr_plan_reg_stats(self.h, v, _stream()))
        return {"evals": int(v[0]), "samples": int(v[1]), "evals_exact": int(v[2]),
                "samples_exact": int(v[3])}

    # -- per-patch motion bookkeeping (pvr_motion_*) ---------------------------------
    def motion_frame(self, v, inverse=False, base=None, out=None):
        """out = base + A v (or A^-1 v), A = diag(rho F^T, F^T) per patch."""
        import torch
        out = torch.empty_like(v) if out is None else out
        _check(load().pvr_motion_frame(self.h, _ptr(v), 1 if inverse else 0, _ptr(base),
                                       _ptr(out), _stream()))
        return out

    def motion_step(self, theta, grad_theta, delta, step_min, trial):
        _check(load().pvr_motion_step(self.h, _ptr(theta), _ptr(grad_theta), _ptr(delta),
                                      float(step_min), _ptr(trial), _stream()))

    def motion_accept(self, cand, score_cand, theta, score, delta=None, step0=1.0,
                      step_min=0.0, n_live=None):
        _check(load().pvr_motion_accept(self.h, _ptr(cand), _ptr(score_cand), _ptr(theta),
                                        _ptr(score), _ptr(delta), float(step0), float(step_min),
                                        _ptr(n_live), _stream()))

    def motion_init_step(self, y_obs, step0, min_std, delta):
        _check(load().pvr_motion_init_step(self.h, _ptr(y_obs), float(step0), float(min_std),
                                           _ptr(delta), _stream()))

    def motion_live(self, delta, step_min, live, active=None):
        _check(load().pvr_motion_live(self.h, _ptr(delta), float(step_min), _ptr(active),
                                      _ptr(live), _stream()))

    def motion_fallback(self, score, tau, theta_ref, theta, flag, score_ref=None, active=None,
                        keep=None):
        _check(load().pvr_motion_fallback(self.h, _ptr(score), float(tau), _ptr(score_ref),
                                          _ptr(theta_ref), _ptr(theta), _ptr(active), _ptr(flag),
                                          _ptr(keep), _stream()))

    def grad_theta(self, X, grad_y, grad_theta):
        import torch
        f = (load().pvr_simulate_grad_theta_f64 if X.dtype == torch.float64
             else load().pvr_simulate_grad_theta)
        _check(f(self.h, _ptr(X), _ptr(grad_y), _ptr(grad_theta), _stream()))

    def ncc_grad(self, y_obs, y_sim, grad_y=None, ncc=None):
        _check(load().pvr_ncc_grad(self.h, _ptr(y_obs), _ptr(y_sim), _ptr(grad_y), _ptr(ncc),
                                   _stream()))

    # -- EM state helpers ---------------------------------------------------------------
    def em_state(self, device="cuda"):
        import torch
        return torch.zeros(self.P * ctypes.sizeof(EMState), dtype=torch.uint8, device=device)

    @staticmethod
    def read_em(em) -> List[EMState]:
        raw = em.detach().cpu().numpy().tobytes()
        n = len(raw) // ctypes.sizeof(EMState)
        return [EMState.from_buffer_copy(raw, i * ctypes.sizeof(EMState)) for i in range(n)]


class SRGraph:
    """`iters` SR iterations recorded once in a HIP graph by the library
    (pvr_sr_graph_create); launch() replays them on the current stream.  The
    tensors passed in are kept referenced for the graph's lifetime."""

    def __init__(self, plan: Plan, X, X_alt, y, resid, p, pbar, W, num, den, em,
                 params: Optional[SRParams] = None, iters: int = 2):
        self.plan = plan
        self.prm = params or SRParams.make()
        self._keep = (X, X_alt, y, resid, p, pbar, W, num, den, em)
        h = ctypes.c_void_p()
        _check(load().pvr_sr_graph_create(plan.h, _ptr(X), _ptr(X_alt), _ptr(y), _ptr(resid),
                                          _ptr(p), _ptr(pbar), _ptr(W), _ptr(num), _ptr(den),
                                          _ptr(em), ctypes.byref(self.prm), int(iters),
                                          _stream(), ctypes.byref(h)))
        self.h = h
        self.iters = int(iters)

    def launch(self):
        _check(load().pvr_sr_graph_launch(self.h, _stream()))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().pvr_sr_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
