"""Reconstruction driver: the cycle of registration and SR iterations built
from the library's calls (paper Sec. II: patches are repeatedly registered to
the current volume and reintegrated by iterative super-resolution; EM-based
outlier removal weights samples and patches).

Order of a cycle: register every patch against the current volume, rebuild
the plan at the new motion, restart EM, run n_sr SR iterations.  The first
volume is the PSF-weighted average X_0 = A^T y / A^T 1.  Every arithmetic step
runs in libpvr.so; torch only holds device buffers.
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np

from . import pvr


class Buffers:
    def __init__(self, plan, device="cuda"):
        import torch
        f32 = dict(dtype=torch.float32, device=device)
        self.e = torch.empty(plan.N, **f32)
        self.p = torch.empty(plan.N, **f32)
        self.pbar = torch.empty(plan.M, **f32)
        self.W = torch.empty(plan.M, **f32)
        self.num = torch.empty(plan.V, **f32)
        self.den = torch.empty(plan.V, **f32)
        self.Xn = torch.empty(plan.V, **f32)
        self.ncc = torch.empty(plan.M, **f32)
        self.em = plan.em_state(device)


def initial_volume(plan, y, buf: Buffers):
    import torch
    X = torch.zeros(plan.V, dtype=torch.float32, device=y.device)
    plan.backproject(y, None, None, buf.num, buf.den)
    plan.sr_update(X, buf.num, buf.den, buf.Xn, pvr.SRParams.make(lam=0.0))
    return buf.Xn.clone()


def sr_iterations(plan, X, y, buf: Buffers, n_sr: int, params: Optional[pvr.SRParams] = None,
                  fresh_em: bool = True):
    """n_sr SR iterations in place on X (returns the final volume tensor)."""
    prm = params or pvr.SRParams.make()
    cur, nxt = X, buf.Xn
    for it in range(n_sr):
        plan.simulate(cur, y_obs=y, resid=buf.e)
        flags = pvr.PVR_EM_INIT if (fresh_em and it == 0) else 0
        plan.robust_weights(buf.e, y, buf.em, buf.p, buf.pbar, buf.W, flags)
        plan.backproject(buf.e, buf.p, buf.W, buf.num, buf.den)
        plan.sr_update(cur, buf.num, buf.den, nxt, prm)
        cur, nxt = nxt, cur
    if cur is not X:
        X.copy_(cur)
    return X


def reconstruct(plan, y, theta0, cycles: int = 3, n_sr: int = 10,
                reg_params: Optional[pvr.RegParams] = None,
                sr_params: Optional[pvr.SRParams] = None, register: bool = True,
                init_fn=None):
    """Full reconstruction; theta0 is [M, 6] float32 on the device and is
    updated in place.  ``init_fn(plan, X, y, theta)``, when given, runs before
    each registration (a learned initialiser).  Returns (X, theta, history)."""
    import torch
    buf = Buffers(plan, y.device)
    theta = theta0
    timings = {"build": 0.0, "register": 0.0, "sr": 0.0, "init_fn": 0.0}

    def tick():
        torch.cuda.synchronize()
        return time.perf_counter()

    t = tick()
    plan.build(theta)
    X = initial_volume(plan, y, buf)
    t1 = tick(); timings["build"] += t1 - t
    hist = {"ncc": [], "excluded": []}
    ymax = float(y.abs().max())
    rp = reg_params or pvr.RegParams.make(min_std=0.01 * ymax)
    for c in range(cycles):
        if register:
            if init_fn is not None:
                t = tick()
                init_fn(plan, X, y, theta)
                timings["init_fn"] += tick() - t
            t = tick()
            plan.register(X, y, theta, buf.ncc, params=rp)
            t1 = tick(); timings["register"] += t1 - t
            hist["ncc"].append(float(buf.ncc.mean()))
            t = tick()
            plan.build(theta)
            timings["build"] += tick() - t
        t = tick()
        sr_iterations(plan, X, y, buf, n_sr, sr_params)
        timings["sr"] += tick() - t
        hist["excluded"].append(pvr.Plan.read_em(buf.em)[0].n_excluded)
    hist["timings"] = timings
    return X, theta, hist


def psnr(X, X_true, plan, dilate_vox: int = 5) -> float:
    """Volume PSNR against the synthetic truth over the truth's support
    dilated by ``dilate_vox`` voxels (cube), I_max = max(truth) (paper Sec.
    IV-A eq. PSNR, base-10 logarithm)."""
    import torch
    import torch.nn.functional as F
    vals = []
    for b in range(plan.P):
        a, z = int(plan.vol_off[b]), int(plan.vol_off[b + 1])
        g = plan._g[b]
        T = X_true[a:z].reshape(1, 1, g.nz, g.ny, g.nx).float()
        R = X[a:z].reshape(1, 1, g.nz, g.ny, g.nx).float()
        m = F.max_pool3d((T > 0).float(), 2 * dilate_vox + 1, stride=1, padding=dilate_vox) > 0
        mse = float(((R - T)[m] ** 2).mean())
        imax = float(T.max())
        vals.append(10 * np.log10(imax * imax / mse) if mse > 0 else float("inf"))
    return float(np.mean(vals))
