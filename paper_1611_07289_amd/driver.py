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
    # X_0 = A^T y / A^T 1 as it stands (no clamp at 0: noisy background can
    # average below 0, and the update's clamp belongs to the SR iterations)
    plan.sr_update(X, buf.num, buf.den, buf.Xn, pvr.SRParams.make(lam=0.0, use_clamp=False))
    return buf.Xn.clone()


def uncertainty_maps(plan, p, pbar, buf: Buffers):
    """Rigidity / uncertainty maps (paper Sec. II, "Patch Potentials"): the
    sample posteriors p and the patch potentials p_bar integrated into the
    volume with the reconstruction's PSF, each normalised by A^T 1:
    map_p = A^T p / A^T 1 and map_pbar = A^T p_bar(s) / A^T 1 (zero where
    A^T 1 <= 1e-6).  High values mark regions that fit the rigid patch
    model.  Returns (map_p, map_pbar) as new tensors [V]."""
    import torch
    zero = torch.zeros(plan.V, dtype=torch.float32, device=p.device)
    prm = pvr.SRParams.make(lam=0.0)
    plan.backproject(p, None, None, buf.num, buf.den)  # A^T p and A^T 1
    plan.sr_update(zero, buf.num, buf.den, buf.Xn, prm)
    map_p = buf.Xn.clone()
    ones = torch.ones(plan.N, dtype=torch.float32, device=p.device)
    plan.backproject(ones, None, pbar, buf.num, None)  # A^T p_bar(s), den kept
    plan.sr_update(zero, buf.num, buf.den, buf.Xn, prm)
    return map_p, buf.Xn.clone()


def sr_iterations(plan, X, y, buf: Buffers, n_sr: int, params: Optional[pvr.SRParams] = None,
                  fresh_em: bool = True):
    """n_sr SR iterations in place on X (returns the final volume tensor)."""
    prm = params or pvr.SRParams.make()
    cur, nxt = X, buf.Xn
    for it in range(n_sr):
        plan.simulate(cur, y_obs=y, resid=buf.e)
        flags = ((pvr.PVR_EM_INIT if (fresh_em and it == 0) else 0) | pvr.PVR_EM_RESID_FRESH
                 | pvr.PVR_EM_PREP_ADJOINT)
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
                init_fn=None, active_schedule=None, sample_mask=None, X0=None,
                first_cycle: int = 0, on_cycle=None, fallback_tau: Optional[float] = None,
                fallback_params: Optional[pvr.RegParams] = None, register_fn=None,
                fallback_relative: bool = False):
    """Full reconstruction; theta0 is [M, 6] float32 on the device and is
    updated in place.  ``init_fn(plan, X, y, theta)``, when given, runs before
    each registration (a learned initialiser) with the keyword arguments
    active and mask of the cycle's build; it returns the per-patch NCC before
    the prediction and at the motion it leaves (device tensors), or None.
    With ``fallback_tau`` that NCC decides: patches where it is below tau
    (below the NCC before the prediction plus tau with
    ``fallback_relative``) are registered from their motion before the
    prediction with ``fallback_params`` (default the same parameters), the
    others refine the prediction with ``reg_params``.
    ``register_fn(plan, X, y, theta, ncc, active,
    mask)``, when given, replaces the per-patch registration
    (pvr_register_patches), e.g. the joint gradient-based registration.
    ``active_schedule``, when given, is a list of per-patch uint8 device masks used cycle by cycle (in
    turn): multi-scale patches (paper Sec. II, eq. Y_i), where cycle c
    registers and reconstructs from the patches of one scale only.
    ``sample_mask`` (uint8 [N] on the device), when given, applies at every
    build: the samples of arbitrarily shaped patches (superpixels) inside
    their rectangular boxes.
    Resuming: ``X0`` (a volume [V] on the device) replaces the initial volume
    and the cycles are numbered from ``first_cycle`` (the active schedule
    follows the numbering); EM restarts every cycle, so (X, theta, cycle) is
    the whole state between cycles (see save_checkpoint / load_checkpoint).
    ``on_cycle(record)``, when given, receives after every cycle a dict of
    its statistics: cycle, mean NCC after registration, EM sigma^2, c, m and
    excluded patches, and the cumulative timings.
    Returns (X, theta, history)."""
    import torch
    buf = Buffers(plan, y.device)
    theta = theta0
    timings = {"build": 0.0, "register": 0.0, "sr": 0.0, "init_fn": 0.0}

    def active(c):
        return None if not active_schedule else active_schedule[c % len(active_schedule)]

    def tick():
        torch.cuda.synchronize()
        return time.perf_counter()

    t = tick()
    plan.build(theta, active=active(first_cycle), mask=sample_mask)
    X = initial_volume(plan, y, buf) if X0 is None else X0.clone()
    t1 = tick(); timings["build"] += t1 - t
    hist = {"ncc": [], "excluded": [], "fallback": []}
    ymax = float(y.abs().max())
    # default: the exact NCC gradient (the same registrations as central
    # differences at a third of the time); the sinc PSF has only the latter
    rp = reg_params or pvr.RegParams.make(
        min_std=0.01 * ymax, exact=getattr(plan, "psf", pvr.PVR_PSF_GAUSSIAN) == pvr.PVR_PSF_GAUSSIAN)
    for c in range(first_cycle, first_cycle + cycles):
        if register:
            scores = None
            if init_fn is not None:
                t = tick()
                theta_pre = theta.clone()
                scores = init_fn(plan, X, y, theta, active=active(c), mask=sample_mask)
                timings["init_fn"] += tick() - t
            t = tick()
            if register_fn is not None:
                register_fn(plan, X, y, theta, buf.ncc, active(c), sample_mask)
            elif scores is not None and fallback_tau is not None:
                # the NCC after the prediction decides: where it stays below
                # the threshold (tau, or the NCC before the prediction plus
                # tau with fallback_relative) the plain registration takes
                # over from the motion before the prediction, elsewhere the
                # registration refines the prediction
                n_old, n_pred = scores
                flag = torch.empty(plan.M, dtype=torch.uint8, device=theta.device)
                keep = torch.empty_like(flag)
                plan.motion_fallback(n_pred, fallback_tau, theta_pre, theta, flag,
                                     score_ref=n_old if fallback_relative else None,
                                     active=active(c), keep=keep)
                plan.register(X, y, theta, buf.ncc, reg=keep, params=rp)
                plan.register(X, y, theta, buf.ncc, reg=flag, params=fallback_params or rp)
                hist["fallback"].append(int(flag.sum()))
            else:
                plan.register(X, y, theta, buf.ncc, reg=active(c), params=rp)
            t1 = tick(); timings["register"] += t1 - t
            hist["ncc"].append(float(buf.ncc.mean()))
            t = tick()
            plan.build(theta, active=active(c), mask=sample_mask)
            timings["build"] += tick() - t
        elif active_schedule:
            plan.build(theta, active=active(c), mask=sample_mask)
        t = tick()
        sr_iterations(plan, X, y, buf, n_sr, sr_params)
        timings["sr"] += tick() - t
        em = pvr.Plan.read_em(buf.em)
        hist["excluded"].append(em[0].n_excluded)
        if on_cycle is not None:
            on_cycle({"cycle": c, "mean_ncc": hist["ncc"][-1] if register else None,
                      "sigma2": [e.sigma2 for e in em], "c": [e.c for e in em],
                      "m": [e.m for e in em], "excluded": [e.n_excluded for e in em],
                      "timings": dict(timings)})
    hist["timings"] = timings
    return X, theta, hist


def save_checkpoint(path: str, X, theta, cycle: int) -> None:
    """The state between two cycles (EM restarts every cycle): the volume,
    the motion and the index of the next cycle, as an .npz file."""
    np.savez(path, X=X.detach().cpu().numpy(), theta=theta.detach().cpu().numpy(),
             next_cycle=np.int64(cycle))


def load_checkpoint(path: str, device="cuda"):
    """(X, theta, next_cycle) of save_checkpoint, tensors on ``device``."""
    import torch
    with np.load(path, allow_pickle=False) as d:
        return (torch.from_numpy(d["X"]).to(device), torch.from_numpy(d["theta"]).to(device),
                int(d["next_cycle"]))


def json_lines(stream):
    """An on_cycle callback writing one JSON line per cycle to ``stream``."""
    import json

    def write(record):
        stream.write(json.dumps(record) + "\n")
        stream.flush()
    return write


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


def patch_table(plan) -> np.ndarray:
    """The plan's patch descriptors as an int32 array [M][6] (stack, slice,
    x0, y0, w, h; stack indices global over the plan's problems)."""
    return np.frombuffer(plan._p, dtype=np.int32).reshape(-1, 6)


def patch_radius(plan):
    """Half-diagonal (mm) of every patch: the scale of the rotation variables
    of the registration optimisers (a unit step moves the farthest pixel by
    about 1 mm)."""
    sp = np.array([np.linalg.norm(np.asarray(list(s.pix2world), float).reshape(3, 4)[:, :3], axis=0)
                   for s in plan._s])
    tab = patch_table(plan)
    su, sv = sp[tab[:, 0], 0], sp[tab[:, 0], 1]
    rho = 0.5 * np.hypot((tab[:, 4] - 1) * su, (tab[:, 5] - 1) * sv)
    return np.maximum(rho, 1.0)


def register_gradient(plan, X, y, theta, iters: int = 30, step0: float = 1.0,
                      step_min: float = 0.01, min_std: float = 0.0, active=None, mask=None):
    """Joint gradient-based registration of all patches with the
    differentiable forward model: d NCC_s / d theta_s is the NCC derivative
    with respect to the simulated samples (pvr_ncc_grad) pulled back through
    pvr_simulate_grad_theta.  Each patch takes a normalised ascent step in the
    radius-scaled variables (pvr_motion_step), kept on strict NCC improvement
    (the step then doubles, capped at step0) and halved otherwise
    (pvr_motion_accept).  Patches with std(y_s) < min_std and patches whose
    step fell below step_min stay put (pvr_motion_init_step).  Every build
    takes ``active`` and ``mask`` (uint8 device arrays, nullable) as
    driver.reconstruct passes them.  theta ([M, 6] float32 on the device) is
    updated in place; the plan is left built at the final theta.  Returns the
    final per-patch NCC."""
    import torch
    dev = theta.device
    ysim = torch.empty(plan.N, dtype=torch.float32, device=dev)
    g = torch.empty_like(ysim)
    ncc = torch.empty(plan.M, dtype=torch.float32, device=dev)
    ncc_t = torch.empty_like(ncc)
    ncc_c = torch.empty_like(ncc)
    G = torch.empty(plan.M, 6, dtype=torch.float32, device=dev)
    G_t = torch.empty_like(G)
    trial = torch.empty_like(G)
    delta = torch.empty(plan.M, dtype=torch.float32, device=dev)
    live = torch.empty(plan.M, dtype=torch.uint8, device=dev)

    def evaluate(th, score, grad, act):
        plan.build(th, active=act, mask=mask)
        plan.simulate(X, y_sim=ysim)
        plan.ncc_grad(y, ysim, g, score)
        plan.grad_theta(X, g, grad)

    # NCC and gradient at every trial: an accepted trial becomes the patch's
    # motion with the NCC and gradient just computed there, a rejected one
    # leaves the motion, NCC and gradient as they were, so the motion is
    # never evaluated twice.  Only the patches whose step is still at least
    # step_min are evaluated (pvr_motion_live); the others could not move
    # anyway, and their NCC and motion stay as they are.
    n_live = torch.zeros(1, dtype=torch.int32, device=dev)
    evaluate(theta, ncc, G, active)
    plan.motion_init_step(y, step0, min_std, delta)
    plan.motion_live(delta, step_min, live, active)
    for it in range(iters):
        plan.motion_step(theta, G, delta, step_min, trial)
        evaluate(trial, ncc_t, G_t, live)
        # the gradient follows the motion: the same strict-improvement test
        # (on a copy of the scores, which the motion's acceptance updates);
        # a patch not evaluated may pass it (its trial score reads 0), but its
        # gradient is never used again, as its step stays below step_min
        ncc_c.copy_(ncc)
        plan.motion_accept(G_t, ncc_t, G, ncc_c)
        n_live.zero_()
        plan.motion_accept(trial, ncc_t, theta, ncc, delta, step0, step_min, n_live)
        plan.motion_live(delta, step_min, live, active)
        if it % 4 == 3 and int(n_live.item()) == 0:  # every patch has converged
            break
    plan.build(theta, active=active, mask=mask)
    return ncc
