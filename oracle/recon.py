"""SR iteration and reconstruction cycles, FP64 -- TEST INFRASTRUCTURE ONLY.

Order of one SR iteration k (a reading; the paper gives the parts but not
their order, Sec. II):
  1. e = y - A X_k over valid samples;
  2. m = 1 / (max e - min e);
  3. E-step p(e) with sigma^2, c of the previous iteration (or the cycle start);
  4. patch potentials p_bar and patch weights W from the patch mixture;
  5. num = A^T(W p e), den = A^T(W p);
  6. X_{k+1} = update(X_k, num, den);
  7. M-step for the next iteration from the same e, p, W.
A cycle is: register every patch against the current X (Sec. II "Patch to
Volume Registration"), then restart EM and run n_sr SR iterations.
The initial volume is the PSF-weighted average X_0 = A^T y / A^T 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import em
from .update import sr_update


@dataclasses.dataclass
class SRParams:
    alpha: float = 1.0
    lam: float = 0.02
    delta: float = 150.0
    clamp_min: float = 0.0
    den_eps: float = 1e-6


@dataclasses.dataclass
class EMState:
    sigma2: float = 1.0
    c: float = em.C_START
    started: bool = False


def initial_volume(ctx, y, theta, mask=None, active=None, den_eps=1e-6):
    num = ctx.backproject(theta, y, mask, active)
    den = ctx.backproject(theta, np.ones(ctx.N), mask, active)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(den > den_eps, num / np.where(den > den_eps, den, 1.0), 0.0)


def robust_weights(e, y, valid, state: EMState, patch_of_sample, M, active=None,
                   W_override=None):
    """E-step, potentials, patch weights and next-iteration M-step; returns
    (p, pbar, W, pi, new_state, diagnostics).  Arrays are per sample / patch.
    ``W_override`` replaces the classified patch weights (used by parity
    checks to pin patches whose posterior sits on the 0.5 threshold)."""
    ev = e[valid]
    yabs = float(np.max(np.abs(y[valid]))) if ev.size else 0.0
    floor = (1e-4 * yabs) ** 2
    if not state.started:
        s2, c = em.init_state(ev)
        state = EMState(max(s2, floor) if s2 > 0 else max(floor, 1.0), c, True)
    m = em.outlier_density(ev, yabs)
    p = np.where(valid, em.posterior(e, state.sigma2, state.c, m), 0.0)
    pbar, n_s, _, _ = em.patch_potentials(p, valid, patch_of_sample, M)
    W, pi = em.patch_weights(pbar, n_s, active)
    if W_override is not None:
        W = np.asarray(W_override, np.float64)
    Ws = W[patch_of_sample]
    s2, c = em.mstep(e, p, valid, Ws, n_s, W, state.sigma2, state.c, yabs)
    diag = dict(m=m, sigma2=state.sigma2, c=state.c, excluded=int(np.sum((n_s > 0) & (W == 0))))
    return p, pbar, W, pi, EMState(s2, c, True), diag


def sr_iteration(ctx, X, y, theta, state: EMState, params: SRParams,
                 mask=None, active=None, W_override: Optional[np.ndarray] = None):
    yhat, Z, valid = ctx.simulate(X, theta, mask, active)
    e = np.where(valid, np.asarray(y, np.float64) - yhat, 0.0)
    p, pbar, W, pi, new_state, diag = robust_weights(
        e, np.asarray(y, np.float64), valid, state, ctx.patch_of_sample, ctx.M,
        active, W_override)
    Ws = W[ctx.patch_of_sample]
    num = ctx.backproject(theta, Ws * p * e, mask, active)
    den = ctx.backproject(theta, Ws * p, mask, active)
    Xn = sr_update(X, num, den, params.alpha, params.lam, params.delta,
                   params.clamp_min, params.den_eps)
    diag.update(W=W, pbar=pbar, pi=pi, e=e, p=p, valid=valid)
    return Xn, new_state, diag


def reconstruct(ctx, y, theta0, cycles=1, n_sr=10, params: SRParams = SRParams(),
                register=True, mask=None, reg_kw=None, X0=None, trace=None):
    """C cycles of [register every patch against X -> restart EM -> n_sr SR
    iterations] from X_0 = A^T y / A^T 1 at theta0.  Returns (X, theta,
    per-iteration diagnostics).  ``trace``, when a list, receives one dict
    per cycle: the volume the cycle's SR iterations start from (after its
    registration), the motion they use and the NCC the registration reached."""
    theta = np.array(theta0, dtype=np.float64).reshape(-1, 6).copy()
    X = initial_volume(ctx, y, theta, mask) if X0 is None else np.asarray(X0, np.float64)
    hist = []
    for cyc in range(cycles):
        ncc = None
        if register:
            theta, ncc = ctx.register(X, y, theta, mask=mask, **(reg_kw or {}))
        if trace is not None:
            trace.append(dict(X=np.array(X, copy=True), theta=theta.copy(), ncc=ncc))
        state = EMState()
        for it in range(n_sr):
            X, state, diag = sr_iteration(ctx, X, y, theta, state, params, mask)
            hist.append(diag)
    return X, theta, hist


def psnr(X, X_true, mask=None) -> float:
    """10 log10(I_max^2 / MSE) with I_max = max(X_true) (Sec. IV-A eq. PSNR,
    base-10 logarithm read)."""
    X = np.asarray(X, np.float64); T = np.asarray(X_true, np.float64)
    if mask is None:
        mask = np.ones(T.shape, bool)
    mse = float(np.mean((X[mask] - T[mask]) ** 2))
    imax = float(T.max())
    return float("inf") if mse == 0 else 10.0 * math.log10(imax * imax / mse)
