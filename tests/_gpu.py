"""Helpers shared by the GPU parity tests (device transfers, the per-sample
bar and an SR-iteration loop through the C ABI that can take the patch
weights from the oracle)."""
import numpy as np
import torch

from paper_1611_07289_amd import pvr


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def sample_close(g, o, rel=1e-5):
    """Worst per-sample error against the bar 1e-5 max(|y_ora|, 1e-3 max|y_ora|)
    (returned relative to that scale) and the per-sample errors."""
    g = np.asarray(g, np.float64); o = np.asarray(o, np.float64)
    scale = np.maximum(np.abs(o), 1e-3 * np.abs(o).max())
    err = np.abs(g - o) / scale
    return float(err.max()), err


def sr_loop(plan, X0, y, n_iter, params=None, fix_w_list=None):
    """n_iter SR iterations from the volume X0 (host array) on observations y
    (host): simulate, robust weights (EM restarted at the first iteration),
    back-projection, update.  With fix_w_list, iteration i takes the patch
    weights fix_w_list[i] (PVR_EM_FIX_W) instead of classifying: the patch
    classification is a hard threshold at posterior 0.5, so a patch whose
    posterior sits within rounding of it may flip between FP32 and FP64, and
    pinning W keeps a volume comparison meaningful.  Returns the final volume
    and the patch weights of every iteration (host)."""
    prm = params or pvr.SRParams.make()
    X = dev(np.asarray(X0, np.float32).reshape(-1))
    Xn = torch.empty_like(X)
    yd = dev(np.asarray(y, np.float32))
    e = torch.empty(plan.N, dtype=torch.float32, device="cuda")
    p = torch.empty_like(e)
    pbar = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    W = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    num = torch.empty(plan.V, dtype=torch.float32, device="cuda")
    den = torch.empty_like(num)
    emg = plan.em_state()
    Ws = []
    for it in range(n_iter):
        plan.simulate(X, y_obs=yd, resid=e)
        flags = pvr.PVR_EM_INIT if it == 0 else 0
        if fix_w_list is not None:
            W.copy_(dev(np.asarray(fix_w_list[it], np.float32)))
            flags |= pvr.PVR_EM_FIX_W
        plan.robust_weights(e, yd, emg, p, pbar, W, flags)
        Ws.append(host(W).copy())
        plan.backproject(e, p, W, num, den)
        plan.sr_update(X, num, den, Xn, prm)
        X, Xn = Xn, X
    return host(X), Ws
