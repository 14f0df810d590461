"""The multi-GPU design, emulated on the CPU with the oracle: the patches are
split into shards (one per GPU), each shard simulates its own patches and
back-projects into its own num / den, the EM runs on the gathered residuals
(its scalars and patch potentials are what the all-reduce and all-gather
would exchange), and num / den are summed over the shards.  One SR iteration
built that way equals the unsharded iteration to FP64 rounding."""
import numpy as np

import oracle
from oracle import recon
from oracle.update import sr_update
from paper_1611_07289_amd import synth


def _sub(pat, a, b):
    return synth.Patches(*[np.asarray(getattr(pat, k)[a:b], np.int32)
                           for k in ("stack", "slice", "x0", "y0", "w", "h")])


def test_sharded_sr_iteration_equals_unsharded():
    P = synth.tiny_problem()
    ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
    th = P.theta_true
    yc, _, _ = ctx.simulate(P.x_true, th)
    y = synth.corrupt(yc, P.patches, P.outlier_patch, 0.01, 3, 5).astype(np.float64)
    X0 = recon.initial_volume(ctx, y, th)
    prm = recon.SRParams()
    X1, _, diag = recon.sr_iteration(ctx, X0, y, th, recon.EMState(), prm)

    bounds = [0, 61, 140, P.M]  # uneven shards
    off = P.patches.sample_off
    shards = [(a, b, oracle.Ctx(P.grid, P.stacks, _sub(P.patches, a, b)))
              for a, b in zip(bounds[:-1], bounds[1:])]
    yh = np.concatenate([c.simulate(X0, th[a:b])[0] for a, b, c in shards])
    valid = np.concatenate([c.simulate(X0, th[a:b])[2] for a, b, c in shards])
    assert np.array_equal(valid, diag["valid"])
    e = np.where(valid, y - yh, 0.0)
    assert np.allclose(e, diag["e"], rtol=0, atol=1e-9 * np.abs(y).max())
    p, pbar, W, pi, _, _ = recon.robust_weights(e, y, valid, recon.EMState(),
                                                ctx.patch_of_sample, P.M)
    assert np.array_equal(W > 0, diag["W"] > 0)
    r = W[ctx.patch_of_sample] * p
    num = sum(c.backproject(th[a:b], (r * e)[off[a]:off[b]]) for a, b, c in shards)
    den = sum(c.backproject(th[a:b], r[off[a]:off[b]]) for a, b, c in shards)
    X1s = sr_update(X0, num, den, prm.alpha, prm.lam, prm.delta, prm.clamp_min, prm.den_eps)
    assert np.linalg.norm(X1s - X1) <= 1e-12 * np.linalg.norm(X1)
