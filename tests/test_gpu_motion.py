"""The per-patch motion bookkeeping calls (pvr_motion_*) against numpy
statements of their rules on the 32^3 workload's 216 patches (three
orthogonal stacks) plus an oblique stack: the patch-frame map
A = diag(rho F^T, F^T) and its inverse, the normalised ascent trial, the
accept / halve rule with its live count, the live set, the flat-patch test
and the fallback selection."""
import math

import numpy as np
import pytest
import torch

from paper_1611_07289_amd import pvr, synth
from tests._gpu import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    g = synth.iso_grid(32)
    c = synth.grid_center(g)
    stacks = [synth.make_stack(c, *fr, 32, 32, 8, (1, 1), 4.0, (1.0, 1.0, 4.0))
              for fr in synth.orthogonal_frames([30.0])]
    stacks.append(synth.make_stack(c, *synth.orthogonal_frames()[0], 30, 28, 6, (0.8, 1.2), 3.0,
                                   (0.8, 1.2, 3.0)))
    P = synth.square_patches(stacks, 16, 8)
    plan = pvr.Plan([g], [stacks], [P])
    F = []
    rho = []
    for s in P.stack:
        L = np.asarray(stacks[s].pix2world, float)[:, :3]
        sp = np.linalg.norm(L, axis=0)
        F.append(L / sp)
        rho.append(max(0.5 * math.hypot(15 * sp[0], 15 * sp[1]), 1.0))
    A = np.zeros((P.M, 6, 6))
    for i, (Fi, r) in enumerate(zip(F, rho)):
        A[i, :3, :3] = r * Fi.T
        A[i, 3:, 3:] = Fi.T
    return plan, P, np.array(rho), A


def test_frame_map_and_inverse(case):
    plan, P, rho, A = case
    rng = np.random.default_rng(1)
    v = rng.normal(size=(P.M, 6)).astype(np.float32)
    base = rng.normal(size=(P.M, 6)).astype(np.float32)
    fw = host(plan.motion_frame(dev(v)))
    ref = np.einsum("mij,mj->mi", A, v.astype(np.float64))
    assert np.abs(fw - ref).max() <= 1e-5 * np.abs(ref).max()
    inv = host(plan.motion_frame(dev(v), inverse=True, base=dev(base)))
    ref = base + np.einsum("mij,mj->mi", np.linalg.inv(A), v.astype(np.float64))
    assert np.abs(inv - ref).max() <= 1e-5 * np.abs(ref).max()
    # a translation along the slice normal is the sixth target; a small
    # rotation about the normal the third, scaled by rho
    for i in (0, P.M // 2, P.M - 1):
        n = A[i, 5, 3:]
        off = np.zeros((P.M, 6), np.float32)
        off[i, 3:] = n
        off[i, :3] = 1e-3 * n
        out = host(plan.motion_frame(dev(off)))[i]
        assert np.allclose(out, [0, 0, 1e-3 * rho[i], 0, 0, 1], atol=1e-6)


def test_step_accept_and_live_count(case):
    plan, P, rho, A = case
    rng = np.random.default_rng(2)
    th = rng.normal(scale=0.1, size=(P.M, 6)).astype(np.float32)
    G = rng.normal(size=(P.M, 6)).astype(np.float32)
    delta = rng.choice([0.0, 0.005, 0.3, 1.0], size=P.M).astype(np.float32)
    step_min, step0 = 0.01, 1.0
    trial = torch.empty(P.M, 6, device="cuda")
    plan.motion_step(dev(th), dev(G), dev(delta), step_min, trial)
    sc = np.c_[np.repeat(rho[:, None], 3, 1), np.ones((P.M, 3))]
    gq = G / sc
    ref = th + np.where((delta >= step_min)[:, None],
                        delta[:, None] * gq / np.linalg.norm(gq, axis=1, keepdims=True) / sc, 0)
    assert np.abs(host(trial) - ref).max() <= 1e-6
    score = rng.uniform(size=P.M).astype(np.float32)
    score_c = rng.uniform(size=P.M).astype(np.float32)
    tt, ss, dd = dev(th), dev(score), dev(delta)
    n_live = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.motion_accept(trial, dev(score_c), tt, ss, dd, step0, step_min, n_live)
    live = delta >= step_min
    acc = live & (score_c > score)
    assert np.array_equal(host(tt), np.where(acc[:, None], host(trial), th))
    assert np.array_equal(host(ss), np.where(acc, score_c, score))
    d_ref = np.where(acc, np.minimum(2 * delta, step0), np.where(live, 0.5 * delta, delta))
    assert np.array_equal(host(dd), d_ref.astype(np.float32))
    assert int(n_live.item()) == int(np.sum(live & (d_ref >= step_min)))
    # without step lengths: a plain selection of the higher score
    tt, ss = dev(th), dev(score)
    plan.motion_accept(trial, dev(score_c), tt, ss)
    sel = score_c > score
    assert np.array_equal(host(tt), np.where(sel[:, None], host(trial), th))
    # the live set: step at least step_min, within an active set (or all)
    live = torch.empty(P.M, dtype=torch.uint8, device="cuda")
    plan.motion_live(dev(delta), step_min, live)
    assert np.array_equal(host(live), (delta >= step_min).astype(np.uint8))
    active = (rng.uniform(size=P.M) < 0.6).astype(np.uint8)
    plan.motion_live(dev(delta), step_min, live, dev(active))
    assert np.array_equal(host(live), ((delta >= step_min) & (active > 0)).astype(np.uint8))


def test_flat_patches_and_fallback(case):
    plan, P, rho, A = case
    rng = np.random.default_rng(3)
    y = rng.normal(100, 5, size=P.n_samples).astype(np.float32)
    off = P.sample_off
    flat = rng.uniform(size=P.M) < 0.3
    for s in np.nonzero(flat)[0]:
        y[off[s]:off[s + 1]] = 7.0 + 1e-4 * rng.normal(size=off[s + 1] - off[s])
    mask = np.ones(P.n_samples, np.uint8)
    mask[off[3]:off[3] + 100] = 0  # a masked part of patch 3 does not count
    y[off[3]:off[3] + 100] = 1e6 if flat[3] else y[off[3]:off[3] + 100]
    plan.build(dev(np.zeros((P.M, 6), np.float32)), mask=dev(mask))
    delta = torch.empty(P.M, device="cuda")
    plan.motion_init_step(dev(y), 0.5, 1.0, delta)
    sd = np.array([y[off[s]:off[s + 1]][mask[off[s]:off[s + 1]] > 0].astype(np.float64).std()
                   for s in range(P.M)])
    assert np.array_equal(host(delta), np.where(sd >= 1.0, 0.5, 0.0).astype(np.float32))
    score = rng.uniform(size=P.M).astype(np.float32)
    score_ref = rng.uniform(size=P.M).astype(np.float32)
    active = (rng.uniform(size=P.M) < 0.7).astype(np.uint8)
    th = rng.normal(size=(P.M, 6)).astype(np.float32)
    ref = rng.normal(size=(P.M, 6)).astype(np.float32)
    flag = torch.empty(P.M, dtype=torch.uint8, device="cuda")
    keep = torch.empty_like(flag)
    # a fixed threshold over every patch
    tt = dev(th)
    plan.motion_fallback(dev(score), 0.4, dev(ref), tt, flag)
    back = score < 0.4
    assert np.array_equal(host(flag), back.astype(np.uint8))
    assert np.array_equal(host(tt), np.where(back[:, None], ref, th))
    # a threshold relative to a reference score, over an active set
    tt = dev(th)
    plan.motion_fallback(dev(score), 0.05, dev(ref), tt, flag, score_ref=dev(score_ref),
                         active=dev(active), keep=keep)
    back = (active > 0) & (score < score_ref + np.float32(0.05))
    assert np.array_equal(host(flag), back.astype(np.uint8))
    assert np.array_equal(host(keep), ((active > 0) & ~back).astype(np.uint8))
    assert np.array_equal(host(tt), np.where(back[:, None], ref, th))
