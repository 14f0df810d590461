#!/usr/bin/env python3
"""Benchmark of the PVR super-resolution hot path on one MI355X.

Workloads: uterus256 (default) below; sinc256 the same with the paper's sinc
PSF (pvr_plan_set_psf); batched, diff48, learned and multiscale as their
functions say.

Workload (default): the 256^3 whole-uterus case -- 1 mm grid, 4 stacks of
256x256x60 slices at 1x1x4 mm (3 orthogonal + 1 oblique at 30 deg), PSF FWHM
(1, 1, 4) mm, 64x64 patches with stride 32 (11 760 patches, 48.2 M samples),
per-patch motion <= 10 deg / <= 5 mm, 1 % noise, 10 % outlier patches.  All
inputs are seeded synthetic stand-ins for the paper's fetal data.

A step is one SR iteration over the whole batch: simulate (residuals), EM
robust weights, gather back-projection, volume update, all through the C ABI
of libpvr.so with inputs resident in HBM.  Reported value: valid patch
samples processed per second (whole job).

Extra objects on the JSON line:
  hbm_equivalent  the iteration time against the HBM floor of a stored-weight
                implementation of the same iteration (bytes it would move /
                8 TB/s);
  roofline      dominant kernel (k_simulate or k_backproject): algorithmic
                work per launch / its average duration from the event pairs
                the library records around each launch on its stream, against
                the chip's peak; traffic = counter-measured HBM-side bytes
                per launch when taken on the current library sources;
  kernels_ms    average duration of every call of the step (HIP events on
                the library's stream);
  hot_kernels_ms  the two PSF kernels alone;
  cpu_baseline  the FP64 oracle timed on the host on a bounded sample;
  full_pvr      (uterus256 and sinc256, unless --no-full-pvr) seconds and
                PSNR of a whole reconstruction from zero motion -- initial
                volume, then 3 cycles of [registration, 10 SR iterations] --
                with plain registration and (uterus256) with the learned
                initialiser (trained first on --learned-pairs forward-model
                pairs of another phantom; training time reported apart), each
                with the registration gradient by central differences and
                (uterus256) exact ("_exact");
  superpixel_pvr  (uterus256, unless --no-superpixel) whole slices observed
                under per-slice motion, reconstructed (exact registration,
                same schedule) from 64x64 stride-32 square patches and from
                SLIC superpixel patches (a = 32 and a = 64, dilation 60 % of
                a) of the same slices: patch and sample counts, extraction
                time, seconds and PSNR of each.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP32 peak without packed-FP32 instructions (the library is built with them
# disabled): 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz.
FP32_VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
# Algorithmic FP32 work of one PSF nonzero (one sample-voxel pair): offset
# along the 3 stack axes (3), scaling by 1/sigma (3), squared norm (5), the
# exponential (1), cut-off shift (1), and the accumulation (forward: weight sum
# 1 + weighted value 2; adjoint: two weighted sums 4).
FLOP_PER_NNZ_FWD = 16
FLOP_PER_NNZ_ADJ = 17
# The sinc PSF: offsets (3), scaling (3), two Taylor series in (pi t)^2 to the
# 8th power (2 x 18), the slice profile (square, scale, exponential, cut-off:
# 4), the product (2), accumulation (forward 3, adjoint 4).
FLOP_PER_NNZ_SINC_FWD = 51
FLOP_PER_NNZ_SINC_ADJ = 52
# HBM-side bytes per launch of the hot kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by a 1 GiB device copy; valid only for the library
# sources they were taken on (their SHA-256 is stored beside the figures).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_uterus256.json")


def library_source_sha() -> str:
    """Hash of the sources the two PSF kernels are compiled from (their
    translation units, the plan that lays out their inputs, every header)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1611_07289_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.h")) +
                   [os.path.join(csrc, f) for f in ("pvr_forward.hip", "pvr_adjoint.hip",
                                                    "pvr_plan.hip")])
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """Counter-measured bytes per launch of `kernel`, or None when none were
    taken on the current sources for this workload."""
    if workload != "uterus256":
        return None
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != library_source_sha():
        return None
    e = d.get("kernels", {}).get(kernel)
    return None if e is None else float(e["fetch_bytes"]) + float(e["write_bytes"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name: str):
    from paper_1611_07289_amd import synth
    if name in ("uterus256", "sinc256"):
        return [synth.full_problem()]
    if name == "uterus384":
        # the same construction at 384^3 (4 stacks of 384 x 384 x 90)
        return [synth.full_problem(n=384, slices=90)]
    if name == "tiny32":
        return [synth.tiny_problem()]
    if name == "batched":
        return synth.batched_problems()
    if name == "diff48":
        return [synth.diff_problem()]
    if name == "learned":
        return [synth.full_problem()]
    if name == "multiscale":
        return [synth.multiscale_problem(n=128, slices=32, sizes=(32, 64))]
    raise SystemExit(f"unknown workload {name}")


def nnz_estimate(probs, n_valid, sinc=False):
    """Expected PSF support size times the valid samples: a support is the
    lattice points inside the ellipsoid of semi-axes k sigma, on average its
    volume 4/3 pi k^3 prod(sigma) over the voxel volume (k = 3); for the sinc
    PSF inside the box of half widths (w_u, w_v, k sigma_n), w = in-plane
    FWHM."""
    P = probs[0]
    vox = abs(np.linalg.det(P.grid.vox2world[:, :3]))
    fw = np.asarray(P.stacks[0].fwhm_mm, float)
    sig = fw / (2 * math.sqrt(2 * math.log(2)))
    if sinc:
        return 8.0 * fw[0] * fw[1] * 3.0 * sig[2] / vox * n_valid
    return 4.0 / 3.0 * math.pi * 27.0 * float(np.prod(sig)) / vox * n_valid


def hbm_equivalent(nnz, nnz_adj, n_valid, V, ms_step):
    """The SR iteration against the memory floor of a stored-weight design:
    the bytes such an implementation moves per iteration (the PSF weight
    lists read at 6 B per nonzero -- FP32 weight and 16-bit local index --
    forward for every valid sample and backward for those of the patches the
    EM keeps, 16 B per valid sample for y, e and its re-reads,
    32 B per voxel for X, num, den and X') over the chip's 8 TB/s, as a
    fraction of the measured iteration time.  This path stores no weights,
    so the figure is a like-for-like time budget, not a count of its own
    traffic (see roofline.traffic for that)."""
    b = (nnz + nnz_adj) * 6 + n_valid * 16 + V * 32
    floor_ms = b / (HBM_PEAK_GBS * 1e9) * 1e3
    return {"bytes_per_iteration": b, "floor_ms": floor_ms, "frac": floor_ms / ms_step}


def _oracle_sample(P, n_patch_sample: int, seed: int):
    """Seconds of one FP64 SR iteration restricted to n_patch_sample patches
    (simulate, EM, two back-projections) and of the full-volume update, and
    the valid samples of the sample."""
    import oracle
    from oracle import recon
    from oracle.update import sr_update
    from paper_1611_07289_amd import synth
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(P.M, size=min(n_patch_sample, P.M), replace=False))
    tab = P.patches.table()[sel]
    sub = synth.Patches(*[tab[:, i].copy() for i in range(6)])
    ctx = oracle.Ctx(P.grid, P.stacks, sub)
    th = P.theta_true[sel]
    X = np.asarray(P.x_true, np.float64)
    t0 = time.perf_counter()
    yh, _, val = ctx.simulate(X, th)
    y = yh * 1.01
    e = np.where(val, y - yh, 0.0)
    p, pbar, W, pi, st, _ = recon.robust_weights(e, y, val, recon.EMState(),
                                                 ctx.patch_of_sample, ctx.M)
    Ws = W[ctx.patch_of_sample]
    num = ctx.backproject(th, Ws * p * e)
    den = ctx.backproject(th, Ws * p)
    t_samples = time.perf_counter() - t0
    t1 = time.perf_counter()
    sr_update(X, num, den)
    t_volume = time.perf_counter() - t1
    return len(sel), int(val.sum()), t_samples, t_volume


def cpu_baseline(P, n_patch_sample: int = 2048, n_patch_single: int = 48):
    """FP64 oracle on a bounded sample of the same workload: one SR
    iteration restricted to n_patch_sample patches (simulate, EM, two
    back-projections) plus the update of the full volume, extrapolated to all
    patches, on all the host threads the oracle uses; and the same on one
    thread over n_patch_single patches.  Value in patch-samples/s."""
    import oracle
    cores = oracle.num_threads()
    n_sel, n_sub, t_s, t_v = _oracle_sample(P, n_patch_sample, 7)
    frac = P.M / n_sel
    t_full = t_s * frac + t_v
    out = {
        "value": n_sub * frac / t_full,
        "unit": "patch-samples/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"one FP64 SR iteration over {n_sel} of {P.M} patches "
                   f"({n_sub} valid samples; simulate, EM, 2 back-projections: "
                   f"{t_s:.1f} s) plus the full-volume update ({t_v:.1f} s) on {cores} "
                   f"threads, sample part extrapolated x{frac:.1f}"),
        "seconds_measured": t_s + t_v,
        "full_iteration_s_estimate": t_full,
    }
    oracle.set_num_threads(1)
    try:
        n1, s1, t1s, t1v = _oracle_sample(P, n_patch_single, 8)
    finally:
        oracle.set_num_threads(cores)
    f1 = P.M / n1
    out["single_core"] = {
        "value": s1 * f1 / (t1s * f1 + t1v), "cores": 1,
        "sample": (f"the same over {n1} patches ({s1} valid samples: {t1s:.1f} s) plus the "
                   f"full-volume update ({t1v:.1f} s) on one thread, extrapolated x{f1:.1f}"),
        "seconds_measured": t1s + t1v,
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uterus256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-pvr", action="store_true",
                    help="skip the whole-reconstruction comparison (plain vs learned init)")
    ap.add_argument("--learned-pairs", type=int, default=1_000_000,
                    help="training pairs of the learned initialiser for the full-PVR "
                         "comparison (0: plain reconstruction only)")
    ap.add_argument("--no-training", action="store_true",
                    help="learned workload: time inference only")
    ap.add_argument("--no-superpixel", action="store_true",
                    help="skip the superpixel-versus-square-patch reconstruction")
    ap.add_argument("--learned-seeds", default="5005:7800",
                    help="comma-separated NET:TRAIN seed pairs of the learned initialiser; "
                         "the first gives the learned runs, every pair is reported under "
                         "full_pvr.learned_seeds (the spread of the learned result)")
    ap.add_argument("--full-pvr-runs", default=None,
                    help="comma-separated subset of the whole-reconstruction runs (e.g. "
                         "plain,plain_exact), a profiling aid")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched workload: skip the one-after-another comparison")
    ap.add_argument("--fixed-launch", default=None,
                    help="batched workload: launch shapes instead of the autotuner, "
                         "'walk:G,BPG' or 'tiles:WxH,BPG'")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, see the documentation)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1611_07289_amd import pvr, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    probs = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: generated in {time.time() - t0:.1f} s")
    if args.workload == "batched":
        batched_bench(args, probs, dev)
        return
    if args.workload == "diff48":
        diff_bench(args, probs[0], dev)
        return
    if args.workload == "learned":
        learned_bench(args, probs[0], dev)
        return
    if args.workload == "multiscale":
        multiscale_bench(args, *probs[0], dev)
        return
    plan = pvr.Plan.from_problems(probs)
    sinc = args.workload == "sinc256"
    if sinc:
        plan.set_psf(pvr.PVR_PSF_SINC)
    log(f"[bench] plan: N={plan.N} M={plan.M} V={plan.V} problems={plan.P}")

    theta = torch.from_numpy(np.concatenate([P.theta_true for P in probs]).astype(np.float32)).to(dev)
    Xtrue = torch.from_numpy(np.concatenate([P.x_true.reshape(-1) for P in probs])).to(dev)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    plan.build(theta)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - tb
    log(f"[bench] build (geometry, normalisers) {t_build * 1e3:.1f} ms")

    # observations: the forward model at the true motion, then noise and
    # outlier patches drawn by the generator
    yc = torch.empty(plan.N, dtype=torch.float32, device=dev)
    plan.simulate(Xtrue, y_sim=yc)
    ych = yc.cpu().numpy()
    y_parts = []
    for b, P in enumerate(probs):
        a, z = plan.sample_off[plan_patch_begin(plan, probs, b)], plan.sample_off[plan_patch_begin(plan, probs, b + 1)]
        y_parts.append(synth.corrupt(ych[a:z], P.patches, P.outlier_patch, P.noise_frac,
                                     P.seed_base + 3, P.seed_base + 5))
    y = torch.from_numpy(np.concatenate(y_parts)).to(dev)
    del yc, ych
    # valid samples (inverse normaliser > 0)
    ones = torch.ones(plan.V, dtype=torch.float32, device=dev)
    ysim1 = torch.empty(plan.N, dtype=torch.float32, device=dev)
    plan.simulate(ones, y_sim=ysim1)
    valid = ysim1 > 0.5
    n_valid = int(valid.sum().item())
    del ysim1, ones

    e = torch.empty(plan.N, dtype=torch.float32, device=dev)
    p = torch.empty_like(e)
    pbar = torch.empty(plan.M, dtype=torch.float32, device=dev)
    W = torch.empty_like(pbar)
    num = torch.empty(plan.V, dtype=torch.float32, device=dev)
    den = torch.empty_like(num)
    em = plan.em_state()
    # initial volume X0 = A^T y / A^T 1 (the update with X = 0, lambda = 0)
    X = torch.zeros(plan.V, dtype=torch.float32, device=dev)
    Xn = torch.empty_like(X)
    # (the first back-projection after the build also builds the adjoint's
    # brick index: its extra time over a second, identical call is reported)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    plan.backproject(y, None, None, num, den)
    torch.cuda.synchronize()
    t_bp_first = time.perf_counter() - tb
    tb = time.perf_counter()
    plan.backproject(y, None, None, num, den)
    torch.cuda.synchronize()
    t_index = max(t_bp_first - (time.perf_counter() - tb), 0.0)
    info = plan.info()
    log(f"[bench] adjoint index: {t_index * 1e3:.2f} ms, sub-brick/patch pairs {info.n_bin_pairs} "
        f"(capacity {info.sub_capacity})")
    plan.sr_update(X, num, den, Xn, pvr.SRParams.make(lam=0.0, use_clamp=False))
    X, Xn = Xn, X
    prm = pvr.SRParams.make()

    def step(first=False, ev=None):
        if ev is not None:
            ev[0].record()
        plan.simulate(X_ref[0], y_obs=y, resid=e)
        if ev is not None:
            ev[1].record()
        plan.robust_weights(e, y, em, p, pbar, W,
                            (pvr.PVR_EM_INIT if first else 0) | pvr.PVR_EM_RESID_FRESH
                            | pvr.PVR_EM_PREP_ADJOINT)
        if ev is not None:
            ev[2].record()
        plan.backproject(e, p, W, num, den)
        if ev is not None:
            ev[3].record()
        plan.sr_update(X_ref[0], num, den, X_ref[1], prm)
        if ev is not None:
            ev[4].record()
        X_ref.reverse()

    X_ref = [X, Xn]
    for i in range(args.warmup):
        step(first=(i == 0))
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    plan.set_timing(True)
    for kid in (pvr.PVR_KERNEL_SIMULATE, pvr.PVR_KERNEL_BACKPROJECT):
        plan.kernel_time(kid)  # start the counts at the timed region
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(first=(args.warmup == 0 and i == 0), ev=evs[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    names = ["simulate", "robust_weights", "backproject", "sr_update"]
    per = {n: 0.0 for n in names}
    for ev in evs:
        for k, n in enumerate(names):
            per[n] += ev[k].elapsed_time(ev[k + 1])
    per = {n: v / args.steps for n, v in per.items()}
    ms_step = elapsed * 1e3 / args.steps
    value = n_valid * args.steps / elapsed
    log(f"[bench] {ms_step:.3f} ms/step, {value / 1e9:.3f} G samples/s; "
        + ", ".join(f"{n} {v:.3f} ms" for n, v in per.items()))

    # the hot kernels alone (event pairs the library records around each
    # launch on its stream during the timed steps)
    kern = {}
    for name, kid in (("k_simulate", pvr.PVR_KERNEL_SIMULATE),
                      ("k_backproject", pvr.PVR_KERNEL_BACKPROJECT)):
        tot, n = plan.kernel_time(kid)
        kern[name] = tot / max(n, 1)
    plan.set_timing(False)
    nnz = nnz_estimate(probs, n_valid, sinc)
    # the adjoint skips patches the EM excludes (W = 0): its work is the
    # nonzeros of the valid samples of the kept patches
    counts = torch.from_numpy(np.diff(plan.sample_off)).to(dev)
    kept = torch.repeat_interleave(W > 0, counts)
    n_kept = int((valid & kept).sum().item())
    del valid, kept, counts
    nnz_adj = nnz * n_kept / max(n_valid, 1)
    dom = max(kern, key=kern.get)
    if sinc:
        fpn = FLOP_PER_NNZ_SINC_FWD if dom == "k_simulate" else FLOP_PER_NNZ_SINC_ADJ
    else:
        fpn = FLOP_PER_NNZ_FWD if dom == "k_simulate" else FLOP_PER_NNZ_ADJ
    nnz_dom = nnz if dom == "k_simulate" else nnz_adj
    achieved = nnz_dom * fpn / (kern[dom] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved,
                "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS,
                "traffic": measured_traffic(dom, args.workload),
                "kernel_ms": kern[dom], "nnz_per_launch": nnz_dom, "flop_per_nnz": fpn,
                "valid_samples_kept": n_kept}

    st = pvr.Plan.read_em(em)
    out = {
        "metric": "SR-iteration patch-samples/s",
        "value": value,
        "unit": "patch-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "problems": plan.P, "patches": plan.M,
                   "samples": plan.N, "valid_samples": n_valid, "voxels": plan.V,
                   "patch": ("64x64 stride 32" if args.workload in ("uterus256", "uterus384")
                             else "mixed"),
                   "psf_fwhm_mm": [1, 1, 4], "psf": "sinc" if sinc else "gaussian",
                   "plan_device_bytes": int(plan.info().device_bytes),
                   "parallelism": "single GPU"},
        "kernels_ms": per,
        "hot_kernels_ms": kern,
        "build_ms": t_build * 1e3,
        "index_build_ms": t_index * 1e3,
        "index_pairs": {"sub_brick_patch": int(info.n_bin_pairs),
                        "capacity": int(info.sub_capacity)},
        "roofline": roofline,
        "hbm_equivalent": hbm_equivalent(nnz, nnz_adj, n_valid, plan.V, ms_step),  # same bytes per nonzero
        "em": {"sigma2": st[0].sigma2, "c": st[0].c, "excluded": st[0].n_excluded},
    }

    if not args.no_full_pvr and args.workload == "uterus256":
        seeds = [tuple(int(v) for v in kv.split(":")) for kv in args.learned_seeds.split(",")]
        out["full_pvr"] = full_pvr(plan, probs, y, Xtrue, dev, learned_pairs=args.learned_pairs,
                                   learned_seeds=seeds,
                                   only=args.full_pvr_runs.split(",") if args.full_pvr_runs
                                   else None)
    if not args.no_full_pvr and args.workload == "sinc256":
        # the sinc PSF registers with the central-difference gradient only
        out["full_pvr"] = full_pvr(plan, probs, y, Xtrue, dev, exact=False)
    if not args.no_superpixel and args.workload == "uterus256":
        out["superpixel_pvr"] = superpixel_pvr(probs[0], Xtrue, dev)

    if args.copy_calibration:
        a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = a.numel() * 4
        del a, b

    if not args.no_cpu_baseline and args.workload != "batched":
        log("[bench] timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(probs[0])
    print(json.dumps(out), flush=True)


def batched_bench(args, probs, dev):
    """Batched form: all problems in one plan, launch shapes of the two PSF
    kernels chosen by the autotuner (or given with --fixed-launch), two SR
    iterations per HIP-graph replay; the roofline of the dominant kernel from
    event pairs around eager iterations of the same plan; compared with the
    same problems run one after another, each in its own plan, eagerly
    (skipped with --no-sequential)."""
    import torch
    from paper_1611_07289_amd import autotune, pvr, synth
    from paper_1611_07289_amd.batch import GraphedSR
    plan = pvr.Plan.from_problems(probs)
    theta = torch.from_numpy(np.concatenate([P.theta_true for P in probs]).astype(np.float32)).to(dev)
    Xt = torch.from_numpy(np.concatenate([P.x_true.reshape(-1) for P in probs])).to(dev)
    plan.build(theta)
    yc = torch.empty(plan.N, dtype=torch.float32, device=dev)
    plan.simulate(Xt, y_sim=yc)
    ych = yc.cpu().numpy()
    parts = []
    for b, P in enumerate(probs):
        a = plan.sample_off[plan_patch_begin(plan, probs, b)]
        z = plan.sample_off[plan_patch_begin(plan, probs, b + 1)]
        parts.append(synth.corrupt(ych[a:z], P.patches, P.outlier_patch, P.noise_frac,
                                   P.seed_base + 3, P.seed_base + 5))
    y = torch.from_numpy(np.concatenate(parts)).to(dev)
    ones = torch.ones(plan.V, dtype=torch.float32, device=dev)
    plan.simulate(ones, y_sim=yc)
    valid = yc > 0.5
    n_valid = int(valid.sum().item())
    X0 = Xt * 0.9
    if args.fixed_launch:
        fwd, g = args.fixed_launch.split(",")
        kind, val = fwd.split(":")
        if kind == "walk":
            plan.set_tiles(0, 0)
            plan.set_granules(int(val), int(g))
        else:
            tw, th = (int(v) for v in val.split("x"))
            plan.set_granules(1, int(g))
            plan.set_tiles(tw, th)
        tuned = {"fixed": args.fixed_launch}
    else:
        tuned = autotune.tune(plan, X0, y, cache=None)
    log(f"[bench] batched: {plan.P} problems, N={plan.N} M={plan.M} V={plan.V}; launch {tuned}")
    gs = GraphedSR(plan, y, X0.clone())
    gs.start()
    gs.capture()
    pairs = max(1, args.steps // 2)
    gs.replay_pairs(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gs.replay_pairs(pairs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    it = 2 * pairs
    value = n_valid * it / el
    # kernel durations: eager iterations of the same plan with the library's
    # event pairs around the two PSF kernels
    plan.set_timing(True)
    for kid in (pvr.PVR_KERNEL_SIMULATE, pvr.PVR_KERNEL_BACKPROJECT):
        plan.kernel_time(kid)
    for k in range(4):
        gs._iter(gs.X, gs.Xn) if k % 2 == 0 else gs._iter(gs.Xn, gs.X)
    kern = {}
    for name, kid in (("k_simulate", pvr.PVR_KERNEL_SIMULATE),
                      ("k_backproject", pvr.PVR_KERNEL_BACKPROJECT)):
        tot, n = plan.kernel_time(kid)
        kern[name] = tot / max(n, 1)
    plan.set_timing(False)
    nnz = nnz_estimate(probs, n_valid)
    counts = torch.from_numpy(np.diff(plan.sample_off)).to(dev)
    n_kept = int((valid & torch.repeat_interleave(gs.W > 0, counts)).sum().item())
    nnz_adj = nnz * n_kept / max(n_valid, 1)
    dom = max(kern, key=kern.get)
    fpn = FLOP_PER_NNZ_FWD if dom == "k_simulate" else FLOP_PER_NNZ_ADJ
    nnz_dom = nnz if dom == "k_simulate" else nnz_adj
    achieved = nnz_dom * fpn / (kern[dom] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved,
                "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                "kernel_ms": kern[dom], "nnz_per_launch": nnz_dom, "flop_per_nnz": fpn,
                "valid_samples_kept": n_kept}
    out = {
        "metric": "SR-iteration patch-samples/s (batched, graph)",
        "value": value, "unit": "patch-samples/s", "n_gpus": 1, "steps": it,
        "warmup": 2, "ms_per_step": el * 1e3 / it, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched", "problems": plan.P, "patches": plan.M,
                   "samples": plan.N, "valid_samples": n_valid, "voxels": plan.V,
                   "sizes": [P.grid.nx for P in probs],
                   "stacks": [len(P.stacks) for P in probs], "parallelism": "single GPU"},
        "launch": tuned, "hot_kernels_ms": kern, "roofline": roofline,
    }
    if not args.no_sequential:
        # the same problems one after another, eagerly, each in its own plan
        seq_t = 0.0
        for b, P in enumerate(probs):
            pl = pvr.Plan.from_problems([P])
            pl.build(torch.from_numpy(P.theta_true.astype(np.float32)).to(dev))
            a = plan.sample_off[plan_patch_begin(plan, probs, b)]
            z = plan.sample_off[plan_patch_begin(plan, probs, b + 1)]
            yb = y[a:z].contiguous()
            g1 = GraphedSR(pl, yb, torch.from_numpy(P.x_true.reshape(-1) * 0.9).to(dev))
            g1.start()
            g1._iter(g1.X, g1.Xn)
            g1._iter(g1.Xn, g1.X)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(pairs):
                g1._iter(g1.X, g1.Xn)
                g1._iter(g1.Xn, g1.X)
            torch.cuda.synchronize()
            seq_t += time.perf_counter() - t1
            pl.close()
        out["sequential_ms_per_step"] = seq_t * 1e3 / it
        out["speedup_vs_sequential"] = seq_t / el
    print(json.dumps(out), flush=True)


def diff_bench(args, P, dev):
    """Differentiable simulation on the 48^3 case: one forward + backward of
    the autograd function (y = A(theta) X, then d/dX and d/dtheta of a scalar
    loss) per step, FP64 and FP32."""
    import torch
    from paper_1611_07289_amd import pvr
    from paper_1611_07289_amd.autograd import simulate
    plan = pvr.Plan.from_problems([P], f64=True)
    res = {}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        X = torch.tensor(P.x_true.reshape(-1), dtype=dt, device=dev, requires_grad=True)
        th = torch.tensor(P.theta_true, dtype=dt, device=dev, requires_grad=True)
        g = torch.randn(plan.N, dtype=dt, device=dev, generator=torch.Generator(device=dev).manual_seed(1))

        def one():
            X.grad = None
            th.grad = None
            (simulate(X, th, plan) * g).sum().backward()

        for _ in range(args.warmup):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one()
        torch.cuda.synchronize()
        res[name] = args.steps / (time.perf_counter() - t0)
        log(f"[bench] diff48 {name}: {res[name]:.1f} gradient evaluations/s")
    out = {"metric": "gradient evaluations/s (forward + d/dX + d/dtheta)", "value": res["f32"],
           "unit": "evaluations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 / res["f32"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "diff48", "patches": plan.M, "samples": plan.N,
                      "voxels": plan.V, "parallelism": "single GPU"},
           "f64_evaluations_per_s": res["f64"]}
    print(json.dumps(out), flush=True)


def learned_bench(args, P, dev):
    """The learned initialiser's network on MFMA: inference over all 11 760
    patches of the uterus workload and training steps (forward, backward,
    Adam) at batch 256; TFLOP/s against the dense BF16 MFMA peak."""
    import torch
    from paper_1611_07289_amd import learned, pvr, synth
    plan = pvr.Plan.from_problems([P])
    X = torch.from_numpy(P.x_true.reshape(-1)).to(dev)
    ref = torch.from_numpy(P.theta_true.astype(np.float32)).to(dev)
    off = torch.from_numpy(synth.random_motion_batch(plan.M, 10.0, 5.0, 77).astype(np.float32)).to(dev)
    y_obs, y_sim = learned.make_pairs(plan, X, ref, off, 0.01 * float(X.max()), 78)
    net = learned.Net(seed=5)
    flop_fwd = 2 * learned.macs_per_pair()
    # inference, batches of 1024
    B = 1024
    ids = torch.arange(plan.M, dtype=torch.int32, device=dev)

    def infer():
        for b0 in range(0, plan.M, B):
            n = min(B, plan.M - b0)
            net.predict(plan, y_obs, y_sim, ids[b0:b0 + n].contiguous(), n)

    infer()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infer()
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / args.steps
    tf_inf = flop_fwd * plan.M / t_inf / 1e12
    gbs_inf = learned.activation_bytes_per_pair() * plan.M / t_inf / 1e9
    # training steps
    Bt = 256
    if args.no_training:
        log(f"[bench] learned: inference {plan.M / t_inf:.0f} pairs/s ({tf_inf:.1f} TFLOP/s)")
        return
    tgt = torch.zeros(Bt * 6, device=dev)
    bf = net.buffers(Bt)
    bf["ids"].copy_(ids[:Bt])
    net.pack(plan, bf["ids"], y_obs, y_sim, Bt)

    def train_step():
        net.forward(Bt, tgt)
        net.backward(Bt)
        net.adam(1e-4)

    train_step()
    torch.cuda.synchronize()
    n_tr = 20 * args.steps
    t0 = time.perf_counter()
    for _ in range(n_tr):
        train_step()
    torch.cuda.synchronize()
    t_tr = (time.perf_counter() - t0) / n_tr
    tf_tr = 3 * flop_fwd * Bt / t_tr / 1e12
    log(f"[bench] learned: inference {plan.M / t_inf:.0f} pairs/s ({tf_inf:.1f} TFLOP/s), "
        f"training {Bt / t_tr:.0f} pairs/s ({tf_tr:.1f} TFLOP/s)")
    out = {"metric": "learned-initialiser inference pairs/s (BF16 MFMA)", "value": plan.M / t_inf,
           "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": t_inf * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "learned", "pairs_per_step": plan.M, "batch": B,
                      "parallelism": "single GPU"},
           # at 64x64 inputs and <= 64 channels the network moves more bytes
           # than the matrix cores need time for (~110 flop per byte against
           # the chip's ~310), so the HBM roofline bounds inference; MFMA
           # utilisation is reported beside it
           "roofline": {"bound": "hbm", "achieved": gbs_inf, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": gbs_inf / HBM_PEAK_GBS, "traffic": None,
                        "bytes_per_pair": learned.activation_bytes_per_pair()},
           "mfma": {"achieved_tflops": tf_inf, "peak_tflops": BF16_MFMA_PEAK_TFLOPS,
                    "utilisation": tf_inf / BF16_MFMA_PEAK_TFLOPS},
           "training": {"pairs_per_s": Bt / t_tr, "tflops": tf_tr,
                        "frac": tf_tr / BF16_MFMA_PEAK_TFLOPS, "batch": Bt}}
    print(json.dumps(out), flush=True)


def multiscale_bench(args, P, scale, dev):
    """Multi-scale patches: whole reconstructions (3 cycles x 10 SR
    iterations from zero motion) with the 64-pixel patches only, and with the
    scales alternating cycle by cycle (32, 64, 32), in one plan holding both."""
    import torch
    from paper_1611_07289_amd import driver, pvr, synth
    plan = pvr.Plan.from_problems([P])
    th = torch.from_numpy(P.theta_true.astype(np.float32)).to(dev)
    Xt = torch.from_numpy(P.x_true.reshape(-1)).to(dev)
    plan.build(th)
    yc = torch.empty(plan.N, dtype=torch.float32, device=dev)
    plan.simulate(Xt, y_sim=yc)
    y = torch.from_numpy(synth.corrupt(yc.cpu().numpy(), P.patches, P.outlier_patch, 0.01,
                                       P.seed_base + 3, P.seed_base + 5)).to(dev)
    masks = [torch.from_numpy((scale == k).astype(np.uint8)).to(dev) for k in (0, 1)]
    res = {}
    for name, sched in (("single_64", [masks[1]]), ("alternating_32_64", [masks[0], masks[1]])):
        th0 = torch.zeros(plan.M, 6, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, _, hist = driver.reconstruct(plan, y, th0, cycles=3, n_sr=10, active_schedule=sched)
        torch.cuda.synchronize()
        res[name] = {"seconds": time.perf_counter() - t0, "psnr_db": driver.psnr(X, Xt, plan),
                     "timings": hist["timings"]}
        log(f"[bench] multiscale {name}: {res[name]['seconds']:.2f} s, PSNR {res[name]['psnr_db']:.2f} dB")
    out = {"metric": "full PVR seconds (multi-scale schedule vs single scale)",
           "value": res["alternating_32_64"]["seconds"], "unit": "s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": res["alternating_32_64"]["seconds"] * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "multiscale", "voxels": plan.V, "patches": plan.M,
                      "patches_32": int((scale == 0).sum()), "patches_64": int((scale == 1).sum()),
                      "parallelism": "single GPU"},
           "runs": res}
    print(json.dumps(out), flush=True)


def plan_patch_begin(plan, probs, b):
    return int(sum(P.M for P in probs[:b]))


# Algorithmic FP32 work of a registration evaluation per PSF nonzero of a
# walked sample: plain NCC evaluation as the forward walk (16); exact
# gradient: the forward walk plus the accumulation of the weight's nine
# offset moments of e^-Q/2 (X - X_b) and of e^-Q/2 (8 more: the two products
# em (X - X_b) and em wc, and six sums); per walked sample the NCC sums
# (plain 10; exact 10 + the six derivatives from the moments and their
# three sums each, 100).
FLOP_PER_NNZ_REG = 16
FLOP_PER_NNZ_REG_EXACT = 24
FLOP_PER_SAMPLE_REG = 10
FLOP_PER_SAMPLE_REG_EXACT = 100


def register_roofline(stats, reg_ms, nnz_per_sample):
    """Algorithmic FP32 rate of the registration kernel over a run: the
    samples its NCC evaluations walked (counted by the kernel) times the work
    per walked sample, over the summed duration of its launches."""
    flop = (stats["samples"] * (nnz_per_sample * FLOP_PER_NNZ_REG + FLOP_PER_SAMPLE_REG)
            + stats["samples_exact"] * (nnz_per_sample * FLOP_PER_NNZ_REG_EXACT
                                        + FLOP_PER_SAMPLE_REG_EXACT))
    ach = flop / max(reg_ms * 1e-3, 1e-12) / 1e12
    return {"bound": "alu", "kernel": "k_register", "achieved": ach,
            "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TFLOPS,
            "kernel_ms": reg_ms, "work": stats, "nnz_per_sample": nnz_per_sample}


def full_pvr(plan, probs, y, Xtrue, dev, cycles=3, n_sr=10, learned_pairs=0, exact=True,
             tight=(0.25, 5), fallback_tau=0.3, only=None, learned_seeds=((5005, 7800),)):
    """Seconds and PSNR of a whole reconstruction from the motion-corrupted
    start (zero motion), each with its registration kernel's time, work and
    roofline: plain registration with the full budget (step0 1, 40 trial
    steps) and with a tight one (step0 and trial steps of `tight`,
    "_tight"), the control of the learned runs; with learned_pairs > 0 the
    learned initialiser (trained first, on a phantom of another seed) whose
    prediction the tight budget refines, except where the patch's NCC after
    the prediction stays below fallback_tau: there plain registration takes
    over with the full budget from the motion before the prediction; and
    (exact only) the
    joint gradient-based registration through the differentiable forward
    model (driver.register_gradient) in place of the per-patch one.  `only`,
    when given, names the runs to make (a profiling aid).  Every (network,
    training) seed pair of `learned_seeds` trains its own network; the first
    gives the "learned" runs, and all are listed under "learned_seeds"."""
    import torch
    from paper_1611_07289_amd import driver, learned, pvr, synth
    res = {}
    ymax = float(y.abs().max())
    nnz_ps = nnz_estimate(probs, 1)

    def run(key, rp, init_fn=None, register_fn=None):
        if only and key.split("@")[0] not in only:
            return
        th0 = torch.zeros(plan.M, 6, dtype=torch.float32, device=dev)
        plan.set_timing(True)
        plan.kernel_time(pvr.PVR_KERNEL_REGISTER)
        plan.reg_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, th, hist = driver.reconstruct(
            plan, y, th0, cycles=cycles, n_sr=n_sr, reg_params=rp, init_fn=init_fn,
            fallback_tau=fallback_tau if init_fn is not None else None,
            fallback_params=pvr.RegParams.make(min_std=0.01 * ymax, exact=rp.gradient == 1),
            register_fn=register_fn)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        reg_ms, n_reg = plan.kernel_time(pvr.PVR_KERNEL_REGISTER)
        stats = plan.reg_stats()
        plan.set_timing(False)
        for kid in (pvr.PVR_KERNEL_SIMULATE, pvr.PVR_KERNEL_BACKPROJECT):
            plan.kernel_time(kid)
        res[key] = {"seconds": sec, "psnr_db": driver.psnr(X, Xtrue, plan),
                    "timings": hist["timings"], "mean_ncc": hist["ncc"],
                    "register_launches": n_reg}
        if init_fn is not None:
            res[key]["fallback_patches"] = hist["fallback"]
        if register_fn is None:
            res[key]["register_roofline"] = register_roofline(stats, reg_ms, nnz_ps)
        log(f"full PVR {key}: {sec:.3f} s, PSNR {res[key]['psnr_db']:.2f} dB"
            + (f", registration kernel {reg_ms:.1f} ms "
               f"({res[key]['register_roofline']['frac']:.3f} of the FP32 ALU peak)"
               if register_fn is None else "")
            + (f", fallback {hist['fallback']}" if init_fn is not None else ""))

    full = dict(min_std=0.01 * ymax)
    short = dict(step0=tight[0], max_iter=tight[1], min_std=0.01 * ymax)
    # central-difference gradient (12 NCC evaluations per gradient), then the
    # exact gradient (one evaluation)
    run("plain", pvr.RegParams.make(**full))
    run("plain_tight", pvr.RegParams.make(**short))
    if exact:
        run("plain_exact", pvr.RegParams.make(**full, exact=True))
        run("plain_tight_exact", pvr.RegParams.make(**short, exact=True))

        def joint(pl, X, yy, th, ncc, act, mask):
            ncc.copy_(driver.register_gradient(pl, X, yy, th, iters=30, min_std=0.01 * ymax,
                                               active=act, mask=mask))
        run("joint_gradient", pvr.RegParams.make(**full), register_fn=joint)
    if learned_pairs > 0 and exact and (not only or any(k.startswith("learned") for k in only)):
        P = probs[0]
        Xtr = torch.from_numpy(synth.phantom_uterus(P.grid.nx, 7700, 7701).reshape(-1)).to(dev)
        res["learned_seeds"] = []
        for i, (net_seed, train_seed) in enumerate(learned_seeds):
            net = learned.Net(seed=net_seed)
            tr = learned.train(net, plan, [Xtr], n_pairs=learned_pairs, batch=256, lr=1e-3,
                               seed=train_seed, log=log)
            init_fn = learned.init_fn_factory(net)
            sfx = "" if i == 0 else f"@{net_seed}"
            run("learned" + sfx, pvr.RegParams.make(**short), init_fn)
            run("learned_exact" + sfx, pvr.RegParams.make(**short, exact=True), init_fn)
            if i == 0:
                res["training"] = {"pairs": tr["pairs"], "seconds": tr["seconds"],
                                   "data_seconds": tr["data_seconds"],
                                   "loss_first_last": [tr["loss"][0][1], tr["loss"][-1][1]]
                                   if tr["loss"] else None}
            entry = {"net_seed": net_seed, "train_seed": train_seed}
            for k in ("learned", "learned_exact"):
                if k + sfx in res:
                    r = res[k + sfx] if i == 0 else res.pop(k + sfx)
                    entry[k] = {"seconds": r["seconds"], "psnr_db": r["psnr_db"]}
            res["learned_seeds"].append(entry)
        del Xtr
        for sfx in ("", "_exact"):
            if any(k + sfx not in res for k in ("learned", "plain", "plain_tight")):
                continue
            lr_, pl_, pt_ = res["learned" + sfx], res["plain" + sfx], res["plain_tight" + sfx]
            res["learned_vs_plain" + sfx] = {
                "delta_psnr_db": lr_["psnr_db"] - pl_["psnr_db"],
                "speedup": pl_["seconds"] / lr_["seconds"]}
            res["learned_vs_plain_tight" + sfx] = {
                "delta_psnr_db": lr_["psnr_db"] - pt_["psnr_db"],
                "speedup": pt_["seconds"] / lr_["seconds"]}
    res["budgets"] = {"full": {"step0": 1.0, "max_iter": 40},
                      "tight": {"step0": tight[0], "max_iter": tight[1]}}
    res["fallback_tau"] = fallback_tau
    res["cycles"] = cycles
    res["sr_iterations"] = n_sr
    res["paper_runtime_s"] = "2000-4000 (whole PVR, unspecified NVIDIA GPU machines; Sec. V)"
    return res


def superpixel_pvr(P, Xtrue, dev, sizes=((32, 19), (64, 38)), cycles=3, n_sr=10,
                   max_rot_deg=4.0, max_trans_mm=4.0, square=True, ms_schedule=(32, 64, 32)):
    """Square versus superpixel patches on the same observed slices (paper
    Sec. II "Patch Extraction").  Every slice of the four stacks is simulated
    whole under its own rigid motion about the slice centre (<= max_rot_deg,
    <= max_trans_mm), with 1 % noise; square patches (64x64, stride 32) and
    SLIC superpixels (step a, dilation gamma = 60 % of a, compactness t0 = 40
    adapting per superpixel, t_min = 5, 10 iterations) for every (a, gamma) in
    `sizes` are cut from these slices, and each set is reconstructed from zero
    motion with exact registration; then all sizes together in one plan as
    multi-scale superpixels, cycle c using the size ms_schedule[c], and the
    square patches of the same sizes (stride a/2) on the same schedule.  Overlapping patches share their pixels'
    noise here (unlike the per-patch observations of the main workload), so
    the PSNR ceiling is lower."""
    import torch
    from paper_1611_07289_amd import driver, pvr, superpixel, synth
    ns = sum(s.nslices for s in P.stacks)
    h, w = P.stacks[0].ny, P.stacks[0].nx
    whole = synth.square_patches(P.stacks, max(h, w), max(h, w))
    assert whole.M == ns and int(whole.w[0]) == w and int(whole.h[0]) == h
    plan_sl = pvr.Plan([P.grid], [P.stacks], [whole])
    th_sl = synth.random_motion(ns, max_rot_deg, max_trans_mm, P.seed_base + 40)
    plan_sl.build(torch.from_numpy(th_sl.astype(np.float32)).to(dev))
    ysl = torch.empty(plan_sl.N, dtype=torch.float32, device=dev)
    plan_sl.simulate(Xtrue, y_sim=ysl)
    ych = synth.corrupt(ysl.cpu().numpy(), whole, np.zeros(ns, bool), 0.01, P.seed_base + 41,
                        P.seed_base + 42)
    img = torch.from_numpy(ych).to(dev).reshape(ns, h, w)
    del plan_sl, ysl, ych
    image_of = np.zeros(len(P.stacks) + 1, np.int64)
    image_of[1:] = np.cumsum([s.nslices for s in P.stacks])
    iss = np.array([(si, k) for si, s in enumerate(P.stacks) for k in range(s.nslices)], np.int32)
    res = {"slices": ns,
           "slice_motion": f"<= {max_rot_deg:g} deg, <= {max_trans_mm:g} mm per slice"}

    def recon(key, patches, y, mask, schedule=None):
        plan = pvr.Plan([P.grid], [P.stacks], [patches])
        ymax = float(y.abs().max())
        th0 = torch.zeros(plan.M, 6, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, th, hist = driver.reconstruct(plan, y, th0, cycles=cycles, n_sr=n_sr,
                                         reg_params=pvr.RegParams.make(min_std=0.01 * ymax,
                                                                       exact=True),
                                         sample_mask=mask, active_schedule=schedule)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        n_in = plan.N if mask is None else int(mask.sum())
        res[key] = {"patches": plan.M, "samples": plan.N, "samples_in_patches": n_in,
                    "seconds": sec, "psnr_db": driver.psnr(X, Xtrue, plan),
                    "timings": hist["timings"]}
        log(f"superpixel_pvr {key}: M={plan.M} N={plan.N} {sec:.3f} s, "
            f"PSNR {res[key]['psnr_db']:.2f} dB")
        del plan

    if square:
        # square patches: the pack call with one label covering every slice
        zero = torch.zeros(ns, h, w, dtype=torch.int32, device=dev)

        def cut(sq):
            tab = np.column_stack([image_of[sq.stack] + sq.slice, np.zeros(sq.M, np.int32),
                                   sq.x0, sq.y0, sq.w, sq.h]).astype(np.int32)
            return superpixel.pack(img, zero, 0, tab)[0]

        sq = synth.square_patches(P.stacks, 64, 32)
        recon("square", sq, cut(sq), None)
        if ms_schedule:
            # multi-scale squares of the same two scales (a, stride a/2),
            # the same schedule
            sizes_sq = sorted(set(ms_schedule))
            parts = [synth.square_patches(P.stacks, a, a // 2) for a in sizes_sq]
            both = synth.concat_patches(parts)
            scale = np.concatenate([np.full(q.M, i, np.uint8) for i, q in enumerate(parts)])
            act = {a: torch.from_numpy((scale == i).astype(np.uint8)).to(dev)
                   for i, a in enumerate(sizes_sq)}
            recon("square_ms", both, cut(both), None, schedule=[act[a] for a in ms_schedule])
            res["square_ms"]["schedule_a"] = list(ms_schedule)
        del zero
    extracted = {}
    for a, gamma in sizes:
        key = f"superpixel_a{a}"
        superpixel.superpixel_patches(img[:4], a, gamma, 40.0, 5.0, 10, iss[:4])  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cols, y_sp, m_sp, tab, lab, C = superpixel.superpixel_patches(img, a, gamma, 40.0, 5.0,
                                                                      10, iss)
        torch.cuda.synchronize()
        ext = (time.perf_counter() - t0) * 1e3
        recon(key, synth.Patches(**{k: np.asarray(v, np.int32) for k, v in cols.items()}),
              y_sp, m_sp)
        res[key].update({"a": a, "gamma": gamma, "extraction_ms": ext})
        if square:
            res[key]["delta_psnr_db"] = res[key]["psnr_db"] - res["square"]["psnr_db"]
            res[key]["speedup"] = res["square"]["seconds"] / res[key]["seconds"]
        extracted[a] = (cols, y_sp, m_sp)
        del lab, C
    # multi-scale superpixels (paper Sec. II, eq. Y_i over superpixel sizes):
    # every size's patches in one plan, each cycle registering and
    # reconstructing from one size (schedule `ms_schedule`, sizes in order)
    if ms_schedule and all(a in extracted for a in ms_schedule):
        sizes_ms = sorted(set(ms_schedule))
        cols = {k: np.concatenate([np.asarray(extracted[a][0][k], np.int32) for a in sizes_ms])
                for k in ("stack", "slice", "x0", "y0", "w", "h")}
        y_ms = torch.cat([extracted[a][1] for a in sizes_ms])
        m_ms = torch.cat([extracted[a][2] for a in sizes_ms])
        scale = np.concatenate([np.full(len(extracted[a][0]["x0"]), i, np.uint8)
                                for i, a in enumerate(sizes_ms)])
        act = {a: torch.from_numpy((scale == i).astype(np.uint8)).to(dev)
               for i, a in enumerate(sizes_ms)}
        key = "superpixel_ms"
        recon(key, synth.Patches(**cols), y_ms, m_ms,
              schedule=[act[a] for a in ms_schedule])
        res[key]["schedule_a"] = list(ms_schedule)
        if square:
            ref = "square_ms" if "square_ms" in res else "square"
            res[key]["delta_psnr_db_vs_" + ref] = res[key]["psnr_db"] - res[ref]["psnr_db"]
            res[key]["speedup_vs_" + ref] = res[ref]["seconds"] / res[key]["seconds"]
    return res


if __name__ == "__main__":
    main()
