/*
 * pvr.h -- C ABI of the MI355X (gfx950) patch-to-volume reconstruction
 * hot path.  Method: Alansary, Kainz et al., "PVR: Patch-to-Volume
 * Reconstruction for Large Area Motion Correction of Fetal MRI",
 * arXiv 1611.07289.
 *
 * The library reconstructs one or more independent volumes X from many
 * overlapping 2D patches cut out of stacks of slices, each patch moved by its
 * own rigid transform (Sec. II, eq. for Y = {y_s}).  It exposes the steps of
 * one super-resolution (SR) iteration and the per-patch registration:
 *
 *   pvr_plan_build        per-patch motion geometry, PSF normalisers and the
 *                         brick -> patch index used by the adjoint
 *   pvr_simulate          y_hat = A X, residual e = y - y_hat
 *                         (observation model x_i = W_i y + n_i,
 *                         W_i = D B T_i, Sec. I eq. (1))
 *   pvr_backproject       num = A^T(W p e), den = A^T(W p), a gather
 *                         (every voxel sums over the samples whose PSF
 *                         covers it; no atomics, fixed summation order)
 *   pvr_robust_weights    EM outlier model: m = 1/(max e - min e), inlier
 *                         posterior p, patch potential p_bar, patch
 *                         classification W, M-step for sigma^2 and c
 *                         (Sec. II "EM-Based Outlier Removal")
 *   pvr_sr_update         X' = max(clamp, X + a num/den + a l R(X)) with an
 *                         edge-preserving 26-neighbour regulariser
 *                         (Sec. II gradient-descent SR; anisotropic
 *                         diffusion of the cited method, Sec. I-A)
 *   pvr_register_patches  per-patch rigid 2D-3D registration maximising the
 *                         cross-correlation of Sec. IV-A eq. CC
 *                         (Sec. II "Patch to Volume Registration",
 *                         Sec. III parallelisation level I)
 *
 * Conventions
 *  - Pointers are DEVICE pointers unless marked (host).  The caller owns all
 *    device memory: every buffer passed in and the plan's workspace, which
 *    the caller allocates at the size pvr_plan_workspace_size reports and
 *    hands over with pvr_plan_attach.  The library allocates no device
 *    memory; it keeps the host descriptors it is given (copied), a second
 *    stream and two events per plan.  Device arrays are aligned to their
 *    element size (FP32 and int32 4 bytes, FP64 and pvr_em_state 8); a
 *    misaligned pointer gives PVR_EINVAL.
 *  - Calls are asynchronous on `stream` except where noted.  A plan is used on
 *    one stream at a time (thread-compatible, not thread-safe).
 *  - Every function returns a pvr_status; no exception crosses the ABI.  On
 *    error pvr_last_error() returns a message (thread-local, valid until the
 *    next call on the same thread).  Invalid arguments are rejected before any
 *    launch.
 *  - Volume layout: problem b occupies X[vol_off[b] .. vol_off[b+1]) with voxel
 *    (i, j, k) at vol_off[b] + (k*ny + j)*nx + i.  Sample layout: patch s
 *    occupies samples [sample_off[s], sample_off[s+1]) row-major inside the
 *    patch.  Both offset tables come from pvr_plan_offsets.
 *  - Motion theta: [M][6] = (rx, ry, rz [rad], tx, ty, tz [mm]);
 *    R = Rz Ry Rx; a patch rotates about its centre c_s:
 *    x = R (P - c_s) + c_s + t.
 *  - PSF: Gaussian along the moved stack axes with the stack's FWHMs,
 *    support sum (d_a/sigma_a)^2 <= k^2, weight exp(-Q/2) - exp(-k^2/2)
 *    (continuous at the cut-off), normalised over in-volume voxels.  A sample
 *    is valid iff its moved centre lies in [-1/2, n-1/2)^3, its normaliser is
 *    positive, its mask byte is non-zero and its patch is active; invalid
 *    samples simulate to 0 and contribute nothing.
 */
#ifndef PVR_H
#define PVR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest number of patches of one problem (the patch classification of a
 * problem runs in one workgroup: its potentials sit in LDS up to 12288
 * patches, beyond that in the plan's scratch array). */
#define PVR_MAX_PROBLEM_PATCHES (1 << 20)

typedef enum {
  PVR_OK = 0,
  PVR_EINVAL = 1,       /* null / inconsistent argument */
  PVR_ESHAPE = 2,       /* sizes or layouts do not fit */
  PVR_ENOMEM = 3,       /* device allocation failed */
  PVR_EHIP = 4,         /* a HIP runtime call failed (message attached) */
  PVR_ENUMERIC = 5,     /* non-finite input detected */
  PVR_EUNSUPPORTED = 6  /* valid request the library does not implement */
} pvr_status;

/* Volume grid of one reconstruction: voxel index -> world mm affine, row-major
 * 3x4.  The three linear columns must be linearly independent. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t pad_;
  double vox2world[12];
} pvr_grid;

/* A stack of 2D slices (Sec. I: LR images; Sec. II: input stacks).
 * pix2world maps (u, v, slice) to world mm, row-major 3x4; its three linear
 * columns must be mutually orthogonal (in-plane axes x spacing, slice normal x
 * slice spacing).  fwhm_mm: PSF full widths at half maximum along the
 * in-plane x, in-plane y and normal axes. */
typedef struct {
  int32_t problem;          /* reconstruction this stack belongs to */
  int32_t nx, ny, nslices;
  double pix2world[12];
  double fwhm_mm[3];
} pvr_stack;

/* A rectangular patch y_s (Sec. II "Patch Extraction": square patches of size
 * a, stride omega) on one slice: pixels (x0+u, y0+v, slice), u < w, v < h. */
typedef struct {
  int32_t stack, slice, x0, y0, w, h;
} pvr_patch;

typedef struct {
  int64_t n_samples;        /* N = sum over patches of w*h */
  int64_t n_voxels;         /* total over problems */
  int32_t n_patches;        /* M */
  int32_t n_problems;
  int32_t n_stacks;
  int32_t n_bricks;         /* 8x8x8 voxel bricks over all problems */
  int64_t n_bin_pairs;      /* sub-brick/patch pairs of the adjoint's index
                               (0 until a back-projection built it) */
  int64_t device_bytes;     /* bytes of the attached workspace (0 if none) */
  int64_t bin_capacity;     /* brick/patch pairs the workspace holds */
  int64_t sub_capacity;     /* sub-brick/patch pairs the workspace holds */
} pvr_plan_sizes;

/* EM state of one reconstruction, kept on the device so that an SR iteration
 * needs no host round trip (one entry per problem, caller-allocated). */
typedef struct {
  double sigma2;            /* inlier variance sigma^2 */
  double c;                 /* inlier proportion c */
  double m;                 /* outlier density of the last E-step */
  double y_abs_max;         /* max |y| over valid samples */
  double sum_wp, sum_wpe2, sum_w;  /* M-step sums of the last iteration */
  int32_t n_used;           /* patches entering the patch classification */
  int32_t n_excluded;       /* patches with W = 0 among them */
  int32_t started;          /* sigma2 / c hold a value */
  int32_t pad_;
} pvr_em_state;

/* pvr_robust_weights flags */
#define PVR_EM_INIT  1      /* start of a cycle: sigma^2 = mean(e^2), c = 0.9 */
#define PVR_EM_FIX_W 2      /* use patch_w as given instead of classifying */
#define PVR_EM_RESID_FRESH 4 /* resid (with y_obs) is exactly what the plan's last
                                pvr_simulate wrote, unmodified: its residual
                                statistics, reduced by the forward kernel, are
                                reused instead of a pass over resid (the
                                library also checks the two pointers; with a
                                mismatch, LDS-tiled simulation or a build in
                                between it passes over resid as usual) */
#define PVR_EM_PREP_ADJOINT 8 /* also prepare the adjoint's per-sample inputs
                                 (p e / Z, p / Z) for a pvr_backproject(resid,
                                 p, patch_w, ...) that follows with these same
                                 resid and p buffers, unmodified: the
                                 preparation runs on the plan's second stream
                                 while the patch classification runs on
                                 `stream` (joined before the call returns on
                                 `stream`), and pvr_backproject skips its own
                                 pass.  Needs p != NULL; a pvr_simulate or a
                                 build in between cancels it */

typedef struct {
  float alpha;              /* step length (default 1) */
  float lambda;             /* regularisation weight (default 0.02) */
  float delta;              /* edge threshold of the diffusion (default 150) */
  float clamp_min;          /* lower bound of X' (default 0) */
  float den_eps;            /* voxels with den <= den_eps get no data step */
  int32_t use_clamp;        /* 1: apply clamp_min */
} pvr_sr_params;

typedef struct {
  double step0;             /* initial / largest step (default 1.0) */
  double step_min;          /* stop when the step falls below (0.01) */
  double fd_h;              /* central-difference step (0.05) */
  double min_std;           /* patches with std(y) below keep theta */
  int32_t max_iter;         /* trial steps (40) */
  int32_t gradient;         /* PVR_REG_GRAD_FD (0, default) or PVR_REG_GRAD_EXACT */
} pvr_reg_params;

/* Gradient of the registration optimiser: central differences of the NCC
 * with step fd_h (12 NCC evaluations), or the exact derivative of the NCC
 * through every PSF weight of the simulated patch (one evaluation that walks
 * each sample's support twice; fd_h is then unused). */
#define PVR_REG_GRAD_FD 0
#define PVR_REG_GRAD_EXACT 1

typedef struct pvr_plan pvr_plan;

/* Thread-local text of the last error. */
const char *pvr_last_error(void);

/* Library version string. */
const char *pvr_version(void);

/* Create a plan (host work only: the problem, stack and patch tables of
 * Sec. II "Patch Extraction", the forward work list and the capacity of the
 * adjoint's index).  All arrays are (host) and copied.  Patches must
 * reference valid stacks and lie inside their slice; every stack names a
 * valid problem.  cutoff_k: PSF support radius in standard deviations (> 0,
 * default 3).  No HIP call is made; the plan is usable once a workspace is
 * attached.
 * Errors: PVR_EINVAL for null pointers or out-of-range indices, PVR_ESHAPE
 * for non-orthogonal stack axes, empty sizes, a grid beyond 2^28 voxels, a
 * problem with more than PVR_MAX_PROBLEM_PATCHES patches, or a patch beyond
 * 32767 pixels per side or 2^26 pixels. */
pvr_status pvr_plan_create(const pvr_grid *grids, int32_t n_problems,
                           const pvr_stack *stacks, int32_t n_stacks,
                           const pvr_patch *patches, int32_t n_patches,
                           double cutoff_k, pvr_plan **out);

/* Workspace flags: PVR_WS_F64 adds room for the FP64 calls (the FP64
 * normalisers of pvr_plan_build_f64 and the FP64 adjoint inputs; 24 bytes
 * per sample). */
#define PVR_WS_F64 1

/* (host) Bytes of device workspace the plan needs with `flags`: its device
 * tables, the per-build motion state, the adjoint's brick index at a
 * capacity bounded over every motion (so no build reads a count back or
 * grows a list), and per-sample / per-patch scratch. */
pvr_status pvr_plan_workspace_size(const pvr_plan *plan, int32_t flags, size_t *bytes);

/* Hand the plan its workspace: `bytes` >= pvr_plan_workspace_size(flags),
 * 256-byte aligned, on the current device (the plan stays on the device of
 * its first workspace; the first attach also creates the plan's second
 * stream and its events).  The plan's tables are uploaded on `stream`,
 * which is synchronised before the call returns.  The workspace must stay allocated until the plan is
 * destroyed (or another workspace is attached, which synchronises `stream`
 * first); the plan then counts as unbuilt.  Errors: PVR_EINVAL (NULL,
 * misaligned, unknown flags, wrong device), PVR_ESHAPE (too small),
 * PVR_EHIP. */
pvr_status pvr_plan_attach(pvr_plan *plan, void *workspace, size_t bytes, int32_t flags,
                           hipStream_t stream);

/* Free a plan (NULL is a no-op).  Synchronises the device first when a
 * workspace is attached; the caller may free the workspace afterwards. */
void pvr_plan_destroy(pvr_plan *plan);

/* (host) sizes.  Synchronises the device to read n_bin_pairs when the
 * adjoint's index is built. */
pvr_status pvr_plan_info(const pvr_plan *plan, pvr_plan_sizes *out);

/* (host) sample_off[M+1] and vol_off[n_problems+1]; either may be NULL. */
pvr_status pvr_plan_offsets(const pvr_plan *plan, int64_t *sample_off,
                            int64_t *vol_off);

/* Build the motion-dependent state of the observation model of Sec. I
 * eq. (1), x_i = W_i y + n_i with W_i = D B T_i, for theta (float [M][6] or
 * double [M][6]): per patch the rigid transform T_s and the PSF B moved
 * with it, per sample the inverse PSF normaliser (0 marks an invalid
 * sample).  active ([M], nullable = all) and sample_mask ([N], nullable =
 * all) are read here.  The adjoint's brick -> patch index follows lazily
 * with the first pvr_backproject after a build, so loops that only simulate
 * (registration) do not pay for it; neither synchronises (the index lists
 * have capacities bounded at plan creation).  With LDS forward tiles
 * enabled (pvr_plan_set_tiles) the build synchronises `stream` once to size
 * the staged boxes.  pvr_plan_build_f64 also writes FP64 normalisers when
 * the workspace was attached with PVR_WS_F64 (needed by the _f64 calls).
 * Errors: PVR_EINVAL (NULL, misaligned, no workspace), PVR_EHIP. */
pvr_status pvr_plan_build(pvr_plan *plan, const float *theta,
                          const uint8_t *active, const uint8_t *sample_mask,
                          hipStream_t stream);
pvr_status pvr_plan_build_f64(pvr_plan *plan, const double *theta,
                              const uint8_t *active, const uint8_t *sample_mask,
                              hipStream_t stream);

/* PSF of the plan's forward model (Sec. II, "Patch to Volume Registration").
 *   PVR_PSF_GAUSSIAN (default): a 3D Gaussian along the moved stack axes with
 *     the stacks' FWHMs, truncated at k standard deviations and shifted to 0
 *     there (the approximation of the method the paper builds on).
 *   PVR_PSF_SINC: the paper's own PSF, a sinc in-plane times the slice
 *     profile through-plane.  In the moved patch frame (offsets d_u, d_v, d_n
 *     in mm) the weight is s(d_u / w_u) s(d_v / w_v) (exp(-d_n^2 / 2 sigma_n^2)
 *     - exp(-k^2 / 2)) on |d_u| < w_u, |d_v| < w_v, |d_n| <= k sigma_n, where
 *     s(t) = sin(pi t) / (pi t) is a polynomial in (pi t)^2 (in FP32 its
 *     degree-6 Chebyshev interpolant on |t| <= 1, within 1e-9 of s; in FP64
 *     the Taylor series through (pi t)^22), w = the in-plane FWHMs (the sinc's first zero;
 *     main lobe only) and sigma_n the slice profile's deviation from the
 *     through-plane FWHM.  Normalised over in-volume voxels like the Gaussian.
 *     Registration runs with the central-difference gradient only: the
 *     exact gradient (PVR_REG_GRAD_EXACT) and the theta-derivatives
 *     (pvr_simulate_grad_theta*) return PVR_EUNSUPPORTED for this PSF; the
 *     LDS-tiled forward pass is not used with it.
 * Takes effect at the next pvr_plan_build (the plan counts as unbuilt until
 * then).  (host) */
#define PVR_PSF_GAUSSIAN 0
#define PVR_PSF_SINC 1
pvr_status pvr_plan_set_psf(pvr_plan *plan, int32_t kind);

/* Forward tile shape.  By default the simulation walks every sample's PSF
 * support in global memory (one workgroup per 1024-sample chunk of a patch).
 * With tile_w x tile_h > 0 it instead splits every patch into tile_w x tile_h
 * pixel rectangles, one workgroup each, and stages each tile's voxel box in
 * LDS (tile_w * tile_h <= 256; tiles whose box exceeds 64 KiB walk global
 * memory); 0 x 0 returns to the global walk.  Used by the autotuner.
 * Synchronises `stream` when tiles are enabled. */
pvr_status pvr_plan_set_tiles(pvr_plan *plan, int32_t tile_w, int32_t tile_h,
                              hipStream_t stream);

/* Launch order of the two PSF kernels (a tuning knob, used by the
 * autotuner): workgroups are dealt to the 8 XCDs round-robin, each XCD with
 * its own L2; the work lists (forward chunks of 1024 samples, patch-major;
 * adjoint bricks of 8^3 voxels, x fastest) are regrouped into granules of
 * g consecutive items so that XCD x takes granules x, x + 8, ....  Defaults:
 * forward 1, adjoint 64.  Results do not depend on the granules (every
 * output keeps its summation order).  Both in [1, 4096].  (host) */
pvr_status pvr_plan_set_granules(pvr_plan *plan, int32_t sim_granule, int32_t bp_granule);

/* Kernel timing, a profiling aid.  With on != 0 the plan records a HIP
 * event pair on the launch stream around every launch of the kernel named by
 * `kernel` (PVR_KERNEL_SIMULATE: the forward kernel of pvr_simulate;
 * PVR_KERNEL_REGISTER: the registration of pvr_register_patches, both
 * volume layouts and the volume copy between them;
 * PVR_KERNEL_BACKPROJECT: the gather kernel of pvr_backproject, without its
 * operand preparation), up to 256 launches per kernel between reads.
 * pvr_plan_kernel_time synchronises on the recorded events and returns the
 * summed milliseconds and the launch count since the previous read, then
 * starts a new count.  Not for use while a stream is being captured into a
 * graph.  Enabling creates the events (host call); disabling keeps them. */
#define PVR_KERNEL_SIMULATE 0
#define PVR_KERNEL_BACKPROJECT 1
#define PVR_KERNEL_REGISTER 2
pvr_status pvr_plan_set_timing(pvr_plan *plan, int32_t on);
pvr_status pvr_plan_kernel_time(pvr_plan *plan, int32_t kernel, double *total_ms,
                                int32_t *launches);

/* Work of the registrations since the previous read (a profiling aid, Sec.
 * II "Patch to Volume Registration"): out[0] NCC evaluations and out[1]
 * valid samples they walked (plain evaluations: the gradient by central
 * differences and every trial step), out[2] and out[3] the same for
 * evaluations with the exact gradient.  Synchronises `stream`, then starts
 * a new count. */
pvr_status pvr_plan_reg_stats(pvr_plan *plan, int64_t out[4], hipStream_t stream);

/* (device) inverse normalisers 1/Z_j of the last build, [N] float
 * (0 for invalid samples).  The pointer stays valid until the next build. */
const float *pvr_plan_inv_z(const pvr_plan *plan);

/* Forward simulation ("volume-pixel"): y_sim = A X over valid samples.
 * X [V], y_obs [N] (nullable), y_sim [N] (nullable), resid [N] (nullable;
 * requires y_obs) = y_obs - y_sim for valid samples, 0 otherwise. */
pvr_status pvr_simulate(const pvr_plan *plan, const float *X,
                        const float *y_obs, float *y_sim, float *resid,
                        hipStream_t stream);
pvr_status pvr_simulate_f64(const pvr_plan *plan, const double *X,
                            const double *y_obs, double *y_sim, double *resid,
                            hipStream_t stream);

/* Adjoint ("pixel-volume", Sec. III level II) of the forward model, the
 * reintegration step of the SR iterations (Sec. II, "EM-Based Outlier
 * Removal": samples weighted by their posteriors and patch weights enter the
 * volume update), in gather form: for every voxel i
 *   num_i = sum_j psi_ji W_s(j) p_j e_j,   den_i = sum_j psi_ji W_s(j) p_j
 * e [N] (required), p [N] (nullable = 1), patch_w [M] (nullable = 1),
 * num [V] (required), den [V] (nullable).  Deterministic: the summation order
 * is fixed (patch order, then pixel order).  The first call after a build
 * also builds the adjoint's brick -> patch index on `stream`. */
pvr_status pvr_backproject(const pvr_plan *plan, const float *e,
                           const float *p, const float *patch_w, float *num,
                           float *den, hipStream_t stream);
pvr_status pvr_backproject_f64(const pvr_plan *plan, const double *e,
                               const double *p, const double *patch_w,
                               double *num, double *den, hipStream_t stream);

/* EM robust weights of one SR iteration (per problem):
 *   m = 1/max(max e - min e, 1e-6 max|y|) over valid samples,
 *   p_j = c G(e_j) / (c G(e_j) + m (1 - c)),  G zero-mean Gaussian (sigma^2),
 *   p_bar_s = sqrt(sum_{j in s} p_j^2 / N_s),
 *   W_s from a two-component Gaussian mixture fitted to {p_bar_s} (20 EM
 *   iterations from a median split; W = inlier posterior if >= 0.5 else 0),
 *   then sigma^2 = sum W p e^2 / sum W p (floored at (1e-4 max|y|)^2) and
 *   c = sum W p / sum_s W_s N_s for the next call.
 * resid, y_obs [N]; em [n_problems] (device, in/out); p [N], pbar [M] and
 * patch_w [M] out (patch_w in with PVR_EM_FIX_W). */
pvr_status pvr_robust_weights(pvr_plan *plan, const float *resid,
                              const float *y_obs, pvr_em_state *em, float *p,
                              float *pbar, float *patch_w, int32_t flags,
                              hipStream_t stream);

/* SR update of every volume (Jacobi: reads X only, writes X_out; X_out must
 * not alias X):
 *   X'_i = max(clamp, X_i + alpha num_i/den_i [den_i > den_eps]
 *                        + alpha lambda R_i(X))
 *   R_i = sum over the 26 neighbours d inside the grid of
 *         b_d D_d / sqrt(1 + (D_d/delta)^2),  D_d = X_{i+d} - X_i,
 *         b_d = 1/|d| (voxel units).
 * params (host). */
pvr_status pvr_sr_update(const pvr_plan *plan, const float *X,
                         const float *num, const float *den,
                         const pvr_sr_params *params, float *X_out,
                         hipStream_t stream);

/* Per-patch rigid registration (one workgroup per patch): maximise
 * NCC(y_s, A_s(theta) X) over the six parameters, where the simulated patch
 * uses the full PSF forward model and NCC runs over samples valid at theta.
 * Optimiser: variables (rho * angles, translations) with rho the patch
 * half-diagonal in mm; gradient by central differences with step fd_h or
 * exact (params->gradient, PVR_REG_GRAD_*; exact needs the Gaussian PSF,
 * PVR_EUNSUPPORTED otherwise); a normalised
 * step of length delta is accepted on strict improvement (delta doubles,
 * capped at step0) or delta halves; stop below step_min or after max_iter
 * trial steps.  Patches with std(y_s) < min_std keep theta.
 * theta [M][6] in/out; ncc [M] out (nullable); reg [M] (nullable = all):
 * only patches with reg != 0 move; params (host); sample_mask of the last
 * build applies.  With max_iter = 0 it only evaluates NCC at theta.  The
 * patches whose rows run closer to voxel y than to x are registered on the
 * plan's second stream, concurrently with the others; `stream` waits for
 * them before any later work. */
pvr_status pvr_register_patches(const pvr_plan *plan, const float *X,
                                const float *y_obs, float *theta, float *ncc,
                                const uint8_t *reg,
                                const pvr_reg_params *params,
                                hipStream_t stream);

/* Derivative of the forward model with respect to the per-patch motion
 * (differentiable simulation; the derivative of the PSF weights of
 * eq. (1)'s W_i = D B T_i through T_i):
 *   grad_theta[s][k] = sum_{j in s} grad_y[j] * d y_sim_j / d theta_s[k]
 * at the theta of the last build (radians and mm), with the normalisers
 * Z_j differentiated too.  The derivative with respect to X is the adjoint:
 * pvr_backproject(grad_y, NULL, NULL, grad_X, NULL).  X [V], grad_y [N],
 * grad_theta [M][6] out. */
pvr_status pvr_simulate_grad_theta(const pvr_plan *plan, const float *X,
                                   const float *grad_y, float *grad_theta,
                                   hipStream_t stream);
pvr_status pvr_simulate_grad_theta_f64(const pvr_plan *plan, const double *X,
                                       const double *grad_y,
                                       double *grad_theta, hipStream_t stream);

/* Cross-correlation of every patch with its simulation (Sec. IV-A eq. CC,
 * population statistics over the samples valid at the last build) and its
 * derivative with respect to the simulated samples:
 *   d NCC_s / d y_sim_j = ((y_j - mu_y)/(sd_y sd_sim)
 *                          - NCC_s (y_sim_j - mu_sim)/sd_sim^2) / n_s.
 * Chained through pvr_simulate_grad_theta it gives d NCC_s / d theta_s for
 * gradient-based registration.  y_obs, y_sim [N]; grad_y [N] out (nullable);
 * ncc [M] out (nullable).  Flat patches give 0. */
pvr_status pvr_ncc_grad(const pvr_plan *plan, const float *y_obs,
                        const float *y_sim, float *grad_y, float *ncc,
                        hipStream_t stream);

/* Per-patch motion bookkeeping of the optimisers built on the forward model
 * (one lane per patch; M = the plan's patches; theta-like arrays [M][6]).
 * rho_s is the patch half-diagonal in mm (at least 1), the scale of the
 * rotation variables of the registration (Sec. II, "Patch to Volume
 * Registration": each patch's rigid parameters are optimised on its own).
 *
 * pvr_motion_frame: the motion in the patch's own frame, used as the
 *   learned initialiser's target: out_s = base_s + A_s in_s (inverse = 0) or
 *   base_s + A_s^-1 in_s (inverse != 0), A_s = diag(rho_s F_s^T, F_s^T) with
 *   F_s the unit axes of the patch's stack (in-plane u, in-plane v, normal)
 *   as columns.  base nullable (= 0); out may alias base, not in.
 * pvr_motion_step: a normalised gradient-ascent trial in the variables
 *   (rho angles, translations): trial_s = theta_s + delta_s g~_s / |g~_s|
 *   mapped back (g~ = grad_theta with the angle part divided by rho_s) for
 *   patches with delta_s >= step_min, else theta_s.
 * pvr_motion_accept: where score_cand_s > score_s (and, when delta is given,
 *   delta_s >= step_min): theta_s = cand_s and score_s = score_cand_s; with
 *   delta, an accepted step doubles (capped at step0) and a rejected one
 *   halves (patches below step_min are left alone); n_live (int32 [1],
 *   nullable) is increased by the number of patches whose step is still
 *   >= step_min afterwards (the caller zeroes it).
 * pvr_motion_init_step: delta_s = step0 for patches whose observed samples
 *   (those the last build's mask keeps) have a population standard
 *   deviation >= min_std, else 0 (flat patches keep their motion).  Needs a
 *   built plan.
 * pvr_motion_fallback: the threshold is tau, or score_ref_s + tau when
 *   score_ref is given (nullable); for the patches with active_s != 0
 *   (active nullable = all) and score_s below their threshold: theta_s =
 *   theta_ref_s and flag_s = 1 -- the patches a plain registration takes
 *   over from their reference motion; every other patch gets flag_s = 0 and
 *   keep_s = 1 if active (keep nullable; flag and keep uint8 [M]).
 * pvr_motion_live: live_s = 1 where delta_s >= step_min and active_s != 0
 *   (active nullable = all), else 0 (live uint8 [M]): the patches whose
 *   optimiser still moves, the active set of a build that evaluates only
 *   them. */
pvr_status pvr_motion_frame(const pvr_plan *plan, const float *in, int32_t inverse,
                            const float *base, float *out, hipStream_t stream);
pvr_status pvr_motion_step(const pvr_plan *plan, const float *theta, const float *grad_theta,
                           const float *delta, float step_min, float *trial, hipStream_t stream);
pvr_status pvr_motion_accept(const pvr_plan *plan, const float *cand, const float *score_cand,
                             float *theta, float *score, float *delta, float step0,
                             float step_min, int32_t *n_live, hipStream_t stream);
pvr_status pvr_motion_init_step(const pvr_plan *plan, const float *y_obs, float step0,
                                double min_std, float *delta, hipStream_t stream);
pvr_status pvr_motion_fallback(const pvr_plan *plan, const float *score, float tau,
                               const float *score_ref, const float *theta_ref, float *theta,
                               const uint8_t *active, uint8_t *flag, uint8_t *keep,
                               hipStream_t stream);
pvr_status pvr_motion_live(const pvr_plan *plan, const float *delta, float step_min,
                           const uint8_t *active, uint8_t *live, hipStream_t stream);

/* Numeric faults.  The SR update raises PVR_FAULT_VOLUME when a voxel of the
 * new volume is not finite before the clamp (which would otherwise hide a
 * NaN); the robust weights raise PVR_FAULT_RESIDUAL when a problem's residual
 * statistics (sum of e^2, range of e, max |y|) are not finite -- a NaN or an
 * infinity in X, y or on the way.  The flags accumulate on the device over
 * calls; pvr_check synchronises `stream`, reads and clears them, and returns
 * PVR_ENUMERIC with the raised flags named in pvr_last_error(), PVR_OK when
 * none was raised. */
#define PVR_FAULT_VOLUME 1u
#define PVR_FAULT_RESIDUAL 2u
#define PVR_FAULT_INDEX 4u  /* the adjoint's index outgrew its capacity (the
                               host bound rules this out; pvr_check then
                               returns PVR_ESHAPE) */
pvr_status pvr_check(pvr_plan *plan, hipStream_t stream);

/* Debug mode, for callers tracking down bad inputs (it costs a device scan
 * and a stream synchronisation per checked array).  When on, the entry
 * points below check their input arrays on the device before launching and
 * synchronise `stream`; the first offending element gives PVR_EINVAL with
 * the function, the array and the index in pvr_last_error():
 *   pvr_plan_build[_f64]            theta [6M] finite
 *   pvr_simulate[_f64]              X [V], y_obs [N] finite
 *   pvr_backproject[_f64]           e [N], p [N] finite; patch_w [M] finite
 *                                   and >= 0
 *   pvr_robust_weights              resid [N], y_obs [N] finite
 *   pvr_sr_update                   X, num, den [V] finite
 *   pvr_register_patches            X [V], y_obs [N], theta [6M] finite
 *   pvr_simulate_grad_theta[_f64]   X [V], grad_y [N] finite
 * Null (optional) arrays are not checked, and no check runs while `stream`
 * is being captured into a graph (the graph's launches are the ones of the
 * calls made during the capture, checked or not).  The mode is process-wide
 * (every plan, every thread); it starts on when the environment variable
 * PVR_DEBUG is set to anything other than "" or "0" when first consulted, and
 * pvr_set_debug switches it (on != 0) at any time.  Always PVR_OK. */
pvr_status pvr_set_debug(int32_t on);
/* 1 when the debug mode is on, else 0. */
int32_t pvr_get_debug(void);

/* Captured SR iterations (the batched form of Sec. III level II: every
 * problem of the plan in each launch).  Records `iters` SR iterations into a
 * HIP graph: iteration i simulates from the current volume (X for even i,
 * X_alt for odd i) with residuals into resid, runs the robust weights with
 * PVR_EM_RESID_FRESH | PVR_EM_PREP_ADJOINT (the preparation branch of the
 * adjoint is a second branch of the graph; EM continues from em's state: start a cycle with an
 * eager call with PVR_EM_INIT first), back-projects into num / den and writes
 * the update into the other volume; after a launch the volume is in X when
 * iters is even, else in X_alt.  All buffers are device memory of the sizes
 * of the corresponding calls and must stay allocated while the graph lives;
 * params is read at capture.  Before capturing, the call prepares the
 * adjoint's brick index and synchronises `stream`; kernel timing must be off.
 * A graph records the plan as it is: after pvr_plan_build*, pvr_plan_set_psf,
 * pvr_plan_set_tiles, pvr_plan_set_granules or an index rebuild
 * pvr_sr_graph_launch returns
 * PVR_EINVAL (capture again).  Destroy graphs before their plan.  Launches
 * are asynchronous on `stream`. */
typedef struct pvr_sr_graph pvr_sr_graph;
pvr_status pvr_sr_graph_create(pvr_plan *plan, float *X, float *X_alt, const float *y_obs,
                               float *resid, float *p, float *pbar, float *patch_w,
                               float *num, float *den, pvr_em_state *em,
                               const pvr_sr_params *params, int32_t iters,
                               hipStream_t stream, pvr_sr_graph **out);
pvr_status pvr_sr_graph_launch(const pvr_sr_graph *graph, hipStream_t stream);
void pvr_sr_graph_destroy(pvr_sr_graph *graph); /* NULL is a no-op */

#ifdef __cplusplus
}
#endif

#endif /* PVR_H */
