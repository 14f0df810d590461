/*
 * FP64 CPU oracle for patch-to-volume reconstruction (PVR), Alansary, Kainz
 * et al., "PVR: Patch-to-Volume Reconstruction for Large Area Motion
 * Correction of Fetal MRI" (arXiv 1611.07289).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the HIP path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the product path never does.
 * It shares no source with the HIP library.
 *
 * What it computes (section / equation of the paper in brackets):
 *  - the observation model x_i = W_i y + n_i with W_i = D B T_i
 *    [Sec. I, eq. (1)]: every observed patch sample is the PSF-weighted
 *    average of the volume around its rigidly moved centre;
 *  - the PSF is a 3D Gaussian aligned with the moved stack axes
 *    [Sec. II "Patch to Volume Registration" names an accurate PSF; the
 *    Gaussian approximation of the cited reconstruction method is used],
 *    truncated at Mahalanobis radius k and shifted to zero there so that the
 *    truncated kernel is continuous, normalised over in-volume voxels;
 *  - simulate (y_hat = A X), the adjoint back-projection (A^T r);
 *  - the cross-correlation similarity [Sec. IV-A, eq. CC] of a patch and
 *    its simulation, and the per-patch rigid 2D-3D registration by gradient
 *    ascent on it [Sec. II "Patch to Volume Registration", Sec. III level I].
 *
 * Conventions (these are readings where the paper is silent):
 *  - theta_s = (rx, ry, rz [rad], tx, ty, tz [mm]); R = Rz Ry Rx; the patch
 *    rotates about its own centre c_s: x = R (P - c_s) + c_s + t;
 *  - PSF frame F = R [e1 e2 n] (unit stack axes), sigma = FWHM / 2.3548;
 *  - support: Q = sum_a (d_a / sigma_a)^2 <= k^2 with d = F^T (v - x);
 *    weight g_hat = exp(-Q/2) - exp(-k^2/2); Z = sum over in-volume voxels;
 *  - a sample is valid iff its moved centre lies in the half-open voxel box
 *    [-1/2, n - 1/2)^3, Z > 0, its mask byte is non-zero and its patch is
 *    active; invalid samples simulate to 0 and contribute nothing.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int dims[3];          /* nx, ny, nz */
  double v2w[12];       /* voxel index -> world mm, row-major 3x4 */
  double w2v[12];       /* inverse */
  int n_stacks;
  int *sdims;           /* [n_stacks][3] nx, ny, nslices */
  double *p2w;          /* [n_stacks][12] */
  double *fwhm;         /* [n_stacks][3] */
  int M;
  int *pat;             /* [M][6] stack, slice, x0, y0, w, h */
  int64_t *off;         /* [M+1] */
  int64_t N;
  double k;             /* support radius in standard deviations */
  int psf;              /* 0: Gaussian, 1: sinc in-plane x slice profile */
} ora_ctx;

typedef struct {
  double R[9];          /* rotation, row-major */
  double c[3];          /* patch centre, world */
  double t[3];          /* translation */
  double A[9];          /* stack pix2world linear part */
  double o[3];          /* stack pix2world origin */
  double E[9];          /* [e1 e2 n]: unit stack axes as columns */
  double F[9];          /* R * [e1 e2 n] : columns are the moved PSF axes */
  double sig[3];        /* PSF standard deviations (mm) */
  double wz[2];         /* sinc PSF: in-plane first zeros (mm) = in-plane FWHM */
  double ext[3];        /* support half-extent along voxel axes (voxels) */
  double reach;         /* radius (mm) of a ball around the centre holding the support */
  int st, slice, x0, y0, w, h;
} pgeo;

static void inv_affine(const double *a, double *out) {
  /* inverse of [L | b] is [L^-1 | -L^-1 b] */
  double L[9] = {a[0], a[1], a[2], a[4], a[5], a[6], a[8], a[9], a[10]};
  double det = L[0] * (L[4] * L[8] - L[5] * L[7]) -
               L[1] * (L[3] * L[8] - L[5] * L[6]) +
               L[2] * (L[3] * L[7] - L[4] * L[6]);
  double I[9];
  I[0] = (L[4] * L[8] - L[5] * L[7]) / det;
  I[1] = (L[2] * L[7] - L[1] * L[8]) / det;
  I[2] = (L[1] * L[5] - L[2] * L[4]) / det;
  I[3] = (L[5] * L[6] - L[3] * L[8]) / det;
  I[4] = (L[0] * L[8] - L[2] * L[6]) / det;
  I[5] = (L[2] * L[3] - L[0] * L[5]) / det;
  I[6] = (L[3] * L[7] - L[4] * L[6]) / det;
  I[7] = (L[1] * L[6] - L[0] * L[7]) / det;
  I[8] = (L[0] * L[4] - L[1] * L[3]) / det;
  for (int r = 0; r < 3; ++r) {
    out[4 * r + 0] = I[3 * r + 0];
    out[4 * r + 1] = I[3 * r + 1];
    out[4 * r + 2] = I[3 * r + 2];
    out[4 * r + 3] = -(I[3 * r + 0] * a[3] + I[3 * r + 1] * a[7] +
                       I[3 * r + 2] * a[11]);
  }
}

static void apply_affine(const double *a, const double p[3], double out[3]) {
  for (int r = 0; r < 3; ++r)
    out[r] = a[4 * r] * p[0] + a[4 * r + 1] * p[1] + a[4 * r + 2] * p[2] +
             a[4 * r + 3];
}

/* R = Rz(rz) Ry(ry) Rx(rx) */
void ora_rotation(const double *th, double *R) {
  double cx = cos(th[0]), sx = sin(th[0]);
  double cy = cos(th[1]), sy = sin(th[1]);
  double cz = cos(th[2]), sz = sin(th[2]);
  double Rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx};
  double Ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
  double Rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1};
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += Ry[3 * i + m] * Rx[3 * m + j];
      T[3 * i + j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += Rz[3 * i + m] * T[3 * m + j];
      R[3 * i + j] = s;
    }
}

ora_ctx *ora_ctx_create(const int *dims, const double *v2w, int n_stacks,
                        const int *sdims, const double *p2w,
                        const double *fwhm, int M, const int *pat, double k) {
  ora_ctx *C = (ora_ctx *)calloc(1, sizeof(ora_ctx));
  memcpy(C->dims, dims, sizeof(int) * 3);
  memcpy(C->v2w, v2w, sizeof(double) * 12);
  inv_affine(C->v2w, C->w2v);
  C->n_stacks = n_stacks;
  C->sdims = (int *)malloc(sizeof(int) * 3 * n_stacks);
  memcpy(C->sdims, sdims, sizeof(int) * 3 * n_stacks);
  C->p2w = (double *)malloc(sizeof(double) * 12 * n_stacks);
  memcpy(C->p2w, p2w, sizeof(double) * 12 * n_stacks);
  C->fwhm = (double *)malloc(sizeof(double) * 3 * n_stacks);
  memcpy(C->fwhm, fwhm, sizeof(double) * 3 * n_stacks);
  C->M = M;
  C->pat = (int *)malloc(sizeof(int) * 6 * (M > 0 ? M : 1));
  memcpy(C->pat, pat, sizeof(int) * 6 * M);
  C->off = (int64_t *)malloc(sizeof(int64_t) * (M + 1));
  C->off[0] = 0;
  for (int s = 0; s < M; ++s)
    C->off[s + 1] = C->off[s] + (int64_t)pat[6 * s + 4] * pat[6 * s + 5];
  C->N = C->off[M];
  C->k = k;
  return C;
}

void ora_ctx_free(ora_ctx *C) {
  if (!C) return;
  free(C->sdims); free(C->p2w); free(C->fwhm); free(C->pat); free(C->off);
  free(C);
}

int64_t ora_n_samples(const ora_ctx *C) { return C->N; }

/* Patch geometry for motion parameters th[6] (Sec. II: each patch is
 * rigidly registered; rotation about the patch centre is the reading). */
static void patch_geometry(const ora_ctx *C, int s, const double *th,
                           pgeo *g) {
  const int *p = C->pat + 6 * s;
  g->st = p[0]; g->slice = p[1]; g->x0 = p[2]; g->y0 = p[3];
  g->w = p[4]; g->h = p[5];
  const double *P = C->p2w + 12 * g->st;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) g->A[3 * r + c] = P[4 * r + c];
    g->o[r] = P[4 * r + 3];
  }
  double pc[3] = {g->x0 + 0.5 * (g->w - 1), g->y0 + 0.5 * (g->h - 1),
                  (double)g->slice};
  apply_affine(P, pc, g->c);
  ora_rotation(th, g->R);
  for (int a = 0; a < 3; ++a) g->t[a] = th[3 + a];
  /* unit stack axes e_a = column a of A / |column a| */
  double *E = g->E;
  for (int a = 0; a < 3; ++a) {
    double n = sqrt(g->A[a] * g->A[a] + g->A[3 + a] * g->A[3 + a] +
                    g->A[6 + a] * g->A[6 + a]);
    for (int r = 0; r < 3; ++r) E[3 * r + a] = g->A[3 * r + a] / n;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int m = 0; m < 3; ++m) acc += g->R[3 * i + m] * E[3 * m + j];
      g->F[3 * i + j] = acc;
    }
  for (int a = 0; a < 3; ++a)
    g->sig[a] = C->fwhm[3 * g->st + a] / (2.0 * sqrt(2.0 * log(2.0)));
  for (int a = 0; a < 2; ++a) g->wz[a] = C->fwhm[3 * g->st + a];
  if (C->psf == 1) {
    /* support box x + F (t_u w_u, t_v w_v, t_n sig_n), |t_u|, |t_v| < 1,
     * |t_n| <= k: half extent along voxel axis b is the sum of the box's
     * half widths times |W2V_lin F|_{b,a} */
    const double hw[3] = {g->wz[0], g->wz[1], C->k * g->sig[2]};
    for (int b = 0; b < 3; ++b) {
      double acc = 0;
      for (int a = 0; a < 3; ++a) {
        double m = 0;
        for (int q = 0; q < 3; ++q) m += C->w2v[4 * b + q] * g->F[3 * q + a];
        acc += fabs(m) * hw[a];
      }
      g->ext[b] = acc;
    }
    g->reach = sqrt(hw[0] * hw[0] + hw[1] * hw[1] + hw[2] * hw[2]);
    return;
  }
  /* support ellipsoid x + F diag(sig) u, |u| <= k, in voxel coordinates:
   * half extent along voxel axis b is k * |row_b(W2V_lin F diag(sig))| */
  for (int b = 0; b < 3; ++b) {
    double acc = 0;
    for (int a = 0; a < 3; ++a) {
      double m = 0;
      for (int q = 0; q < 3; ++q) m += C->w2v[4 * b + q] * g->F[3 * q + a];
      m *= g->sig[a];
      acc += m * m;
    }
    g->ext[b] = C->k * sqrt(acc);
  }
  g->reach = C->k * fmax(g->sig[0], fmax(g->sig[1], g->sig[2]));
}

/* sin(R) / R by its Taylor series 1 - R^2/3! + R^4/5! - ... (Sec. II, the
 * PSF paragraph), summed until the next term is below 1e-15 of the partial
 * sum (an alternating series with decreasing terms errs by less than its
 * first omitted term) or after 40 terms; |R| <= pi here. */
static double sinc_taylor(double R) {
  const double r2 = R * R;
  double term = 1.0, sum = 1.0;
  for (int m = 1; m < 40; ++m) {
    term *= -r2 / ((2.0 * m) * (2.0 * m + 1.0));
    sum += term;
    if (fabs(term) < 1e-15 * fabs(sum)) break;
  }
  return sum;
}

void ora_set_psf(ora_ctx *C, int kind) { C->psf = kind; }
double ora_sinc_taylor(double R) { return sinc_taylor(R); }

/* World centre of sample (u, v) of the patch after motion. */
static void sample_centre(const pgeo *g, int u, int v, double x[3]) {
  double P[3], d[3];
  for (int r = 0; r < 3; ++r)
    P[r] = g->A[3 * r] * u + g->A[3 * r + 1] * v + g->A[3 * r + 2] * g->slice +
           g->o[r];
  for (int r = 0; r < 3; ++r) d[r] = P[r] - g->c[r];
  for (int r = 0; r < 3; ++r)
    x[r] = g->R[3 * r] * d[0] + g->R[3 * r + 1] * d[1] + g->R[3 * r + 2] * d[2] +
           g->c[r] + g->t[r];
}

/* Shifted, truncated Gaussian weight of voxel (i, j, kk) for a sample at x.
 * Returns a negative value when the voxel is outside the support. */
static double psf_hat(const ora_ctx *C, const pgeo *g, const double x[3],
                      int i, int j, int kk) {
  double ip[3] = {(double)i, (double)j, (double)kk}, v[3], dv[3];
  apply_affine(C->v2w, ip, v);
  for (int r = 0; r < 3; ++r) dv[r] = v[r] - x[r];
  if (C->psf == 1) {
    /* sinc in-plane (first zero at the in-plane FWHM) x the slice profile (a
     * Gaussian of the through-plane FWHM, cut at k sigma and shifted to 0) */
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = g->F[a] * dv[0] + g->F[3 + a] * dv[1] + g->F[6 + a] * dv[2];
    const double tu = d[0] / g->wz[0], tv = d[1] / g->wz[1], qn = (d[2] / g->sig[2]) * (d[2] / g->sig[2]);
    if (!(fabs(tu) < 1.0) || !(fabs(tv) < 1.0) || qn > C->k * C->k) return -1.0;
    return sinc_taylor(M_PI * tu) * sinc_taylor(M_PI * tv) *
           (exp(-0.5 * qn) - exp(-0.5 * C->k * C->k));
  }
  double Q = 0;
  for (int a = 0; a < 3; ++a) {
    double d = g->F[a] * dv[0] + g->F[3 + a] * dv[1] + g->F[6 + a] * dv[2];
    Q += (d / g->sig[a]) * (d / g->sig[a]);
  }
  if (Q > C->k * C->k) return -1.0;
  return exp(-0.5 * Q) - exp(-0.5 * C->k * C->k);
}

/* Voxel index box holding the support; returns 0 if the centre is outside
 * the half-open voxel box (the sample is then invalid). */
static int support_box(const ora_ctx *C, const pgeo *g, const double x[3],
                       int lo[3], int hi[3]) {
  double xv[3];
  apply_affine(C->w2v, x, xv);
  int inside = 1;
  for (int b = 0; b < 3; ++b) {
    if (!(xv[b] >= -0.5 && xv[b] < C->dims[b] - 0.5)) inside = 0;
    double l = ceil(xv[b] - g->ext[b]), h = floor(xv[b] + g->ext[b]);
    if (l < 0) l = 0;
    if (h > C->dims[b] - 1) h = C->dims[b] - 1;
    lo[b] = (int)l;
    hi[b] = (int)h;
  }
  return inside;
}

/* Simulate one sample: returns validity, writes y_hat and Z. */
static int sim_sample(const ora_ctx *C, const pgeo *g, const double *X,
                      int u, int v, double *yhat, double *Zout) {
  double x[3];
  int lo[3], hi[3];
  sample_centre(g, u, v, x);
  int inside = support_box(C, g, x, lo, hi);
  double Z = 0, acc = 0;
  const int nx = C->dims[0], ny = C->dims[1];
  if (inside) {
    for (int kk = lo[2]; kk <= hi[2]; ++kk)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          double w = psf_hat(C, g, x, i, j, kk);
          if (w < 0) continue;
          Z += w;
          if (X) acc += w * X[((int64_t)kk * ny + j) * nx + i];
        }
  }
  *Zout = Z;
  if (!inside || !(Z > 0)) {
    *yhat = 0;
    return 0;
  }
  *yhat = acc / Z;
  return 1;
}

static int patch_of(const ora_ctx *C, int64_t j) {
  int lo = 0, hi = C->M - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (C->off[mid] <= j) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* Validity of every sample by the rule of sim_sample (centre inside the
 * voxel box and Z > 0, unmasked, patch active), without the support walk
 * where it is not needed: Z >= the weight of any one voxel, so a positive
 * weight at the nearest voxel settles Z > 0; only otherwise is Z summed. */
void ora_valid(const ora_ctx *C, const double *theta, const uint8_t *mask,
               const uint8_t *active, uint8_t *valid) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int s = 0; s < C->M; ++s) {
    pgeo g;
    patch_geometry(C, s, theta + 6 * s, &g);
    for (int64_t l = 0; l < (int64_t)g.w * g.h; ++l) {
      const int64_t j = C->off[s] + l;
      int ok = !(mask && !mask[j]) && !(active && !active[s]);
      if (ok) {
        const int u = g.x0 + (int)(l % g.w), v = g.y0 + (int)(l / g.w);
        double x[3], xv[3];
        int lo[3], hi[3];
        sample_centre(&g, u, v, x);
        ok = support_box(C, &g, x, lo, hi);
        if (ok) {
          apply_affine(C->w2v, x, xv);
          int n[3];
          for (int b = 0; b < 3; ++b) {
            n[b] = (int)floor(xv[b] + 0.5);
            if (n[b] < 0) n[b] = 0;
            if (n[b] > C->dims[b] - 1) n[b] = C->dims[b] - 1;
          }
          if (!(psf_hat(C, &g, x, n[0], n[1], n[2]) > 0)) {
            double yh, Z;
            ok = sim_sample(C, &g, NULL, u, v, &yh, &Z);
          }
        }
      }
      valid[j] = (uint8_t)ok;
    }
  }
}

/* y_hat = A X for the listed samples (all when list == NULL); Z and valid
 * are written for the same samples.  theta is [M][6]. */
void ora_simulate(const ora_ctx *C, const double *X, const double *theta,
                  const uint8_t *mask, const uint8_t *active, int64_t n_list,
                  const int64_t *list, double *yhat, double *Z,
                  uint8_t *valid) {
  int64_t n = list ? n_list : C->N;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t q = 0; q < n; ++q) {
    int64_t j = list ? list[q] : q;
    int s = patch_of(C, j);
    pgeo g;
    patch_geometry(C, s, theta + 6 * s, &g);
    int64_t l = j - C->off[s];
    int u = g.x0 + (int)(l % g.w), v = g.y0 + (int)(l / g.w);
    double yh, z;
    int ok = sim_sample(C, &g, X, u, v, &yh, &z);
    if (mask && !mask[j]) ok = 0;
    if (active && !active[s]) ok = 0;
    yhat[q] = ok ? yh : 0.0;
    if (Z) Z[q] = z;
    if (valid) valid[q] = (uint8_t)ok;
  }
}

/* Sparse row of A for one sample: voxel indices and normalised weights
 * psi = g_hat / Z.  Returns nnz (or -1 if cap is too small); 0 if invalid. */
int ora_sample_row(const ora_ctx *C, const double *theta, int64_t j,
                   int64_t *idx, double *wt, int cap) {
  int s = patch_of(C, j);
  pgeo g;
  patch_geometry(C, s, theta + 6 * s, &g);
  int64_t l = j - C->off[s];
  int u = g.x0 + (int)(l % g.w), v = g.y0 + (int)(l / g.w);
  double x[3], yh, Z;
  int lo[3], hi[3];
  if (!sim_sample(C, &g, NULL, u, v, &yh, &Z)) return 0;
  sample_centre(&g, u, v, x);
  support_box(C, &g, x, lo, hi);
  int n = 0;
  const int nx = C->dims[0], ny = C->dims[1];
  for (int kk = lo[2]; kk <= hi[2]; ++kk)
    for (int jj = lo[1]; jj <= hi[1]; ++jj)
      for (int i = lo[0]; i <= hi[0]; ++i) {
        double w = psf_hat(C, &g, x, i, jj, kk);
        if (w < 0) continue;
        if (n >= cap) return -1;
        idx[n] = ((int64_t)kk * ny + jj) * nx + i;
        wt[n] = w / Z;
        ++n;
      }
  return n;
}

/* out = A^T r (the adjoint, "pixel-volume" direction): every valid sample j
 * adds psi_ji * r_j to voxel i.  Patches are split into a fixed number of
 * chunks with private accumulators summed in chunk order, so the result does
 * not depend on the thread count. */
/* indicator = 0: (A^T r)_i = sum_j psi_ji r_j.  indicator = 1: the same sum
 * with psi_ji replaced by 1/Z_j on the support (the transpose of the
 * support indicator, scaled by 1/Z_j), used to size the rounding error of
 * the weights near the support edge. */
static void backproject_impl(const ora_ctx *C, const double *theta, const uint8_t *mask,
                             const uint8_t *active, const double *r, int indicator,
                             double *out) {
  const int64_t V = (int64_t)C->dims[0] * C->dims[1] * C->dims[2];
  /* one private accumulator per thread (patch ranges in order), summed in
     chunk order afterwards */
  int NCH = omp_get_max_threads();
  if (NCH < 1) NCH = 1;
  if (NCH > 64) NCH = 64;
  double *buf = (double *)calloc((size_t)NCH * V, sizeof(double));
  const int nx = C->dims[0], ny = C->dims[1];
#pragma omp parallel for schedule(static, 1)
  for (int ch = 0; ch < NCH; ++ch) {
    double *acc = buf + (size_t)ch * V;
    int s0 = (int)((int64_t)C->M * ch / NCH), s1 = (int)((int64_t)C->M * (ch + 1) / NCH);
    for (int s = s0; s < s1; ++s) {
      if (active && !active[s]) continue;
      pgeo g;
      patch_geometry(C, s, theta + 6 * s, &g);
      for (int64_t l = 0; l < (int64_t)g.w * g.h; ++l) {
        int64_t j = C->off[s] + l;
        if (mask && !mask[j]) continue;
        int u = g.x0 + (int)(l % g.w), v = g.y0 + (int)(l / g.w);
        double yh, Z, x[3];
        int lo[3], hi[3];
        if (!sim_sample(C, &g, NULL, u, v, &yh, &Z)) continue;
        sample_centre(&g, u, v, x);
        support_box(C, &g, x, lo, hi);
        for (int kk = lo[2]; kk <= hi[2]; ++kk)
          for (int jj = lo[1]; jj <= hi[1]; ++jj)
            for (int i = lo[0]; i <= hi[0]; ++i) {
              double w = psf_hat(C, &g, x, i, jj, kk);
              if (w < 0) continue;
              acc[((int64_t)kk * ny + jj) * nx + i] += (indicator ? 1.0 : w) / Z * r[j];
            }
      }
    }
  }
  for (int64_t i = 0; i < V; ++i) {
    double s = 0;
    for (int ch = 0; ch < NCH; ++ch) s += buf[(size_t)ch * V + i];
    out[i] = s;
  }
  free(buf);
}

/* (A^T r)_i for a list of voxels, computed one voxel at a time straight from
 * the definition: every sample whose support holds the voxel contributes
 * psi_ji r_j.  A patch is skipped only when the voxel is farther from its
 * centre than the patch half-diagonal plus the largest support radius. */
static void backproject_voxels_impl(const ora_ctx *C, const double *theta,
                                    const uint8_t *mask, const uint8_t *active,
                                    const double *r, int indicator, int64_t n_vox,
                                    const int64_t *vox, double *out) {
  const int nx = C->dims[0], ny = C->dims[1];
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < n_vox; ++q) {
    int64_t id = vox[q];
    int i = (int)(id % nx), jj = (int)((id / nx) % ny), kk = (int)(id / ((int64_t)nx * ny));
    double ip[3] = {(double)i, (double)jj, (double)kk}, vw[3];
    apply_affine(C->v2w, ip, vw);
    double acc = 0;
    for (int s = 0; s < C->M; ++s) {
      if (active && !active[s]) continue;
      pgeo g;
      patch_geometry(C, s, theta + 6 * s, &g);
      double cen[3];
      for (int a = 0; a < 3; ++a) cen[a] = g.c[a] + g.t[a];
      double su = sqrt(g.A[0] * g.A[0] + g.A[3] * g.A[3] + g.A[6] * g.A[6]);
      double sv = sqrt(g.A[1] * g.A[1] + g.A[4] * g.A[4] + g.A[7] * g.A[7]);
      double half = 0.5 * sqrt((g.w - 1) * (g.w - 1) * su * su +
                               (g.h - 1) * (g.h - 1) * sv * sv);
      double dd = 0;
      for (int a = 0; a < 3; ++a) dd += (vw[a] - cen[a]) * (vw[a] - cen[a]);
      double lim = half + g.reach + 1e-9;
      if (dd > lim * lim) continue;
      for (int64_t l = 0; l < (int64_t)g.w * g.h; ++l) {
        int64_t j = C->off[s] + l;
        if (mask && !mask[j]) continue;
        int u = g.x0 + (int)(l % g.w), v = g.y0 + (int)(l / g.w);
        double x[3];
        sample_centre(&g, u, v, x);
        double w = psf_hat(C, &g, x, i, jj, kk);
        if (w < 0) continue;
        double yh, Z;
        if (!sim_sample(C, &g, NULL, u, v, &yh, &Z)) continue;
        acc += (indicator ? 1.0 : w) / Z * r[j];
      }
    }
    out[q] = acc;
  }
}

void ora_backproject(const ora_ctx *C, const double *theta, const uint8_t *mask,
                     const uint8_t *active, const double *r, double *out) {
  backproject_impl(C, theta, mask, active, r, 0, out);
}

void ora_support_backproject(const ora_ctx *C, const double *theta, const uint8_t *mask,
                             const uint8_t *active, const double *r, double *out) {
  backproject_impl(C, theta, mask, active, r, 1, out);
}

void ora_backproject_voxels(const ora_ctx *C, const double *theta,
                            const uint8_t *mask, const uint8_t *active,
                            const double *r, int64_t n_vox,
                            const int64_t *vox, double *out) {
  backproject_voxels_impl(C, theta, mask, active, r, 0, n_vox, vox, out);
}

void ora_support_backproject_voxels(const ora_ctx *C, const double *theta,
                                    const uint8_t *mask, const uint8_t *active,
                                    const double *r, int64_t n_vox,
                                    const int64_t *vox, double *out) {
  backproject_voxels_impl(C, theta, mask, active, r, 1, n_vox, vox, out);
}

/* Cross-correlation of the observed patch and its simulation at th
 * (Sec. IV-A eq. CC with population standard deviations), over samples valid
 * at th.  NCC is 0 when either standard deviation is 0. */
static double patch_ncc(const ora_ctx *C, int s, const double *th,
                        const double *X, const double *y, const uint8_t *mask) {
  pgeo g;
  patch_geometry(C, s, th, &g);
  int64_t n = (int64_t)g.w * g.h, cnt = 0;
  double *a = (double *)malloc(sizeof(double) * n);
  double *b = (double *)malloc(sizeof(double) * n);
  for (int64_t l = 0; l < n; ++l) {
    int64_t j = C->off[s] + l;
    if (mask && !mask[j]) continue;
    double yh, Z;
    int u = g.x0 + (int)(l % g.w), v = g.y0 + (int)(l / g.w);
    if (!sim_sample(C, &g, X, u, v, &yh, &Z)) continue;
    a[cnt] = y[j];
    b[cnt] = yh;
    ++cnt;
  }
  double res = 0;
  if (cnt > 0) {
    double ma = 0, mb = 0;
    for (int64_t q = 0; q < cnt; ++q) { ma += a[q]; mb += b[q]; }
    ma /= cnt; mb /= cnt;
    double va = 0, vb = 0, cab = 0;
    for (int64_t q = 0; q < cnt; ++q) {
      va += (a[q] - ma) * (a[q] - ma);
      vb += (b[q] - mb) * (b[q] - mb);
      cab += (a[q] - ma) * (b[q] - mb);
    }
    if (va > 0 && vb > 0) res = cab / sqrt(va * vb);
  }
  free(a);
  free(b);
  return res;
}

double ora_ncc_patch(const ora_ctx *C, int s, const double *th,
                     const double *X, const double *y, const uint8_t *mask) {
  return patch_ncc(C, s, th, X, y, mask);
}

void ora_ncc(const ora_ctx *C, const double *X, const double *y,
             const double *theta, const uint8_t *mask, double *ncc) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < C->M; ++s) ncc[s] = patch_ncc(C, s, theta + 6 * s, X, y, mask);
}

/* Partial derivatives of R = Rz Ry Rx with respect to rx, ry, rz, each the
 * product with the one elementary factor replaced by its derivative. */
static void rotation_derivatives(const double *th, double dR[3][9]) {
  double cx = cos(th[0]), sx = sin(th[0]);
  double cy = cos(th[1]), sy = sin(th[1]);
  double cz = cos(th[2]), sz = sin(th[2]);
  double Rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx};
  double Ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
  double Rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1};
  double dRx[9] = {0, 0, 0, 0, -sx, -cx, 0, cx, -sx};
  double dRy[9] = {-sy, 0, cy, 0, 0, 0, -cy, 0, -sy};
  double dRz[9] = {-sz, -cz, 0, cz, -sz, 0, 0, 0, 0};
  const double *f[3][3] = {{Rz, Ry, dRx}, {Rz, dRy, Rx}, {dRz, Ry, Rx}};
  for (int k = 0; k < 3; ++k) {
    double T[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int m = 0; m < 3; ++m) s += f[k][1][3 * i + m] * f[k][2][3 * m + j];
        T[3 * i + j] = s;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int m = 0; m < 3; ++m) s += f[k][0][3 * i + m] * T[3 * m + j];
        dR[k][3 * i + j] = s;
      }
  }
}

/* Cross-correlation of patch s at th (as patch_ncc) and its exact gradient
 * with respect to th (the six raw parameters), by the chain rule through
 * every simulated sample:
 *   d NCC / d b_q = (a_q - mean a) / sqrt(va vb) - NCC (b_q - mean b) / vb
 * (va, vb: sums of squared deviations), b_q = A_q / Z_q with
 * A_q = sum_i g_i X_i and Z_q = sum_i g_i over the sample's support, and
 *   d g_i / d th = -1/2 exp(-Q_i / 2) dQ_i / d th,
 *   Q = sum_a (d_a / sigma_a)^2,  d_a = F_a . (v_i - x),
 *   d d_a / d r_k = (dR_k E)_a . (v_i - x) - F_a . (dR_k (P - c)),
 *   d d_a / d t_m = -F[m][a].
 * The support and the set of valid samples are held fixed (their changes
 * have measure zero in th).  grad is zero where NCC is defined as zero. */
static double patch_ncc_grad(const ora_ctx *C, int s, const double *th,
                             const double *X, const double *y,
                             const uint8_t *mask, double grad[6]) {
  pgeo g;
  patch_geometry(C, s, th, &g);
  double dR[3][9], dF[3][9];
  rotation_derivatives(th, dR);
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0;
        for (int m = 0; m < 3; ++m) acc += dR[k][3 * i + m] * g.E[3 * m + j];
        dF[k][3 * i + j] = acc;
      }
  int64_t n = (int64_t)g.w * g.h, cnt = 0;
  double *a = (double *)malloc(sizeof(double) * n);
  double *b = (double *)malloc(sizeof(double) * n);
  double *db = (double *)malloc(sizeof(double) * 6 * n);
  const int nx = C->dims[0], ny = C->dims[1];
  for (int64_t l = 0; l < n; ++l) {
    int64_t j = C->off[s] + l;
    if (mask && !mask[j]) continue;
    int u = g.x0 + (int)(l % g.w), v = g.y0 + (int)(l / g.w);
    double yh, Z;
    if (!sim_sample(C, &g, X, u, v, &yh, &Z)) continue;
    /* the sample centre and its derivatives */
    double P[3], d[3], x[3], dx[6][3];
    for (int r = 0; r < 3; ++r)
      P[r] = g.A[3 * r] * u + g.A[3 * r + 1] * v + g.A[3 * r + 2] * g.slice + g.o[r];
    for (int r = 0; r < 3; ++r) d[r] = P[r] - g.c[r];
    for (int r = 0; r < 3; ++r)
      x[r] = g.R[3 * r] * d[0] + g.R[3 * r + 1] * d[1] + g.R[3 * r + 2] * d[2] +
             g.c[r] + g.t[r];
    for (int k = 0; k < 3; ++k)
      for (int r = 0; r < 3; ++r)
        dx[k][r] = dR[k][3 * r] * d[0] + dR[k][3 * r + 1] * d[1] + dR[k][3 * r + 2] * d[2];
    for (int m = 0; m < 3; ++m)
      for (int r = 0; r < 3; ++r) dx[3 + m][r] = r == m ? 1.0 : 0.0;
    int lo[3], hi[3];
    support_box(C, &g, x, lo, hi);
    double A = 0, Zs = 0, dA[6] = {0}, dZ[6] = {0};
    for (int kk = lo[2]; kk <= hi[2]; ++kk)
      for (int jj = lo[1]; jj <= hi[1]; ++jj)
        for (int ii = lo[0]; ii <= hi[0]; ++ii) {
          double w = psf_hat(C, &g, x, ii, jj, kk);
          if (w < 0) continue;
          double ip[3] = {(double)ii, (double)jj, (double)kk}, vw[3], dv[3];
          apply_affine(C->v2w, ip, vw);
          for (int r = 0; r < 3; ++r) dv[r] = vw[r] - x[r];
          double pr[3], Q = 0;
          for (int q = 0; q < 3; ++q) {
            pr[q] = g.F[q] * dv[0] + g.F[3 + q] * dv[1] + g.F[6 + q] * dv[2];
            Q += (pr[q] / g.sig[q]) * (pr[q] / g.sig[q]);
          }
          const double e = exp(-0.5 * Q);
          const double Xi = X[((int64_t)kk * ny + jj) * nx + ii];
          A += w * Xi;
          Zs += w;
          for (int p = 0; p < 6; ++p) {
            double dQ = 0;
            for (int q = 0; q < 3; ++q) {
              double dp = -(g.F[q] * dx[p][0] + g.F[3 + q] * dx[p][1] + g.F[6 + q] * dx[p][2]);
              if (p < 3)
                dp += dF[p][q] * dv[0] + dF[p][3 + q] * dv[1] + dF[p][6 + q] * dv[2];
              dQ += 2.0 * pr[q] * dp / (g.sig[q] * g.sig[q]);
            }
            const double dg = -0.5 * e * dQ;
            dA[p] += dg * Xi;
            dZ[p] += dg;
          }
        }
    a[cnt] = y[j];
    b[cnt] = A / Zs;
    for (int p = 0; p < 6; ++p) db[6 * cnt + p] = (dA[p] * Zs - A * dZ[p]) / (Zs * Zs);
    ++cnt;
  }
  double res = 0;
  for (int p = 0; p < 6; ++p) grad[p] = 0;
  if (cnt > 0) {
    double ma = 0, mb = 0;
    for (int64_t q = 0; q < cnt; ++q) { ma += a[q]; mb += b[q]; }
    ma /= cnt; mb /= cnt;
    double va = 0, vb = 0, cab = 0;
    for (int64_t q = 0; q < cnt; ++q) {
      va += (a[q] - ma) * (a[q] - ma);
      vb += (b[q] - mb) * (b[q] - mb);
      cab += (a[q] - ma) * (b[q] - mb);
    }
    if (va > 0 && vb > 0) {
      res = cab / sqrt(va * vb);
      for (int64_t q = 0; q < cnt; ++q) {
        const double dn = (a[q] - ma) / sqrt(va * vb) - res * (b[q] - mb) / vb;
        for (int p = 0; p < 6; ++p) grad[p] += dn * db[6 * q + p];
      }
    }
  }
  free(a);
  free(b);
  free(db);
  return res;
}

void ora_ncc_grad(const ora_ctx *C, const double *X, const double *y,
                  const double *theta, const uint8_t *mask, double *ncc,
                  double *grad) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < C->M; ++s)
    ncc[s] = patch_ncc_grad(C, s, theta + 6 * s, X, y, mask, grad + 6 * s);
}

/* Per-patch rigid registration by gradient ascent on NCC.  The paper names
 * "patch-wise gradient descent" (Sec. III, level I) and CC as the cost
 * (Sec. II); the optimiser is a reading.  Variables are q = (rho * angles,
 * translations): the three angles (radians) are scaled by the patch radius
 * rho (half-diagonal, mm) so that a unit change of any variable moves the
 * farthest patch pixel by about 1 mm.  Central finite-difference gradient
 * with step fd_h; a normalised trial step of length delta is accepted only on
 * strict improvement (then delta doubles, capped at step0, and the gradient is
 * recomputed), otherwise delta is halved; stop when delta < step_min, the
 * gradient vanishes, or after max_iter trial steps.  With grad_mode = 1 the
 * gradient is the exact one of patch_ncc_grad instead of the central
 * differences (d/dq_a = d/dth_a / scale_a).  Patches whose observed
 * standard deviation is below min_std keep their parameters.  Only patches
 * with reg[s] != 0 are registered (all when reg == NULL). */
void ora_register(const ora_ctx *C, const double *X, const double *y,
                  double *theta, const uint8_t *mask, const uint8_t *reg,
                  double step0, double step_min, double fd_h, int max_iter,
                  double min_std, int grad_mode, double *ncc_out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < C->M; ++s) {
    double *th = theta + 6 * s;
    if (reg && !reg[s]) {
      if (ncc_out) ncc_out[s] = patch_ncc(C, s, th, X, y, mask);
      continue;
    }
    /* observed standard deviation over unmasked samples */
    int64_t n = C->off[s + 1] - C->off[s], cnt = 0;
    double m = 0, m2 = 0;
    for (int64_t l = 0; l < n; ++l) {
      int64_t j = C->off[s] + l;
      if (mask && !mask[j]) continue;
      m += y[j]; ++cnt;
    }
    if (cnt) m /= cnt;
    for (int64_t l = 0; l < n; ++l) {
      int64_t j = C->off[s] + l;
      if (mask && !mask[j]) continue;
      m2 += (y[j] - m) * (y[j] - m);
    }
    double sd = cnt ? sqrt(m2 / cnt) : 0.0;
    double f0 = patch_ncc(C, s, th, X, y, mask);
    if (sd < min_std) {
      if (ncc_out) ncc_out[s] = f0;
      continue;
    }
    pgeo g0;
    patch_geometry(C, s, th, &g0);
    double su = sqrt(g0.A[0] * g0.A[0] + g0.A[3] * g0.A[3] + g0.A[6] * g0.A[6]);
    double sv = sqrt(g0.A[1] * g0.A[1] + g0.A[4] * g0.A[4] + g0.A[7] * g0.A[7]);
    double rho = 0.5 * sqrt((g0.w - 1) * (g0.w - 1) * su * su +
                            (g0.h - 1) * (g0.h - 1) * sv * sv);
    if (rho < 1.0) rho = 1.0;
    double sc[6] = {rho, rho, rho, 1, 1, 1};
    double q[6], tt[6], grad[6];
    for (int a = 0; a < 6; ++a) q[a] = th[a] * sc[a];
    double delta = step0;
    int have_grad = 0, moved = 0;
    for (int it = 0; it < max_iter; ++it) {
      if (delta < step_min) break;
      if (!have_grad && grad_mode == 1) {
        for (int b = 0; b < 6; ++b) tt[b] = q[b] / sc[b];
        double gth[6];
        patch_ncc_grad(C, s, tt, X, y, mask, gth);
        for (int a = 0; a < 6; ++a) grad[a] = gth[a] / sc[a];
        have_grad = 1;
      } else if (!have_grad) {
        for (int a = 0; a < 6; ++a) {
          for (int b = 0; b < 6; ++b) tt[b] = q[b] / sc[b];
          tt[a] = (q[a] + fd_h) / sc[a];
          double fp = patch_ncc(C, s, tt, X, y, mask);
          tt[a] = (q[a] - fd_h) / sc[a];
          double fm = patch_ncc(C, s, tt, X, y, mask);
          grad[a] = (fp - fm) / (2 * fd_h);
        }
        have_grad = 1;
      }
      double gn = 0;
      for (int a = 0; a < 6; ++a) gn += grad[a] * grad[a];
      gn = sqrt(gn);
      if (!(gn > 0)) break;
      double trial[6];
      for (int a = 0; a < 6; ++a) {
        trial[a] = q[a] + delta * grad[a] / gn;
        tt[a] = trial[a] / sc[a];
      }
      double ft = patch_ncc(C, s, tt, X, y, mask);
      if (ft > f0) {
        memcpy(q, trial, sizeof q);
        f0 = ft;
        have_grad = 0;
        moved = 1;
        delta = fmin(2.0 * delta, step0);
      } else {
        delta *= 0.5;
      }
    }
    if (moved)
      for (int a = 0; a < 6; ++a) th[a] = q[a] / sc[a];
    if (ncc_out) ncc_out[s] = f0;
  }
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following calls (n >= 1); a timing aid. */
void ora_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
