/*
 * pvr_slic.h -- C ABI of the superpixel patch extraction (paper Sec. II,
 * "Patch Extraction"): simple linear iterative clustering (SLIC) of every
 * observed slice with the distance
 *     D^2 = d_c^2 + (d_s / a)^2 t^2
 * (d_c intensity, d_s spatial Euclidean distance in pixels, a the initial grid
 * step, t a compactness that adapts per superpixel).
 *
 * Images: FP32 [n_img][h][w] row-major, device.  Centres: FP32
 * [n_img][K][4] = (x, y, intensity, t), 16-byte aligned, K = ceil(h / a) *
 * ceil(w / a) per image, one per a x a grid cell in row-major cell order.
 * Labels: int32 [n_img][h][w], the centre index within the image, -1 where
 * no centre's window reaches.  Scratch: at least n_img uint64 elements of
 * device workspace.  The caller owns all memory; calls are asynchronous on
 * `stream`.
 *
 *  init:   centres at their cell's middle pixel position (the cell clipped to
 *          the image), intensity of the nearest pixel, t = t0;
 *  assign: every pixel takes, among the centres whose 2a x 2a window covers
 *          it (|x - c_x| <= a and |y - c_y| <= a), the one of least D^2 (FP32),
 *          ties to the lower index; the result does not depend on the order
 *          of evaluation (a packed atomic minimum);
 *  update: every centre becomes the mean (x, y, intensity) of its pixels (FP64
 *          sums in a fixed order) and t the largest |I_p - mean intensity|
 *          over them, at least t_min; a centre without pixels is unchanged.
 *          The labels must come from pvr_slic_assign with the same centres
 *          (a centre only looks for its pixels inside its own window);
 *  pvr_slic: init, then `iters` rounds of assign + update, then assign.
 *
 * Superpixel patches (the paper dilates every superpixel by gamma pixels
 * before it becomes a patch; here with the square (2 gamma + 1)^2 element):
 *  boxes:  int32 [n_img][K][4] = (x0, y0, bw, bh), the bounding box of
 *          superpixel k dilated by gamma and clipped to the image, (0,0,0,0)
 *          for a superpixel without pixels; labels and centres as left by
 *          pvr_slic (the final assignment's centres);
 *  pack:   for M patches given on the host as int32 [M][6] = (image, label,
 *          x0, y0, bw, bh), writes the patches' samples, patch s at
 *          [off_s, off_s + bw_s bh_s) row-major with off the exclusive prefix
 *          sum of bw bh: y[j] = the image's pixel, mask[j] = 1 where the
 *          pixel lies in the dilation of the label's pixels inside the box
 *          (for a box from pvr_slic_boxes: the dilated superpixel), else 0.
 *          Boxes must lie in the image and hold at most 65536 pixels.
 *          The table is staged into the caller's device workspace
 *          (pvr_slic_pack_workspace(M) bytes, 16-byte aligned) through a
 *          host array on the stack, synchronising `stream` once per 1024
 *          patches before the packing kernel is launched; the workspace
 *          must stay allocated until that kernel has run.  The library
 *          allocates no memory.
 * Errors: PVR_EINVAL for NULL pointers, non-positive sizes, a beyond 2^20 or
 * gamma < 0, PVR_ESHAPE when n_img * h * w exceeds 2^31, h or w exceeds
 * 2^20, K exceeds 2^20, n_img exceeds 65535, a packed box leaves its image
 * or holds more than 65536 pixels, or the pack workspace is too small.  Centres of any value (NaN included) are
 * safe: a centre whose window misses the image takes no pixel.
 */
#ifndef PVR_SLIC_H
#define PVR_SLIC_H

#include <stdint.h>

#include "pvr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Centres per image for an h x w image and step a (host; 0 on invalid sizes). */
int64_t pvr_slic_centres(int32_t h, int32_t w, int32_t a);

pvr_status pvr_slic_init(const float *img, int32_t n_img, int32_t h, int32_t w, int32_t a,
                         float t0, float *centres, hipStream_t stream);

pvr_status pvr_slic_assign(const float *img, int32_t n_img, int32_t h, int32_t w, int32_t a,
                           const float *centres, uint64_t *scratch, int32_t *labels,
                           hipStream_t stream);

pvr_status pvr_slic_update(const float *img, int32_t n_img, int32_t h, int32_t w, int32_t a,
                           const int32_t *labels, float t_min, float *centres,
                           hipStream_t stream);

pvr_status pvr_slic(const float *img, int32_t n_img, int32_t h, int32_t w, int32_t a,
                    float t0, float t_min, int32_t iters, uint64_t *scratch, float *centres,
                    int32_t *labels, hipStream_t stream);

pvr_status pvr_slic_boxes(const int32_t *labels, int32_t n_img, int32_t h, int32_t w, int32_t a,
                          const float *centres, int32_t gamma, int32_t *boxes,
                          hipStream_t stream);

/* Device workspace bytes of pvr_slic_pack for M patches (host; 0 for M <= 0). */
size_t pvr_slic_pack_workspace(int32_t M);

pvr_status pvr_slic_pack(const float *img, const int32_t *labels, int32_t n_img, int32_t h,
                         int32_t w, int32_t gamma, int32_t M, const int32_t *table,
                         void *workspace, size_t workspace_bytes, float *y, uint8_t *mask,
                         hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * pvr_slic_pack without a workspace.  The descriptor table goes to a
 * library-resident device array of PVR_SLIC_PACK_NOALLOC_MAX entries (2 MiB,
 * held by every device the library runs on until the process ends); more
 * patches give PVR_ESHAPE.  No device memory is allocated or freed.  Same
 * arguments, output and errors as pvr_slic_pack otherwise; synchronises
 * `stream` before returning, so calls made one after another may use any
 * streams, but calls that overlap in time on one device (other threads)
 * share the array and race. */
#define PVR_SLIC_PACK_NOALLOC_MAX 65536
pvr_status pvr_slic_pack_noalloc(const float *img, const int32_t *labels, int32_t n_img,
                                 int32_t h, int32_t w, int32_t gamma, int32_t M,
                                 const int32_t *table, float *y, uint8_t *mask,
                                 hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PVR_SLIC_H */
