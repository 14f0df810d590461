/*
 * pvr_cnn.h -- C ABI of the learned registration initialiser.
 *
 * Not a part of the paper's method: the paper registers every patch by
 * gradient-based optimisation of the cross-correlation (Sec. II, Sec. III
 * level I).  This network only proposes a starting motion for that
 * registration: from the pair (observed 64 x 64 patch, the same patch
 * simulated from the current volume at the current motion) it regresses the
 * 6-DoF correction; the NCC registration then refines the proposal and
 * replaces it when its NCC is worse than the unchanged motion.
 *
 * Network: 8 convolutions 3x3 (pad 1, ReLU) with channels 32, 32, 64, 64, 64,
 * 64, 64, 64 and stride 2 at layers 2, 4 and 6, then one fully connected
 * layer from the whole 8 x 8 x 64 map to 6 outputs (position-dependent
 * weights: a rotation displaces the image differently across the patch).  Activations and weights BF16 (MFMA),
 * accumulation and training state FP32.
 *
 * Conventions: device pointers; BF16 values are stored as uint16_t (upper
 * half of the FP32 bit pattern, round to nearest even); activations NHWC
 * ([B][H][W][C]); conv weights [Cout][3][3][Cin] (forward and FP32 master)
 * and [3][3][Cin][Cout] (data gradient).  BF16 activations, weights,
 * activation gradients and the FP32 scratch arrays are 16-byte aligned (they
 * are read 16 bytes at a time), other FP32 and int32 arrays 4-byte aligned;
 * a misaligned pointer gives PVR_EINVAL.  All calls are asynchronous on
 * `stream` and return pvr_status (pvr_last_error() explains failures).
 * Supported (cin, cout, stride): (2,32,1) (32,32,2) (32,64,1) (64,64,2)
 * (64,64,1) (32,32,1) (64,32,1); the data gradient needs cin >= 16.
 */
#ifndef PVR_CNN_H
#define PVR_CNN_H

#include <stdint.h>

#include "pvr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PVR_CNN_SIDE 64

/* out = relu(conv3x3(in) + bias) (relu = 0: no ReLU).  in [B][H][W][cin],
 * w [cout][3][3][cin], bias [cout] FP32, out [B][Ho][Wo][cout] with
 * Ho = (H - 1)/stride + 1. */
pvr_status pvr_cnn_conv_fwd(const uint16_t *in, const uint16_t *w,
                            const float *bias, uint16_t *out, int32_t B,
                            int32_t H, int32_t W, int32_t cin, int32_t cout,
                            int32_t stride, int32_t relu, hipStream_t stream);

/* Gradient with respect to the layer input: gin = conv^T(gout * [out > 0]).
 * gout, out [B][Ho][Wo][cout] (out = the layer's ReLU output), wt
 * [3][3][cin][cout], gin [B][H][W][cin]. */
pvr_status pvr_cnn_conv_dgrad(const uint16_t *gout, const uint16_t *out,
                              const uint16_t *wt, uint16_t *gin, int32_t B,
                              int32_t H, int32_t W, int32_t cin, int32_t cout,
                              int32_t stride, hipStream_t stream);

/* Bytes of FP32 scratch pvr_cnn_conv_wgrad needs for this layer shape
 * (host, no device call). */
int64_t pvr_cnn_wgrad_scratch(int32_t B, int32_t H, int32_t W, int32_t cin,
                              int32_t cout, int32_t stride);

/* Weight and bias gradients: dw [cout][3][3][cin], db [cout] (FP32) from
 * gout and out (as in dgrad) and the layer input in.  Per-chunk partial sums
 * in `scratch` are added in a fixed order (deterministic). */
pvr_status pvr_cnn_conv_wgrad(const uint16_t *gout, const uint16_t *out,
                              const uint16_t *in, float *scratch, float *dw,
                              float *db, int32_t B, int32_t H, int32_t W,
                              int32_t cin, int32_t cout, int32_t stride,
                              hipStream_t stream);

/* Network input for B patches of a built plan: out [B][64][64][2], channel 0
 * the observed patch, channel 1 the simulated one, each standardised over
 * the patch's valid samples (invalid samples 0).  patch_ids [B] (device);
 * an id outside [0, M) gives an all-zero pair.  Every patch of the plan must
 * be 64 x 64. */
pvr_status pvr_cnn_pack_pairs(const pvr_plan *plan, const int32_t *patch_ids,
                              int32_t B, const float *y_obs, const float *y_sim,
                              uint16_t *out, hipStream_t stream);

/* Bytes of FP32 scratch pvr_cnn_head needs in training (host). */
int64_t pvr_cnn_head_scratch(int32_t B);

/* Head: pred[b][k] = sum_{q,c} act[b][q][c] wfc[q][c][k] + bfc[k] with act
 * [B][hw][64], wfc [hw][64][6] FP32, bfc [6], pred [B][6].  With target
 * [B][6] (nullable for inference) and per-output loss weights loss_w [6]:
 * loss [1] = sum_b sum_k loss_w[k] (pred - target)^2 / (2 B), and the
 * gradients gact (w.r.t. act, BF16), dwfc [hw][64][6], dbfc [6] (sums over
 * the batch in sample order). */
pvr_status pvr_cnn_head(const uint16_t *act, int32_t B, int32_t hw,
                        const float *wfc, const float *bfc, const float *target,
                        const float *loss_w, float *pred, float *loss,
                        uint16_t *gact, float *dwfc, float *dbfc,
                        float *scratch, hipStream_t stream);

/* Adam step `step` (>= 1) on FP32 master weights w [n] with gradient g,
 * moments m, v; refreshes w_bf16 [n] (nullable) and, for conv weights,
 * wt_bf16 ([3][3][cin][cout], nullable; needs n = cout * 9 * cin).
 * step = 0 only refreshes the BF16 copies. */
pvr_status pvr_cnn_adam(float *w, const float *g, float *m, float *v, int32_t n,
                        float lr, float beta1, float beta2, float eps,
                        int32_t step, uint16_t *w_bf16, uint16_t *wt_bf16,
                        int32_t cout, int32_t cin, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PVR_CNN_H */
