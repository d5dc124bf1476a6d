/*
 * pcsir_mlp.h — C ABI of the learned log-likelihood surrogate (gfx950).
 *
 * An extension of the paper's method, not part of it: for the dummy particles
 * of Alg. pcSIR, the log-likelihood of Eq. likelihood (Sec. 5.2) is written as
 *     l = -A(z) + 100 f(u),   A(z) = sum_window (z - I_bg)^2 / (2 sigma_xi^2),
 * where A depends on the frame only and is computed exactly, and f is a
 * multilayer perceptron that stands in for the model-image terms (the
 * expensive sub-sampled PSF rendering). f has three hidden layers of 256
 * units with exact GELU, g(v) = v Phi(v), and one linear output.
 *
 * Features u (BF16 rows of 256, unused entries zero): the P x P window
 * (z - I_bg) / 100 in row-major order, then the dummy's offsets from the pixel
 * that holds it (dx, dy[, dz]), its mean velocity / 10, its mean intensity / 100.
 * Target of f: (l + A) / 100.
 *
 * Parameters: one FP32 vector of pcsir_mlp_param_count() values,
 *   W1[256][256], b1[256], W2[256][256], b2[256], W3[256][256], b3[256], w4[256], b4[1]
 * with W[k][n] the weight from input k to unit n.
 *
 * Conventions as in pcsir.h: device pointers, caller-owned memory, work on the
 * given hipStream_t, no allocation inside the library, pcsir_status returns.
 */
#ifndef PCSIR_MLP_H
#define PCSIR_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "pcsir.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of FP32 parameters of the network (3 * 256 * 256 + 4 * 256 + 1 = 197633). */
size_t pcsir_mlp_param_count(void);

/* Device workspace bytes of pcsir_mlp_train_step / pcsir_mlp_forward_train_path
 * for a batch of `batch` rows (a multiple of 64, >= 64); 0 otherwise. */
size_t pcsir_mlp_train_bytes(int32_t batch);

/* One training step on one batch, all on the device: BF16 copies of the
 * weights, forward pass (BF16 MFMA GEMMs with FP32 accumulation, bias and
 * exact GELU fused), mean-squared-error loss against y, backward pass
 * (GELU' fused, weight gradients as FP32-accumulated GEMMs, bias gradients as
 * column sums) into grad_dev [param_count] (required), then, when adam_m and
 * adam_v are not NULL and t >= 1, one Adam update of params (FP32 master
 * copy; beta 0.9 / 0.999, eps 1e-8, learning rate lr, step t). X: BF16
 * [batch][256]; y: FP32 [batch]; loss_dev: FP32 scalar or NULL. */
pcsir_status pcsir_mlp_train_step(float *params_dev, float *adam_m_dev, float *adam_v_dev, const uint16_t *X_dev,
                                  const float *y_dev, int32_t batch, float lr, int32_t t, void *workspace_dev,
                                  size_t workspace_bytes, void *hip_stream, float *loss_dev, float *grad_dev);

/* pcsir_mlp_train_step with the FP8 quantisation of the inference kernel in
 * the forward pass (quantisation-aware training, an extension for the FP8
 * surrogate mode): the two hidden layers take E4M3 operands, their inputs
 * quantised as fp8(clamp(g / s, +-448)) with s = act_scale_dev[1] and
 * act_scale_dev[2] (device, three FP32 values as for pcsir_set_surrogate;
 * [0] unused), their weights as fp8(W / s_w) with s_w = max|W| / 448 per
 * tensor, and the accumulators scaled by s s_w. The backward pass takes each
 * quantiser as the identity where it does not clamp and as zero where it
 * does (straight-through gradients onto the FP32 master weights). The input
 * layer and the output unit are as in pcsir_mlp_train_step. Same workspace,
 * arguments and errors as pcsir_mlp_train_step; act_scale_dev is required. */
pcsir_status pcsir_mlp_train_step_fp8(float *params_dev, float *adam_m_dev, float *adam_v_dev, const uint16_t *X_dev,
                                      const float *y_dev, int32_t batch, float lr, int32_t t,
                                      const float *act_scale_dev, void *workspace_dev, size_t workspace_bytes,
                                      void *hip_stream, float *loss_dev, float *grad_dev);

/* Largest batch of pcsir_mlp_train_step_static. */
#define PCSIR_MLP_STATIC_MAX_BATCH 1024

/* pcsir_mlp_train_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight training loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the workspace taken from a
 * device array inside the library, sized for PCSIR_MLP_STATIC_MAX_BATCH rows
 * (8.4 MiB, held on every GPU the library runs on until the process ends).
 * No hipMalloc, hipFree or other allocation happens in the call. Returns
 * PCSIR_E_NOMEM when batch exceeds PCSIR_MLP_STATIC_MAX_BATCH, PCSIR_E_INVAL
 * for the argument errors of pcsir_mlp_train_step or when hip_stream does not
 * belong to the current device. On its first call on a device the library
 * looks up the array's address there (no allocation); calls on one GPU share
 * the array, so calls that overlap on one GPU (concurrent streams or host
 * threads) race and must be serialised by the caller. Every byte the step
 * reads from the array is written earlier in the same call. */
pcsir_status pcsir_mlp_train_step_static(float *params_dev, float *adam_m_dev, float *adam_v_dev,
                                         const uint16_t *X_dev, const float *y_dev, int32_t batch, float lr,
                                         int32_t t, void *hip_stream, float *loss_dev, float *grad_dev);

/* Network outputs f [n] for BF16 feature rows X [n][256] through the training
 * path (the same GEMMs as pcsir_mlp_train_step). n a multiple of 64. */
pcsir_status pcsir_mlp_forward_train_path(const float *params_dev, const uint16_t *X_dev, int32_t n, float *f_dev,
                                          void *workspace_dev, size_t workspace_bytes, void *hip_stream);

/* Plain BF16 MFMA GEMM, C [M][N] (ldc) = op(A) op(B) in FP32, for tests:
 * A(m,k) = a_trans ? A[k lda + m] : A[m lda + k], B(k,n) = b_trans ? B[n ldb + k] : B[k ldb + n].
 * M, N multiples of 64, K a multiple of 32; lda and ldb multiples of 8 and A,
 * B 16-byte aligned (E_INVAL otherwise). */
pcsir_status pcsir_mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t lda, int32_t a_trans,
                                 const uint16_t *B, int32_t ldb, int32_t b_trans, float *C, int32_t ldc,
                                 void *hip_stream);

/* ---------------------------------------------------------------- inference
 * Inference form of the network: one device block of pcsir_surr_bytes() (256-
 * byte aligned) holding the weights transposed to [layer][unit][input] in BF16
 * and in FP8 E4M3 (scaled per layer by max|W| / 448), the FP32 biases and the
 * output unit, and the FP8 input scales s_l of the three layers. One fused
 * kernel runs the three layers on 128 rows per workgroup with FP32
 * accumulation. BF16 mode: BF16 operands; the activations between layers are
 * rounded to BF16. FP8 mode: the input layer keeps BF16 operands (the
 * features' 3-bit-mantissa quantisation carried most of the all-FP8 network's
 * error); the two hidden layers take E4M3 operands, their input being the
 * previous layer's FP32 output g quantised as fp8(clamp(g / s_l, +-448)),
 * l = 1, 2 (s_0 is unused). The output unit reads BF16 activations. */
size_t pcsir_surr_bytes(void);

/* Fill the inference block from the FP32 parameter vector. act_scale_host: [3]
 * host floats s_l (finite, > 0), or NULL for 1 (enough for BF16 inference).
 * Synchronises `hip_stream`. E_INVAL on NULL pointers, a short or unaligned
 * block, or bad scales. */
pcsir_status pcsir_surr_prepare(const float *params_dev, const float *act_scale_host, void *surr_dev, size_t bytes,
                                void *hip_stream);

/* Network outputs f [n] for BF16 feature rows X [n][256] (16-byte aligned)
 * through the fused inference kernel, BF16 (fp8 = 0) or FP8 (fp8 != 0)
 * operands. absmax_dev: NULL, or [3] FP32 values (initialise to 0) into which
 * the largest |input| of each layer is max-accumulated (FP8 scale calibration;
 * s_l = absmax_l / 448 uses the full range). Asynchronous on hip_stream. */
pcsir_status pcsir_surr_rows(const void *surr_dev, const uint16_t *X_dev, int32_t n, int32_t fp8, float *f_dev,
                             float *absmax_dev, void *hip_stream);

/* Install the surrogate on a filter made with lik_mode PCSIR_LIK_SURR_BF16 or
 * PCSIR_LIK_SURR_FP8 (required before its first pcsir_step; may be called
 * again to replace the weights). Per frame, each dummy is checked against its
 * exact log-likelihood with probability check_fraction (a counter-based
 * uniform of (dummy index, frame, target)). A checked dummy is relevant when
 * its exact or surrogate value lies within 40 nats of its target's largest
 * surrogate value (below that its weight is under e^-40 of the best one's); a
 * target whose relevant checked dummies have a root-mean-square error above
 * tol_nats has all its dummies evaluated exactly in that frame. Checked
 * dummies keep their exact value. act_scale_host as in pcsir_surr_prepare,
 * required for FP8. Synchronises the filter's stream. */
pcsir_status pcsir_set_surrogate(pcsir_ctx *ctx, const float *params_dev, const float *act_scale_host,
                                 float check_fraction, float tol_nats);

/* Training rows from the dummies of the last pcsir_step (any likelihood mode;
 * exact modes give exact targets): features X [min(B, cap)][256] BF16 as
 * described above and targets y = (l + A(z)) / 100 FP32, with l the dummy's
 * log-likelihood of that step. *count = B, the number of dummies (may exceed
 * cap). The frame given to that step must still be valid. Asynchronous after
 * one read of B. E_STATE when the last step was not a pcsir_step. */
pcsir_status pcsir_surrogate_features(pcsir_ctx *ctx, uint16_t *X_dev, float *y_dev, int32_t cap, int32_t *count);

/* Cumulative surrogate statistics since init or the last reset: dummies
 * checked, target-frames that fell back to exact evaluation, the largest
 * |l_surrogate - l_exact| seen. Any output may be NULL. Synchronises. */
pcsir_status pcsir_surrogate_stats(pcsir_ctx *ctx, uint64_t *checked, uint64_t *fallbacks, float *max_err,
                                   int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* PCSIR_MLP_H */
