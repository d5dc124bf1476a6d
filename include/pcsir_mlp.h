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

/* Network outputs f [n] for BF16 feature rows X [n][256] through the training
 * path (the same GEMMs as pcsir_mlp_train_step). n a multiple of 64. */
pcsir_status pcsir_mlp_forward_train_path(const float *params_dev, const uint16_t *X_dev, int32_t n, float *f_dev,
                                          void *workspace_dev, size_t workspace_bytes, void *hip_stream);

/* Plain BF16 MFMA GEMM, C [M][N] (ldc) = op(A) op(B) in FP32, for tests:
 * A(m,k) = a_trans ? A[k lda + m] : A[m lda + k], B(k,n) = b_trans ? B[n ldb + k] : B[k ldb + n].
 * M, N multiples of 64, K a multiple of 32. */
pcsir_status pcsir_mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t lda, int32_t a_trans,
                                 const uint16_t *B, int32_t ldb, int32_t b_trans, float *C, int32_t ldc,
                                 void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PCSIR_MLP_H */
