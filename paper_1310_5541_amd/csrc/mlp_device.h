// Device pieces of the log-likelihood surrogate shared by the training GEMMs
// and the fused inference kernel of the pcSIR step: BF16 / FP8 conversions,
// exact GELU, the gfx950 MFMA fragment layout and the per-dummy features.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcsir {

constexpr int MLP_H = 256;        // hidden width
constexpr int MLP_F = 256;        // padded input width
constexpr int MLP_N_PARAMS = 3 * MLP_H * MLP_H + 4 * MLP_H + 1;
// offsets of the packed FP32 parameter vector (W[k][n]: input k -> unit n)
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_F * MLP_H;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H * MLP_H;
constexpr int MLP_OFF_W4 = MLP_OFF_B3 + MLP_H;
constexpr int MLP_OFF_B4 = MLP_OFF_W4 + MLP_H;
constexpr float MLP_OUT_SCALE = 100.0f;  // f predicts (l + A) / 100
constexpr float MLP_IN_SCALE = 0.01f;    // (z - I_bg) / 100, I / 100
constexpr float MLP_VEL_SCALE = 0.1f;    // v / 10

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t u) { return __builtin_bit_cast(float, (uint32_t)u << 16); }

// Exact GELU g(u) = u Phi(u) and g'(u) = Phi(u) + u phi(u).
__device__ __forceinline__ float gelu(float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float u) {
  return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) + u * expf(-0.5f * u * u) * 0.39894228040143268f;
}

// gfx950 v_mfma_f32_32x32x16_bf16: A 32x16, B 16x32, C 32x32 (FP32).
// Lane l holds A[l % 32][8 (l / 32) + i] and B[8 (l / 32) + i][l % 32],
// i = 0..7, and C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32], r = 0..15.
__device__ __forceinline__ int mfma_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
__device__ __forceinline__ int mfma_col(int lane) { return lane & 31; }
__device__ __forceinline__ int mfma_k0(int lane) { return 8 * (lane >> 5); }

__device__ __forceinline__ f32x16 mfma_bf16(const uint4 &a, const uint4 &b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}
// FP8 (E4M3) variant, same lane layout with 8 one-byte values per operand.
__device__ __forceinline__ f32x16 mfma_fp8(const uint2 &a, const uint2 &b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0,
                                                    0, 0);
}

// Two floats to two FP8 E4M3 bytes (hardware conversion, round to nearest,
// saturating to the largest finite value).
__device__ __forceinline__ uint32_t f2fp8x2(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

}  // namespace pcsir
