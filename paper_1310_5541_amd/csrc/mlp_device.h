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

// Standard normal tail Phi(-|u|) without branches, from the rational-times-
// exponential form of erfc in Abramowitz & Stegun (1964), formula 7.1.26
// (absolute error of erf below 1.5e-7): for x = |u| / sqrt 2 and
// t = 1 / (1 + p x), erfc(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-x^2),
// and Phi(-|u|) = erfc(x) / 2. The 1 / sqrt 2 is folded into p and the 1 / 2
// into the a_i. Also returns e = e^(-u^2 / 2) for the density.
constexpr float AS_P2 = 0.3275911f * 0.70710678118654752f;
constexpr float AS_H1 = 0.5f * 0.254829592f, AS_H2 = 0.5f * -0.284496736f, AS_H3 = 0.5f * 1.421413741f,
                AS_H4 = 0.5f * -1.453152027f, AS_H5 = 0.5f * 1.061405429f;
__device__ __forceinline__ float norm_tail(float u, float &e) {
  const float t = __builtin_amdgcn_rcpf(fmaf(fabsf(u), AS_P2, 1.0f));
  const float poly = t * fmaf(fmaf(fmaf(fmaf(AS_H5, t, AS_H4), t, AS_H3), t, AS_H2), t, AS_H1);
  e = __builtin_amdgcn_exp2f((u * -0.72134752044448170f) * u);  // 2^(-u^2 / (2 ln 2))
  return poly * e;
}

// GELU g(u) = u Phi(u) = max(u, 0) - |u| Phi(-|u|), two hardware
// transcendentals (reciprocal, exp2) and ten FP32 operations, a third of the
// library erff's cost, whose two ranges diverge; and its derivative
// g'(u) = Phi(u) + u phi(u), phi(u) = e^(-u^2 / 2) / sqrt(2 pi).
__device__ __forceinline__ float gelu(float u) {
  float e;
  const float h = norm_tail(u, e);
  return fmaf(-fabsf(u), h, fmaxf(u, 0.0f));
}
__device__ __forceinline__ float gelu_grad(float u) {
  float e;
  const float h = norm_tail(u, e);
  const float c = u < 0.0f ? h : 1.0f - h;
  return fmaf(u * e, 0.39894228040143268f, c);
}

// Two floats to two BF16 (round to nearest even) in one word, a low.
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  const f32x2v v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
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

// gfx950 v_mfma_scale_f32_32x32x64_f8f6f4 with E4M3 operands and unit block
// scales (exponent 127): A 32x64, B 64x32, C 32x32 (FP32), C laid out as in
// the BF16 instruction. Lane l supplies 32 bytes of row l % 32 of A and of
// column l % 32 of B; the instruction pairs byte j of A in lane l with byte j
// of B in the lane of the same half (l / 32), so any assignment of the 64 k
// values to (half, byte) that both operands share gives A B. Here lane l takes
// k = 32 (l / 32) + j, j = 0..31.
typedef int i32x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f32x16 mfma_fp8_k64(const uint4 &a0, const uint4 &a1, const uint4 &b0, const uint4 &b1,
                                               f32x16 c) {
  const i32x8 a = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
  const i32x8 b = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// Two floats to two FP8 E4M3 bytes (hardware conversion, round to nearest,
// saturating to the largest finite value).
__device__ __forceinline__ uint32_t f2fp8x2(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}
constexpr float FP8_MAX = 448.0f;  // largest finite E4M3 value

// v rounded to E4M3 (after the clamp to +-FP8_MAX that the FP8 paths apply),
// as a float: every E4M3 value is exact in binary32 and in BF16.
__device__ __forceinline__ float fp8_value(float v) {
  const float q = fminf(fmaxf(v, -FP8_MAX), FP8_MAX);
  return __builtin_amdgcn_cvt_f32_fp8((int)f2fp8x2(q, 0.0f), 0);
}

}  // namespace pcsir
