// Fused surrogate inference for the dummies of a pcSIR step (and for feature
// rows, for tests and calibration): features -> three MFMA layers with GELU
// -> output unit -> l = 100 f - A(z). BF16 or FP8 (E4M3, per-tensor scales)
// operands, FP32 accumulation.
//
// One block of eight waves takes SURR_ROWS = 128 rows at a time; wave w owns
// units [32 w, 32 w + 32) of every layer, so each weight read from L2 serves
// all 128 rows, and two blocks per compute unit (four waves per SIMD) let one
// wave's matrix products run while another evaluates its GELUs. The product is formed transposed, C^T = W^T X^T: the MFMA's
// first operand is the weights (k contiguous in the inference layout), the
// second the activations in LDS, and each lane's accumulators then hold four
// consecutive units of one row, which the epilogue (bias, GELU, rounding)
// stores as one 8-byte (BF16) or 4-byte (FP8) LDS write. The last layer's
// epilogue forms the output unit directly from registers.
#pragma once
#include "device_util.h"
#include "kernels.h"
#include "mlp_device.h"

namespace pcsir {

constexpr int SURR_NW = 8;                // waves per block
constexpr int SURR_WU = MLP_H / SURR_NW;  // units per wave (a multiple of 32)
constexpr int SURR_NJ = SURR_WU / 32;     // 32-unit MFMA tiles per wave
constexpr int SURR_TPB = 64 * SURR_NW;
constexpr int SURR_ROWS = 128;            // rows per block
constexpr int SURR_RT = SURR_ROWS / 32;   // 32-row MFMA tiles
constexpr int SURR_LD = MLP_F + 8;        // LDS row stride (bf16 elements)
constexpr int SURR_LD8 = MLP_F + 16;      // LDS row stride (fp8 bytes)

// LDS bytes of the activations of SURR_ROWS rows (BF16 layout; the FP8
// layout of the hidden layers' inputs, SURR_ROWS x SURR_LD8 bytes, fits in it)
constexpr int SURR_ACT_BYTES = SURR_ROWS * SURR_LD * 2;
static_assert(SURR_ROWS * SURR_LD8 <= SURR_ACT_BYTES, "FP8 activations fit the buffer");

// Loads through global-address-space pointers (see as_global).
typedef uint32_t u32v4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32v2 __attribute__((ext_vector_type(2)));
typedef float f32v4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 gload_u4(const void *ptr) {
  const u32v4 v = *(const __attribute__((address_space(1))) u32v4 *)ptr;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 gload_u2(const void *ptr) {
  const u32v2 v = *(const __attribute__((address_space(1))) u32v2 *)ptr;
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float4 gload_f4(const float *ptr) {
  const f32v4 v = *(const __attribute__((address_space(1))) f32v4 *)ptr;
  return make_float4(v.x, v.y, v.z, v.w);
}

// Weights in inference layout, prepared on the device from the FP32 master
// vector: WT[l][n][k] (k contiguous, so a lane's 8 k values are one load).
// One device block of surr_block_bytes(), sub-arrays at 256-byte boundaries.
struct SurrWeights {
  const uint16_t *wt;     // [3][256][256] bf16
  const uint8_t *wt8;     // [3][256][256] fp8 (W / s_w)
  const float *bias;      // [3][256]
  const float *w4;        // [256]
  const float *b4;        // [1]
  const float *scale_w;   // [3] FP8 weight scales
  const float *scale_x;   // [3] FP8 input scales of each layer
};

constexpr size_t surr_align(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t SURR_OFF_WT = 0;
constexpr size_t SURR_OFF_WT8 = SURR_OFF_WT + surr_align(2 * 3 * (size_t)MLP_H * MLP_F);
constexpr size_t SURR_OFF_BIAS = SURR_OFF_WT8 + surr_align(3 * (size_t)MLP_H * MLP_F);
constexpr size_t SURR_OFF_W4 = SURR_OFF_BIAS + surr_align(4 * 3 * (size_t)MLP_H);
constexpr size_t SURR_OFF_B4 = SURR_OFF_W4 + surr_align(4 * (size_t)MLP_H);
constexpr size_t SURR_OFF_SW = SURR_OFF_B4 + 256;
constexpr size_t SURR_OFF_SX = SURR_OFF_SW + 256;
constexpr size_t SURR_BYTES = SURR_OFF_SX + 256;

inline SurrWeights surr_view(void *base) {
  char *b = (char *)base;
  SurrWeights w;
  w.wt = (const uint16_t *)(b + SURR_OFF_WT);
  w.wt8 = (const uint8_t *)(b + SURR_OFF_WT8);
  w.bias = (const float *)(b + SURR_OFF_BIAS);
  w.w4 = (const float *)(b + SURR_OFF_W4);
  w.b4 = (const float *)(b + SURR_OFF_B4);
  w.scale_w = (const float *)(b + SURR_OFF_SW);
  w.scale_x = (const float *)(b + SURR_OFF_SX);
  return w;
}

// The dummies of a pcSIR step as the surrogate reads them.
struct DummyView {
  const int32_t *dpix;   // [dim][NT]
  const float *doff;     // [dim][NT]
  const float *dvel;     // [dim][NT]
  const float *dint;     // [NT]
  const int32_t *seg_t;  // [NT]
};

template <int DIM>
__device__ __forceinline__ float dummy_feature(const Params &p, const DummyView &dv, const float *frame, uint32_t s,
                                               int f) {
  const int P2 = p.P * p.P;
  const uint32_t NT = p.NT;
  if (f < P2) {
    const int t = dv.seg_t[s];
    const gfloat *fr = as_global(frame) + (p.per_target_frames ? (size_t)t * p.H * p.W : 0);
    const int c = dv.dpix[s] + f % p.P - p.R;
    const int r = dv.dpix[(size_t)NT + s] + f / p.P - p.R;
    const float zb = (c >= 0 && c < p.W && r >= 0 && r < p.H) ? fr[(size_t)r * p.W + c] - p.i_bg : 0.0f;
    return zb * MLP_IN_SCALE;
  }
  f -= P2;
  // in-plane offsets from the pixel; the axial coordinate (3D) in full / 10
  if (f < 2) return dv.doff[(size_t)f * NT + s];
  if (f < DIM) return ((float)dv.dpix[(size_t)f * NT + s] + dv.doff[(size_t)f * NT + s]) * MLP_VEL_SCALE;
  f -= DIM;
  if (f < DIM) return dv.dvel[(size_t)f * NT + s] * MLP_VEL_SCALE;
  f -= DIM;
  if (f == 0) return dv.dint[s] * MLP_IN_SCALE;
  return 0.0f;
}

template <int DIM>
__device__ __forceinline__ double dummy_data_term(const Params &p, const DummyView &dv, const float *frame, uint32_t s) {
  const int t = dv.seg_t[s];
  const gfloat *fr = as_global(frame) + (p.per_target_frames ? (size_t)t * p.H * p.W : 0);
  const int c0 = dv.dpix[s], r0 = dv.dpix[(size_t)p.NT + s];
  double a = 0.0;
  for (int r = r0 - p.R; r <= r0 + p.R; ++r)
    for (int c = c0 - p.R; c <= c0 + p.R; ++c)
      if (c >= 0 && c < p.W && r >= 0 && r < p.H) {
        const double zb = (double)fr[(size_t)r * p.W + c] - (double)p.i_bg;
        a += zb * zb;
      }
  return a * p.inv2sxi2;
}

// One layer's product for this wave's SURR_WU units and the block's SURR_ROWS
// rows: acc[j][i] is the 32-unit tile j (units SURR_WU w + 32 j + ...) of row
// tile i (rows 32 i + ...), transposed: lane l holds units
// 8 (r / 4) + 4 (l / 32) + r % 4 of row l % 32. Weights stream from L2 three
// k-steps ahead of the MFMAs; activations come from LDS.
template <bool FP8>
__device__ __forceinline__ void surr_gemm(const SurrWeights &sw, int l, const uint8_t *act,
                                          f32x16 (&acc)[SURR_NJ][SURR_RT]) {
  const int lane = lane_id(), w = wave_id();
#pragma unroll
  for (int j = 0; j < SURR_NJ; ++j)
#pragma unroll
    for (int i = 0; i < SURR_RT; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[j][i][r] = 0.0f;
  constexpr int KS = MLP_F / 16;  // k-steps of 16
  constexpr int PF = 3;           // weight k-steps in flight
  const size_t wrow = (size_t)(SURR_WU * w + mfma_col(lane)) * MLP_F + mfma_k0(lane);
  if (!FP8) {
    const uint16_t *W = sw.wt + (size_t)l * MLP_H * MLP_F + wrow;
    const uint16_t *X = (const uint16_t *)act + mfma_col(lane) * SURR_LD + mfma_k0(lane);
    uint4 wq[PF][SURR_NJ];
#pragma unroll
    for (int s = 0; s < PF; ++s)
#pragma unroll
      for (int j = 0; j < SURR_NJ; ++j) wq[s][j] = gload_u4(W + 32 * j * MLP_F + 16 * s);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      uint4 a[SURR_NJ];
#pragma unroll
      for (int j = 0; j < SURR_NJ; ++j) {
        a[j] = wq[ks % PF][j];
        if (ks + PF < KS) wq[ks % PF][j] = gload_u4(W + 32 * j * MLP_F + 16 * (ks + PF));
      }
#pragma unroll
      for (int i = 0; i < SURR_RT; ++i) {
        const uint4 xb = *reinterpret_cast<const uint4 *>(X + 32 * i * SURR_LD + 16 * ks);
#pragma unroll
        for (int j = 0; j < SURR_NJ; ++j) acc[j][i] = mfma_bf16(a[j], xb, acc[j][i]);
      }
    }
  } else {
    // K = 64 per instruction: lane l takes k = 64 ks + 32 (l / 32) + 0..31
    constexpr int KS8 = MLP_F / 64, PF8 = 2;
    const size_t w8row = (size_t)(SURR_WU * w + mfma_col(lane)) * MLP_F + 32 * (lane >> 5);
    const uint8_t *W = sw.wt8 + (size_t)l * MLP_H * MLP_F + w8row;
    const uint8_t *X = act + mfma_col(lane) * SURR_LD8 + 32 * (lane >> 5);
    uint4 wq[PF8][SURR_NJ][2];
#pragma unroll
    for (int s = 0; s < PF8; ++s)
#pragma unroll
      for (int j = 0; j < SURR_NJ; ++j) {
        wq[s][j][0] = gload_u4(W + 32 * j * MLP_F + 64 * s);
        wq[s][j][1] = gload_u4(W + 32 * j * MLP_F + 64 * s + 16);
      }
#pragma unroll
    for (int ks = 0; ks < KS8; ++ks) {
      uint4 a[SURR_NJ][2];
#pragma unroll
      for (int j = 0; j < SURR_NJ; ++j) {
        a[j][0] = wq[ks % PF8][j][0];
        a[j][1] = wq[ks % PF8][j][1];
        if (ks + PF8 < KS8) {
          wq[ks % PF8][j][0] = gload_u4(W + 32 * j * MLP_F + 64 * (ks + PF8));
          wq[ks % PF8][j][1] = gload_u4(W + 32 * j * MLP_F + 64 * (ks + PF8) + 16);
        }
      }
#pragma unroll
      for (int i = 0; i < SURR_RT; ++i) {
        const uint4 x0 = *reinterpret_cast<const uint4 *>(X + 32 * i * SURR_LD8 + 64 * ks);
        const uint4 x1 = *reinterpret_cast<const uint4 *>(X + 32 * i * SURR_LD8 + 64 * ks + 16);
#pragma unroll
        for (int j = 0; j < SURR_NJ; ++j) acc[j][i] = mfma_fp8_k64(a[j][0], a[j][1], x0, x1, acc[j][i]);
      }
    }
  }
}

// Pre-activation of the lane's unit n (bias b) from accumulator value a.
template <bool FP8>
__device__ __forceinline__ float surr_pre(float a, float sc, float b) {
  return fmaf(a, FP8 ? sc : 1.0f, b);
}

// Epilogue of hidden layer l < 2: g = gelu(acc * scale + bias) into the
// activations for layer l + 1, rounded to BF16, or (FP8) quantised directly
// with that layer's input scale, fp8(clamp(g / s_{l+1})). IN8: this layer's
// operands were FP8 (the accumulator then carries the scales). With
// `absmax` (BF16), the largest |bf16(g)| is max-accumulated into absmax[l + 1].
template <bool IN8, bool FP8>
__device__ __forceinline__ void surr_store(const SurrWeights &sw, int l, const f32x16 (&acc)[SURR_NJ][SURR_RT],
                                           uint8_t *act, unsigned int *absmax) {
  const int lane = lane_id(), w = wave_id();
  const float sc = IN8 ? sw.scale_x[l] * sw.scale_w[l] : 1.0f;
  const float inv = FP8 ? 1.0f / sw.scale_x[l + 1] : 1.0f;
  const float *bias = sw.bias + l * MLP_H;
  float mx = 0.0f;
#pragma unroll
  for (int j = 0; j < SURR_NJ; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = SURR_WU * w + 32 * j + 8 * q + 4 * (lane >> 5);
      const float4 b = gload_f4(bias + n);
#pragma unroll
      for (int i = 0; i < SURR_RT; ++i) {
        const int m = 32 * i + mfma_col(lane);
        const float g0 = gelu(surr_pre<IN8>(acc[j][i][4 * q + 0], sc, b.x));
        const float g1 = gelu(surr_pre<IN8>(acc[j][i][4 * q + 1], sc, b.y));
        const float g2 = gelu(surr_pre<IN8>(acc[j][i][4 * q + 2], sc, b.z));
        const float g3 = gelu(surr_pre<IN8>(acc[j][i][4 * q + 3], sc, b.w));
        if (FP8) {
          const float q0 = fminf(fmaxf(g0 * inv, -FP8_MAX), FP8_MAX);
          const float q1 = fminf(fmaxf(g1 * inv, -FP8_MAX), FP8_MAX);
          const float q2 = fminf(fmaxf(g2 * inv, -FP8_MAX), FP8_MAX);
          const float q3 = fminf(fmaxf(g3 * inv, -FP8_MAX), FP8_MAX);
          *reinterpret_cast<uint32_t *>(act + m * SURR_LD8 + n) = f2fp8x2(q0, q1) | (f2fp8x2(q2, q3) << 16);
        } else {
          uint2 v;
          v.x = f2bf2(g0, g1);
          v.y = f2bf2(g2, g3);
          if (absmax)
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(__uint_as_float(v.x << 16)), fabsf(__uint_as_float(v.x & 0xFFFF0000u))),
                                 fmaxf(fabsf(__uint_as_float(v.y << 16)), fabsf(__uint_as_float(v.y & 0xFFFF0000u)))));
          *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(act) + m * SURR_LD + n) = v;
        }
      }
    }
  if (!FP8 && absmax) {
    mx = wave_max(mx);
    if (lane == 0) atomicMax(&absmax[l + 1], __float_as_uint(mx));
  }
}

// Epilogue of the last hidden layer fused with the output unit: this wave's
// share sum_n bf16(gelu(z_n)) w4_n of every row into fpart[w][row].
template <bool FP8>
__device__ __forceinline__ void surr_head(const SurrWeights &sw, const f32x16 (&acc)[SURR_NJ][SURR_RT],
                                          float (*fpart)[SURR_ROWS]) {
  const int lane = lane_id(), w = wave_id();
  const float sc = FP8 ? sw.scale_x[2] * sw.scale_w[2] : 1.0f;
  const float *bias = sw.bias + 2 * MLP_H;
  float part[SURR_RT];
#pragma unroll
  for (int i = 0; i < SURR_RT; ++i) part[i] = 0.0f;
#pragma unroll
  for (int j = 0; j < SURR_NJ; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = SURR_WU * w + 32 * j + 8 * q + 4 * (lane >> 5);
      const float4 b = gload_f4(bias + n);
      const float4 v = gload_f4(sw.w4 + n);
#pragma unroll
      for (int i = 0; i < SURR_RT; ++i) {
        const uint32_t h01 = f2bf2(gelu(surr_pre<FP8>(acc[j][i][4 * q + 0], sc, b.x)),
                                   gelu(surr_pre<FP8>(acc[j][i][4 * q + 1], sc, b.y)));
        const uint32_t h23 = f2bf2(gelu(surr_pre<FP8>(acc[j][i][4 * q + 2], sc, b.z)),
                                   gelu(surr_pre<FP8>(acc[j][i][4 * q + 3], sc, b.w)));
        part[i] = fmaf(__uint_as_float(h01 << 16), v.x, part[i]);
        part[i] = fmaf(__uint_as_float(h01 & 0xFFFF0000u), v.y, part[i]);
        part[i] = fmaf(__uint_as_float(h23 << 16), v.z, part[i]);
        part[i] = fmaf(__uint_as_float(h23 & 0xFFFF0000u), v.w, part[i]);
      }
    }
#pragma unroll
  for (int i = 0; i < SURR_RT; ++i) {
    // lanes l and l + 32 hold the two halves of the wave's units of row l % 32
    const float both = part[i] + __shfl_xor(part[i], 32, WAVE);
    if (lane < 32) fpart[w][32 * i + lane] = both;
  }
}

// The three layers and the output unit on the block's rows in `act` (BF16
// features); the network output of row m is sw.b4 + sum_w fpart[w][m] (fixed
// order). FP8: the input layer keeps BF16 operands (quantising the window's
// pixels to a 3-bit mantissa carried most of the FP8 network's error) and
// quantises its output for the two FP8 hidden layers.
template <bool FP8>
__device__ __forceinline__ void surr_layers(const SurrWeights &sw, uint8_t *act, float (*fpart)[SURR_ROWS],
                                            unsigned int *absmax) {
  f32x16 acc[SURR_NJ][SURR_RT];
  for (int l = 0; l < 3; ++l) {
    const bool in8 = FP8 && l > 0;
    if (in8)
      surr_gemm<true>(sw, l, act, acc);
    else
      surr_gemm<false>(sw, l, act, acc);
    __syncthreads();  // every wave has read the layer's input
    if (l < 2) {
      if (in8)
        surr_store<true, FP8>(sw, l, acc, act, absmax);
      else
        surr_store<false, FP8>(sw, l, acc, act, absmax);
      __syncthreads();
    } else {
      surr_head<FP8>(sw, acc, fpart);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ float surr_out(const SurrWeights &sw, const float (*fpart)[SURR_ROWS], int m) {
  float f = sw.b4[0];
#pragma unroll
  for (int w = 0; w < SURR_NW; ++w) f += fpart[w][m];
  return f;
}

// One feature value into the activations (BF16).
__device__ __forceinline__ void surr_put(uint8_t *act, int m, int f, float v) {
  reinterpret_cast<uint16_t *>(act)[m * SURR_LD + f] = f2bf(v);
}

// Surrogate log-likelihood of every dummy of the step: ll[s] = 100 f - A(z),
// and every target's largest surrogate value (tmax, ordered bits, atomic max;
// dummies are sorted by target, so a block's rows span consecutive targets).
// Features: wave w takes rows w, w + SURR_NW, ..., SURR_FR rows at a time; a
// row's P^2 window pixels are spread over the lanes (pixel k = lane + 64 j),
// and every pixel of the SURR_FR rows is loaded before any is used (from
// clamped coordinates, pixels outside the frame then reading as the
// background), so that the loads overlap instead of waiting one by one. The
// squared residuals of a row add up for A(z) in binary64, in a fixed order
// (per lane, then the wave's butterfly).
constexpr int SURR_WJ = (MLP_F + WAVE - 1) / WAVE;  // window pixels per lane (P^2 < 256)
constexpr int SURR_FR = 2;                          // rows whose windows are loaded together
// PP: the window side when known at compile time (0: p.P).
template <int DIM, bool FP8, int PP = 0>
__global__ __launch_bounds__(SURR_TPB) __attribute__((amdgpu_waves_per_eu(4))) void k_surr_infer(Params p, DummyView dv, const uint64_t *__restrict__ meta,
                                                            const StepDesc *__restrict__ desc, SurrWeights sw,
                                                            double *__restrict__ ll,
                                                            unsigned long long *__restrict__ tmax) {
  static_assert((SURR_ROWS / SURR_NW) % SURR_FR == 0, "rows of a wave in groups of SURR_FR");
  __shared__ __attribute__((aligned(16))) uint8_t act[SURR_ACT_BYTES];
  __shared__ float fpart[SURR_NW][SURR_ROWS];
  __shared__ double aw[SURR_ROWS];
  __shared__ int rinfo[4][SURR_ROWS];  // frame offset, c0, r0, valid
  __shared__ unsigned long long tmx[SURR_ROWS];
  const uint32_t B = (uint32_t)meta[META_B];
  const uint32_t NT = p.NT;
  const gfloat *frame = as_global(desc->frame);
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
  const int P = PP ? PP : p.P, R = PP ? (PP - 1) / 2 : p.R, P2 = P * P, NF = P2 + 2 * DIM + 1;
  for (uint32_t s0 = blockIdx.x * SURR_ROWS; s0 < B; s0 += gridDim.x * SURR_ROWS) {
    if (tid < SURR_ROWS) {
      const uint32_t s = s0 + tid;
      const bool valid = s < B;
      const uint32_t sc = valid ? s : B - 1;  // clamped: unconditional loads
      const int t = dv.seg_t[sc];
      const int c0 = dv.dpix[sc], r0 = dv.dpix[(size_t)NT + sc];
      // state features: offsets from the pixel (in-plane), the axial
      // coordinate in full / 10 (3D), velocities / 10, intensity / 100
      float st[2 * DIM + 1];
#pragma unroll
      for (int a = 0; a < 2; ++a) st[a] = dv.doff[(size_t)a * NT + sc];
      if (DIM == 3) st[2] = ((float)dv.dpix[2 * (size_t)NT + sc] + dv.doff[2 * (size_t)NT + sc]) * MLP_VEL_SCALE;
#pragma unroll
      for (int a = 0; a < DIM; ++a) st[DIM + a] = dv.dvel[(size_t)a * NT + sc] * MLP_VEL_SCALE;
      st[2 * DIM] = dv.dint[sc] * MLP_IN_SCALE;
      rinfo[0][tid] = p.per_target_frames ? t * p.H * p.W : 0;
      rinfo[1][tid] = valid ? c0 : 0;
      rinfo[2][tid] = valid ? r0 : 0;
      rinfo[3][tid] = valid;
#pragma unroll
      for (int a = 0; a < 2 * DIM + 1; ++a) surr_put(act, tid, P2 + a, valid ? st[a] : 0.0f);
      for (int f = NF; f < MLP_F; ++f) surr_put(act, tid, f, 0.0f);
    }
    __syncthreads();
    // this lane's window pixels: offsets (dx, dy) from the window's corner,
    // formed anew for every group of rows (the empty asm keeps the compiler
    // from hoisting them out of the loop, which would keep them in registers
    // across the layers and spill)
    int wdx[SURR_WJ], wdy[SURR_WJ];
#pragma unroll
    for (int j = 0; j < SURR_WJ; ++j) {
      int k = min(lane + WAVE * j, P2 - 1);
      asm volatile("" : "+v"(k));
      wdy[j] = k / P;
      wdx[j] = k - wdy[j] * P;
    }
    for (int i0 = 0; i0 < SURR_ROWS / SURR_NW; i0 += SURR_FR) {
      float z[SURR_FR][SURR_WJ];
      bool in[SURR_FR][SURR_WJ];
#pragma unroll
      for (int r = 0; r < SURR_FR; ++r) {
        const int m = w + SURR_NW * (i0 + r);
        const int base = rinfo[0][m], c0 = rinfo[1][m] - R, r0 = rinfo[2][m] - R;
        const bool valid = rinfo[3][m] != 0;
#pragma unroll
        for (int j = 0; j < SURR_WJ; ++j) {
          const int rr = r0 + wdy[j], cc = c0 + wdx[j];
          in[r][j] = valid && lane + WAVE * j < P2 && rr >= 0 && rr < p.H && cc >= 0 && cc < p.W;
          z[r][j] = frame[base + (ptrdiff_t)min(max(rr, 0), p.H - 1) * p.W + min(max(cc, 0), p.W - 1)];
        }
      }
#pragma unroll
      for (int r = 0; r < SURR_FR; ++r) {
        const int m = w + SURR_NW * (i0 + r);
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < SURR_WJ; ++j) {
          const int k = lane + WAVE * j;
          const float v = in[r][j] ? z[r][j] : p.i_bg;
          if (k < P2) surr_put(act, m, k, (v - p.i_bg) * MLP_IN_SCALE);
          if (in[r][j]) {
            const double zb = (double)v - (double)p.i_bg;
            a += zb * zb;
          }
        }
        a = wave_sum(a);
        if (lane == 0) aw[m] = a;
      }
    }
    __syncthreads();
    const double az = tid < SURR_ROWS ? aw[tid] * p.inv2sxi2 : 0.0;
    surr_layers<FP8>(sw, act, fpart, nullptr);
    if (tid < SURR_ROWS) tmx[tid] = 0ull;
    __syncthreads();
    const int t_first = dv.seg_t[s0];
    if (tid < SURR_ROWS) {
      const uint32_t s = s0 + tid;
      if (s < B) {
        const double v = (double)MLP_OUT_SCALE * (double)surr_out(sw, fpart, tid) - az;
        ll[s] = v;
        atomicMax(&tmx[dv.seg_t[s] - t_first], ordered_bits(v));
      }
    }
    __syncthreads();
    if (tid < SURR_ROWS && tmx[tid] != 0ull) atomicMax(&tmax[t_first + tid], tmx[tid]);
    __syncthreads();
  }
}

// Network outputs f for BF16 feature rows X [n][256] (tests, calibration, evaluation).
template <bool FP8>
__global__ __launch_bounds__(SURR_TPB) __attribute__((amdgpu_waves_per_eu(4))) void k_surr_rows(int n, const uint16_t *__restrict__ Xg, SurrWeights sw,
                                                           float *__restrict__ f_out,
                                                           unsigned int *__restrict__ absmax) {
  __shared__ __attribute__((aligned(16))) uint8_t act[SURR_ACT_BYTES];
  __shared__ float fpart[SURR_NW][SURR_ROWS];
  const int tid = threadIdx.x;
  for (int r0 = blockIdx.x * SURR_ROWS; r0 < n; r0 += gridDim.x * SURR_ROWS) {
    float mx = 0.0f;
    for (int e = tid; e < SURR_ROWS * (MLP_F / 8); e += SURR_TPB) {
      const int m = e / (MLP_F / 8), k = 8 * (e % (MLP_F / 8));
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (r0 + m < n) v = gload_u4(Xg + (size_t)(r0 + m) * MLP_F + k);
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint16_t lo = (uint16_t)(wv[u] & 0xFFFF), hi = (uint16_t)(wv[u] >> 16);
        mx = fmaxf(mx, fmaxf(fabsf(bf2f(lo)), fabsf(bf2f(hi))));
        surr_put(act, m, k + 2 * u, bf2f(lo));
        surr_put(act, m, k + 2 * u + 1, bf2f(hi));
      }
    }
    if (absmax) {
      mx = wave_max(mx);
      if (lane_id() == 0) atomicMax(&absmax[0], __float_as_uint(mx));
    }
    __syncthreads();
    surr_layers<FP8>(sw, act, fpart, absmax);
    if (tid < SURR_ROWS && r0 + tid < n) f_out[r0 + tid] = surr_out(sw, fpart, tid);
    __syncthreads();
  }
}

// Training rows from the dummies of an exact pcSIR step: features and the
// target f = (l + A(z)) / 100 of the network.
template <int DIM>
__global__ __launch_bounds__(256) void k_surr_features(Params p, DummyView dv, const uint64_t *__restrict__ meta,
                                                       const StepDesc *__restrict__ desc,
                                                       const double *__restrict__ ll, uint32_t cap,
                                                       uint16_t *__restrict__ X, float *__restrict__ y) {
  const uint32_t B = (uint32_t)meta[META_B];
  const uint32_t n = B < cap ? B : cap;
  const float *frame = desc->frame;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * MLP_F;
       e += (size_t)gridDim.x * blockDim.x) {
    const uint32_t s = (uint32_t)(e / MLP_F);
    const int f = (int)(e % MLP_F);
    X[e] = f2bf(dummy_feature<DIM>(p, dv, frame, s, f));
    if (f == 0) y[s] = (float)((ll[s] + dummy_data_term<DIM>(p, dv, frame, s)) / (double)MLP_OUT_SCALE);
  }
}

// Inference layouts from the FP32 master vector: bf16 WT[l][n][k], biases,
// output unit; with FP8, per-tensor weight scales s_w = max|W| / 448 and
// WT8 = fp8(W / s_w). One block per layer for the scales (fixed-order max).
__global__ __launch_bounds__(256) void k_surr_scales(const float *__restrict__ params, float *__restrict__ scale_w) {
  __shared__ float lds[4];
  const int l = blockIdx.x;
  const float *W = params + (l == 0 ? MLP_OFF_W1 : l == 1 ? MLP_OFF_W2 : MLP_OFF_W3);
  float mx = 0.0f;
  for (int i = threadIdx.x; i < MLP_F * MLP_H; i += 256) mx = fmaxf(mx, fabsf(W[i]));
  mx = block_max<256, float>(mx, lds);
  if (threadIdx.x == 0) scale_w[l] = mx > 0.0f ? mx / FP8_MAX : 1.0f;
}

__global__ void k_surr_prep(const float *__restrict__ params, const float *__restrict__ scale_w,
                            uint16_t *__restrict__ wt, uint8_t *__restrict__ wt8, float *__restrict__ bias,
                            float *__restrict__ w4, float *__restrict__ b4) {
  const int offW[3] = {MLP_OFF_W1, MLP_OFF_W2, MLP_OFF_W3};
  const int offB[3] = {MLP_OFF_B1, MLP_OFF_B2, MLP_OFF_B3};
  const int total = 3 * MLP_H * MLP_F;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int l = i / (MLP_H * MLP_F), r = i % (MLP_H * MLP_F);
    const int n = r / MLP_F, k = r % MLP_F;
    const float v = params[offW[l] + k * MLP_H + n];
    wt[i] = f2bf(v);
    const float q = fminf(fmaxf(v / scale_w[l], -FP8_MAX), FP8_MAX);
    wt8[i] = (uint8_t)(f2fp8x2(q, 0.0f) & 0xFF);
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * MLP_H; i += gridDim.x * blockDim.x)
    bias[i] = params[offB[i / MLP_H] + i % MLP_H];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_H; i += gridDim.x * blockDim.x)
    w4[i] = params[MLP_OFF_W4 + i];
  if (blockIdx.x == 0 && threadIdx.x == 0) b4[0] = params[MLP_OFF_B4];
}

}  // namespace pcsir
