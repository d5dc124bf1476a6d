// Fused surrogate inference for the dummies of a pcSIR step (and for feature
// rows, for tests and calibration): features -> three MFMA layers with exact
// GELU -> output unit -> l = 100 f - A(z). BF16 or FP8 (E4M3, per-tensor
// scales) operands, FP32 accumulation. One block of four waves per 64 rows;
// each wave owns 64 of the 256 output units of a layer, so every weight read
// from L2 serves all the block's rows. (128 rows per block halve the weight
// traffic but need 288 registers per lane: one wave per SIMD, slower.)
#pragma once
#include "device_util.h"
#include "kernels.h"
#include "mlp_device.h"

namespace pcsir {

constexpr int SURR_ROWS = 64;       // rows per block, FP8
constexpr int SURR_ROWS_BF16 = 64;  // rows per block, BF16
template <bool FP8>
struct SurrRows {
  static constexpr int N = FP8 ? SURR_ROWS : SURR_ROWS_BF16;
};
constexpr int SURR_LD = MLP_F + 8;      // LDS row stride (bf16 elements)
constexpr int SURR_LD8 = MLP_F + 16;    // LDS row stride (fp8 bytes)
constexpr float FP8_MAX = 448.0f;       // largest finite E4M3 value

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

// Three hidden layers on the 64 rows held in LDS (X: bf16 activations; X8:
// fp8 copy when FP8), then the output unit; f of row m goes to fout[m].
// With `absmax`, the largest |input| of each layer is max-accumulated into it
// (FP8 scale calibration).
template <bool FP8>
__device__ __forceinline__ void surr_layers(const SurrWeights &sw, uint16_t (*X)[SURR_LD], uint8_t (*X8)[SURR_LD8],
                                            float *fout, unsigned int *absmax = nullptr) {
  constexpr int ROWS = SurrRows<FP8>::N;
  constexpr int RT = ROWS / 32;  // 32-row MFMA tiles
  const int lane = lane_id(), w = wave_id(), tid = threadIdx.x;
  for (int l = 0; l < 3; ++l) {
    if (absmax) {
      float mx = 0.0f;
      for (int e = tid; e < ROWS * MLP_F; e += 256) mx = fmaxf(mx, fabsf(bf2f(X[e / MLP_F][e % MLP_F])));
      mx = wave_max(mx);
      if (lane == 0) atomicMax(&absmax[l], __float_as_uint(mx));
    }
    if (FP8) {
      // quantize this layer's input with its per-tensor scale
      const float inv = 1.0f / sw.scale_x[l];
      for (int e = tid; e < ROWS * (MLP_F / 2); e += 256) {
        const int m = e / (MLP_F / 2), k = 2 * (e % (MLP_F / 2));
        const float a = fminf(fmaxf(bf2f(X[m][k]) * inv, -FP8_MAX), FP8_MAX);
        const float b = fminf(fmaxf(bf2f(X[m][k + 1]) * inv, -FP8_MAX), FP8_MAX);
        const uint32_t pk = f2fp8x2(a, b);
        X8[m][k] = (uint8_t)(pk & 0xFF);
        X8[m][k + 1] = (uint8_t)(pk >> 8);
      }
      __syncthreads();
    }
    f32x16 acc[RT][2];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int nb = 64 * w;
    if (FP8) {
      const uint8_t *W8 = sw.wt8 + (size_t)l * MLP_H * MLP_F;
#pragma unroll 4
      for (int kk = 0; kk < MLP_F; kk += 16) {
        const int k = kk + mfma_k0(lane);
        const uint2 b0 = *reinterpret_cast<const uint2 *>(W8 + (size_t)(nb + mfma_col(lane)) * MLP_F + k);
        const uint2 b1 = *reinterpret_cast<const uint2 *>(W8 + (size_t)(nb + 32 + mfma_col(lane)) * MLP_F + k);
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const uint2 a = *reinterpret_cast<const uint2 *>(&X8[32 * i + mfma_col(lane)][k]);
          acc[i][0] = mfma_fp8(a, b0, acc[i][0]);
          acc[i][1] = mfma_fp8(a, b1, acc[i][1]);
        }
      }
    } else {
      const uint16_t *Wt = sw.wt + (size_t)l * MLP_H * MLP_F;
#pragma unroll 2
      for (int kk = 0; kk < MLP_F; kk += 16) {
        const int k = kk + mfma_k0(lane);
        const uint4 b0 = *reinterpret_cast<const uint4 *>(Wt + (size_t)(nb + mfma_col(lane)) * MLP_F + k);
        const uint4 b1 = *reinterpret_cast<const uint4 *>(Wt + (size_t)(nb + 32 + mfma_col(lane)) * MLP_F + k);
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const uint4 a = *reinterpret_cast<const uint4 *>(&X[32 * i + mfma_col(lane)][k]);
          acc[i][0] = mfma_bf16(a, b0, acc[i][0]);
          acc[i][1] = mfma_bf16(a, b1, acc[i][1]);
        }
      }
    }
    __syncthreads();  // every wave has read this layer's input
    const float sc = FP8 ? sw.scale_x[l] * sw.scale_w[l] : 1.0f;
    const float *bias = sw.bias + l * MLP_H;
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = 32 * i + mfma_row(lane, r);
          const int n = nb + 32 * j + mfma_col(lane);
          X[m][n] = f2bf(gelu(fmaf(acc[i][j][r], sc, bias[n])));
        }
    __syncthreads();
  }
  if (tid < ROWS) {
    float f = sw.b4[0];
    for (int n = 0; n < MLP_H; ++n) f = fmaf(bf2f(X[tid][n]), sw.w4[n], f);
    fout[tid] = f;
  }
  __syncthreads();
}

// Surrogate log-likelihood of every dummy of the step: ll[s] = 100 f - A(z),
// and every target's largest surrogate value (tmax, ordered bits, atomic max;
// dummies are sorted by target, so a block's rows span consecutive targets).
template <int DIM, bool FP8>
__global__ __launch_bounds__(256) void k_surr_infer(Params p, DummyView dv, const uint64_t *__restrict__ meta,
                                                    const StepDesc *__restrict__ desc, SurrWeights sw,
                                                    double *__restrict__ ll, unsigned long long *__restrict__ tmax) {
  constexpr int ROWS = SurrRows<FP8>::N;
  __shared__ __attribute__((aligned(16))) uint16_t X[ROWS][SURR_LD];
  __shared__ __attribute__((aligned(16))) uint8_t X8[FP8 ? SURR_ROWS : 1][SURR_LD8];
  __shared__ float fout[ROWS];
  __shared__ double az[ROWS];
  const uint32_t B = (uint32_t)meta[META_B];
  const float *frame = desc->frame;
  for (uint32_t s0 = blockIdx.x * ROWS; s0 < B; s0 += gridDim.x * ROWS) {
    for (int e = threadIdx.x; e < ROWS * MLP_F; e += 256) {
      const int m = e / MLP_F, f = e % MLP_F;
      const uint32_t s = s0 + m;
      X[m][f] = f2bf(s < B ? dummy_feature<DIM>(p, dv, frame, s, f) : 0.0f);
    }
    if (threadIdx.x < ROWS) {
      const uint32_t s = s0 + threadIdx.x;
      az[threadIdx.x] = s < B ? dummy_data_term<DIM>(p, dv, frame, s) : 0.0;
    }
    __syncthreads();
    surr_layers<FP8>(sw, X, X8, fout);
    // tmx[j]: largest value among rows of target t_first + j (at most ROWS targets)
    __shared__ unsigned long long tmx[ROWS];
    if (threadIdx.x < ROWS) tmx[threadIdx.x] = 0ull;
    __syncthreads();
    const int t_first = dv.seg_t[s0];
    if (threadIdx.x < ROWS) {
      const uint32_t s = s0 + threadIdx.x;
      if (s < B) {
        const double v = (double)MLP_OUT_SCALE * (double)fout[threadIdx.x] - az[threadIdx.x];
        ll[s] = v;
        atomicMax(&tmx[dv.seg_t[s] - t_first], ordered_bits(v));
      }
    }
    __syncthreads();
    if (threadIdx.x < ROWS && tmx[threadIdx.x] != 0ull)
      atomicMax(&tmax[t_first + threadIdx.x], tmx[threadIdx.x]);
    __syncthreads();
  }
}

// Network outputs f for BF16 feature rows X [n][256] (tests, calibration, evaluation).
template <bool FP8>
__global__ __launch_bounds__(256) void k_surr_rows(int n, const uint16_t *__restrict__ Xg, SurrWeights sw,
                                                   float *__restrict__ f_out, unsigned int *__restrict__ absmax) {
  constexpr int ROWS = SurrRows<FP8>::N;
  __shared__ __attribute__((aligned(16))) uint16_t X[ROWS][SURR_LD];
  __shared__ __attribute__((aligned(16))) uint8_t X8[FP8 ? SURR_ROWS : 1][SURR_LD8];
  __shared__ float fout[ROWS];
  for (int r0 = blockIdx.x * ROWS; r0 < n; r0 += gridDim.x * ROWS) {
    for (int e = threadIdx.x; e < ROWS * MLP_F; e += 256) {
      const int m = e / MLP_F, f = e % MLP_F;
      X[m][f] = r0 + m < n ? Xg[(size_t)(r0 + m) * MLP_F + f] : (uint16_t)0;
    }
    __syncthreads();
    surr_layers<FP8>(sw, X, X8, fout, absmax);
    if (threadIdx.x < ROWS && r0 + threadIdx.x < n) f_out[r0 + threadIdx.x] = fout[threadIdx.x];
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
