// Device helpers for the gfx950 pcSIR kernels: counter-based RNG, exact cell
// index, wave64 reductions and scans. Wave size is 64 on CDNA; every helper
// here assumes it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcsir {

constexpr int WAVE = 64;

// ---------------------------------------------------------------- address spaces
// A pointer read from memory (rather than passed as a kernel argument) is
// generic to the compiler, and loads through it become flat loads, which are
// counted with the LDS operations as well: every wait for a lane shuffle then
// also waits for them. Pointers known to address device memory are cast to
// the global address space before use.
typedef const float __attribute__((address_space(1))) gfloat;
__device__ __forceinline__ const gfloat *as_global(const float *ptr) { return (const gfloat *)ptr; }

// ---------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two
// 32x32->64 products (multipliers 0xD2511F53, 0xCD9E8D57) with a Weyl key
// schedule (0x9E3779B9, 0xBB67AE85). The 32-bit variant runs on the native
// 32-bit multiplier; the 64-bit one needs four partial products per multiply.
// The key (k0, k1) must be the same in every lane of a wave (here always the
// seed, a kernel argument): it enters the rounds from scalar registers.
struct U32x4 {
  uint32_t v[4];
};

// a ^ b ^ k in one instruction (the compiler emits two XORs for it): the
// three-input bitwise operation with truth table 0x96 (bit 4a + 2b + c of the
// table is a ^ b ^ c), for a key k that is the same in every lane of the wave
// (held in a scalar register)
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 64-bit product is one multiply instruction giving both halves
    const uint64_t p0 = (uint64_t)c0 * M0, p1 = (uint64_t)c2 * M1;
    const uint32_t n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += W0;
    k1 += W1;
  }
  U32x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// Key of every draw: the 64-bit seed as two words.
__device__ __forceinline__ uint32_t seed_lo(uint64_t seed) { return (uint32_t)seed; }
__device__ __forceinline__ uint32_t seed_hi(uint64_t seed) { return (uint32_t)(seed >> 32); }

// A uniform on (0,1) from one word: its top 23 bits plus one half, times
// 2^-23; exact in binary32.
__device__ __forceinline__ float u01(uint32_t w) { return ((float)(w >> 9) + 0.5f) * 0x1p-23f; }

// [0, 1) with 53 random bits from two words: (w1 2^32 + w0) >> 11, times 2^-53.
__device__ __forceinline__ double u01_53(uint32_t w0, uint32_t w1) {
  return (double)((((uint64_t)w1 << 32) | (uint64_t)w0) >> 11) * 0x1p-53;
}

// NPAIRS pairs of N(0,1) draws (binary32 Box-Muller) for particle i of target
// t at frame k: blocks with counters (i, k, t, 0) and (i, k, t, 1); pair p
// takes (u1, u2) from words 2p and 2p + 1 of the eight. k enters modulo 2^32.
template <int NPAIRS>
__device__ __forceinline__ void normal_pairs(uint64_t seed, uint32_t i, uint64_t k, uint32_t t, float *z) {
  static_assert(NPAIRS >= 1 && NPAIRS <= 4, "two blocks give at most four pairs");
  uint32_t w[8];
  const U32x4 a = philox4x32_10(i, (uint32_t)k, t, 0u, seed_lo(seed), seed_hi(seed));
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = a.v[q];
  if (NPAIRS > 2) {
    const U32x4 b = philox4x32_10(i, (uint32_t)k, t, 1u, seed_lo(seed), seed_hi(seed));
#pragma unroll
    for (int q = 0; q < 4; ++q) w[4 + q] = b.v[q];
  }
#pragma unroll
  for (int p = 0; p < NPAIRS; ++p) {
    const float u1 = u01(w[2 * p]);
    const float u2 = u01(w[2 * p + 1]);
    // hardware log2, and sine / cosine of 2 pi u2 (the instructions take the
    // angle in turns); about one ulp each, far inside the tolerance of the
    // propagated states
    const float r = sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(u1));
    z[2 * p] = r * __builtin_amdgcn_cosf(u2);
    z[2 * p + 1] = r * __builtin_amdgcn_sinf(u2);
  }
}

// Resampling uniform of target t at frame k: counter (0, k, t, 2), words 0
// and 1, in [0, 1).
__device__ __forceinline__ double resample_uniform(uint64_t seed, uint64_t k, uint64_t t) {
  const U32x4 b = philox4x32_10(0u, (uint32_t)k, (uint32_t)t, 2u, seed_lo(seed), seed_hi(seed));
  return u01_53(b.v[0], b.v[1]);
}

// ---------------------------------------------------------------- exact cell index
// floor((x + 1/2) * m) of the binary32 value x, exactly. x is clamped to
// [-2^24, 2^24] (NaN -> 2^24), the result to [-2^30, 2^30]; 1 <= m <= 4096.
// For |x| >= 2^-17, x + 1/2 has at most 40 significant bits and m at most
// 13, so (x + 1/2) m is exact in binary64 and so is its floor. Below, |x m|
// < 2^-5 and the floor is m/2 rounded down, less one when m is even and
// x < 0 (x in (-2^-17, 0) pushes (x + 1/2) m just below m/2).
// The clamp of cell_index: NaN -> 2^24, then into [-2^24, 2^24].
__device__ __forceinline__ float clamp_position(float xf) {
  float x = xf;
  if (x != x) x = 16777216.0f;
  return fminf(fmaxf(x, -16777216.0f), 16777216.0f);
}

__device__ __forceinline__ int32_t cell_index(float xf, int32_t m) {
  const float x = clamp_position(xf);
  if (fabsf(x) >= 0x1p-17f) {
    double v = floor(((double)x + 0.5) * (double)m);
    v = fmin(fmax(v, -1073741824.0), 1073741824.0);
    return (int32_t)v;
  }
  return (m >> 1) - (((m & 1) == 0 && x < 0.0f) ? 1 : 0);
}

// Order-preserving map of doubles to unsigned integers (for atomic max); 0
// is below every mapped value.
__device__ __forceinline__ unsigned long long ordered_bits(double d) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered_bits(unsigned long long u) {
  return __longlong_as_double((long long)((u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u));
}

__device__ __forceinline__ int32_t floor_div(int32_t a, int32_t m) {
  int32_t q = a / m;
  if ((a % m) != 0 && (a < 0)) q -= 1;
  return q;
}

// ---------------------------------------------------------------- wave / block primitives
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x / WAVE); }
// A value that every lane of the wave holds, moved to a scalar register.
__device__ __forceinline__ int32_t wave_uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T y = __shfl_xor(v, o, WAVE);
    v = y > v ? y : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T y = __shfl_xor(v, o, WAVE);
    v = y < v ? y : v;
  }
  return v;
}

// Inclusive wave scan (Kogge-Stone over shfl_up).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T y = __shfl_up(v, o, WAVE);
    if (lane >= o) v += y;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_incl_max_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T y = __shfl_up(v, o, WAVE);
    if (lane >= o) v = y > v ? y : v;
  }
  return v;
}

// Data-parallel-primitive lane moves within a row of 16 lanes (GCN / CDNA
// dpp_ctrl codes): quad permutations [1,0,3,2] and [2,3,0,1], the mirror of
// each half-row of 8 (lane i <-> 7 - i) and of the row (i <-> 15 - i). Each
// pairs every lane with one in the other half of its group of 2, 4, 8, 16,
// so that four of them in this order give every lane its row's total. They
// move data in the vector ALU, without the LDS crossbar of a shuffle.
constexpr int DPP_QUAD_XOR1 = 0xB1;
constexpr int DPP_QUAD_XOR2 = 0x4E;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// One level of the compensated pair sum: (s, e) += (s2, e2), the rounding
// error of s + s2 (TwoSum) joining e.
__device__ __forceinline__ void pair_sum_level(float &s, float &e, float s2, float e2) {
  const float t = s + s2;
  const float bp = t - s;
  const float err = (s - (t - bp)) + (s2 - bp);
  s = t;
  e = e + e2 + err;
}

// Compensated wave reduction that keeps the result as an unevaluated pair
// (hi, lo), returned in FP64 registers of every lane: four levels by lane
// moves within rows of 16, then two shuffles across rows.
__device__ __forceinline__ void wave_sum_pair(float s, float e, double &hi, double &lo) {
  pair_sum_level(s, e, dpp_move<DPP_QUAD_XOR1>(s), dpp_move<DPP_QUAD_XOR1>(e));
  pair_sum_level(s, e, dpp_move<DPP_QUAD_XOR2>(s), dpp_move<DPP_QUAD_XOR2>(e));
  pair_sum_level(s, e, dpp_move<DPP_ROW_HALF_MIRROR>(s), dpp_move<DPP_ROW_HALF_MIRROR>(e));
  pair_sum_level(s, e, dpp_move<DPP_ROW_MIRROR>(s), dpp_move<DPP_ROW_MIRROR>(e));
#pragma unroll
  for (int o = 16; o < WAVE; o <<= 1) pair_sum_level(s, e, __shfl_xor(s, o, WAVE), __shfl_xor(e, o, WAVE));
  hi = (double)s;
  lo = (double)e;
}

// Block (NT threads) reduction helpers using a small LDS scratch.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *lds) {
  v = wave_sum(v);
  if (lane_id() == 0) lds[wave_id()] = v;
  __syncthreads();
  T r = lds[0];
#pragma unroll
  for (int w = 1; w < NT / WAVE; ++w) r += lds[w];
  __syncthreads();
  return r;
}
template <int NT, typename T>
__device__ __forceinline__ T block_max(T v, T *lds) {
  v = wave_max(v);
  if (lane_id() == 0) lds[wave_id()] = v;
  __syncthreads();
  T r = lds[0];
#pragma unroll
  for (int w = 1; w < NT / WAVE; ++w) r = lds[w] > r ? lds[w] : r;
  __syncthreads();
  return r;
}
template <int NT, typename T>
__device__ __forceinline__ T block_min(T v, T *lds) {
  v = wave_min(v);
  if (lane_id() == 0) lds[wave_id()] = v;
  __syncthreads();
  T r = lds[0];
#pragma unroll
  for (int w = 1; w < NT / WAVE; ++w) r = lds[w] < r ? lds[w] : r;
  __syncthreads();
  return r;
}

// Exclusive block scan of integers; *total receives the block sum.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *lds, T *total) {
  const int lane = lane_id(), w = wave_id();
  const T incl = wave_incl_scan(v);
  if (lane == WAVE - 1) lds[w] = incl;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) {
    if (i < w) pre += lds[i];
    tot += lds[i];
  }
  __syncthreads();
  *total = tot;
  return pre + incl - v;
}

// Exclusive block scan of non-negative doubles whose results are forced to be
// non-decreasing in thread order (a running maximum after the sum scan), so
// that boundaries derived from them never cross. *total is the block sum.
template <int NT>
__device__ __forceinline__ double block_excl_scan_monotone(double v, double *lds, double *total) {
  const int lane = lane_id(), w = wave_id();
  const double incl = wave_incl_scan(v);
  double ex = __shfl_up(incl, 1, WAVE);
  if (lane == 0) ex = 0.0;
  if (lane == WAVE - 1) lds[w] = incl;
  __syncthreads();
  double pre = 0.0, tot = 0.0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) {
    if (i < w) pre += lds[i];
    tot += lds[i];
  }
  __syncthreads();
  double r = pre + ex;
  r = wave_incl_max_scan(r);
  // running maximum across waves: last lane of each earlier wave
  if (lane == WAVE - 1) lds[w] = r;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i)
    if (i < w) r = lds[i] > r ? lds[i] : r;
  __syncthreads();
  *total = tot;
  return r;
}

}  // namespace pcsir
