// Surrogate-network training on gfx950: BF16 MFMA GEMMs with FP32
// accumulation and fused epilogues (bias + GELU forward, GELU' backward,
// weight gradients), the output unit, column sums for the bias gradients,
// and Adam on FP32 master parameters. C ABI in include/pcsir_mlp.h.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "../../include/pcsir_mlp.h"
#include "device_util.h"
#include "mlp_device.h"

using namespace pcsir;

namespace {

constexpr int GT = 64;    // GEMM block tile (rows and columns)
constexpr int GK = 32;    // k chunk staged in LDS
constexpr int GPAD = 8;   // LDS row padding (bf16 elements)

enum { EPI_FWD = 0, EPI_BWD = 1, EPI_STORE = 2 };

// 8 consecutive BF16 elements of a tile row into LDS row `dst` (16 bytes).
__device__ __forceinline__ uint4 ld16(const uint16_t *p) { return *reinterpret_cast<const uint4 *>(p); }

// Stage one GT x GK tile of op(X) into Xs[row][k], with op(X)(row, k) =
// x_t ? X[k ld + row] : X[row ld + k]: one 16-byte load per thread (8
// consecutive elements of the contiguous index); the transposed case
// scatters its 8 values down a column of the tile.
__device__ __forceinline__ uint4 stage_load(const uint16_t *X, int ld, int x_t, int r0, int k0, int tid) {
  if (x_t) {
    const int k = tid / (GT / 8), r8 = 8 * (tid % (GT / 8));
    return ld16(X + (size_t)(k0 + k) * ld + r0 + r8);
  }
  const int r = tid / (GK / 8), k8 = 8 * (tid % (GK / 8));
  return ld16(X + (size_t)(r0 + r) * ld + k0 + k8);
}
__device__ __forceinline__ void stage_store(uint16_t (*Xs)[GK + GPAD], int x_t, int tid, const uint4 &v) {
  if (x_t) {
    const int k = tid / (GT / 8), r8 = 8 * (tid % (GT / 8));
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Xs[r8 + 2 * i][k] = (uint16_t)(w[i] & 0xFFFF);
      Xs[r8 + 2 * i + 1][k] = (uint16_t)(w[i] >> 16);
    }
  } else {
    const int r = tid / (GK / 8), k8 = 8 * (tid % (GK / 8));
    *reinterpret_cast<uint4 *>(&Xs[r][k8]) = v;
  }
}

// C = op(A) op(B), A(m,k) = a_t ? A[k lda + m] : A[m lda + k], B(k,n) = b_t ? B[n ldb + k] : B[k ldb + n],
// BF16 inputs, FP32 accumulation. M, N multiples of 64, K a multiple of 32,
// lda and ldb multiples of 8 and 16-byte aligned operands. Block (x, y, z)
// computes the 64 x 64 tile (y, x) over the z-th of gridDim.z equal shares
// of K; the next k-chunk is loaded while the current one is multiplied.
// EPI_FWD:   z = acc + bias[n]; Zout[m][n] = z; Hout[m][n] = bf16(gelu(z))
// EPI_BWD:   Hout[m][n] = bf16(acc * gelu'(Zin[m][n]))
// EPI_STORE: Cout[z M ldc + m ldc + n] = acc (the z-th partial with a K split)
// With FP8 quantisation in the forward pass (qs, two device floats, else null):
// EPI_FWD:   z = acc qs[0] + bias[n] (operands holding E4M3 values of scaled
//            tensors); with qs[1] > 0, Hout = the E4M3 value of
//            clamp(gelu(z) / qs[1]) (the next layer's quantised input)
// EPI_BWD:   Hout = bf16(acc qs[0] gelu'(z) [|gelu(z) / qs[1]| <= FP8_MAX])
//            (the straight-through gradient of the quantiser, zero where it clamps)
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t *__restrict__ A, int lda, int a_t,
                                              const uint16_t *__restrict__ B, int ldb, int b_t,
                                              const float *__restrict__ bias, const float *__restrict__ Zin,
                                              float *__restrict__ Zout, uint16_t *__restrict__ Hout,
                                              float *__restrict__ Cout, int ldc, const float *__restrict__ qs) {
  static_assert(GT * GK / 8 == 256, "one 16-byte load per thread and operand");
  __shared__ __attribute__((aligned(16))) uint16_t As[GT][GK + GPAD];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GT][GK + GPAD];  // [n][k]
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int kz = K / (int)gridDim.z, kb = kz * (int)blockIdx.z, ke = kb + kz;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  uint4 va = stage_load(A, lda, a_t, m0, kb, tid);
  uint4 vb = stage_load(B, ldb, !b_t, n0, kb, tid);
  for (int k0 = kb; k0 < ke; k0 += GK) {
    __syncthreads();  // the previous chunk has been read
    stage_store(As, a_t, tid, va);
    stage_store(Bs, !b_t, tid, vb);
    __syncthreads();
    if (k0 + GK < ke) {
      va = stage_load(A, lda, a_t, m0, k0 + GK, tid);
      vb = stage_load(B, ldb, !b_t, n0, k0 + GK, tid);
    }
#pragma unroll
    for (int kk = 0; kk < GK; kk += 16) {
      const uint4 a = *reinterpret_cast<const uint4 *>(&As[wm + mfma_col(lane)][kk + mfma_k0(lane)]);
      const uint4 b = *reinterpret_cast<const uint4 *>(&Bs[wn + mfma_col(lane)][kk + mfma_k0(lane)]);
      acc = mfma_bf16(a, b, acc);
    }
  }
  float *Cz = EPI == EPI_STORE ? Cout + (size_t)blockIdx.z * M * ldc : nullptr;
  // quantisation: the accumulator's scale, and the output quantiser's scale
  // and reciprocal (the inference kernel's form, g * (1 / s))
  const float qa = qs ? qs[0] : 1.0f, qo = qs ? qs[1] : 0.0f;
  const float qinv = qo > 0.0f ? 1.0f / qo : 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm + mfma_row(lane, r);
    const int n = n0 + wn + mfma_col(lane);
    const size_t o = (size_t)m * ldc + n;
    if (EPI == EPI_FWD) {
      const float z = fmaf(acc[r], qa, bias[n]);
      Zout[o] = z;
      const float g = gelu(z);
      Hout[o] = f2bf(qo > 0.0f ? fp8_value(g * qinv) : g);
    } else if (EPI == EPI_BWD) {
      const float z = Zin[o];
      float d = acc[r] * qa * gelu_grad(z);
      if (qo > 0.0f && !(fabsf(gelu(z) * qinv) <= FP8_MAX)) d = 0.0f;
      Hout[o] = f2bf(d);
    } else {
      Cz[o] = acc[r];
    }
  }
}

// out[i] = sum over the S partials part[s][i], s = 0..S-1 in order (K split),
// times *scale when scale is not null.
__global__ void k_split_sum(int n, int S, const float *__restrict__ part, float *__restrict__ out,
                            const float *__restrict__ scale) {
  const float sc = scale ? *scale : 1.0f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float v = part[i];
    for (int s = 1; s < S; ++s) v += part[(size_t)s * n + i];
    out[i] = scale ? v * sc : v;
  }
}

// FP8 quantisation of the hidden layers for training (quantisation-aware):
// block l - 1 (l = 1, 2) scales W_l per tensor as the inference kernel does,
// sw = max|W_l| / FP8_MAX, and writes the E4M3 values of W_l / sw as BF16
// into wq[l - 1]; sw into q[6 + l - 1].
__global__ __launch_bounds__(256) void k_qat_weights(const float *__restrict__ params, uint16_t *__restrict__ wq1,
                                                     uint16_t *__restrict__ wq2, float *__restrict__ q) {
  __shared__ float lds[4];
  const int l = blockIdx.x + 1;
  const float *W = params + (l == 1 ? MLP_OFF_W2 : MLP_OFF_W3);
  uint16_t *out = l == 1 ? wq1 : wq2;
  float mx = 0.0f;
  for (int i = threadIdx.x; i < MLP_H * MLP_H; i += 256) mx = fmaxf(mx, fabsf(W[i]));
  mx = block_max<256, float>(mx, lds);
  const float sw = mx > 0.0f ? mx / FP8_MAX : 1.0f;
  for (int i = threadIdx.x; i < MLP_H * MLP_H; i += 256) out[i] = f2bf(fp8_value(W[i] / sw));
  if (threadIdx.x == 0) q[6 + l - 1] = sw;
}
// The per-GEMM factors from the activation scales sx (sx[1], sx[2]: inputs of
// hidden layers 1 and 2) and the weight scales q[6], q[7]:
// forward l = 0, 1, 2 at q[2l] (accumulator scale, output quantiser scale),
// backward through W_1, W_2 at q[8], q[10] (weight scale, quantiser scale),
// weight gradients of W_1, W_2 at q[12], q[13].
__global__ void k_qat_factors(const float *__restrict__ sx, float *__restrict__ q) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const float s1 = sx[1], s2 = sx[2], w1 = q[6], w2 = q[7];
  q[0] = 1.0f;
  q[1] = s1;
  q[2] = s1 * w1;
  q[3] = s2;
  q[4] = s2 * w2;
  q[5] = 0.0f;
  q[8] = w1;
  q[9] = s1;
  q[10] = w2;
  q[11] = s2;
  q[12] = s1;
  q[13] = s2;
}

__global__ void k_f32_to_bf16(int n, const float *__restrict__ src, uint16_t *__restrict__ dst) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = f2bf(src[i]);
}

// Output unit, one thread per row: f = H3 . w4 + b4; with targets, the loss
// residual r = f - y, the row's share of d loss / d f = 2 r / M, and
// dZ3[m][n] = (2 r / M) w4[n] gelu'(Z3[m][n]). Per-block sums of r^2 for the loss.
__global__ __launch_bounds__(256) void k_head(int M, const uint16_t *__restrict__ H3, const float *__restrict__ Z3,
                                              const float *__restrict__ params, const float *__restrict__ y,
                                              float *__restrict__ f_out, float *__restrict__ df,
                                              uint16_t *__restrict__ dZ3, float *__restrict__ loss_part) {
  __shared__ float lds[4];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const float *w4 = params + MLP_OFF_W4;
  float r2 = 0.0f;
  if (m < M) {
    float f = params[MLP_OFF_B4];
    for (int n = 0; n < MLP_H; ++n) f = fmaf(bf2f(H3[(size_t)m * MLP_H + n]), w4[n], f);
    if (f_out) f_out[m] = f;
    if (y) {
      const float r = f - y[m];
      r2 = r * r;
      const float d = 2.0f * r / (float)M;
      df[m] = d;
      for (int n = 0; n < MLP_H; ++n)
        dZ3[(size_t)m * MLP_H + n] = f2bf(d * w4[n] * gelu_grad(Z3[(size_t)m * MLP_H + n]));
    }
  }
  if (loss_part) {
    const float s = block_sum<256, float>(r2, lds);
    if (threadIdx.x == 0) loss_part[blockIdx.x] = s;
  }
}

// Column sums out[n] = sum_m X[m][n] * (v ? v[m] : 1) in FP32, in a fixed
// order: block (x, y) sums rows [128 y, 128 y + 128) of columns
// [32 x, 32 x + 32), thread (g, c) every eighth row from g, the eight partial
// sums then in order of g, into part[y][n]; k_colsum_fin adds the row blocks
// in order of y.
constexpr int CS_ROWS = 128;
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const uint16_t *__restrict__ X,
                                                const float *__restrict__ v, float *__restrict__ part) {
  __shared__ float lds[8][32];
  const int c = threadIdx.x % 32, g = threadIdx.x / 32;
  const int n = 32 * blockIdx.x + c, m0 = CS_ROWS * blockIdx.y;
  float s = 0.0f;
  for (int m = m0 + g; m < min(M, m0 + CS_ROWS); m += 8) s = fmaf(bf2f(X[(size_t)m * N + n]), v ? v[m] : 1.0f, s);
  lds[g][c] = s;
  __syncthreads();
  if (g == 0) {
    float t = lds[0][c];
    for (int i = 1; i < 8; ++i) t += lds[i][c];
    part[(size_t)blockIdx.y * N + n] = t;
  }
}
__global__ void k_colsum_fin(int N, int parts, const float *__restrict__ part, float *__restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float t = part[n];
  for (int y = 1; y < parts; ++y) t += part[(size_t)y * N + n];
  out[n] = t;
}

__global__ void k_sum(int n, const float *__restrict__ v, float *__restrict__ out, float scale) {
  __shared__ float lds[4];
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) s += v[i];
  s = block_sum<256, float>(s, lds);
  if (threadIdx.x == 0) *out = s * scale;
}

// Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
__global__ void k_adam(int n, float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float mi = b1 * m[i] + (1.0f - b1) * g[i];
    const float vi = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

struct TrainLayout {
  size_t wb[3], Z[3], Hh[3], dZ[3], f, df, loss_part, part, cs, q, total;
};

// Shares of the batch dimension for the weight-gradient GEMMs (K = batch):
// up to 8, each a multiple of 32 rows.
constexpr int wgrad_splits(int B) {
  int S = 8;
  while (S > 1 && B % (32 * S) != 0) S /= 2;
  return S;
}

constexpr TrainLayout train_layout(int B) {
  TrainLayout L{};
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o += (bytes + 255) / 256 * 256;
    return at;
  };
  for (int l = 0; l < 3; ++l) L.wb[l] = take(2 * (size_t)MLP_H * MLP_H);
  for (int l = 0; l < 3; ++l) L.Z[l] = take(4 * (size_t)B * MLP_H);
  for (int l = 0; l < 3; ++l) L.Hh[l] = take(2 * (size_t)B * MLP_H);
  for (int l = 0; l < 3; ++l) L.dZ[l] = take(2 * (size_t)B * MLP_H);
  L.f = take(4 * (size_t)B);
  L.df = take(4 * (size_t)B);
  L.loss_part = take(4 * (size_t)((B + 255) / 256));
  L.part = take(4 * (size_t)wgrad_splits(B) * MLP_H * MLP_H);
  L.cs = take(4 * (size_t)((B + CS_ROWS - 1) / CS_ROWS) * MLP_H);
  L.q = take(4 * 16);  // FP8 quantisation factors (quantisation-aware step)
  L.total = o;
  return L;
}

}  // namespace

// Workspace of the no-allocation training step: a file-scope device array
// sized for the largest batch it accepts (8.4 MiB). Each GPU holds its own
// copy from module load until the process ends. Host code never passes the
// array's name to a kernel: it is a host-side stand-in there, and the device
// address comes from hipGetSymbolAddress, taken once per device.
constexpr size_t MLP_STATIC_BYTES = train_layout(PCSIR_MLP_STATIC_MAX_BATCH).total;
static __device__ __align__(256) unsigned char scratch[MLP_STATIC_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the device that owns `stream` (which must be
// the current device), looked up on the first call for that device.
pcsir_status scratch_address(void *stream, void **out) {
  int cur = -1, dev = -1;
  if (hipGetDevice(&cur) != hipSuccess) return PCSIR_E_HIP;
  if (hipStreamGetDevice((hipStream_t)stream, &dev) != hipSuccess) return PCSIR_E_HIP;
  if (dev != cur || cur < 0 || cur >= MAX_DEVICES) return PCSIR_E_INVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[cur]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return PCSIR_E_HIP;
    g_scratch_dev[cur] = p;
  }
  *out = g_scratch_dev[cur];
  return PCSIR_OK;
}

template <int EPI>
void gemm(hipStream_t st, int M, int N, int K, const uint16_t *A, int lda, int a_t, const uint16_t *B, int ldb, int b_t,
          const float *bias, const float *Zin, float *Zout, uint16_t *Hout, float *Cout, int ldc, int splits = 1,
          const float *qs = nullptr) {
  dim3 grid(N / GT, M / GT, splits);
  k_gemm<EPI><<<grid, 256, 0, st>>>(M, N, K, A, lda, a_t, B, ldb, b_t, bias, Zin, Zout, Hout, Cout, ldc, qs);
}

// out[n] = sum_m X[m][n] (v ? v[m] : 1) for the N = 256 columns, fixed order; part: workspace.
void colsum(hipStream_t st, int M, const uint16_t *X, const float *v, float *part, float *out) {
  const int parts = (M + CS_ROWS - 1) / CS_ROWS;
  k_colsum<<<dim3(MLP_H / 32, parts), 256, 0, st>>>(M, MLP_H, X, v, part);
  k_colsum_fin<<<1, MLP_H, 0, st>>>(MLP_H, parts, part, out);
}

// The training step of pcsir_mlp_train_step in a workspace at `ws` (device
// memory of at least train_layout(batch).total bytes); arguments validated.
// act_scale (device, three floats, or null): the forward pass quantises the
// two hidden layers as the FP8 inference does, with these input scales
// (act_scale[1], act_scale[2]) and per-tensor weight scales, and the
// backward pass takes the quantisers as the identity where they do not clamp.
pcsir_status train_step(float *params, float *adam_m, float *adam_v, const uint16_t *X, const float *y, int32_t batch,
                        float lr, int32_t t, void *ws, void *stream, float *loss_dev, float *grad_dev,
                        const float *act_scale = nullptr) {
  const TrainLayout L = train_layout(batch);
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  auto at16 = [&](size_t o) { return (uint16_t *)(w + o); };
  auto at32 = [&](size_t o) { return (float *)(w + o); };
  const int H = MLP_H, M = batch;
  const int offW[3] = {MLP_OFF_W1, MLP_OFF_W2, MLP_OFF_W3};
  const int offB[3] = {MLP_OFF_B1, MLP_OFF_B2, MLP_OFF_B3};
  const bool q8 = act_scale != nullptr;
  float *q = at32(L.q);
  for (int l = 0; l < (q8 ? 1 : 3); ++l) k_f32_to_bf16<<<64, 256, 0, st>>>(H * H, params + offW[l], at16(L.wb[l]));
  if (q8) {
    k_qat_weights<<<2, 256, 0, st>>>(params, at16(L.wb[1]), at16(L.wb[2]), q);
    k_qat_factors<<<1, 64, 0, st>>>(act_scale, q);
  }
  // forward
  const uint16_t *in = X;
  for (int l = 0; l < 3; ++l) {
    gemm<EPI_FWD>(st, M, H, H, in, H, 0, at16(L.wb[l]), H, 0, params + offB[l], nullptr, at32(L.Z[l]),
                  at16(L.Hh[l]), nullptr, H, 1, q8 ? q + 2 * l : nullptr);
    in = at16(L.Hh[l]);
  }
  const int hb = (M + 255) / 256;
  k_head<<<hb, 256, 0, st>>>(M, at16(L.Hh[2]), at32(L.Z[2]), params, y, at32(L.f), at32(L.df), at16(L.dZ[2]),
                             at32(L.loss_part));
  if (loss_dev) k_sum<<<1, 256, 0, st>>>(hb, at32(L.loss_part), loss_dev, 1.0f / (float)M);
  // backward: output unit
  float *g = grad_dev;
  colsum(st, M, at16(L.Hh[2]), at32(L.df), at32(L.cs), g + MLP_OFF_W4);
  k_sum<<<1, 256, 0, st>>>(M, at32(L.df), g + MLP_OFF_B4, 1.0f);
  const int S = wgrad_splits(M);
  for (int l = 2; l >= 0; --l) {
    const uint16_t *hin = l > 0 ? at16(L.Hh[l - 1]) : X;
    // dW_l = H_{l-1}^T dZ_l (K = batch, in S shares whose partial products are added in order)
    gemm<EPI_STORE>(st, H, H, M, hin, H, 1, at16(L.dZ[l]), H, 0, nullptr, nullptr, nullptr, nullptr, at32(L.part), H,
                    S);
    // (quantised: the activations hold E4M3 values of H_{l-1} / s_l)
    k_split_sum<<<64, 256, 0, st>>>(H * H, S, at32(L.part), g + offW[l], q8 && l > 0 ? q + 11 + l : nullptr);
    colsum(st, M, at16(L.dZ[l]), nullptr, at32(L.cs), g + offB[l]);
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l^T) * gelu'(Z_{l-1})
      gemm<EPI_BWD>(st, M, H, H, at16(L.dZ[l]), H, 0, at16(L.wb[l]), H, 1, nullptr, at32(L.Z[l - 1]), nullptr,
                    at16(L.dZ[l - 1]), nullptr, H, 1, q8 ? q + 6 + 2 * l : nullptr);
    }
  }
  if (adam_m && adam_v && t >= 1) {
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    k_adam<<<256, 256, 0, st>>>(MLP_N_PARAMS, params, adam_m, adam_v, g, lr, c1, c2);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PCSIR_OK : PCSIR_E_HIP;
}

}  // namespace

extern "C" {

size_t pcsir_mlp_param_count(void) { return (size_t)MLP_N_PARAMS; }

size_t pcsir_mlp_train_bytes(int32_t batch) {
  if (batch < 64 || batch % 64) return 0;
  return train_layout(batch).total;
}

pcsir_status pcsir_mlp_train_step(float *params, float *adam_m, float *adam_v, const uint16_t *X, const float *y,
                                  int32_t batch, float lr, int32_t t, void *ws, size_t ws_bytes, void *stream,
                                  float *loss_dev, float *grad_dev) {
  if (!params || !X || !y || !ws || batch < 64 || batch % 64) return PCSIR_E_INVAL;
  // the caller provides the gradient buffer (used for Adam too)
  if (!grad_dev) return PCSIR_E_INVAL;
  if (ws_bytes < train_layout(batch).total) return PCSIR_E_NOMEM;
  return train_step(params, adam_m, adam_v, X, y, batch, lr, t, ws, stream, loss_dev, grad_dev);
}

pcsir_status pcsir_mlp_train_step_fp8(float *params, float *adam_m, float *adam_v, const uint16_t *X, const float *y,
                                      int32_t batch, float lr, int32_t t, const float *act_scale_dev, void *ws,
                                      size_t ws_bytes, void *stream, float *loss_dev, float *grad_dev) {
  if (!params || !X || !y || !ws || !act_scale_dev || batch < 64 || batch % 64) return PCSIR_E_INVAL;
  if (!grad_dev) return PCSIR_E_INVAL;
  if (ws_bytes < train_layout(batch).total) return PCSIR_E_NOMEM;
  return train_step(params, adam_m, adam_v, X, y, batch, lr, t, ws, stream, loss_dev, grad_dev, act_scale_dev);
}

pcsir_status pcsir_mlp_train_step_static(float *params, float *adam_m, float *adam_v, const uint16_t *X,
                                         const float *y, int32_t batch, float lr, int32_t t, void *stream,
                                         float *loss_dev, float *grad_dev) {
  if (!params || !X || !y || !grad_dev || batch < 64 || batch % 64) return PCSIR_E_INVAL;
  if (batch > PCSIR_MLP_STATIC_MAX_BATCH) return PCSIR_E_NOMEM;
  void *ws = nullptr;
  const pcsir_status s = scratch_address(stream, &ws);
  if (s != PCSIR_OK) return s;
  return train_step(params, adam_m, adam_v, X, y, batch, lr, t, ws, stream, loss_dev, grad_dev);
}

pcsir_status pcsir_mlp_forward_train_path(const float *params, const uint16_t *X, int32_t n, float *f_out, void *ws,
                                          size_t ws_bytes, void *stream) {
  if (!params || !X || !f_out || !ws || n < 64 || n % 64) return PCSIR_E_INVAL;
  const TrainLayout L = train_layout(n);
  if (ws_bytes < L.total) return PCSIR_E_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  auto at16 = [&](size_t o) { return (uint16_t *)(w + o); };
  auto at32 = [&](size_t o) { return (float *)(w + o); };
  const int H = MLP_H;
  const int offW[3] = {MLP_OFF_W1, MLP_OFF_W2, MLP_OFF_W3};
  const int offB[3] = {MLP_OFF_B1, MLP_OFF_B2, MLP_OFF_B3};
  for (int l = 0; l < 3; ++l) k_f32_to_bf16<<<64, 256, 0, st>>>(H * H, params + offW[l], at16(L.wb[l]));
  const uint16_t *in = X;
  for (int l = 0; l < 3; ++l) {
    gemm<EPI_FWD>(st, n, H, H, in, H, 0, at16(L.wb[l]), H, 0, params + offB[l], nullptr, at32(L.Z[l]),
                  at16(L.Hh[l]), nullptr, H, 1);
    in = at16(L.Hh[l]);
  }
  k_head<<<(n + 255) / 256, 256, 0, st>>>(n, at16(L.Hh[2]), at32(L.Z[2]), params, nullptr, f_out, nullptr, nullptr,
                                         nullptr);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PCSIR_OK : PCSIR_E_HIP;
}

pcsir_status pcsir_mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t lda, int32_t a_trans,
                                 const uint16_t *B, int32_t ldb, int32_t b_trans, float *C, int32_t ldc, void *stream) {
  if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0 || M % GT || N % GT || K % GK) return PCSIR_E_INVAL;
  if (lda % 8 || ldb % 8 || ((uintptr_t)A) % 16 || ((uintptr_t)B) % 16) return PCSIR_E_INVAL;
  gemm<EPI_STORE>((hipStream_t)stream, M, N, K, A, lda, a_trans ? 1 : 0, B, ldb, b_trans ? 1 : 0, nullptr, nullptr,
                  nullptr, nullptr, C, ldc);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PCSIR_OK : PCSIR_E_HIP;
}

}  // extern "C"
