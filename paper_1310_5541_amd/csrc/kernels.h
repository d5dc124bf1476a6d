// gfx950 kernels of one SIR / pcSIR frame. Particles are SoA float32 in HBM,
// one thread per particle for the streaming stages, one wave64 per likelihood
// evaluation. Binning: the distinct cell keys of every tile (LDS hash set),
// an LSD radix sort of that list, runs of equal keys as bins.
#pragma once
#include "device_util.h"

namespace pcsir {

constexpr int TPB = 256;            // threads per block of the streaming kernels
constexpr int KEYS_TPB = 512;       // threads per block of the key dedup (k_keys)
constexpr int KEYS_TILE = 8192;     // particles of one target per tile of the key dedup
constexpr int BINS_TPB = 512;       // threads per block of the bin sums (k_bin_sums)
constexpr int LIST_BLOCKS_MAX = 2048;  // most workgroups of the sort / segment passes over the key list
constexpr int SCAN_ITEMS = 8;       // particles per thread in the weight scan and resampling
constexpr int SCAN_TILE = TPB * SCAN_ITEMS;
constexpr int RS_ITEMS = 4;         // new particles per thread in the resampling search
constexpr int RS_TILE = TPB * RS_ITEMS;
constexpr int RS_LIGHT_DEFAULT = 4096;  // most offspring a scan tile resolves itself (tunable)
constexpr int RS_LIGHT_MAX = 4096;     // run slots of the on-chip decode
constexpr int RS_SEARCH_BLOCKS = 2048;  // most workgroups of the heavy-tile search (grid-stride)
constexpr int MAX_QUAD = 16;        // largest number of sub-samples per pixel axis
constexpr int PROP_TILES = 2;       // propagate tiles (TPB particles each) per block
constexpr int LIK_WAVES = 4;        // likelihood evaluations per block (one per wave)
constexpr int BIN_TILE_MAX = 4096;   // largest bin-sum tile: consecutive particles of one target

// Fixed-point scales of the bin sums (integer sums are exact and order-free).
constexpr float FX_POS = 4294967296.0f;  // 2^32: offsets from the cell's pixel, |d| <= 1/2
constexpr float FX_VEL = 16777216.0f;    // 2^24: velocities, |v| < 2^7
constexpr float FX_INT = 1048576.0f;     // 2^20: intensity, |I| < 2^15
constexpr double FX_SQ = 4294967296.0;   // 2^32: second moments of the offsets, (d 2^16)^2 rounded
constexpr float LIM_VEL = 128.0f;
constexpr float LIM_INT = 32768.0f;

// Device-side status bits (meta[META_ERR]).
constexpr uint64_t ERR_KEY_RANGE = 1;    // compacted cell range of all targets >= 2^32
constexpr uint64_t ERR_FIXED_SAT = 2;    // a velocity or intensity outside the fixed-point range
constexpr uint64_t ERR_NONFINITE = 4;    // a target's normalisation was not finite

enum {
  META_PASSES = 0, META_RANGE = 1, META_B = 2, META_ERR = 3, META_DIGIT = 4, META_DIRTY = 5,
  META_CHECKED = 6,   // surrogate: dummies checked against the exact likelihood (cumulative)
  META_MAXERR = 7,    // surrogate: largest |l_surrogate - l_exact| seen (float bits)
  META_FALLBACK = 8,  // surrogate: target-frames recomputed exactly (cumulative)
  META_L = 9,         // length of this frame's list of distinct (tile, cell) keys
  META_NCHK = 10,     // surrogate: dummies picked for the exact check this frame
  META_NFB = 11,      // surrogate: dummies of fallback targets this frame
  // arrival counters of kernels whose last workgroup finishes a reduction of
  // all workgroups' results (back to 0 at the end of every launch)
  META_ARRIVE_BBOX = 12, META_ARRIVE_KEYS = 13, META_ARRIVE_SEG = 14,
  META_N = 15
};

// Cell-occupancy bitmap: one bit per compacted cell key, 64 keys per word, as
// many words as cover every 32-bit key, so it holds any key range the step
// accepts. Each word sits in a 16-byte entry with the number of the first bin
// it holds, so that a particle's bin takes one load (1 GB in all).
struct __attribute__((aligned(16))) BmWord {
  unsigned long long bits;
  uint32_t first;
  uint32_t pad;
};
constexpr uint64_t BM_WORDS = 1ull << 26;
// Words in use for a key range of `range` keys:
__device__ __host__ __forceinline__ uint32_t bm_words(uint64_t range) {
  const uint64_t r = range < (1ull << 32) ? range : (1ull << 32);
  return (uint32_t)((r + 63) >> 6);
}
// A frame whose cell range of all targets does not fit 32-bit keys (reported
// as ERR_KEY_RANGE) gets no bins: its keys and key bases have wrapped, and
// bins numbered from them would not be ordered by target.
__device__ __forceinline__ bool key_range_overflow(const uint64_t *meta) {
  return meta[META_RANGE] > 0xFFFFFFFFull;
}

// Values one workgroup hands to another within a launch go through memory,
// not through the XCD's own L2 (which the other workgroup's XCD does not
// see): an agent-scope store writes through, and once the storing thread's
// memory counter has drained (stores_done) the value is visible to an
// agent-scope load on any XCD. Only the handed-over values take this path;
// an agent-scope fence instead would write back the XCD's whole L2.
template <typename T>
__device__ __forceinline__ void store_agent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_done() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Whether this workgroup is the last of its launch to get here: true in
// exactly one workgroup, which may then read with load_agent what every
// workgroup stored with store_agent before its call (the storing threads
// call stores_done first; the workgroup's count follows its barrier). Every
// workgroup calls it once, with all its threads; the last one resets the
// counter for the next launch. This fuses a reduction over all workgroups
// into the kernel that produces its inputs, instead of a separate
// one-workgroup launch.
__device__ __forceinline__ bool last_block(uint64_t *counter) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long n =
        __hip_atomic_fetch_add((unsigned long long *)counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = n + 1ull == (unsigned long long)gridDim.x * gridDim.y * gridDim.z;
    if (last) store_agent((unsigned long long *)counter, 0ull);
  }
  __syncthreads();
  return last != 0;
}
constexpr int MAX_DIGIT_BITS = 11;  // radix digit of at most 2048 buckets (LDS histogram)
constexpr int MIN_DIGIT_BITS = 6;
constexpr int MAX_BUCKETS = 1 << MAX_DIGIT_BITS;

struct Params {
  int dim, D, T;
  uint32_t NT;
  int m[3];                 // configured cells per pixel (fixed bin size)
  double bins_per_sigma;    // > 0: adaptive bin size, about this many bins per standard deviation
  int bins_max;             // adaptive: at most this many cells per pixel
  const int32_t *tm;        // [T][3] cells per pixel of every target in the current frame
  int acc_rows;             // rows of the bin sums (1 + D, plus 3 second moments for second-order dummies)
  int P, R, q;
  int psf, dummy_mode, per_target_frames, H, W;
  float sigma_psf, astig_gamma, astig_d, i_bg;
  double inv2sxi2;  // 1 / (2 sigma_xi^2)
  float proc_sigma[7];
  uint64_t seed;
  const int32_t *bbox_cur;  // [T][6] (x0, y0, z0, wx, wy, wz) of the current frame's cells
};

// Per-step values that change from frame to frame. They live in device memory
// (written by k_set_desc before each step) so that the kernel sequence of a
// step can be captured once in a HIP graph and replayed.
struct StepDesc {
  const float *frame;
  int64_t k;
};

__global__ void k_set_desc(StepDesc *__restrict__ d, const float *frame, int64_t k) {
  d->frame = frame;
  d->k = k;
}

struct Tile {
  int32_t t;     // target
  uint32_t i0;   // first particle of the tile, index within the target
  uint32_t base; // the target's first particle in storage
  uint32_t n;    // the target's particle count
};

// Bin-sum work item: up to BIN_TILE_MAX consecutive particles of one target.
struct BinTile {
  int32_t t;
  uint32_t i0, i1;  // particles [i0, i1) of target t
  uint32_t base;    // the target's first particle in storage
};

// ---------------------------------------------------------------- propagation
// Alg. SIR / Alg. pcSIR "draw a sample from pi": bootstrap proposal with the
// nearly-constant-velocity dynamics of Sec. 5.1. The gather x_j <- x~_{s(j)}
// of the previous frame's resampling is fused into the load. With KEYS
// (pcSIR), each tile of TPB particles writes the extremes of its new
// positions as the cell index clamps them (and, with adaptive bins, their
// sums and squares) for k_bbox_reduce, and the bin accumulators that the
// previous frame used (meta[META_DIRTY] of them) are cleared, as are the words
// of the cell-occupancy bitmap (bm) below the previous frame's key range, the
// only ones its key pass can have set. A block takes PROP_TILES tiles, so that
// their loads are in flight together.
template <int DIM, bool KEYS>
__global__ __launch_bounds__(TPB) void k_propagate(Params p, const Tile *__restrict__ tiles, uint32_t ntiles,
                                                   const uint32_t *__restrict__ off, const float *__restrict__ sin,
                                                   float *__restrict__ sout, const uint32_t *__restrict__ anc,
                                                   int pending, const StepDesc *__restrict__ desc,
                                                   float *__restrict__ bbox_part, double *__restrict__ mom_part,
                                                   unsigned long long *__restrict__ acc,
                                                   const uint64_t *__restrict__ meta, BmWord *__restrict__ bm) {
  constexpr int D = 2 * DIM + 1;
  constexpr int K = PROP_TILES;
  if (KEYS && bm) {
    const uint32_t nw = bm_words(meta[META_RANGE]);
    for (uint32_t w = blockIdx.x * TPB + threadIdx.x; w < nw; w += gridDim.x * TPB) bm[w].bits = 0ull;
  }
  // the block's K tiles: their ancestor loads, then their state loads, are
  // issued together (a duplicate of the last tile pads the last block and
  // writes nothing)
  Tile tl[K];
  bool valid[K];
  uint32_t src[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t tb = blockIdx.x * K + k;
    tl[k] = tiles[min(tb, ntiles - 1)];
    const uint32_t i = tl[k].i0 + threadIdx.x;
    valid[k] = tb < ntiles && i < tl[k].n;
    src[k] = tl[k].base + min(i, tl[k].n - 1);
  }
  if (pending) {
#pragma unroll
    for (int k = 0; k < K; ++k) src[k] = tl[k].base + min(anc[src[k]], tl[k].n - 1);
  }
  float x[K][D];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int d = 0; d < D; ++d) x[k][d] = sin[(size_t)d * p.NT + src[k]];
  const uint32_t dirty = KEYS ? (uint32_t)meta[META_DIRTY] : 0u;
  // extremes of the positions as cell_index clamps them (the cell index is
  // non-decreasing in the clamped value, so the extremes give the cell
  // range for any bin size), and with adaptive bins their sums and squares
  float kmin[K][DIM], kmax[K][DIM];
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      kmin[k][a] = INFINITY;
      kmax[k][a] = -INFINITY;
    }
    if (valid[k]) {
      const uint32_t i = tl[k].i0 + threadIdx.x;
      const uint32_t g = tl[k].base + i;
      float z[2 * ((D + 1) / 2)];
      normal_pairs<(D + 1) / 2>(p.seed, i, (uint64_t)desc->k, (uint32_t)tl[k].t, z);
      float nx[D];
#pragma unroll
      for (int a = 0; a < DIM; ++a) nx[a] = fmaf(p.proc_sigma[a], z[a], x[k][a] + x[k][DIM + a]);
#pragma unroll
      for (int a = 0; a < DIM; ++a) nx[DIM + a] = fmaf(p.proc_sigma[DIM + a], z[DIM + a], x[k][DIM + a]);
      nx[2 * DIM] = fmaf(p.proc_sigma[2 * DIM], z[2 * DIM], x[k][2 * DIM]);
#pragma unroll
      for (int d = 0; d < D; ++d) sout[(size_t)d * p.NT + g] = nx[d];
      if (KEYS) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const float xc = clamp_position(nx[a]);
          kmin[k][a] = xc;
          kmax[k][a] = xc;
        }
        if (g < dirty) {
#pragma unroll
          for (int c = 0; c < p.acc_rows; ++c) acc[(size_t)c * p.NT + g] = 0ull;
        }
      }
    }
  }
  if (KEYS) {
    // per tile: per-wave extremes (and sums), then one barrier and a combine of the block's waves
    __shared__ float wbox[K][TPB / WAVE][6];
    __shared__ double wmom[K][TPB / WAVE][6];
    const bool adaptive = p.bins_per_sigma > 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const float lo = wave_min(kmin[k][a]);
        const float hi = wave_max(kmax[k][a]);
        if (lane_id() == 0) {
          wbox[k][wave_id()][a] = lo;
          wbox[k][wave_id()][3 + a] = hi;
        }
        if (adaptive) {
          const double xd = valid[k] ? (double)kmin[k][a] : 0.0;  // the particle's clamped position
          const double s1 = wave_sum(xd);
          const double s2 = wave_sum(xd * xd);
          if (lane_id() == 0) {
            wmom[k][wave_id()][a] = s1;
            wmom[k][wave_id()][3 + a] = s2;
          }
        }
      }
    }
    __syncthreads();
    if (threadIdx.x < K * 2 * DIM) {
      const int k = threadIdx.x / (2 * DIM);
      const int r = threadIdx.x - k * 2 * DIM;
      const int a = r % DIM;
      const bool mx = r >= DIM;
      const uint32_t tb = blockIdx.x * K + k;
      float v = wbox[k][0][mx ? 3 + a : a];
      double sm = wmom[k][0][mx ? 3 + a : a];
#pragma unroll
      for (int w = 1; w < TPB / WAVE; ++w) {
        const float u = wbox[k][w][mx ? 3 + a : a];
        v = mx ? fmaxf(v, u) : fminf(v, u);
        if (adaptive) sm += wmom[k][w][mx ? 3 + a : a];
      }
      if (tb < ntiles) {
        bbox_part[(size_t)tb * 6 + (mx ? 3 : 0) + a] = v;
        if (adaptive) mom_part[(size_t)tb * 6 + (mx ? 3 : 0) + a] = sm;
      }
    }
  }
}

// Cells per pixel of a target on one axis with adaptive bins: about
// bins_per_sigma cells per standard deviation of its positions,
// m = ceil(bins_per_sigma / sigma) in [1, bins_max] (bins_max for sigma = 0),
// from the population variance S2/n - (S1/n)^2 in binary64.
__device__ __forceinline__ int32_t adaptive_m(double s1, double s2, double n, double c, int32_t m_max) {
  const double mean = s1 / n;
  double var = s2 / n - mean * mean;
  var = var > 0.0 ? var : 0.0;
  const double sd = sqrt(var);
  const double q = c / sd;  // +inf for sd = 0
  if (!(q < (double)m_max)) return m_max;
  const double mc = ceil(q);
  return mc < 1.0 ? 1 : (int32_t)mc;
}

// Exclusive scan of the per-target cell ranges -> compacted key bases, the
// total range, and the radix digit width and number of sort passes it needs;
// also resets the length of the frame's key list. Run by one workgroup of TPB
// threads: the last one of k_bbox_reduce.
__device__ __forceinline__ void bbox_scan(int T, const unsigned long long *__restrict__ range,
                                          uint32_t *__restrict__ kbase, uint64_t *__restrict__ meta, int max_bits) {
  __shared__ unsigned long long lds[TPB / WAVE];
  unsigned long long carry = 0;
  for (int t0 = 0; t0 < T; t0 += TPB) {
    const int t = t0 + threadIdx.x;
    const unsigned long long r = t < T ? load_agent(&range[t]) : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<TPB, unsigned long long>(r, lds, &tot);
    if (t < T) kbase[t] = (uint32_t)(carry + ex);
    carry += tot;
    if (carry > (1ull << 40)) carry = (1ull << 40);
  }
  if (threadIdx.x == 0) {
    kbase[T] = (uint32_t)carry;
    meta[META_RANGE] = carry;
    int bits = 0;
    if (carry > 1) bits = 64 - __clzll((long long)(carry - 1));
    if (carry > 0xFFFFFFFFull) {
      meta[META_ERR] |= ERR_KEY_RANGE;
      bits = 32;
    }
    // fewest passes of at most max_bits bits, digits as narrow as that allows
    // (max_bits = 0: bins numbered from the occupancy bitmap, no sort)
    const int passes = max_bits > 0 ? (bits + max_bits - 1) / max_bits : 0;
    const int width = passes ? (bits + passes - 1) / passes : 1;
    meta[META_PASSES] = (uint64_t)passes;
    meta[META_DIGIT] = (uint64_t)width;
    meta[META_L] = 0;
    meta[META_NCHK] = 0;
    meta[META_NFB] = 0;
  }
}

// Per-target cells per pixel and cell range from the propagate tiles' partial
// extremes (tiles of target t: t256_first[t] .. t256_first[t+1]-1). One
// block per target.
__global__ __launch_bounds__(TPB) void k_bbox_reduce(Params p, const uint32_t *__restrict__ t256_first,
                                                     const uint32_t *__restrict__ off,
                                                     const float *__restrict__ bbox_part,
                                                     const double *__restrict__ mom_part, int32_t *__restrict__ tm,
                                                     int32_t *__restrict__ bbox_cur,
                                                     unsigned long long *__restrict__ range,
                                                     int32_t *__restrict__ tfallback, uint32_t *__restrict__ kbase,
                                                     uint64_t *__restrict__ meta, int max_bits) {
  __shared__ float redf[TPB / WAVE];
  __shared__ double redd[TPB / WAVE];
  const int t = blockIdx.x;
  const uint32_t a0 = t256_first[t], a1 = t256_first[t + 1];
  const double n = (double)(off[t + 1] - off[t]);
  unsigned long long r = 1;
  for (int a = 0; a < 3; ++a) {
    int32_t lo = 0, wdt = 1, m = 1;
    if (a < p.dim) {
      float mn = INFINITY, mx = -INFINITY;
      double s1 = 0.0, s2 = 0.0;
      for (uint32_t b = a0 + threadIdx.x; b < a1; b += TPB) {
        mn = fminf(mn, bbox_part[(size_t)b * 6 + a]);
        mx = fmaxf(mx, bbox_part[(size_t)b * 6 + 3 + a]);
        if (p.bins_per_sigma > 0.0) {
          s1 += mom_part[(size_t)b * 6 + a];
          s2 += mom_part[(size_t)b * 6 + 3 + a];
        }
      }
      const float fl = block_min<TPB>(mn, redf);
      const float fh = block_max<TPB>(mx, redf);
      m = p.m[a];
      if (p.bins_per_sigma > 0.0) {
        const double S1 = block_sum<TPB>(s1, redd);
        const double S2 = block_sum<TPB>(s2, redd);
        m = adaptive_m(S1, S2, n, p.bins_per_sigma, p.bins_max);
      }
      lo = cell_index(fl, m);
      const int32_t hi = cell_index(fh, m);
      long long w64 = (long long)hi - (long long)lo + 1;
      w64 = w64 < 1 ? 1 : (w64 > 0x7FFFFFFFLL ? 0x7FFFFFFFLL : w64);  // flagged by the scan if too wide
      wdt = (int32_t)w64;
    }
    if (threadIdx.x == 0) {
      bbox_cur[t * 6 + a] = lo;
      bbox_cur[t * 6 + 3 + a] = wdt;
      tm[t * 3 + a] = m;
    }
    r *= (unsigned long long)(uint32_t)wdt;
    if (r > (1ull << 40)) r = (1ull << 40);
  }
  if (threadIdx.x == 0) {
    store_agent(&range[t], r);
    stores_done();
    tfallback[t] = 0;
  }
  if (last_block(&meta[META_ARRIVE_BBOX])) bbox_scan(p.T, range, kbase, meta, max_bits);
}

template <int DIM>
__device__ __forceinline__ uint32_t compact_key(const int32_t *c, const int32_t *bb, uint32_t kb) {
  // key = base + ((kz - z0) * wy + (ky - y0)) * wx + (kx - x0): ascending (kz, ky, kx)
  uint32_t l = 0;
  if (DIM == 3) l = (uint32_t)(c[2] - bb[2]);
  l = l * (uint32_t)bb[4] + (uint32_t)(c[1] - bb[1]);
  l = l * (uint32_t)bb[3] + (uint32_t)(c[0] - bb[0]);
  return kb + l;
}

template <int DIM>
__device__ __forceinline__ uint32_t particle_key(const float *__restrict__ s, uint32_t NT, uint32_t g, const int *m,
                                                 const int32_t *bb, uint32_t kb) {
  int32_t c[3];
#pragma unroll
  for (int a = 0; a < DIM; ++a) c[a] = cell_index(s[(size_t)a * NT + g], m[a]);
  return compact_key<DIM>(c, bb, kb);
}

// Distinct cell keys of one key tile (at most KEYS_TILE particles of one
// target), found with an open-addressing hash set in LDS of as many slots
// as the tile has particles: a tile has at most that many distinct keys, so
// every insertion finds its key or an empty slot (typical tiles fill a few
// percent of it), and 32 KB of LDS with two rounds of eight particles per
// thread leave room for eight waves per SIMD. Larger tiles than the bin
// sums' repeat a cell in fewer tiles, so the list to sort is shorter. A tile
// has at most as many distinct keys as particles, so it writes them into its
// own particle range of `sparse` (global index of its first particle on), and its count to
// tcount[tile]; the last workgroup turns the counts into offsets, and
// k_list_compact packs the tiles' keys into one list, in tile order, without
// atomics. The list holds every occupied cell at least once.
// With the occupancy bitmap (bm) a tile instead sets the bits of its distinct
// keys and adds its key count to the list length, which is then only
// reported: the keys are first merged by bitmap word in a second LDS table
// (cells next to each other along x share a word), and each word then takes
// one 64-bit atomic OR to memory; a key that finds no free slot within a few
// probes goes to memory by itself.
constexpr int DEDUP_LOG2 = 13;
constexpr int DEDUP_SLOTS = KEYS_TILE;
constexpr int DEDUP_SHIFT = 32 - DEDUP_LOG2;
static_assert(DEDUP_SLOTS == 1 << DEDUP_LOG2, "hash slots");
constexpr uint32_t KEY_EMPTY = 0xFFFFFFFFu;  // compacted keys are < 2^32 - 1 (checked range)
constexpr int WORD_SLOTS_LOG2 = 11;          // bitmap words of a key tile merged in LDS
constexpr int WORD_SLOTS = 1 << WORD_SLOTS_LOG2;
constexpr int WORD_PROBES = 8;
static_assert(WORD_SLOTS * 12 <= DEDUP_SLOTS * 4, "the word table reuses the key table's LDS");

template <int DIM>
__global__ __launch_bounds__(KEYS_TPB) void k_keys(Params p, const BinTile *__restrict__ tiles,
                                              const uint32_t *__restrict__ off, const float *__restrict__ s,
                                              const int32_t *__restrict__ bbox_cur, const uint32_t *__restrict__ kbase,
                                              uint32_t *__restrict__ sparse, uint32_t *__restrict__ tcount,
                                              uint64_t *__restrict__ meta, BmWord *__restrict__ bm) {
  constexpr int R = KEYS_TILE / KEYS_TPB / 2;  // a thread's positions of a round are loaded before use
  constexpr int PER = DEDUP_SLOTS / KEYS_TPB;
  __shared__ __attribute__((aligned(16))) uint32_t tab[DEDUP_SLOTS];
  __shared__ uint32_t lds[KEYS_TPB / WAVE];
  const BinTile tl = tiles[blockIdx.x];
  const int t = tl.t;
  const uint32_t base = tl.base;
  int32_t bb[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) bb[a] = bbox_cur[t * 6 + a];
  const uint32_t kb = kbase[t];
  for (int i = threadIdx.x; i < DEDUP_SLOTS / 4; i += KEYS_TPB)
    reinterpret_cast<uint4 *>(tab)[i] = make_uint4(KEY_EMPTY, KEY_EMPTY, KEY_EMPTY, KEY_EMPTY);
  __syncthreads();
  for (uint32_t r0 = tl.i0; r0 < tl.i1; r0 += R * KEYS_TPB) {
    // all of the round's positions loaded first, from clamped indices (a load under a bounds
    // branch would be waited for before the next one is issued), then keyed
    float xs[DIM][R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const uint32_t g = base + min(r0 + q * KEYS_TPB + threadIdx.x, tl.i1 - 1);
#pragma unroll
      for (int a = 0; a < DIM; ++a) xs[a][q] = s[(size_t)a * p.NT + g];
    }
    uint32_t kk[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      int32_t c[3];
#pragma unroll
      for (int a = 0; a < DIM; ++a) c[a] = cell_index(xs[a][q], p.tm[t * 3 + a]);
      kk[q] = r0 + q * KEYS_TPB + threadIdx.x < tl.i1 ? compact_key<DIM>(c, bb, kb) : KEY_EMPTY;
    }
    // the compare-and-swap of every key at its home slot at once (R atomics
    // in flight instead of R round trips): it inserts the key or returns what
    // the slot holds; a slot, once filled, never changes, so only a slot
    // holding another key sends the key on to the next slots
    uint32_t hh[R], vv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      hh[q] = (kk[q] * 0x9E3779B1u) >> DEDUP_SHIFT;  // Fibonacci hashing: top bits of the product
      vv[q] = kk[q] == KEY_EMPTY ? KEY_EMPTY : atomicCAS(&tab[hh[q]], KEY_EMPTY, kk[q]);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const uint32_t k = kk[q];
      if (k == KEY_EMPTY) continue;
      uint32_t h = hh[q], v = vv[q];
      while (v != KEY_EMPTY && v != k) {
        h = (h + 1) & (DEDUP_SLOTS - 1);
        v = atomicCAS(&tab[h], KEY_EMPTY, k);
      }
    }
  }
  __syncthreads();
  if (bm) {
    uint32_t ks[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) ks[j] = tab[j * KEYS_TPB + threadIdx.x];
    __syncthreads();
    // the key table's LDS becomes the word table: word numbers, then their masks
    uint32_t *wkey = tab;
    unsigned long long *wmask = reinterpret_cast<unsigned long long *>(tab + WORD_SLOTS);
    for (int i = threadIdx.x; i < WORD_SLOTS; i += KEYS_TPB) {
      wkey[i] = KEY_EMPTY;
      wmask[i] = 0ull;
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t k = ks[j];
      if (k == KEY_EMPTY) continue;
      ++c;
      const uint32_t wd = k >> 6;  // below 2^26: never KEY_EMPTY
      const unsigned long long bit = 1ull << (k & 63u);
      uint32_t h = (wd * 0x9E3779B1u) >> (32 - WORD_SLOTS_LOG2);
      bool merged = false;
      for (int pr = 0; pr < WORD_PROBES; ++pr) {
        const uint32_t v = atomicCAS(&wkey[h], KEY_EMPTY, wd);
        if (v == KEY_EMPTY || v == wd) {
          atomicOr(&wmask[h], bit);
          merged = true;
          break;
        }
        h = (h + 1) & (WORD_SLOTS - 1);
      }
      if (!merged) atomicOr(&bm[wd].bits, bit);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < WORD_SLOTS; i += KEYS_TPB) {
      const uint32_t wd = wkey[i];
      if (wd != KEY_EMPTY) atomicOr(&bm[wd].bits, wmask[i]);
    }
    const uint32_t tot = block_sum<KEYS_TPB, uint32_t>(c, lds);
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)&meta[META_L], (unsigned long long)tot);
    return;
  }
  // thread t reads 16-byte groups t, t + KEYS_TPB, ... of slots (consecutive
  // lanes, consecutive banks), once, and keeps them for the write
  uint4 sl[PER / 4];
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < PER / 4; ++j) {
    sl[j] = reinterpret_cast<const uint4 *>(tab)[j * KEYS_TPB + threadIdx.x];
    c += (sl[j].x != KEY_EMPTY) + (sl[j].y != KEY_EMPTY) + (sl[j].z != KEY_EMPTY) + (sl[j].w != KEY_EMPTY);
  }
  uint32_t tot;
  uint32_t o = base + tl.i0 + block_excl_scan<KEYS_TPB, uint32_t>(c, lds, &tot);
  if (threadIdx.x == 0) {
    store_agent(&tcount[blockIdx.x], tot);
    stores_done();
  }
#pragma unroll
  for (int j = 0; j < PER / 4; ++j) {
    if (sl[j].x != KEY_EMPTY) sparse[o++] = sl[j].x;
    if (sl[j].y != KEY_EMPTY) sparse[o++] = sl[j].y;
    if (sl[j].z != KEY_EMPTY) sparse[o++] = sl[j].z;
    if (sl[j].w != KEY_EMPTY) sparse[o++] = sl[j].w;
  }
  // the last workgroup turns the tiles' key counts into their offsets in the
  // packed list (exclusive scan, in tile order) and sets the list's length
  if (last_block(&meta[META_ARRIVE_KEYS])) {
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < gridDim.x; b0 += KEYS_TPB) {
      const uint32_t b = b0 + threadIdx.x;
      const uint32_t v = b < gridDim.x ? load_agent(&tcount[b]) : 0u;
      uint32_t t2;
      const uint32_t ex = block_excl_scan<KEYS_TPB, uint32_t>(v, lds, &t2);
      if (b < gridDim.x) tcount[b] = carry + ex;
      carry += t2;
    }
    if (threadIdx.x == 0) meta[META_L] = carry;
  }
}

// Pack each tile's keys to its offset in the list (one block per tile).
__global__ __launch_bounds__(TPB) void k_list_compact(const BinTile *__restrict__ tiles,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ toff, uint32_t ntiles,
                                                      const uint64_t *__restrict__ meta,
                                                      const uint32_t *__restrict__ sparse, uint32_t *__restrict__ list) {
  const BinTile tl = tiles[blockIdx.x];
  const uint32_t src = tl.base + tl.i0;
  const uint32_t o = toff[blockIdx.x];
  const uint32_t end = blockIdx.x + 1 < ntiles ? toff[blockIdx.x + 1] : (uint32_t)meta[META_L];
  for (uint32_t i = threadIdx.x; i < end - o; i += TPB) list[o + i] = sparse[src + i];
}

// Contiguous share of a device-sized list for block b of G.
__device__ __forceinline__ void list_range(uint32_t L, uint32_t G, uint32_t b, uint32_t &j0, uint32_t &j1) {
  const uint32_t chunk = (L + G - 1) / G;
  j0 = min(L, b * chunk);
  j1 = min(L, j0 + chunk);
}

// ---------------------------------------------------------------- LSD radix sort
// Sort of the key list (length meta[META_L]) by digits of meta[META_DIGIT]
// bits; pass `pass` runs only if the frame's key range needs it. Each of the
// G workgroups owns one contiguous share of the list.
// Lanes of the wave holding the same digit d (at most MAX_DIGIT_BITS bits;
// invalid lanes carry d = MAX_BUCKETS and match only each other).
__device__ __forceinline__ unsigned long long digit_peers(bool valid, uint32_t d, int width) {
  unsigned long long peers = __ballot(valid);
  if (!valid) peers = ~peers;
  for (int bit = 0; bit < width; ++bit) {
    const unsigned long long bb = __ballot((d >> bit) & 1u);
    peers &= ((d >> bit) & 1u) ? bb : ~bb;
  }
  return peers;
}

// Each pass: per-workgroup digit counts (k_sort_hist), their scan per digit
// across workgroups (k_sort_scan), and the stable scatter (k_sort_scatter).
// A workgroup takes its share of the list in rounds of SORT_ITEMS keys per
// thread, all loaded before use.
constexpr int SORT_ITEMS = 8;

// Per-block digit histograms of pass `pass` over that pass's input order (the
// scatter ranks each block's share of its own input, so the counts must come
// from the same keys in the same order); the digit width comes from the device
// (meta[META_DIGIT]) and the pass runs only if the key range needs it.
__global__ __launch_bounds__(TPB) void k_sort_hist(int pass, const uint32_t *__restrict__ key,
                                                   uint32_t *__restrict__ hist, uint32_t G,
                                                   const uint64_t *__restrict__ meta) {
  if ((uint64_t)pass >= meta[META_PASSES]) return;
  const int width = (int)meta[META_DIGIT];
  const uint32_t nb = 1u << width, mask = nb - 1u;
  __shared__ uint32_t cnt[MAX_BUCKETS];
  for (uint32_t d = threadIdx.x; d < nb; d += TPB) cnt[d] = 0;
  __syncthreads();
  uint32_t j0, j1;
  list_range((uint32_t)meta[META_L], G, blockIdx.x, j0, j1);
  const int sh = width * pass;
  const unsigned long long below = (1ull << lane_id()) - 1ull;
  for (uint32_t r0 = j0; r0 < j1; r0 += SORT_ITEMS * TPB) {
    uint32_t kk[SORT_ITEMS];
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
      const uint32_t j = r0 + i * TPB + threadIdx.x;
      kk[i] = j < j1 ? key[j] : 0u;
    }
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
      const bool valid = r0 + i * TPB + threadIdx.x < j1;
      const uint32_t d = valid ? (kk[i] >> sh) & mask : (uint32_t)MAX_BUCKETS;
      const unsigned long long peers = digit_peers(valid, d, width);
      if (valid && (peers & below) == 0ull) atomicAdd(&cnt[d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < nb; d += TPB) hist[(size_t)d * G + blockIdx.x] = cnt[d];
}

// One block per digit: exclusive scan of that digit's per-block counts.
__global__ __launch_bounds__(TPB) void k_sort_scan(int pass, uint32_t *__restrict__ hist, uint32_t G,
                                                   uint32_t *__restrict__ digit_total,
                                                   const uint64_t *__restrict__ meta) {
  if ((uint64_t)pass >= meta[META_PASSES]) return;
  if (blockIdx.x >= (1u << (int)meta[META_DIGIT])) return;
  __shared__ uint32_t lds[TPB / WAVE];
  uint32_t *h = hist + (size_t)blockIdx.x * G;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < G; b0 += TPB) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < G ? h[b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<TPB, uint32_t>(v, lds, &tot);
    if (b < G) h[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

// Stable scatter of pass `pass`: slots in (round, item, wave, lane) order,
// where an item is TPB consecutive keys of the list; within an item each wave
// ranks its lanes by digit with ballots, waves are ordered through per-wave
// digit counts in LDS, and a per-digit running offset carries the order
// across items. Item i's per-wave counts use wcnt[i & 1], which item i clears
// after its slots are taken and item i + 2 refills (two barriers per item).
__global__ __launch_bounds__(TPB) void k_sort_scatter(int pass, const uint32_t *__restrict__ key_in,
                                                      uint32_t *__restrict__ key_out,
                                                      const uint32_t *__restrict__ hist, uint32_t G,
                                                      const uint32_t *__restrict__ digit_total,
                                                      const uint64_t *__restrict__ meta) {
  if ((uint64_t)pass >= meta[META_PASSES]) return;
  const int width = (int)meta[META_DIGIT];
  const uint32_t nb = 1u << width, mask = nb - 1u;
  constexpr int PER = MAX_BUCKETS / TPB;
  __shared__ uint32_t run[MAX_BUCKETS];
  __shared__ uint32_t wcnt[2][TPB / WAVE][MAX_BUCKETS];
  __shared__ uint32_t lds[TPB / WAVE];
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
  {
    // exclusive scan of the digit totals: each thread owns PER consecutive digits
    uint32_t loc[PER], s = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t d = (uint32_t)(tid * PER + i);
      loc[i] = d < nb ? digit_total[d] : 0u;
      s += loc[i];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<TPB, uint32_t>(s, lds, &tot);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t d = (uint32_t)(tid * PER + i);
      if (d < nb) run[d] = ex + hist[(size_t)d * G + blockIdx.x];
      ex += loc[i];
      for (int ww = 0; ww < TPB / WAVE; ++ww) wcnt[0][ww][d] = wcnt[1][ww][d] = 0;
    }
  }
  __syncthreads();
  uint32_t j0, j1;
  list_range((uint32_t)meta[META_L], G, blockIdx.x, j0, j1);
  const int sh = width * pass;
  const unsigned long long below = (1ull << lane) - 1ull;
  int par = 0;
  for (uint32_t r0 = j0; r0 < j1; r0 += SORT_ITEMS * TPB) {
    uint32_t kk[SORT_ITEMS];
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
      const uint32_t j = r0 + i * TPB + tid;
      kk[i] = j < j1 ? key_in[j] : 0u;
    }
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
      if (r0 + i * TPB >= j1) break;  // the same for the whole workgroup
      const bool valid = r0 + i * TPB + tid < j1;
      const uint32_t d = valid ? (kk[i] >> sh) & mask : (uint32_t)MAX_BUCKETS;
      const unsigned long long peers = digit_peers(valid, d, width);
      const uint32_t rank = (uint32_t)__popcll(peers & below);
      const bool leader = valid && rank == 0;
      const uint32_t cnt = (uint32_t)__popcll(peers);
      if (leader) wcnt[par][w][d] = cnt;
      __syncthreads();
      if (valid) {
        uint32_t pos = run[d] + rank;
        for (int ww = 0; ww < w; ++ww) pos += wcnt[par][ww][d];
        key_out[pos] = kk[i];
      }
      __syncthreads();
      if (leader) {
        atomicAdd(&run[d], cnt);
        wcnt[par][w][d] = 0;
      }
      par ^= 1;
    }
  }
}

struct SortBufs {
  const uint32_t *key_store;  // the unsorted list (0 passes: a single key value)
  const uint32_t *kA, *kB;
};
__device__ __forceinline__ const uint32_t *sorted_keys(const SortBufs &sb, uint64_t passes) {
  return passes == 0 ? sb.key_store : ((passes & 1) ? sb.kB : sb.kA);
}

// ---------------------------------------------------------------- segments (bins)
// A bin is a run of equal keys in the sorted list. Bins are numbered in
// sorted order: per-block head counts, their scan, then one pass that records
// each bin's key and target, and a search for the first bin of every target.
__device__ __forceinline__ bool seg_head(const uint32_t *__restrict__ K, uint32_t j) {
  return j == 0 || K[j] != K[j - 1];
}

// Per-block head counts; the last workgroup scans them (exclusive, in block
// order) into each block's first bin and writes the bin count B.
__global__ __launch_bounds__(TPB) void k_seg_count(uint32_t G, int T, SortBufs sb, uint64_t *__restrict__ meta,
                                                   uint32_t *__restrict__ chunk_heads,
                                                   uint32_t *__restrict__ seg_first) {
  __shared__ uint32_t lds[TPB / WAVE];
  const uint32_t *K = sorted_keys(sb, meta[META_PASSES]);
  uint32_t j0, j1;
  list_range((uint32_t)meta[META_L], G, blockIdx.x, j0, j1);
  uint32_t c = 0;
  for (uint32_t j = j0 + threadIdx.x; j < j1; j += TPB)
    if (seg_head(K, j)) ++c;
  const uint32_t s = block_sum<TPB, uint32_t>(c, lds);
  if (threadIdx.x == 0) {
    store_agent(&chunk_heads[blockIdx.x], s);
    stores_done();
  }
  if (!last_block(&meta[META_ARRIVE_SEG])) return;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < G; b0 += TPB) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < G ? load_agent(&chunk_heads[b]) : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<TPB, uint32_t>(v, lds, &tot);
    if (b < G) chunk_heads[b] = carry + ex;
    carry += tot;
  }
  if (key_range_overflow(meta)) carry = 0;  // no bins (k_seg_mark writes nothing)
  if (threadIdx.x == 0) {
    meta[META_B] = carry;
    meta[META_DIRTY] = carry;  // accumulators [0, B) are written this frame
  }
  // an empty list has no bins: every target's first bin is 0 (k_seg_mark
  // writes seg_first otherwise)
  if (carry == 0)
    for (int t = threadIdx.x; t <= T; t += TPB) seg_first[t] = 0;
}

template <int DIM>
__device__ __forceinline__ void decode_key(uint32_t key, int T, const uint32_t *__restrict__ kbase,
                                           const int32_t *__restrict__ bbox_cur, int &t, int32_t c[3]) {
  // target: last t with kbase[t] <= key
  int lo = 0, hi = T - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (kbase[mid] <= key) lo = mid;
    else hi = mid - 1;
  }
  t = lo;
  uint32_t l = key - kbase[t];
  const int32_t *bb = bbox_cur + t * 6;
  c[0] = bb[0] + (int32_t)(l % (uint32_t)bb[3]);
  l /= (uint32_t)bb[3];
  if (DIM == 3) {
    c[1] = bb[1] + (int32_t)(l % (uint32_t)bb[4]);
    c[2] = bb[2] + (int32_t)(l / (uint32_t)bb[4]);
  } else {
    c[1] = bb[1] + (int32_t)l;
    c[2] = 0;
  }
}

template <typename KB>
__device__ __forceinline__ int key_target(uint32_t key, int T, KB kbase) {
  int lo = 0, hi = T - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (kbase[mid] <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Targets whose key bases k_seg_mark stages in LDS for its searches.
constexpr int KBASE_LDS = 4096;

// Record every bin: its key and its target, and every target's first bin:
// seg_first[t] is the first bin whose key is >= kbase[t] (bins are sorted by
// key and targets own consecutive key ranges), seg_first[T] = B. A bin whose
// target tb differs from that of the bin before it (target tp, or -1 for the
// first bin) is the first bin of every target in (tp, tb], so it writes those
// entries, and the list's last key writes B into those after its target:
// every entry is written once, with no search over the bins. (B = 0 is
// handled by k_seg_count.)
__global__ __launch_bounds__(TPB) void k_seg_mark(Params p, uint32_t G, SortBufs sb, uint64_t *__restrict__ meta,
                                                  const uint32_t *__restrict__ chunk_base,
                                                  const uint32_t *__restrict__ kbase, uint32_t *__restrict__ seg_key,
                                                  int32_t *__restrict__ seg_t, uint32_t *__restrict__ lut,
                                                  uint64_t lut_cap, uint32_t *__restrict__ seg_first) {
  if (key_range_overflow(meta)) return;  // no bins this frame (k_seg_count)
  const bool use_lut = meta[META_RANGE] <= lut_cap;
  __shared__ uint32_t lds[TPB / WAVE];
  __shared__ uint32_t kb_lds[KBASE_LDS];
  const bool kb_in_lds = p.T <= KBASE_LDS;
  if (kb_in_lds)
    for (int t = threadIdx.x; t < p.T; t += TPB) kb_lds[t] = kbase[t];
  __syncthreads();
  const uint32_t *K = sorted_keys(sb, meta[META_PASSES]);
  const uint32_t L = (uint32_t)meta[META_L];
  uint32_t j0, j1;
  list_range(L, G, blockIdx.x, j0, j1);
  uint32_t heads = chunk_base[blockIdx.x];
  for (uint32_t r0 = j0; r0 < j1; r0 += TPB) {
    const uint32_t j = r0 + threadIdx.x;
    const bool h = j < j1 && seg_head(K, j);
    uint32_t tot;
    const uint32_t ex = block_excl_scan<TPB, uint32_t>(h ? 1u : 0u, lds, &tot);
    if (h) {
      const uint32_t kj = K[j];
      const int tb = kb_in_lds ? key_target(kj, p.T, (const uint32_t *)kb_lds) : key_target(kj, p.T, kbase);
      seg_key[heads + ex] = kj;
      seg_t[heads + ex] = tb;
      if (use_lut) lut[kj] = heads + ex;  // bin of every occupied cell key
      // previous bin's target: below tb only if its key is below tb's base
      int tp = tb;
      if (j == 0) tp = -1;
      else if (K[j - 1] < kbase[tb])
        tp = kb_in_lds ? key_target(K[j - 1], p.T, (const uint32_t *)kb_lds) : key_target(K[j - 1], p.T, kbase);
      for (int t = tp + 1; t <= tb; ++t) seg_first[t] = heads + ex;
    }
    if (j + 1 == L && j < j1) {
      const uint32_t kl = K[j];
      const int tl = kb_in_lds ? key_target(kl, p.T, (const uint32_t *)kb_lds) : key_target(kl, p.T, kbase);
      const uint32_t B = (uint32_t)meta[META_B];
      for (int t = tl + 1; t <= p.T; ++t) seg_first[t] = B;
    }
    heads += tot;
  }
}

// ---------------------------------------------------------------- bins from the occupancy bitmap
// The same bins as the sorted list gives (distinct occupied cells, numbered in
// ascending key order), without a sort: a bin is a set bit of the bitmap that
// k_keys fills, and its number is the count of set bits below it. The G
// workgroups each take a contiguous share of the words in use. k_map_count
// counts the bits of its share. k_map_rank sums the counts of the shares
// before its own (at most a few thousand loads, instead of one workgroup
// waiting for all others), then writes every word's first bin, every
// bin's key and target, and the first bin of every target whose key base
// falls in its share; the last workgroup writes the bin count B (and
// seg_first[T] = B). A particle with key k is in its word's first bin plus
// the number of set bits of word k / 64 below bit k % 64.
__global__ __launch_bounds__(TPB) void k_map_count(uint32_t G, const BmWord *__restrict__ bm,
                                                   const uint64_t *__restrict__ meta,
                                                   uint32_t *__restrict__ chunk_count) {
  __shared__ uint32_t lds[TPB / WAVE];
  const uint32_t nw = key_range_overflow(meta) ? 0u : bm_words(meta[META_RANGE]);
  uint32_t j0, j1;
  list_range(nw, G, blockIdx.x, j0, j1);
  uint32_t c = 0;
  for (uint32_t j = j0 + threadIdx.x; j < j1; j += TPB) c += (uint32_t)__popcll(bm[j].bits);
  const uint32_t s = block_sum<TPB, uint32_t>(c, lds);
  if (threadIdx.x == 0) chunk_count[blockIdx.x] = s;
}

// First t in [0, T) with kb[t] >= key (T if none); kb ascending.
template <typename KB>
__device__ __forceinline__ int first_target_at(uint32_t key, int T, KB kb) {
  int lo = 0, hi = T;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kb[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(TPB) void k_map_rank(Params p, uint32_t G, uint64_t *__restrict__ meta,
                                                  const uint32_t *__restrict__ chunk_count,
                                                  const uint32_t *__restrict__ kbase,
                                                  BmWord *__restrict__ bm, uint32_t *__restrict__ seg_key,
                                                  int32_t *__restrict__ seg_t, uint32_t *__restrict__ seg_first) {
  __shared__ uint32_t lds[TPB / WAVE];
  __shared__ uint32_t kb_lds[KBASE_LDS];
  __shared__ uint32_t wpre[TPB];
  __shared__ unsigned long long wbits[TPB];
  __shared__ int32_t wtgt[TPB];
  const bool kb_in_lds = p.T <= KBASE_LDS;
  auto kb_at = [&](int t) -> uint32_t { return kb_in_lds ? kb_lds[t] : kbase[t]; };
  if (kb_in_lds)
    for (int t = threadIdx.x; t < p.T; t += TPB) kb_lds[t] = kbase[t];
  __syncthreads();
  const bool overflow = key_range_overflow(meta);
  const uint32_t nw = overflow ? 0u : bm_words(meta[META_RANGE]);
  if (overflow)  // no bins: every target's first bin is 0
    for (int t = blockIdx.x * TPB + threadIdx.x; t < p.T; t += G * TPB) seg_first[t] = 0;
  uint32_t j0, j1;
  list_range(nw, G, blockIdx.x, j0, j1);
  uint32_t before = 0;
  for (uint32_t b = threadIdx.x; b < blockIdx.x; b += TPB) before += chunk_count[b];
  uint32_t base = block_sum<TPB, uint32_t>(before, lds);
  for (uint32_t r0 = j0; r0 < j1; r0 += TPB) {
    const uint32_t j = r0 + threadIdx.x;
    const unsigned long long wd = j < j1 ? bm[j].bits : 0ull;
    uint32_t tot;
    const uint32_t pre = base + block_excl_scan<TPB, uint32_t>((uint32_t)__popcll(wd), lds, &tot);
    if (j < j1) bm[j].first = pre;
    wpre[threadIdx.x] = pre;
    wbits[threadIdx.x] = wd;
    // target of the word's first bin (by a search, once per word)
    int tw = 0;
    if (wd) {
      const uint32_t k0 = j * 64u + (uint32_t)__builtin_ctzll(wd);
      tw = kb_in_lds ? key_target(k0, p.T, (const uint32_t *)kb_lds) : key_target(k0, p.T, kbase);
    }
    wtgt[threadIdx.x] = tw;
    __syncthreads();
    // the round's bins, consecutive lanes taking consecutive bins: the word
    // that holds bin r is the last one whose first bin is <= r (words after
    // the share have no bits and first bin base + tot), the bin is the n-th
    // set bit of that word (found by halving with popcounts), and its target
    // is the word's first target, moved on past any key base it crosses
    for (uint32_t i = threadIdx.x; i < tot; i += TPB) {
      const uint32_t r = base + i;
      int lo = 0, hi = TPB - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wpre[mid] <= r) lo = mid;
        else hi = mid - 1;
      }
      unsigned long long b = wbits[lo];
      uint32_t n = r - wpre[lo], pos = 0;
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) {
        const uint32_t c = (uint32_t)__popcll(b & ((1ull << sh) - 1ull));
        if (n >= c) {
          n -= c;
          b >>= sh;
          pos += (uint32_t)sh;
        }
      }
      const uint32_t k = (r0 + (uint32_t)lo) * 64u + pos;
      int t = wtgt[lo];
      while (t + 1 < p.T && k >= kb_at(t + 1)) ++t;
      if (r < p.NT) {  // always: every set bit is the cell of a particle of this frame
        seg_key[r] = k;
        seg_t[r] = t;
      }
    }
    // first bin of every target whose key base lies in this round's words
    const uint32_t klo = r0 * 64u;
    const uint64_t khi = (uint64_t)min(r0 + (uint32_t)TPB, j1) * 64u;
    const int t0 = kb_in_lds ? first_target_at(klo, p.T, (const uint32_t *)kb_lds) : first_target_at(klo, p.T, kbase);
    for (int t = t0 + (int)threadIdx.x; t < p.T; t += TPB) {
      const uint32_t kt = kbase[t];
      if ((uint64_t)kt >= khi) break;  // key bases ascend
      if (kt < klo) continue;          // only with an overflowed key range (reported)
      const uint32_t wl = (kt >> 6) - r0;
      seg_first[t] = wpre[wl] + (uint32_t)__popcll(wbits[wl] & ((1ull << (kt & 63u)) - 1ull));
    }
    __syncthreads();
    base += tot;
  }
  if (blockIdx.x == G - 1 && threadIdx.x == 0) {
    meta[META_B] = base;
    meta[META_DIRTY] = base;  // accumulators [0, B) are written this frame
    seg_first[p.T] = base;
  }
}

// Members' sums of every bin as exact fixed-point integers: count, offsets of
// the positions from the pixel that holds them (the pixel of a cell is the
// pixel of each member, so x - pixel is exact and |.| <= 1/2), velocities and
// intensity. Particles are read in storage order (coalesced); a block holds
// one target's tile and recomputes each particle's cell key. The target's
// bins are taken in LDS chunks of BINS: for each chunk, the tile's particles
// whose bin falls in it accumulate in LDS with 64-bit integer atomics, then
// each bin of the chunk is flushed to HBM once. A particle's bin comes from
// the occupancy bitmap (two loads and a popcount) or, with bins from the
// sorted list, from this frame's cell -> bin table when the frame's key range
// fits it (one load); either way the tile is loaded once for all chunks.
// Otherwise it is a binary search over the chunk's keys, staged in LDS, with
// the tile read once per chunk.
// Integer sums are exact, so the result does not depend on order. Also
// writes every particle's bin number.
// MOM2 (second-order dummies, 2D) adds the second moments of the offsets:
// (dx 2^16)^2, (dy 2^16)^2 and (dx 2^16)(dy 2^16), each rounded to an integer.
template <int DIM, bool MOM2 = false>
struct BinLds {
  static constexpr int NC = 2 + 2 * DIM + (MOM2 ? 3 : 0);                // count + D components (+ 3)
  static constexpr int BINS = MOM2 ? 768 : (DIM == 2 ? 1024 : 896);      // table fits in 64 KB with the keys
  // threads per block: more components per particle take 1024 threads with
  // 4 particles each (instead of 512 with 8), which keeps the registers of a
  // thread within what four waves per SIMD allow
  static constexpr int NTH = (DIM == 3 || MOM2) ? 1024 : BINS_TPB;
  static constexpr int R = BIN_TILE_MAX / NTH;  // particles per thread and round, loaded together
};

// One member's fixed-point contributions: count, offsets from its pixel
// (x - pixel is exact, |.| <= 1/2), velocities, intensity, and with MOM2 the
// second moments of the offsets; sets sat where a value is outside its range.
template <int DIM, bool MOM2>
__device__ __forceinline__ void member_values(const float *xq, long long *val, bool &sat) {
  constexpr int NC = BinLds<DIM, MOM2>::NC;
  val[0] = 1;
  float dpos[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    // x - pix is exact and in [-1/2, 1/2), so the scaled value is in [-2^31, 2^31)
    const float pix = (float)cell_index(xq[a], 1);
    dpos[a] = xq[a] - pix;
    val[1 + a] = (long long)__float2int_rn(dpos[a] * FX_POS);
  }
  if (MOM2) {
    // d 2^16 is exact; products of two such values are within 2^30
    const double ux = (double)(dpos[0] * 65536.0f), uy = (double)(dpos[1 % DIM] * 65536.0f);
    val[NC - 3] = __double2ll_rn(ux * ux);
    val[NC - 2] = __double2ll_rn(uy * uy);
    val[NC - 1] = __double2ll_rn(ux * uy);
  }
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    float vel = xq[DIM + a];
    if (!(fabsf(vel) < LIM_VEL)) {
      sat = true;
      vel = 0.0f;
    }
    val[1 + DIM + a] = (long long)__float2int_rn(vel * FX_VEL);  // |v 2^24| < 2^31
  }
  float in = xq[2 * DIM];
  if (!(fabsf(in) < LIM_INT)) {
    sat = true;
    in = 0.0f;
  }
  val[1 + 2 * DIM] = __float2ll_rn(in * FX_INT);
}

template <int DIM, bool MOM2 = false>
__global__ __launch_bounds__((BinLds<DIM, MOM2>::NTH)) void k_bin_sums(Params p, const BinTile *__restrict__ tiles,
                                                  const uint32_t *__restrict__ off, const float *__restrict__ s,
                                                  const int32_t *__restrict__ bbox_cur,
                                                  const uint32_t *__restrict__ kbase,
                                                  const uint32_t *__restrict__ seg_key,
                                                  const uint32_t *__restrict__ seg_first,
                                                  unsigned long long *__restrict__ acc, uint32_t *__restrict__ segid,
                                                  uint64_t *__restrict__ meta, const uint32_t *__restrict__ lut,
                                                  uint64_t lut_cap, const BmWord *__restrict__ bm) {
  constexpr int D = 2 * DIM + 1;
  constexpr int NC = BinLds<DIM, MOM2>::NC;
  static_assert(!MOM2 || DIM == 2, "second moments in 2D only");
  // bins numbered from the occupancy bitmap (bm): a particle's bin is its
  // word's first bin plus a popcount; with the sorted list, the cell -> bin
  // table of this frame (total key range within its capacity) gives it in
  // one load, and otherwise a binary search does
  const bool use_lut = bm != nullptr || meta[META_RANGE] <= lut_cap;
  constexpr int BINS = BinLds<DIM, MOM2>::BINS;
  constexpr int R = BinLds<DIM, MOM2>::R;
  constexpr int NTH = BinLds<DIM, MOM2>::NTH;
  __shared__ uint32_t bkey[BINS];
  __shared__ unsigned long long bacc[NC][BINS];
  const uint32_t NT = p.NT;
  const BinTile tl = tiles[blockIdx.x];
  const int t = tl.t;
  const uint32_t base = tl.base;
  const uint32_t s0 = seg_first[t], nb = seg_first[t + 1] - s0;
  int32_t bb[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) bb[a] = bbox_cur[t * 6 + a];
  const uint32_t kb = kbase[t];
  if (nb == 0) {
    // only when the frame's key range overflowed (reported): keep segid in range
    for (uint32_t i = tl.i0 + threadIdx.x; i < tl.i1; i += NTH) segid[base + i] = 0;
    return;
  }
  bool sat = false;
  if (use_lut) {
    // a tile is one round (at most R NTH particles): each particle is
    // loaded and its bin looked up once, and each LDS chunk of the target's
    // bins then takes the particles whose bin it holds
    static_assert(BIN_TILE_MAX <= R * NTH, "one round per bin-sum tile");
    float x[R][D];
    uint32_t bin[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const uint32_t i = min(tl.i0 + q * NTH + threadIdx.x, tl.i1 - 1);  // clamped: unconditional loads
#pragma unroll
      for (int d = 0; d < D; ++d) x[q][d] = s[(size_t)d * NT + base + i];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      int32_t cc[3];
#pragma unroll
      for (int a = 0; a < DIM; ++a) cc[a] = cell_index(x[q][a], p.tm[t * 3 + a]);
      bin[q] = compact_key<DIM>(cc, bb, kb);
    }
    if (bm) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint32_t k = bin[q];
        const uint4 e = *reinterpret_cast<const uint4 *>(&bm[k >> 6]);
        const unsigned long long bits = ((unsigned long long)e.y << 32) | e.x;
        bin[q] = e.z + (uint32_t)__popcll(bits & ((1ull << (k & 63u)) - 1ull));
      }
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) bin[q] = lut[bin[q]];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const uint32_t i = tl.i0 + q * NTH + threadIdx.x;
      if (i < tl.i1) segid[base + i] = bin[q];
    }
    for (uint32_t c0 = 0; c0 < nb; c0 += BINS) {
      const uint32_t cn = min((uint32_t)BINS, nb - c0);
      for (uint32_t b = threadIdx.x; b < cn; b += NTH) {
#pragma unroll
        for (int c = 0; c < NC; ++c) bacc[c][b] = 0ull;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint32_t lo = bin[q] - (s0 + c0);  // wraps above cn for bins of other chunks
        if (tl.i0 + q * NTH + threadIdx.x >= tl.i1 || lo >= cn) continue;
        long long val[NC];
        member_values<DIM, MOM2>(x[q], val, sat);
#pragma unroll
        for (int c = 0; c < NC; ++c) atomicAdd(&bacc[c][lo], (unsigned long long)val[c]);
      }
      __syncthreads();
      for (uint32_t b = threadIdx.x; b < cn; b += NTH) {
        if (bacc[0][b] == 0ull) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c) atomicAdd(&acc[(size_t)c * NT + s0 + c0 + b], bacc[c][b]);
      }
      __syncthreads();
    }
    if (sat) atomicOr((unsigned long long *)&meta[META_ERR], (unsigned long long)ERR_FIXED_SAT);
    return;
  }
  for (uint32_t c0 = 0; c0 < nb; c0 += BINS) {
    const uint32_t cn = min((uint32_t)BINS, nb - c0);
    for (uint32_t b = threadIdx.x; b < cn; b += NTH) {
      bkey[b] = seg_key[s0 + c0 + b];
#pragma unroll
      for (int c = 0; c < NC; ++c) bacc[c][b] = 0ull;
    }
    __syncthreads();
    const uint32_t klo = bkey[0], khi = bkey[cn - 1];
    const bool first = c0 == 0, last = c0 + cn == nb;
    for (uint32_t r0 = tl.i0; r0 < tl.i1; r0 += R * NTH) {
      float x[R][D];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint32_t i = min(r0 + q * NTH + threadIdx.x, tl.i1 - 1);  // clamped: unconditional loads
#pragma unroll
        for (int d = 0; d < D; ++d) x[q][d] = s[(size_t)d * NT + base + i];
      }
      // each particle's bin within the chunk, by binary search over its keys
      uint32_t lob[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        int32_t cc[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) cc[a] = cell_index(x[q][a], p.tm[t * 3 + a]);
        const uint32_t k = compact_key<DIM>(cc, bb, kb);
        if (k < klo || k > khi) {
          lob[q] = 0xFFFFFFFFu;
        } else {
          uint32_t l0 = 0, h0 = cn - 1;
          while (l0 < h0) {
            const uint32_t mid = (l0 + h0) >> 1;
            if (bkey[mid] < k) l0 = mid + 1;
            else h0 = mid;
          }
          lob[q] = l0;
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint32_t i = r0 + q * NTH + threadIdx.x;
        if (i >= tl.i1) continue;
        const uint32_t g = base + i;
        const uint32_t lo = lob[q];
        if (lo >= cn) {
          // a bin of another chunk; the first chunk gives every particle a
          // valid bin number, which the particle's own chunk overwrites
          if (first && !last) segid[g] = s0;
          continue;
        }
        segid[g] = s0 + c0 + lo;
        long long val[NC];
        member_values<DIM, MOM2>(x[q], val, sat);
#pragma unroll
        for (int c = 0; c < NC; ++c) atomicAdd(&bacc[c][lo], (unsigned long long)val[c]);
      }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < cn; b += NTH) {
      if (bacc[0][b] == 0ull) continue;
#pragma unroll
      for (int c = 0; c < NC; ++c) atomicAdd(&acc[(size_t)c * NT + s0 + c0 + b], bacc[c][b]);
    }
    __syncthreads();
  }
  if (sat) atomicOr((unsigned long long *)&meta[META_ERR], (unsigned long long)ERR_FIXED_SAT);
}

// Weighted member sums of every bin for targets with kept (non-uniform)
// weights: sum w, sum w (x - pixel) per position axis, sum w v, sum w I, with
// w = exp(log-weight - the largest log-weight in the bin), so the bin's
// largest member has w = 1 however small the bin's share of the target's
// weight. wacc [2 + D][NT]: rows 0..D the sums (FP64 atomics), row D + 1 the
// bin's largest log-weight as ordered bits (atomic max). One thread per
// particle over the propagate tiles; the rows are cleared first.
__global__ __launch_bounds__(TPB) void k_wsum_clear(uint32_t NT, int D, const uint64_t *__restrict__ meta,
                                                    double *__restrict__ wacc) {
  const uint32_t B = (uint32_t)meta[META_B];
  for (uint32_t i = blockIdx.x * TPB + threadIdx.x; i < B; i += gridDim.x * TPB)
    for (int c = 0; c <= D + 1; ++c) wacc[(size_t)c * NT + i] = 0.0;  // row D + 1: below every ordered value
}

__global__ __launch_bounds__(TPB) void k_bin_wmax(Params p, const Tile *__restrict__ tiles,
                                                  const uint32_t *__restrict__ off, const uint32_t *__restrict__ segid,
                                                  const double *__restrict__ lw, const int32_t *__restrict__ tuni,
                                                  double *__restrict__ wacc) {
  const Tile tl = tiles[blockIdx.x];
  if (tuni[tl.t]) return;
  const uint32_t base = tl.base;
  const uint32_t i = tl.i0 + threadIdx.x;
  if (i >= tl.n) return;
  unsigned long long *mx = (unsigned long long *)(wacc + (size_t)(1 + p.D) * p.NT);
  atomicMax(&mx[segid[base + i]], ordered_bits(lw[base + i]));
}

template <int DIM>
__global__ __launch_bounds__(TPB) void k_bin_wsums(Params p, const Tile *__restrict__ tiles,
                                                   const uint32_t *__restrict__ off, const float *__restrict__ s,
                                                   const uint32_t *__restrict__ segid, const double *__restrict__ lw,
                                                   const int32_t *__restrict__ tuni, double *__restrict__ wacc) {
  constexpr int D = 2 * DIM + 1;
  const Tile tl = tiles[blockIdx.x];
  const int t = tl.t;
  if (tuni[t]) return;
  const uint32_t base = tl.base;
  const uint32_t i = tl.i0 + threadIdx.x;
  if (i >= tl.n) return;
  const uint32_t g = base + i, NT = p.NT;
  const uint32_t b = segid[g];
  const unsigned long long *mx = (const unsigned long long *)(wacc + (size_t)(1 + D) * NT);
  const double w = exp(lw[g] - from_ordered_bits(mx[b]));
  atomicAdd(&wacc[b], w);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const float x = s[(size_t)a * NT + g];
    atomicAdd(&wacc[(size_t)(1 + a) * NT + b], w * (double)(x - (float)cell_index(x, 1)));  // x - pixel exact
  }
#pragma unroll
  for (int d = DIM; d < D; ++d) atomicAdd(&wacc[(size_t)(1 + d) * NT + b], w * (double)s[(size_t)d * NT + g]);
}

__global__ __launch_bounds__(TPB) void k_copy_i32(int32_t *__restrict__ dst, const int32_t *__restrict__ src,
                                                  uint32_t n) {
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
__global__ __launch_bounds__(TPB) void k_fill_i32(int32_t *__restrict__ dst, int32_t v, uint32_t n) {
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i < n) dst[i] = v;
}

// Dummy particle of every bin: mean of the members (CoM) or the cell centre
// (CoC) for the positions, mean of the other components. Positions are kept
// as (pixel of the cell, offset from it) so the likelihood never subtracts
// large coordinates. Also marks the first bin of every target.
template <int DIM>
__global__ void k_dummy(Params p, const uint64_t *__restrict__ meta, const unsigned long long *__restrict__ acc,
                        const uint32_t *__restrict__ seg_key, const int32_t *__restrict__ seg_t,
                        const uint32_t *__restrict__ kbase, const int32_t *__restrict__ bbox_cur,
                        int32_t *__restrict__ dpix, float *__restrict__ doff, float *__restrict__ dint,
                        float *__restrict__ dlo, float *__restrict__ dvel, const double *__restrict__ wacc,
                        const int32_t *__restrict__ tuni) {
  const uint32_t B = (uint32_t)meta[META_B];
  const uint32_t NT = p.NT;
  for (uint32_t sidx = blockIdx.x * blockDim.x + threadIdx.x; sidx < B; sidx += gridDim.x * blockDim.x) {
    int t;
    int32_t cell[3];
    decode_key<DIM>(seg_key[sidx], p.T, kbase, bbox_cur, t, cell);
    const double n = (double)(long long)acc[sidx];
    // kept (non-uniform) weights: the members' centre of mass weighted by them
    const bool wt = wacc && !tuni[t] && wacc[sidx] > 0.0;
    const double wsum = wt ? wacc[sidx] : 1.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const int32_t ma = p.tm[t * 3 + a];
      const int32_t c0 = floor_div(cell[a], ma);
      dpix[(size_t)a * NT + sidx] = c0;
      double off;
      if (p.dummy_mode == 1) {
        const int32_t r = cell[a] - c0 * ma;  // cell within its pixel, 0..m-1
        off = ((double)r + 0.5) / (double)ma - 0.5;
      } else if (wt) {
        off = wacc[(size_t)(1 + a) * NT + sidx] / wsum;
      } else {
        off = (double)(long long)acc[(size_t)(1 + a) * NT + sidx] / (double)FX_POS / n;
      }
      // the offset as a pair of binary32 words (hi + lo)
      const float oh = (float)off;
      doff[(size_t)a * NT + sidx] = oh;
      dlo[(size_t)a * NT + sidx] = (float)(off - (double)oh);
    }
    const double in0 = wt ? wacc[(size_t)(1 + 2 * DIM) * NT + sidx] / wsum
                          : (double)(long long)acc[(size_t)(1 + 2 * DIM) * NT + sidx] / (double)FX_INT / n;
    const float ih = (float)in0;
    dint[sidx] = ih;
    dlo[(size_t)DIM * NT + sidx] = (float)(in0 - (double)ih);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      dvel[(size_t)a * NT + sidx] =
          wt ? (float)(wacc[(size_t)(1 + DIM + a) * NT + sidx] / wsum)
             : (float)((double)(long long)acc[(size_t)(1 + DIM + a) * NT + sidx] / (double)FX_VEL / n);
  }
}

// ---------------------------------------------------------------- likelihood
// Eq. likelihood with the model image of Eq. object: one wave64 per
// evaluation, lanes over the P x P window; each pixel's model value is the
// PSF averaged over q x q midpoint sub-samples. DIRECT evaluates one exp2
// per sub-sample; SEPARABLE uses g(x, y) = g_x(x) g_y(y) (2 P q exp2 per
// evaluation, then one product per pixel through lane shuffles). The sum of
// squares is reduced with compensated (TwoSum) arithmetic.
struct LikInput {
  // pcSIR: dummies; SIR: particles
  const int32_t *dpix;  // [dim][E] pixel of the cell (pcSIR)
  const float *doff;    // [dim][E] offset from it (pcSIR)
  const float *dint;    // [E] intensity (pcSIR)
  const float *dlo;     // [dim + 1][E] low words of the offsets and of the intensity (pcSIR):
                        // the dummy's mean is offset + low word, intensity + low word
  const int32_t *seg_t; // [E] target (pcSIR)
  const float *state;   // SoA state (SIR)
  const uint32_t *off;  // [T+1] (SIR)
};

// 2^(-a) for a >= 0 in binary32 with unbiased rounding: a = n - f with n the
// nearest integer and f in [-1/2, 1/2] (exact), 2^f from a degree-6
// polynomial fitted to the relative error (csrc/fit_exp2.py; 3.6e-9 before
// rounding), then an exact scaling by 2^-n. Max error 0.75 ulp, mean error
// ~0. The hardware exp2 instruction is not used here: its error, about one ulp
// of consistent sign, adds up over the P^2 q^2 sub-samples of a window into a
// relative error of the sum of squares of a few 1e-7.
__device__ __forceinline__ float exp2_neg(float a) {
  a = fminf(a, 200.0f);
  const float n = rintf(a);
  const float f = n - a;
  float r = 0.00015238006f;
  r = fmaf(r, f, 0.0013391137f);
  r = fmaf(r, f, 0.009618841f);
  r = fmaf(r, f, 0.055503592f);
  r = fmaf(r, f, 0.24022645f);
  r = fmaf(r, f, 0.6931472f);
  r = fmaf(r, f, 1.0f);
  return ldexpf(r, -(int)n);
}

// Exponent scale of exp(-u^2 / 2 s^2) = exp2(-u^2 k), k = log2(e) / (2 s^2), per
// axis. k is formed in FP64 once per evaluation and applied as an FP32 pair
// (hi + lo): a single rounded FP32 k would bias every sub-sample of the
// window the same way and the bias would add up over the P^2 q^2 terms.
struct ExpScale {
  float xh, xl, yh, yl;
};
__device__ __forceinline__ ExpScale psf_scale(const Params &p, double zpos) {
  const double LOG2E = 1.4426950408889634074;
  const double s0 = (double)p.sigma_psf;
  double sx2 = s0 * s0, sy2 = s0 * s0;
  if (p.psf == 1) {
    const double ax = (zpos - (double)p.astig_gamma) / (double)p.astig_d;
    const double ay = (zpos + (double)p.astig_gamma) / (double)p.astig_d;
    sx2 *= 1.0 + ax * ax;
    sy2 *= 1.0 + ay * ay;
  }
  const double kx = LOG2E / (2.0 * sx2), ky = LOG2E / (2.0 * sy2);
  ExpScale e;
  e.xh = (float)kx;
  e.xl = (float)(kx - (double)e.xh);
  e.yh = (float)ky;
  e.yl = (float)(ky - (double)e.yh);
  return e;
}
__device__ __forceinline__ float scaled_sq(float u, float kh, float kl) {
  const float uu = u * u;
  return fmaf(uu, kl, uu * kh);
}
// Sub-sample offset within a pixel: (a + 1/2)/q - 1/2 = (2a + 1 - q) / (2q).
__device__ __forceinline__ float sub_offset(int a, int q) { return (float)(2 * a + 1 - q) / (float)(2 * q); }

// ---------------------------------------------------------------- FP32 pairs
// The separable likelihood carries the model image in unevaluated FP32 pairs
// (hi + lo, about 48 significant bits). A model value rounded to one FP32
// word errs by up to 6e-8 of itself; where a window holds residuals of tens
// of counts (a neighbouring spot the model lacks), that rounding alone moves
// the log-likelihood by about 1e-5, the size of the whole weight tolerance.
// The build disables implicit multiply-add contraction, so each operation
// below rounds where it is written.

// a + b = s + e exactly (Knuth's TwoSum; no condition on the operands).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
// a + b = s + e exactly when |a| >= |b| or a = 0 (Dekker's Fast2Sum).
__device__ __forceinline__ void fast_two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  e = b - (s - a);
}
// (sh, sl) += (eh, el), the sum kept as a pair.
__device__ __forceinline__ void pair_acc(float &sh, float &sl, float eh, float el) {
  float s, e;
  two_sum(sh, eh, s, e);
  sh = s;
  sl += e + el;
}
// (ah, al) (bh, bl) as a pair (al bl dropped: below 2^-46 of the product).
__device__ __forceinline__ void pair_mul(float ah, float al, float bh, float bl, float &ph, float &pl) {
  ph = ah * bh;
  float e = fmaf(ah, bh, -ph);  // ah bh = ph + e exactly
  e = fmaf(ah, bl, e);
  pl = fmaf(al, bh, e);
}

// 2^(j/64) for j = -32..32 as FP32 pairs: one LDS table per block.
constexpr int EXP2_TBL = 65;
__device__ __forceinline__ void exp2_table_fill(float2 *tbl) {
  for (int j = threadIdx.x; j < EXP2_TBL; j += blockDim.x) {
    const double v = exp2((double)(j - 32) / 64.0);
    const float h = (float)v;
    tbl[j] = make_float2(h, (float)(v - (double)h));
  }
}

// 2^-(ah + al) as a pair (rh, rl), for ah >= 0 and |al| <= 2^-20 ah (a pair
// exponent). With n the integer nearest ah, f = n - ah is exact and
// |f| <= 1/2; f = j/64 + t with integer j and |t| <= 1/128, again exact.
// Then 2^(t - al) = e^y = 1 + p, y = (t - al) ln 2 (|y| < 0.0055), with p from
// the Taylor series to degree 4 (remainder below 4e-14 of the result) and y
// formed as a pair; 2^(j/64) comes from the table; the scaling by 2^-n is
// exact. Relative error about 6e-10 (the rounding of the table product).
__device__ __forceinline__ void exp2_neg_pair(float ah, float al, const float2 *tbl, float &rh, float &rl) {
  constexpr float LN2_HI = 0.693147182464599609375f;  // ln 2 rounded to binary32
  constexpr float LN2_LO = (float)(0.69314718055994530942 - 0.693147182464599609375);
  ah = fminf(ah, 200.0f);
  const float n = rintf(ah);
  const float f = n - ah;
  const float j = rintf(f * 64.0f);
  const float t = (f - j * 0.015625f) - al;
  const float yh = t * LN2_HI;
  const float yl = fmaf(t, LN2_HI, -yh) + t * LN2_LO;
  float c = fmaf(yh, 1.0f / 24.0f, 1.0f / 6.0f);
  c = fmaf(yh, c, 0.5f);
  const float qd = (yh * yh) * c;          // y^2/2 + y^3/6 + y^4/24
  const float ph = yh + (yl + qd);
  const float pl = ((yh - ph) + yl) + qd;  // yh - ph is exact
  const float2 tb = tbl[(int)j + 32];
  const float s = fmaf(tb.x, ph, fmaf(tb.x, pl, tb.y));
  float h, l;
  fast_two_sum(tb.x, s, h, l);
  const int e = -(int)n;
  rh = ldexpf(h, e);
  rl = ldexpf(l, e);
}

// exp(-(U - d)^2 / (2 s^2)) = 2^-(k (U - d)^2) as a pair, for an exact
// sub-sample position U, a pair offset d = dh + dl and a pair scale k = kh + kl.
__device__ __forceinline__ void psf_factor_pair(float U, float dh, float dl, float kh, float kl, const float2 *tbl,
                                                float &eh, float &el) {
  float uh, ue;
  two_sum(U, -dh, uh, ue);
  const float ul = ue - dl;           // U - d = uh + ul
  const float sh = uh * uh;
  float sl = fmaf(uh, uh, -sh);
  sl = fmaf(2.0f * uh, ul, sl);       // (U - d)^2 = sh + sl
  const float ah = sh * kh;
  float al = fmaf(sh, kh, -ah);
  al = fmaf(sh, kl, al);
  al = fmaf(sl, kh, al);              // k (U - d)^2 = ah + al
  exp2_neg_pair(ah, al, tbl, eh, el);
}

// The ratio of consecutive factors along an axis: 2^-(k ((U + delta - d)^2 -
// (U - d)^2)) = 2^-(k (2 delta (U - d) + delta^2)) as a pair, for a power of
// two delta (so that 2 delta (U - d) and delta^2 are exact scalings). Then
// e(U + delta) = e(U) r(U) and r(U + delta) = r(U) c, c = 2^-(2 k delta^2),
// which turns all but the first two exp2 of a lane's sub-samples into pair
// products.
__device__ __forceinline__ void psf_ratio_pair(float U, float dh, float dl, float kh, float kl, float delta,
                                               const float2 *tbl, float &rh, float &rl) {
  float uh, ue;
  two_sum(U, -dh, uh, ue);
  const float ul = ue - dl;  // U - d = uh + ul
  const float tw = 2.0f * delta;
  float th, tl;
  two_sum(tw * uh, delta * delta, th, tl);
  tl = fmaf(tw, ul, tl);     // 2 delta (U - d) + delta^2 = th + tl
  const float ah = th * kh;
  float al = fmaf(th, kh, -ah);
  al = fmaf(th, kl, al);
  al = fmaf(tl, kh, al);
  exp2_neg_pair(ah, al, tbl, rh, rl);
}

// Evaluation sets of k_lik: every dummy / particle; the dummies picked for
// the surrogate's exact check (list, see k_surr_pick); the dummies of targets
// whose check failed (list, see k_surr_fallback_list).
// LIK_STENCIL: second-order dummies; entry 9 b + s evaluates dummy b at the
// position shifted by (s % 3 - 1, s / 3 - 1) half cells, in the dummy's
// window, into ll[s NT + b].
enum { LIK_ALL = 0, LIK_CHECK = 1, LIK_FALLBACK = 2, LIK_STENCIL = 3 };
struct SurrCheck {
  float fraction;            // share of dummies checked per frame
  float tol;                 // largest accepted |l_surrogate - l_exact| (nats)
  int32_t *tfallback;        // [T] per-target fallback flag of this frame
  const uint32_t *list;      // dummies to evaluate (CHECK / FALLBACK)
  const unsigned long long *tmax;  // [T] largest surrogate l of each target (ordered bits)
  float *err;                // CHECK: |l_surrogate - l_exact| of list entry i
  unsigned long long *tsse;  // [T] squared errors of relevant checked dummies, fixed point 2^16
  unsigned int *tcnt;        // [T] number of relevant checked dummies
};
constexpr double SSE_FX = 65536.0;      // fixed-point scale of the squared errors (nats^2)
constexpr double SSE_CLAMP = 1.0e9;     // a squared error counts at most this much
// A checked dummy counts only when its exact or surrogate log-likelihood is
// within this many nats of its target's largest surrogate value: below, its
// weight relative to the target's best dummy is under e^-40 whatever the error.
constexpr double SURR_RELEVANT_NATS = 40.0;

// A dummy is checked when the uniform of counter (dummy, k, target, 3) is
// below the check fraction.
__device__ __forceinline__ bool surr_checked(uint64_t seed, uint32_t e, int64_t k, int t, float fraction) {
  const U32x4 b = philox4x32_10(e, (uint32_t)k, (uint32_t)t, 3u, seed_lo(seed), seed_hi(seed));
  return u01_53(b.v[0], b.v[1]) < (double)fraction;
}

// Appends of a block to a global list, staged in LDS: lanes that take an
// element add it to the block's buffer (one LDS atomic per wave), and the
// buffer goes to the list with one global atomic per flush: when a further
// round could overflow it, and at the end. A single counter that every wave
// incremented serialised thousands of same-address atomics per frame.
constexpr int LIST_CAP = 2048;
struct ListStage {
  uint32_t buf[LIST_CAP];
  uint32_t n, base;
};
__device__ __forceinline__ void stage_append(ListStage &ls, bool take, uint32_t e) {
  const unsigned long long m = __ballot(take);
  if (m == 0ull) return;
  const int lane = lane_id();
  const int first = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == first) base = atomicAdd(&ls.n, (uint32_t)__popcll(m));
  base = __shfl(base, first, WAVE);
  if (take) ls.buf[base + __popcll(m & ((1ull << lane) - 1ull))] = e;
}
// Called by every thread of the block after a barrier; flushes when the
// buffer holds more than `keep` entries (keep = 0: whatever it holds).
__device__ __forceinline__ void stage_flush(ListStage &ls, uint32_t keep, uint32_t *__restrict__ list,
                                            uint64_t *__restrict__ count) {
  const uint32_t n = ls.n;
  if (n == 0 || n <= keep) return;
  if (threadIdx.x == 0) ls.base = (uint32_t)atomicAdd((unsigned long long *)count, (unsigned long long)n);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) list[ls.base + i] = ls.buf[i];
  __syncthreads();
  if (threadIdx.x == 0) ls.n = 0;
  __syncthreads();
}

// Dummies picked for this frame's exact check (grid-stride over the dummies;
// the list's order depends on the order of the blocks' flushes, and every use
// of it is independent of that order).
__global__ __launch_bounds__(TPB) void k_surr_pick(Params p, const uint64_t *__restrict__ meta,
                                                   const StepDesc *__restrict__ desc,
                                                   const int32_t *__restrict__ seg_t, float fraction,
                                                   uint32_t *__restrict__ list, uint64_t *__restrict__ count) {
  __shared__ ListStage ls;
  if (threadIdx.x == 0) ls.n = 0;
  __syncthreads();
  const uint32_t B = (uint32_t)meta[META_B];
  const int64_t k = desc->k;
  for (uint32_t e0 = blockIdx.x * TPB; e0 < B; e0 += gridDim.x * TPB) {
    const uint32_t e = e0 + threadIdx.x;
    const bool take = e < B && surr_checked(p.seed, e, k, seg_t[e], fraction);
    stage_append(ls, take, e);
    __syncthreads();
    stage_flush(ls, LIST_CAP - TPB, list, count);
  }
  __syncthreads();
  stage_flush(ls, 0, list, count);
}
__global__ __launch_bounds__(TPB) void k_clear_u64(unsigned long long *__restrict__ a, uint32_t n) {
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i < n) a[i] = 0ull;
}

// Check statistics of the frame: dummies checked, largest error (one block).
__global__ __launch_bounds__(TPB) void k_surr_stats(const float *__restrict__ err, uint64_t *__restrict__ meta) {
  __shared__ float lds[TPB / WAVE];
  const uint32_t n = (uint32_t)meta[META_NCHK];
  float mx = 0.0f;
  for (uint32_t i = threadIdx.x; i < n; i += TPB) mx = fmaxf(mx, err[i]);
  mx = block_max<TPB, float>(mx, lds);
  if (threadIdx.x == 0) {
    meta[META_CHECKED] += n;
    const uint64_t b = (uint64_t)__float_as_uint(mx);
    if (b > meta[META_MAXERR]) meta[META_MAXERR] = b;
  }
}

// Per-target decision after the check: fall back when the mean squared
// error of the target's relevant checked dummies exceeds tol^2; the sums are
// cleared for the next frame.
__global__ __launch_bounds__(TPB) void k_surr_decide(int T, float tol, unsigned long long *__restrict__ tsse,
                                                     unsigned int *__restrict__ tcnt, int32_t *__restrict__ tfallback) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= T) return;
  const unsigned int n = tcnt[t];
  const double mse = n ? (double)tsse[t] / SSE_FX / (double)n : 0.0;
  tfallback[t] = n && !(mse <= (double)tol * (double)tol) ? 1 : 0;
  tsse[t] = 0ull;
  tcnt[t] = 0u;
}

// Dummies of the targets whose check failed.
__global__ __launch_bounds__(TPB) void k_surr_fallback_list(const uint64_t *__restrict__ meta,
                                                            const int32_t *__restrict__ seg_t,
                                                            const int32_t *__restrict__ tfallback,
                                                            uint32_t *__restrict__ list, uint64_t *__restrict__ count) {
  __shared__ ListStage ls;
  if (threadIdx.x == 0) ls.n = 0;
  __syncthreads();
  const uint32_t B = (uint32_t)meta[META_B];
  for (uint32_t e0 = blockIdx.x * TPB; e0 < B; e0 += gridDim.x * TPB) {
    const uint32_t e = e0 + threadIdx.x;
    const bool take = e < B && tfallback[seg_t[e]] != 0;
    stage_append(ls, take, e);
    __syncthreads();
    stage_flush(ls, LIST_CAP - TPB, list, count);
  }
  __syncthreads();
  stage_flush(ls, 0, list, count);
}

template <int DIM, typename T>
__device__ __forceinline__ T lik_uniform(T v) {
  return DIM == 2 ? wave_uniform(v) : v;
}

// 2D: five waves per SIMD fit in the vector registers without spills (3D
// would spill)
// PP: the window side when known at compile time (0: p.P), so that the pixel
// rounds and the per-axis sub-sample loops have constant trip counts.
template <int DIM, bool SIR, bool SEP, int Q, int MODE = LIK_ALL, int PP = 0>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(DIM == 2 ? 5 : 1))) void k_lik(Params p, LikInput in, const uint64_t *__restrict__ meta,
                                             const StepDesc *__restrict__ desc, double *__restrict__ ll,
                                             SurrCheck chk = SurrCheck{0.0f, 0.0f, nullptr, nullptr, nullptr, nullptr,
                                                                       nullptr, nullptr},
                                             uint64_t *__restrict__ stats = nullptr) {
  const float *__restrict__ frame = desc->frame;
  const uint32_t E = SIR ? p.NT
                         : (uint32_t)meta[MODE == LIK_CHECK ? META_NCHK : (MODE == LIK_FALLBACK ? META_NFB : META_B)] *
                               (MODE == LIK_STENCIL ? 9u : 1u);
  const int lane = lane_id();
  const int P = PP ? PP : p.P, R = PP ? (PP - 1) / 2 : p.R, P2 = P * P;
  const int q = Q ? Q : p.q;
  const ExpScale ks_flat = psf_scale(p, 0.0);  // the scale of a z-independent PSF, formed once
  // window column and row of this lane's pixel in round 0; each round of 64
  // pixels then advances them by (64 mod P, 64 div P) with one wrap, instead
  // of an integer division per round
  const int pc_first = lane % P, pr_first = lane / P;
  const int dpc = WAVE % P, dpr = WAVE / P;
  // sub-sample offsets (a + 1/2) / q - 1/2, a < q, formed once per block, and
  // (SEPARABLE) the table of the pair exponential
  __shared__ float soff[MAX_QUAD];
  __shared__ float2 e2tbl[SEP ? EXP2_TBL : 1];
  // SEPARABLE with H >= 1, 2D: each wave's per-axis sums (x scaled by the
  // intensity), read by the pixels as one 8-byte LDS load per axis (in 3D,
  // where every evaluation forms its own PSF scale, shuffles measured faster)
  constexpr bool FAC = SEP && DIM == 2;
  __shared__ float2 fac[FAC ? LIK_WAVES : 1][FAC ? WAVE : 1];
  if (threadIdx.x < MAX_QUAD) soff[threadIdx.x] = (int)threadIdx.x < q ? sub_offset((int)threadIdx.x, q) : 0.0f;
  if (SEP) exp2_table_fill(e2tbl);
  __syncthreads();
  // SEPARABLE with H = 64 / (2P) >= 1 lanes per per-axis sum: this lane's
  // (axis, pixel, first sub-sample), fixed for the launch
  const int H = WAVE / (2 * P);
  const bool s_on = H >= 1 && lane < 2 * P * H;
  const int s_axis = s_on ? lane / (P * H) : 0;
  const int s_rem = lane - s_axis * P * H;
  const int s_pixel = H >= 1 ? s_rem / H : 0;
  const int s_part = s_rem - s_pixel * H;
  const float s_cc = (float)(s_pixel - R);
  const float inv_q2 = 1.0f / (float)(q * q);
  // with a PSF scale that is the same for every evaluation and q and H powers
  // of two, a lane's sub-samples (H / q apart) take the product recurrence of
  // psf_ratio_pair after the first; c of the lane's axis is formed once
  const bool s_rec = SEP && H >= 1 && (H & (H - 1)) == 0 && (DIM == 2 || p.psf != 1) && (q & (q - 1)) == 0 && q > H;
  const float s_delta = (float)H / (float)q;
  float s_ch = 0.0f, s_cl = 0.0f;
  if (s_rec) {
    const float c2 = 2.0f * s_delta * s_delta;  // exact: delta is a power of two
    const float kh = s_axis ? ks_flat.yh : ks_flat.xh, kl = s_axis ? ks_flat.yl : ks_flat.xl;
    const float ah = c2 * kh;
    exp2_neg_pair(ah, fmaf(c2, kh, -ah) + c2 * kl, e2tbl, s_ch, s_cl);
  }
  // one evaluation per wave: in 2D its values are moved to scalar registers
  // once loaded (in 3D the compiler then turned their loads into scalar-cache
  // loads and spilled scalar registers, which measured slower)
  const uint32_t idx0 = blockIdx.x * LIK_WAVES + wave_id();
  for (uint32_t idx = DIM == 2 ? __builtin_amdgcn_readfirstlane(idx0) : idx0; idx < E; idx += gridDim.x * LIK_WAVES) {
    const uint32_t e = MODE == LIK_ALL ? idx : (MODE == LIK_STENCIL ? idx / 9u : chk.list[idx]);
    int t;
    int32_t c0, r0;
    // dummy / particle: offsets from the window's centre pixel and intensity,
    // each as a pair (hi + lo); a particle's are exact in one word
    float dx, dy, I0, dxl = 0.0f, dyl = 0.0f, I0l = 0.0f;
    double zpos = 0.0;
    if (SIR) {
      int lo = 0, hi = p.T - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (in.off[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      t = lo;
      const float x = in.state[e];
      const float y = in.state[(size_t)p.NT + e];
      c0 = cell_index(x, 1);
      r0 = cell_index(y, 1);
      dx = x - (float)c0;  // exact
      dy = y - (float)r0;
      if (DIM == 3) zpos = (double)in.state[(size_t)2 * p.NT + e];
      I0 = in.state[(size_t)(2 * DIM) * p.NT + e];
    } else {
      // wave-uniform values, held in scalar registers (2D)
      t = lik_uniform<DIM>(in.seg_t[e]);
      c0 = lik_uniform<DIM>(in.dpix[e]);
      r0 = lik_uniform<DIM>(in.dpix[(size_t)p.NT + e]);
      dx = lik_uniform<DIM>(in.doff[e]);
      dy = lik_uniform<DIM>(in.doff[(size_t)p.NT + e]);
      dxl = lik_uniform<DIM>(in.dlo[e]);
      dyl = lik_uniform<DIM>(in.dlo[(size_t)p.NT + e]);
      if (DIM == 3)
        zpos = (double)in.dpix[(size_t)2 * p.NT + e] + (double)in.doff[(size_t)2 * p.NT + e] +
               (double)in.dlo[(size_t)2 * p.NT + e];
      I0 = lik_uniform<DIM>(in.dint[e]);
      I0l = lik_uniform<DIM>(in.dlo[(size_t)DIM * p.NT + e]);
      if (MODE == LIK_STENCIL) {
        // the shifted position, formed in binary64 and split into a pair
        const int sidx = (int)(idx - 9u * e);
        const double sx = (double)dx + (double)dxl + (double)(sidx % 3 - 1) * (0.5 / (double)p.tm[t * 3 + 0]);
        const double sy = (double)dy + (double)dyl + (double)(sidx / 3 - 1) * (0.5 / (double)p.tm[t * 3 + 1]);
        dx = (float)sx;
        dxl = (float)(sx - (double)dx);
        dy = (float)sy;
        dyl = (float)(sy - (double)dy);
      }
    }
    const ExpScale ks = (DIM == 3 && p.psf == 1) ? psf_scale(p, zpos) : ks_flat;
    const gfloat *fr = as_global(frame) + (p.per_target_frames ? (size_t)t * p.H * p.W : 0);
    // window pixels of the first ZPRE rounds loaded before the model is
    // formed, so that their latency overlaps it: clamped coordinates, and a
    // 0 / 1 factor instead of a select, so that every value is used and no
    // load is moved under a branch that waits for it (pixel values are
    // finite, so a masked pixel is +-0, which acts as 0 below)
    constexpr int ZPRE = 4;
    float zpre[ZPRE];
    {
      int pc = pc_first, pr = pr_first;
#pragma unroll
      for (int it = 0; it < ZPRE; ++it) {
        const int pix = it * WAVE + lane;
        const int c = c0 + pc - R, r = r0 + pr - R;
        const float v = fr[(size_t)min(max(r, 0), p.H - 1) * p.W + min(max(c, 0), p.W - 1)];
        zpre[it] = v * ((pix < P2 && c >= 0 && c < p.W && r >= 0 && r < p.H) ? 1.0f : 0.0f);
        pc += dpc;
        pr += dpr;
        if (pc >= P) {
          pc -= P;
          ++pr;
        }
      }
    }
    float ssd = 0.0f, err = 0.0f;
    if (SEP) {
      // Per-axis sums g_x(c) = sum_a exp(-(c + o_a - x)^2 / 2 s_x^2) (and g_y) as
      // pairs. With H = 64 / (2P) >= 1 they are spread over the wave, H lanes per
      // sum, each adding every H-th sub-sample; the sum of (axis, pixel c) ends
      // up in lane (axis P + c) H. With 2P > 64, lane j forms both axes' sums of
      // pixel j and, for P > 64, of pixel j + 64. The x sums are then scaled by
      // the intensity per sub-sample, A(c) = I0 g_x(c) / q^2, so that the model
      // value of pixel (c, r) is one pair product A(c) g_y(r).
      float Iqh = I0 * inv_q2;
      float Iql = (fmaf(-Iqh, (float)(q * q), I0) + I0l) * inv_q2;  // I0 - Iqh q^2 is exact
      if ((q & (q - 1)) == 0) Iql = I0l * inv_q2;                     // q^2 a power of two: Iqh exact
      float ah = 0.0f, al = 0.0f, bh = 0.0f, bl = 0.0f;  // H >= 1: (ah, al); else x (a) and y (b) of pixel lane
      float ch = 0.0f, cl = 0.0f, eh = 0.0f, el = 0.0f;  // P > 64: x (c) and y (e) of pixel lane + 64
      if (H >= 1) {
        if (s_on) {
          const float d = s_axis ? dy : dx, dl = s_axis ? dyl : dxl;
          const float kh = s_axis ? ks.yh : ks.xh, kl = s_axis ? ks.yl : ks.xl;
          if (s_rec) {
            float vh, vl, rh, rl;
            psf_factor_pair(s_cc + soff[s_part], d, dl, kh, kl, e2tbl, vh, vl);
            psf_ratio_pair(s_cc + soff[s_part], d, dl, kh, kl, s_delta, e2tbl, rh, rl);
            pair_acc(ah, al, vh, vl);
            for (int a = s_part + H; a < q; a += H) {
              float th, tl;
              pair_mul(vh, vl, rh, rl, th, tl);
              vh = th;
              vl = tl;
              pair_acc(ah, al, vh, vl);
              pair_mul(rh, rl, s_ch, s_cl, th, tl);
              rh = th;
              rl = tl;
            }
          } else {
            for (int a = s_part; a < q; a += H) {
              float vh, vl;
              psf_factor_pair(s_cc + soff[a], d, dl, kh, kl, e2tbl, vh, vl);
              pair_acc(ah, al, vh, vl);
            }
          }
        }
        float th = ah, tl = al;
        if (H == 2) {
          // the sum's other lane is lane ^ 1 (only the even lane's total is read)
          pair_acc(th, tl, dpp_move<DPP_QUAD_XOR1>(ah), dpp_move<DPP_QUAD_XOR1>(al));
        } else {
          for (int h = 1; h < H; ++h) {
            const int src = (lane + h) & (WAVE - 1);
            pair_acc(th, tl, __shfl(ah, src, WAVE), __shfl(al, src, WAVE));
          }
        }
        if (s_axis == 0) pair_mul(Iqh, Iql, th, tl, ah, al);
        else {
          ah = th;
          al = tl;
        }
        if (FAC) {
          if (s_on && s_part == 0) fac[FAC ? wave_id() : 0][s_axis * P + s_pixel] = make_float2(ah, al);
          // the wave's own LDS writes before its reads of other lanes' entries
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      } else {
        if (lane < P) {
          const float cc = (float)(lane - R);
          for (int a = 0; a < q; ++a) {
            float vh, vl;
            psf_factor_pair(cc + soff[a], dx, dxl, ks.xh, ks.xl, e2tbl, vh, vl);
            pair_acc(ah, al, vh, vl);
            psf_factor_pair(cc + soff[a], dy, dyl, ks.yh, ks.yl, e2tbl, vh, vl);
            pair_acc(bh, bl, vh, vl);
          }
          float th, tl;
          pair_mul(Iqh, Iql, ah, al, th, tl);
          ah = th;
          al = tl;
        }
        if (lane + WAVE < P) {
          const float cc = (float)(lane + WAVE - R);
          for (int a = 0; a < q; ++a) {
            float vh, vl;
            psf_factor_pair(cc + soff[a], dx, dxl, ks.xh, ks.xl, e2tbl, vh, vl);
            pair_acc(ch, cl, vh, vl);
            psf_factor_pair(cc + soff[a], dy, dyl, ks.yh, ks.yl, e2tbl, vh, vl);
            pair_acc(eh, el, vh, vl);
          }
          float th, tl;
          pair_mul(Iqh, Iql, ch, cl, th, tl);
          ch = th;
          cl = tl;
        }
      }
      int pc = pc_first, pr = pr_first;
      for (int pix0 = 0, it = 0; pix0 < P2; pix0 += WAVE, ++it) {
        const int pix = pix0 + lane;
        const int pcs = pc < P ? pc : 0, prs = pr < P ? pr : 0;
        float xh, xl, yh, yl;
        if (H >= 1 && FAC) {
          const float2 fx = fac[FAC ? wave_id() : 0][pcs], fy = fac[FAC ? wave_id() : 0][P + prs];
          xh = fx.x;
          xl = fx.y;
          yh = fy.x;
          yl = fy.y;
        } else if (H >= 1) {
          xh = __shfl(ah, pcs * H, WAVE);
          xl = __shfl(al, pcs * H, WAVE);
          yh = __shfl(ah, (P + prs) * H, WAVE);
          yl = __shfl(al, (P + prs) * H, WAVE);
        } else if (P <= WAVE) {
          xh = __shfl(ah, pcs, WAVE);
          xl = __shfl(al, pcs, WAVE);
          yh = __shfl(bh, prs, WAVE);
          yl = __shfl(bl, prs, WAVE);
        } else {
          // every lane takes part in all shuffles; each keeps the slot of its pixel
          const int sc = pcs & (WAVE - 1), sr = prs & (WAVE - 1);
          const float x0h = __shfl(ah, sc, WAVE), x0l = __shfl(al, sc, WAVE);
          const float x1h = __shfl(ch, sc, WAVE), x1l = __shfl(cl, sc, WAVE);
          const float y0h = __shfl(bh, sr, WAVE), y0l = __shfl(bl, sr, WAVE);
          const float y1h = __shfl(eh, sr, WAVE), y1l = __shfl(el, sr, WAVE);
          xh = pcs < WAVE ? x0h : x1h;
          xl = pcs < WAVE ? x0l : x1l;
          yh = prs < WAVE ? y0h : y1h;
          yl = prs < WAVE ? y0l : y1l;
        }
        if (pix < P2) {
          const int c = c0 + pc - R, r = r0 + pr - R;
          const bool inside = c >= 0 && c < p.W && r >= 0 && r < p.H;
          float z = 0.0f;
          if (it < ZPRE) {
#pragma unroll
            for (int u = 0; u < ZPRE; ++u)
              if (u == it) z = zpre[u];
          } else if (inside) {
            z = fr[(size_t)r * p.W + c];
          }
          // frame value minus background (a pixel outside the frame reads as the
          // background) and minus the model image, as pairs
          float zh = 0.0f, zl = 0.0f;
          if (inside) two_sum(z, -p.i_bg, zh, zl);
          float mh, ml;
          pair_mul(xh, xl, yh, yl, mh, ml);
          float dh, de;
          two_sum(zh, -mh, dh, de);
          const float dl = (de + zl) - ml;
          const float sq = dh * dh;
          float sqe = fmaf(dh, dh, -sq);
          sqe = fmaf(2.0f * dh, dl, sqe);  // d^2 = sq + sqe (+ dl^2)
          float s2, e2;
          two_sum(ssd, sq, s2, e2);
          ssd = s2;
          err += e2 + sqe;
        }
        pc += dpc;
        pr += dpr;
        if (pc >= P) {
          pc -= P;
          ++pr;
        }
      }
    } else {
      const float Iq = I0 / (float)(q * q);
      int pc = pc_first, pr = pr_first;
      for (int pix0 = 0, it = 0; pix0 < P2; pix0 += WAVE, ++it) {
        const int pix = pix0 + lane;
        if (pix < P2) {
          float g = 0.0f;
          const float cc = (float)(pc - R), rr = (float)(pr - R);
          if (Q) {
            float ax[Q > 0 ? Q : 1];
#pragma unroll
            for (int a = 0; a < Q; ++a) ax[a] = scaled_sq((cc + sub_offset(a, Q)) - dx, ks.xh, ks.xl);
#pragma unroll
            for (int b = 0; b < Q; ++b) {
              const float ay = scaled_sq((rr + sub_offset(b, Q)) - dy, ks.yh, ks.yl);
#pragma unroll
              for (int a = 0; a < Q; ++a) g += exp2_neg(ax[a] + ay);
            }
          } else {
            for (int b = 0; b < q; ++b) {
              const float ay = scaled_sq((rr + sub_offset(b, q)) - dy, ks.yh, ks.yl);
              for (int a = 0; a < q; ++a)
                g += exp2_neg(scaled_sq((cc + sub_offset(a, q)) - dx, ks.xh, ks.xl) + ay);
            }
          }
          const int c = c0 + pc - R, r = r0 + pr - R;
          // frame value minus background; a pixel outside the frame reads as the background
          const bool inside = c >= 0 && c < p.W && r >= 0 && r < p.H;
          float z = 0.0f;
          if (it < ZPRE) {
#pragma unroll
            for (int u = 0; u < ZPRE; ++u)
              if (u == it) z = zpre[u];
          } else if (inside) {
            z = fr[(size_t)r * p.W + c];
          }
          const float zb = inside ? z - p.i_bg : 0.0f;
          // residual d = zb - Iq g and its square as FP32 (hi, lo) pairs: a residual
          // of ~100 (a spot the model lacks) would otherwise lose 1e-5 of l per particle
          const float mg = Iq * g;
          const float mge = fmaf(Iq, g, -mg);          // Iq g = mg + mge exactly
          const float dh = zb - mg;
          const float bv = dh - zb;
          const float dl = ((zb - (dh - bv)) + (-mg - bv)) - mge;  // zb - mg = dh + (..) exactly
          const float sq = dh * dh;
          const float sqe = fmaf(dh, dh, -sq) + 2.0f * dh * dl;   // d^2 = sq + sqe (+ dl^2)
          const float tsum = ssd + sq;
          const float bp = tsum - ssd;
          err += ((ssd - (tsum - bp)) + (sq - bp)) + sqe;
          ssd = tsum;
        }
        pc += dpc;
        pr += dpr;
        if (pc >= P) {
          pc -= P;
          ++pr;
        }
      }
    }
    // compensated wave sum; the (hi, lo) result is combined and scaled in FP64,
    // the precision of the normalisation that consumes it
    double hi, lo;
    wave_sum_pair(ssd, err, hi, lo);
    const double lx = -(hi + lo) * p.inv2sxi2;
    if (MODE == LIK_CHECK && lane == 0) {
      const double ls = ll[e];
      const float d = (float)fabs(lx - ls);
      const double top = from_ordered_bits(chk.tmax[t]);
      const bool relevant = fmax(lx, ls) >= top - SURR_RELEVANT_NATS || !(top == top);
      if (relevant) {
        // integer sums: the per-target decision does not depend on the order of the atomics
        const double d2 = d == d ? fmin((double)d * (double)d, SSE_CLAMP) : SSE_CLAMP;
        atomicAdd(&chk.tsse[t], (unsigned long long)(d2 * SSE_FX));
        atomicAdd(&chk.tcnt[t], 1u);
      }
      chk.err[idx] = d != d ? INFINITY : d;
    }
    if (lane == 0) ll[MODE == LIK_STENCIL ? (size_t)(idx - 9u * e) * p.NT + e : (size_t)e] = lx;
  }
}

// Second-order dummies: each bin's log-likelihood from the nine stencil
// values (ll9[s][b], s = 3 (sy + 1) + (sx + 1) for shifts of half a cell)
// and the members' position covariance from the fixed-point bin sums:
// ell(mu) + tr(H S)/2 + g'S g/2 with central differences for g and H.
__global__ __launch_bounds__(TPB) void k_second_order(Params p, const uint64_t *__restrict__ meta,
                                                      const unsigned long long *__restrict__ acc,
                                                      const int32_t *__restrict__ seg_t,
                                                      const double *__restrict__ ll9, double *__restrict__ ll) {
  const uint32_t B = (uint32_t)meta[META_B];
  const uint32_t NT = p.NT;
  for (uint32_t b = blockIdx.x * TPB + threadIdx.x; b < B; b += gridDim.x * TPB) {
    const int t = seg_t[b];
    const double dx = 0.5 / (double)p.tm[t * 3 + 0], dy = 0.5 / (double)p.tm[t * 3 + 1];
    double l[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) l[s] = ll9[(size_t)s * NT + b];
    const double gx = (l[5] - l[3]) / (2.0 * dx), gy = (l[7] - l[1]) / (2.0 * dy);
    const double hxx = (l[5] - 2.0 * l[4] + l[3]) / (dx * dx), hyy = (l[7] - 2.0 * l[4] + l[1]) / (dy * dy);
    const double hxy = (l[8] - l[6] - l[2] + l[0]) / (4.0 * dx * dy);
    // covariance: second moments of x - pixel (scale 2^32) minus the square of the mean offset
    const double n = (double)(long long)acc[b];
    const double mx = (double)(long long)acc[(size_t)1 * NT + b] / (double)FX_POS / n;
    const double my = (double)(long long)acc[(size_t)2 * NT + b] / (double)FX_POS / n;
    const double sxx = (double)(long long)acc[(size_t)6 * NT + b] / (double)FX_SQ / n - mx * mx;
    const double syy = (double)(long long)acc[(size_t)7 * NT + b] / (double)FX_SQ / n - my * my;
    const double sxy = (double)(long long)acc[(size_t)8 * NT + b] / (double)FX_SQ / n - mx * my;
    ll[b] = l[4] + 0.5 * (hxx * sxx + hyy * syy + 2.0 * hxy * sxy) +
            0.5 * (gx * gx * sxx + gy * gy * syy + 2.0 * gx * gy * sxy);
  }
}

// ---------------------------------------------------------------- normalisation
// pcSIR, one block per target, at bin level: the members of bin b share its
// log-likelihood, so S = sum_b n_b e^{l_b - M}, sum w^2 = sum_b n_b w_b^2 and
// the posterior mean is sum_b w_b (sum of the members' states), with the
// members' sums taken exactly from the fixed-point bin sums. FP64.
template <int DIM>
__global__ __launch_bounds__(TPB) void k_norm_bins(Params p, const uint32_t *__restrict__ seg_first,
                                                   const double *__restrict__ ll, const unsigned long long *__restrict__ acc,
                                                   const int32_t *__restrict__ dpix, const StepDesc *__restrict__ desc,
                                                   double *__restrict__ wbin, double *__restrict__ tgt,
                                                   double *__restrict__ est, int32_t *__restrict__ tflag,
                                                   uint64_t *__restrict__ meta, const int32_t *__restrict__ tfallback) {
  constexpr int D = 2 * DIM + 1;
  __shared__ double lds[TPB / WAVE];
  const int t = blockIdx.x;
  const uint32_t s0 = seg_first[t], s1 = seg_first[t + 1];
  const uint32_t NT = p.NT;
  double mx = -INFINITY;
  for (uint32_t s = s0 + threadIdx.x; s < s1; s += TPB) mx = fmax(mx, ll[s]);
  const double M = block_max<TPB, double>(mx, lds);
  double S = 0.0, Q = 0.0, X[D];
#pragma unroll
  for (int d = 0; d < D; ++d) X[d] = 0.0;
  for (uint32_t s = s0 + threadIdx.x; s < s1; s += TPB) {
    const double n = (double)(long long)acc[s];
    const double e = exp(ll[s] - M);
    S += n * e;
    Q += n * e * e;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double sum = n * (double)dpix[(size_t)a * NT + s] +
                         (double)(long long)acc[(size_t)(1 + a) * NT + s] / (double)FX_POS;
      X[a] += e * sum;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) X[DIM + a] += e * ((double)(long long)acc[(size_t)(1 + DIM + a) * NT + s] / (double)FX_VEL);
    X[2 * DIM] += e * ((double)(long long)acc[(size_t)(1 + 2 * DIM) * NT + s] / (double)FX_INT);
  }
  S = block_sum<TPB, double>(S, lds);
  Q = block_sum<TPB, double>(Q, lds);
#pragma unroll
  for (int d = 0; d < D; ++d) X[d] = block_sum<TPB, double>(X[d], lds);
  const bool ok = isfinite(M) && isfinite(S) && S > 0.0;
  for (uint32_t s = s0 + threadIdx.x; s < s1; s += TPB) wbin[s] = ok ? exp(ll[s] - M) / S : 0.0;
  if (threadIdx.x == 0) {
    tgt[t * 4 + 0] = M;
    tgt[t * 4 + 1] = S;
    tgt[t * 4 + 2] = S * S / Q;
    tgt[t * 4 + 3] = resample_uniform(p.seed, (uint64_t)desc->k, (uint64_t)t);
#pragma unroll
    for (int d = 0; d < D; ++d) est[t * D + d] = X[d] / S;
    tflag[t] = ok ? 0 : 1;
    if (!ok) atomicOr((unsigned long long *)&meta[META_ERR], (unsigned long long)ERR_NONFINITE);
    if (tfallback && tfallback[t]) atomicAdd((unsigned long long *)&meta[META_FALLBACK], 1ull);
  }
}

// Weight of particle g (target t) in storage order. pcSIR: the weight of the
// bin that holds it (its bin number, from the bin sums); SIR: e^{l_g - M} / S;
// with kept weights, e^{previous log-weight + l - M} / S.
struct WeightSrc {
  const uint32_t *segid;     // pcSIR: bin of every particle, storage order
  const double *wbin;        // pcSIR: [B]
  const double *ll;          // SIR: [NT]; pcSIR: [B]
  const double *tgt;         // [T][4]
  // kept weights (resampling threshold below 1; null otherwise): normalised
  // log-weights of the previous frame, and per target whether they are uniform
  double *lw;                // [NT]
  const int32_t *tuni;       // [T]
};
// Log-weight of particle g before normalisation: its previous log-weight
// (0 when the target's weights are uniform) plus its likelihood term.
template <bool SIR>
__device__ __forceinline__ double particle_logv(const WeightSrc &ws, int t, uint32_t g) {
  const double l = SIR ? ws.ll[g] : ws.ll[ws.segid[g]];
  return (ws.tuni[t] ? 0.0 : ws.lw[g]) + l;
}
template <bool SIR>
__device__ __forceinline__ double particle_weight(const WeightSrc &ws, int t, uint32_t g) {
  if (ws.lw) return exp(particle_logv<SIR>(ws, t, g) - ws.tgt[t * 4]) / ws.tgt[t * 4 + 1];
  if (SIR) return exp(ws.ll[g] - ws.tgt[t * 4]) / ws.tgt[t * 4 + 1];
  return ws.wbin[ws.segid[g]];
}

// Per-particle normalisation: per-tile partials (max, S, Q, X[D]) over the
// particles, then a per-target combine.
template <int DIM, bool SIR>
__device__ __forceinline__ double norm_value(const WeightSrc &ws, int t, uint32_t g) {
  return ws.lw ? particle_logv<SIR>(ws, t, g) : ws.ll[g];
}

// SIR, and pcSIR with kept weights.
template <int DIM, bool SIR>
__global__ __launch_bounds__(TPB) void k_norm_part(Params p, const Tile *__restrict__ tiles,
                                                   const uint32_t *__restrict__ off, WeightSrc ws,
                                                   const float *__restrict__ s, double *__restrict__ part) {
  constexpr int D = 2 * DIM + 1;
  __shared__ double lds[TPB / WAVE];
  const Tile tl = tiles[blockIdx.x];
  const uint32_t base = tl.base, n = tl.n;
  double mx = -INFINITY;
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    const uint32_t i = tl.i0 + it * TPB + threadIdx.x;
    if (i < n) mx = fmax(mx, norm_value<DIM, SIR>(ws, tl.t, base + i));
  }
  const double M = block_max<TPB, double>(mx, lds);
  double S = 0.0, Q = 0.0, X[D];
#pragma unroll
  for (int d = 0; d < D; ++d) X[d] = 0.0;
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    const uint32_t i = tl.i0 + it * TPB + threadIdx.x;
    if (i < n) {
      const uint32_t g = base + i;
      const double e = exp(norm_value<DIM, SIR>(ws, tl.t, g) - M);
      S += e;
      Q += e * e;
#pragma unroll
      for (int d = 0; d < D; ++d) X[d] += e * (double)s[(size_t)d * p.NT + g];
    }
  }
  S = block_sum<TPB, double>(S, lds);
  Q = block_sum<TPB, double>(Q, lds);
#pragma unroll
  for (int d = 0; d < D; ++d) X[d] = block_sum<TPB, double>(X[d], lds);
  if (threadIdx.x == 0) {
    double *o = part + (size_t)blockIdx.x * (3 + D);
    o[0] = M;
    o[1] = S;
    o[2] = Q;
#pragma unroll
    for (int d = 0; d < D; ++d) o[3 + d] = X[d];
  }
}

template <int DIM>
__global__ __launch_bounds__(TPB) void k_norm_comb(Params p, const uint32_t *__restrict__ tfirst,
                                                   const double *__restrict__ part, const StepDesc *__restrict__ desc,
                                                   double *__restrict__ tgt, double *__restrict__ est,
                                                   int32_t *__restrict__ tflag, uint64_t *__restrict__ meta,
                                                   const int32_t *__restrict__ tfallback) {
  constexpr int D = 2 * DIM + 1;
  constexpr int W = 3 + D;
  __shared__ double lds[TPB / WAVE];
  const int t = blockIdx.x;
  const uint32_t a0 = tfirst[t], a1 = tfirst[t + 1];
  double mx = -INFINITY;
  for (uint32_t i = a0 + threadIdx.x; i < a1; i += TPB) mx = fmax(mx, part[(size_t)i * W]);
  const double M = block_max<TPB, double>(mx, lds);
  double S = 0.0, Q = 0.0, X[D];
#pragma unroll
  for (int d = 0; d < D; ++d) X[d] = 0.0;
  for (uint32_t i = a0 + threadIdx.x; i < a1; i += TPB) {
    const double *o = part + (size_t)i * W;
    const double f = exp(o[0] - M);
    if (f > 0.0) {
      S += o[1] * f;
      Q += o[2] * f * f;
#pragma unroll
      for (int d = 0; d < D; ++d) X[d] += o[3 + d] * f;
    }
  }
  S = block_sum<TPB, double>(S, lds);
  Q = block_sum<TPB, double>(Q, lds);
#pragma unroll
  for (int d = 0; d < D; ++d) X[d] = block_sum<TPB, double>(X[d], lds);
  if (threadIdx.x == 0) {
    const bool ok = isfinite(M) && isfinite(S) && S > 0.0;
    tgt[t * 4 + 0] = M;
    tgt[t * 4 + 1] = S;
    tgt[t * 4 + 2] = S * S / Q;
    tgt[t * 4 + 3] = resample_uniform(p.seed, (uint64_t)desc->k, (uint64_t)t);
#pragma unroll
    for (int d = 0; d < D; ++d) est[t * D + d] = X[d] / S;
    tflag[t] = ok ? 0 : 1;
    if (!ok) atomicOr((unsigned long long *)&meta[META_ERR], (unsigned long long)ERR_NONFINITE);
    if (tfallback && tfallback[t]) atomicAdd((unsigned long long *)&meta[META_FALLBACK], 1ull);
  }
}

// ---------------------------------------------------------------- weights, CDF, resampling
// Sum of the broadcast weights of every scan tile. A block takes
// CDF_SUM_TILES consecutive tiles, so that all of their loads (for pcSIR the
// bin numbers, then the bin weights they index) are in flight together; each
// tile's sum is formed in the same order as a block of its own would form it
// (per thread over its items, then the waves in order).
constexpr int CDF_SUM_TILES = 2;

template <bool SIR>
__global__ __launch_bounds__(TPB) void k_cdf_sum(const Tile *__restrict__ tiles, uint32_t ntiles,
                                                 const uint32_t *__restrict__ off, WeightSrc ws,
                                                 double *__restrict__ tile_sum) {
  __shared__ double lds[CDF_SUM_TILES][TPB / WAVE];
  Tile tl[CDF_SUM_TILES];
#pragma unroll
  for (int k = 0; k < CDF_SUM_TILES; ++k) tl[k] = tiles[min(blockIdx.x * CDF_SUM_TILES + k, ntiles - 1)];
  double w[CDF_SUM_TILES][SCAN_ITEMS];
  if (!SIR && !ws.lw) {
    uint32_t b[CDF_SUM_TILES][SCAN_ITEMS];
#pragma unroll
    for (int k = 0; k < CDF_SUM_TILES; ++k)
#pragma unroll
      for (int it = 0; it < SCAN_ITEMS; ++it)  // coalesced; clamped, unconditional loads
        b[k][it] = ws.segid[tl[k].base + min(tl[k].i0 + it * TPB + threadIdx.x, tl[k].n - 1)];
#pragma unroll
    for (int k = 0; k < CDF_SUM_TILES; ++k)
#pragma unroll
      for (int it = 0; it < SCAN_ITEMS; ++it) w[k][it] = ws.wbin[b[k][it]];
  } else {
#pragma unroll
    for (int k = 0; k < CDF_SUM_TILES; ++k)
#pragma unroll
      for (int it = 0; it < SCAN_ITEMS; ++it)
        w[k][it] = particle_weight<SIR>(ws, tl[k].t, tl[k].base + min(tl[k].i0 + it * TPB + threadIdx.x, tl[k].n - 1));
  }
#pragma unroll
  for (int k = 0; k < CDF_SUM_TILES; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it)
      if (tl[k].i0 + it * TPB + threadIdx.x < tl[k].n) acc += w[k][it];
    acc = wave_sum(acc);
    if (lane_id() == 0) lds[k][wave_id()] = acc;
  }
  __syncthreads();
  if (threadIdx.x < CDF_SUM_TILES && blockIdx.x * CDF_SUM_TILES + threadIdx.x < ntiles) {
    double r = lds[threadIdx.x][0];
#pragma unroll
    for (int v = 1; v < TPB / WAVE; ++v) r += lds[threadIdx.x][v];
    tile_sum[blockIdx.x * CDF_SUM_TILES + threadIdx.x] = r;
  }
}

// Per target: exclusive, non-decreasing scan of its tiles' sums.
__global__ __launch_bounds__(TPB) void k_cdf_prefix(const uint32_t *__restrict__ tfirst,
                                                    const double *__restrict__ tile_sum,
                                                    double *__restrict__ tile_pre, uint32_t *__restrict__ rs_count) {
  __shared__ double lds[TPB / WAVE];
  const int t = blockIdx.x;
  if (t == 0 && threadIdx.x == 0) *rs_count = 0;  // this frame's resampling work list starts empty
  const uint32_t a0 = tfirst[t], a1 = tfirst[t + 1];
  __shared__ double last;
  double carry = 0.0;
  for (uint32_t b0 = a0; b0 < a1; b0 += TPB) {
    const uint32_t b = b0 + threadIdx.x;
    const double v = b < a1 ? tile_sum[b] : 0.0;
    double tot;
    const double ex = block_excl_scan_monotone<TPB>(v, lds, &tot);
    const double val = carry + ex;
    if (b < a1) tile_pre[b] = val;
    if (threadIdx.x == TPB - 1) last = val + v;
    __syncthreads();
    // the next chunk starts at or above every value written so far
    const double nc = carry + tot;
    carry = nc > last ? nc : last;
    __syncthreads();
  }
}

// Number of thresholds theta_j = (j + u) / n below c, for j in [0, n)
// (theta_j formed as written: j + u, then divided by n, each rounded), without
// divisions where they cannot change the answer. With x = c n - u,
// theta_j < c holds exactly when j < x, except where j lies within about
// 2^-52 (j + u) < 2^-20 of x (the roundings of j + u and of the division);
// x itself comes from one fma, within 2^-20 of c n - u for x < 2^32. So when
// x is more than 2^-10 from every integer, the count is ceil(x) (clamped to
// [0, n]). Otherwise, with J the integer nearest x, every j <= J - 2 counts
// and no j >= J + 1 does, and the two thresholds between are compared as
// written.
__device__ __forceinline__ uint32_t count_below(double c, double u, uint32_t n) {
  if (!(c > 0.0)) return 0;
  if (!(c < 2.0)) return n;
  const double dn = (double)n;
  const double x = fma(c, dn, -u);
  const double f = ceil(x);
  const double g = 0x1p-10;
  if (f - x > g && f - x < 1.0 - g) return (uint32_t)(f < 0.0 ? 0.0 : (f > dn ? dn : f));
  const double J = rint(x);
  uint32_t r = J < 1.0 ? 0u : (uint32_t)(J > dn ? dn : J - 1.0);  // thresholds below J - 1
  for (int d = -1; d <= 0; ++d) {
    const double j = J + d;
    if (j >= 0.0 && j < dn && (j + u) / dn < c) ++r;
  }
  return r;
}

// LDS position of a tile's l-th cumulative weight: one pad slot per
// SCAN_ITEMS entries, so that a thread's SCAN_ITEMS consecutive entries do
// not collide in banks with its neighbours'.
__device__ __forceinline__ uint32_t cpad(uint32_t l) { return l + l / SCAN_ITEMS; }

// Index of the parent of threshold theta among the m cumulative weights of a
// tile held in LDS (at cpad positions): the first entry above theta, the
// tile's last entry when none of the others is (its C is the next tile's
// start, or it is the target's last particle, which stands for +infinity).
// RS_ITEMS searches advance together, one halving step at a time, so that
// their LDS reads overlap.
__device__ __forceinline__ void tile_search(const double *cl, uint32_t m, const double (&theta)[RS_ITEMS],
                                            uint32_t (&a)[RS_ITEMS]) {
  const uint32_t ns = m - 1;  // entries below the last one
#pragma unroll
  for (int it = 0; it < RS_ITEMS; ++it) a[it] = 0;
  // a = number of those entries <= theta (a prefix: C is non-decreasing)
  for (uint32_t step = ns ? 1u << (31 - __clz(ns)) : 0u; step > 0; step >>= 1) {
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it)
      if (a[it] + step <= ns && cl[cpad(a[it] + step - 1)] <= theta[it]) a[it] += step;
  }
}

// Systematic resampling over the cumulative weights C (non-decreasing across
// the whole target): the new particle j takes the parent
// s(j) = min{ l : C_l > theta_j }, theta_j = (j + u) / n, and the target's last
// particle also takes any j left above C_{n-1} by rounding. So particle l has
// the offspring j in [count_below(C_{l-1}), count_below(C_l)) (the last
// particle up to n), one contiguous run per particle.
//
// One block per scan tile forms the tile's C by a block scan, with every
// boundary taken from one source (the next thread's or tile's start, made
// non-decreasing). Weights are loaded coalesced into LDS first, then each
// thread takes its SCAN_ITEMS consecutive ones; the LDS array has one pad
// slot per SCAN_ITEMS entries so that those strided reads do not collide in
// banks. The tile's offspring are j in [count_below(tile start),
// count_below(next tile's start)).
// - A light tile (at most `light` offspring) decodes the runs on chip: each
//   particle with offspring marks the first slot of its run in LDS, a block
//   max-scan carries every mark to the end of its run, and the slots go out
//   to anc in coalesced stores. C never leaves the chip.
// - A heavy tile (one holding a large share of its target's weight, up to
//   all N offspring) stores its C and appends one (search tile, scan tile)
//   pair for every search tile of RS_TILE new particles that its offspring
//   touch to a work list of `cap` entries; k_resample_search spreads the
//   pairs over its grid.
// A target that keeps its particles (non-finite normalisation, or N_eff at
// or above the threshold) gets identity ancestors and, with kept weights, its
// normalised log-weights. CDF_ONLY (the debug view) stores every tile's C and
// nothing else.
constexpr int DEC_ITEMS = RS_LIGHT_MAX / TPB;  // run slots per thread in the decode
__device__ __forceinline__ uint32_t dpad(uint32_t k) { return k + k / DEC_ITEMS; }

template <bool SIR, bool CDF_ONLY>
__global__ __launch_bounds__(TPB) void k_cdf_scan(const Tile *__restrict__ tiles, const uint32_t *__restrict__ tile_last,
                                                  WeightSrc ws, const double *__restrict__ tile_pre,
                                                  const int32_t *__restrict__ tflag, uint32_t *__restrict__ anc,
                                                  double *__restrict__ cdf, double neff_frac,
                                                  int32_t *__restrict__ tuni_next, const uint32_t *__restrict__ tfirstR,
                                                  uint2 *__restrict__ rs_work, uint32_t *__restrict__ rs_count,
                                                  uint32_t cap, uint32_t light) {
  __shared__ double lds[TPB / WAVE];
  __shared__ uint32_t wmax[TPB / WAVE];
  __shared__ uint32_t wpos;
  __shared__ double wfirst[TPB / WAVE + 1];  // each wave's first thread boundary, and the tile's end
  __shared__ double cl[SCAN_TILE + SCAN_TILE / SCAN_ITEMS];
  static_assert(sizeof(cl) >= sizeof(uint32_t) * (RS_LIGHT_MAX + RS_LIGHT_MAX / DEC_ITEMS), "run slots fit in cl");
  uint32_t *mk = reinterpret_cast<uint32_t *>(cl);  // run slots of a light tile (after C is in registers)
  const Tile tl = tiles[blockIdx.x];
  const int t = tl.t;
  const uint32_t base = tl.base, n = tl.n;
  const uint32_t m = min((uint32_t)SCAN_TILE, n - tl.i0);  // particles in this tile
  // per-tile and per-target values, loaded before the first barrier so that
  // their latency overlaps the weights' (loads are not moved across barriers)
  const double pre = tile_pre[blockIdx.x];
  const bool last_tile = tile_last[blockIdx.x] != 0;
  const double tile_end = last_tile ? INFINITY : tile_pre[blockIdx.x + 1];
  const int32_t flag = tflag[t];
  const double neff = ws.tgt[t * 4 + 2];
  const double u = ws.tgt[t * 4 + 3];
  {
    double wl[SCAN_ITEMS];
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it)
      wl[it] = particle_weight<SIR>(ws, t, base + min(tl.i0 + it * TPB + threadIdx.x, n - 1));
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
      const uint32_t li = it * TPB + threadIdx.x;
      cl[cpad(li)] = tl.i0 + li < n ? wl[it] : 0.0;
    }
  }
  __syncthreads();
  double w[SCAN_ITEMS];
  double loc = 0.0;
#pragma unroll
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    w[it] = cl[cpad(threadIdx.x * SCAN_ITEMS + it)];
    loc += w[it];
  }
  double tot;
  const double ex = block_excl_scan_monotone<TPB>(loc, lds, &tot);
  // thread boundaries: non-decreasing, within [this tile's start, next tile's start]
  // (each thread's end is the next thread's start: the next lane's, or the
  // next wave's first, or the tile's end)
  double start;
  {
    const double b = pre + ex;
    start = b < tile_end ? b : tile_end;
  }
  if (lane_id() == 0) wfirst[wave_id()] = start;
  if (threadIdx.x == 0) wfirst[TPB / WAVE] = tile_end;
  __syncthreads();  // also: every thread has read its weights from cl
  // kept weights: a target resamples only when N_eff < neff_frac * N
  const bool keep = ws.lw && !flag && !(neff < neff_frac * (double)n);
  if (flag || keep) {
    if (CDF_ONLY) return;
    if (tuni_next && tl.i0 == 0 && threadIdx.x == 0) tuni_next[t] = keep ? 0 : 1;
    // the particles stay (identity resampling): after a non-finite
    // normalisation, or when N_eff is above the threshold; then they keep
    // their normalised log-weights for the next frame
    const double lnorm = ws.tgt[t * 4] + log(ws.tgt[t * 4 + 1]);
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
      const uint32_t i = tl.i0 + threadIdx.x * SCAN_ITEMS + it;
      if (i < n) {
        anc[base + i] = i;
        if (keep) ws.lw[base + i] = particle_logv<SIR>(ws, t, base + i) - lnorm;
      }
    }
    return;
  }
  if (!CDF_ONLY && tuni_next && tl.i0 == 0 && threadIdx.x == 0) tuni_next[t] = 1;
  double end = __shfl_down(start, 1, WAVE);
  if (lane_id() == WAVE - 1) end = wfirst[wave_id() + 1];
  if (end < start) end = start;
  double run = 0.0;
  double cprev = start;
  double c[SCAN_ITEMS];
#pragma unroll
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    const uint32_t i = tl.i0 + threadIdx.x * SCAN_ITEMS + it;
    run += w[it];
    double ci;
    if (i + 1 == n) {
      ci = pre + (ex + run);  // the target's total
      ci = ci < cprev ? cprev : ci;
    } else {
      ci = (it == SCAN_ITEMS - 1) ? end : pre + (ex + run);
      ci = ci < cprev ? cprev : (ci > end ? end : ci);
    }
    c[it] = ci;
    cprev = ci;
  }
  // C in LDS, from where a heavy tile stores it (coalesced)
#pragma unroll
  for (int it = 0; it < SCAN_ITEMS; ++it) cl[cpad(threadIdx.x * SCAN_ITEMS + it)] = c[it];
  const uint32_t jlo = count_below(pre, u, n);
  const uint32_t jhi = last_tile ? n : count_below(tile_end, u, n);
  const uint32_t M = jhi - jlo;  // offspring of the tile
  if (CDF_ONLY || M > light) {
    // heavy: C through LDS, so that the stores to global memory are coalesced
    // the search tiles that the offspring touch, appended to the work list
    const uint32_t qa = jlo / RS_TILE, nq = CDF_ONLY ? 0 : (jhi - 1) / RS_TILE - qa + 1;
    if (!CDF_ONLY && threadIdx.x == 0) wpos = atomicAdd(rs_count, nq);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
      const uint32_t li = it * TPB + threadIdx.x;
      if (li < m) cdf[base + tl.i0 + li] = cl[cpad(li)];
    }
    if (CDF_ONLY) return;
    const uint32_t first_rtile = tfirstR[t];
    for (uint32_t k = threadIdx.x; k < nq; k += TPB)
      if (wpos + k < cap) rs_work[wpos + k] = make_uint2(first_rtile + qa + k, blockIdx.x);
    return;
  }
  // light: every particle's run [s, e) of offspring, relative to jlo
  const uint32_t s_abs = count_below(start, u, n);  // the thread's first run starts here
  uint32_t e[SCAN_ITEMS];
  {
    uint32_t s0 = s_abs;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
      const uint32_t i = tl.i0 + threadIdx.x * SCAN_ITEMS + it;
      const uint32_t ei = i >= n ? s0 : (i + 1 == n ? n : count_below(c[it], u, n));
      s0 = ei > s0 ? ei : s0;
      e[it] = s0 - jlo;
    }
  }
  // clear the thread's own slots (every thread is done with C in LDS), then
  // mark the first slot of every run
  __syncthreads();
#pragma unroll
  for (int r = 0; r < DEC_ITEMS; ++r) mk[dpad(threadIdx.x * DEC_ITEMS + r)] = 0u;
  __syncthreads();
  {
    uint32_t sp = s_abs - jlo;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
      if (e[it] > sp) mk[dpad(sp)] = threadIdx.x * SCAN_ITEMS + it + 1;  // local index + 1
      sp = e[it];
    }
  }
  __syncthreads();
  // running maximum over the slots (marks rise with the slot): thread r
  // takes slots [r DEC_ITEMS, (r + 1) DEC_ITEMS)
  uint32_t v[DEC_ITEMS];
  uint32_t mx = 0;
#pragma unroll
  for (int r = 0; r < DEC_ITEMS; ++r) {
    const uint32_t x = mk[dpad(threadIdx.x * DEC_ITEMS + r)];
    mx = x > mx ? x : mx;
    v[r] = mx;
  }
  {
    const uint32_t incl = wave_incl_max_scan(mx);
    uint32_t exw = __shfl_up(incl, 1, WAVE);
    if (lane_id() == 0) exw = 0;
    if (lane_id() == WAVE - 1) wmax[wave_id()] = incl;
    __syncthreads();
    uint32_t pw = 0;
#pragma unroll
    for (int i = 0; i < TPB / WAVE; ++i)
      if (i < wave_id()) pw = wmax[i] > pw ? wmax[i] : pw;
    const uint32_t pre_mx = exw > pw ? exw : pw;
#pragma unroll
    for (int r = 0; r < DEC_ITEMS; ++r) mk[dpad(threadIdx.x * DEC_ITEMS + r)] = (v[r] > pre_mx ? v[r] : pre_mx) - 1u;
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < M; k += TPB) anc[base + jlo + k] = tl.i0 + mk[dpad(k)];
}

// The offspring of heavy scan tiles, spread over the grid: each work-list
// pair (search tile of RS_TILE new particles [j0, j1), heavy scan tile)
// stages the scan tile's stored C in LDS and resolves the j of [j0, j1) in
// [count_below(the tile's start), count_below(next tile's start)) by binary
// search, with the scan kernel's thresholds. Pairs are disjoint in j, so
// their order in the list does not matter.
template <bool SIR>
__global__ __launch_bounds__(TPB) void k_resample_search(const Tile *__restrict__ tilesR,
                                                         const Tile *__restrict__ tilesS, WeightSrc ws,
                                                         const double *__restrict__ cdf,
                                                         const double *__restrict__ tile_pre,
                                                         const uint32_t *__restrict__ tile_last,
                                                         const uint2 *__restrict__ rs_work,
                                                         const uint32_t *__restrict__ rs_count, uint32_t cap,
                                                         uint32_t *__restrict__ anc) {
  __shared__ double cl[SCAN_TILE + SCAN_TILE / SCAN_ITEMS];
  const uint32_t total = min(*rs_count, cap);
  for (uint32_t wi = blockIdx.x; wi < total; wi += gridDim.x) {
    const uint2 pr = rs_work[wi];
    const Tile rt = tilesR[pr.x], st = tilesS[pr.y];
    const uint32_t base = rt.base, n = rt.n;
    const double u = ws.tgt[rt.t * 4 + 3];
    const double dn = (double)n;
    const uint32_t m = min((uint32_t)SCAN_TILE, n - st.i0);
    const uint32_t lo = count_below(tile_pre[pr.y], u, n);
    const uint32_t hi = tile_last[pr.y] ? n : count_below(tile_pre[pr.y + 1], u, n);
    const uint32_t j0 = rt.i0, j1 = min(rt.i0 + RS_TILE, n);
    const uint32_t a0 = max(lo, j0), a1 = min(hi, j1);
    __syncthreads();  // the previous pair's searches are done with cl
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
      const uint32_t li = it * TPB + threadIdx.x;
      if (li < m) cl[cpad(li)] = cdf[base + st.i0 + li];
    }
    __syncthreads();
    double theta[RS_ITEMS];
    uint32_t a[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) theta[it] = ((double)(j0 + it * TPB + threadIdx.x) + u) / dn;
    tile_search(cl, m, theta, a);
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
      const uint32_t j = j0 + it * TPB + threadIdx.x;
      if (j >= a0 && j < a1) anc[base + j] = st.i0 + a[it];
    }
  }
}

// ---------------------------------------------------------------- helpers for the API
// Materialise the current particle set (apply the pending resampling gather).
__global__ __launch_bounds__(TPB) void k_gather(int D, uint32_t NT, const Tile *__restrict__ tiles,
                                                const uint32_t *__restrict__ off, const float *__restrict__ s,
                                                const uint32_t *__restrict__ anc, int pending, float *__restrict__ dst) {
  const Tile tl = tiles[blockIdx.x];
  const uint32_t base = tl.base, n = tl.n;
  const uint32_t i = tl.i0 + threadIdx.x;
  if (i >= n) return;
  const uint32_t g = base + i;
  const uint32_t src = pending ? base + min(anc[g], n - 1) : g;
  for (int d = 0; d < D; ++d) dst[(size_t)d * NT + g] = s[(size_t)d * NT + src];
}

// anc[g] = index within the target (identity resampling).
__global__ __launch_bounds__(TPB) void k_identity(const Tile *__restrict__ tiles, const uint32_t *__restrict__ off,
                                                  uint32_t *__restrict__ anc) {
  const Tile tl = tiles[blockIdx.x];
  const uint32_t base = tl.base, n = tl.n;
  const uint32_t i = tl.i0 + threadIdx.x;
  if (i < n) anc[base + i] = i;
}

// Cell index of every particle with its target's cells per pixel (tm null:
// pixels, m = 1).
__global__ __launch_bounds__(TPB) void k_dbg_keys(int dim, uint32_t NT, const Tile *__restrict__ tiles,
                                                  const int32_t *__restrict__ tm, const float *__restrict__ s,
                                                  int32_t *__restrict__ out) {
  const Tile tl = tiles[blockIdx.x];
  const uint32_t i = tl.i0 + threadIdx.x;
  if (i >= tl.n) return;
  const uint32_t g = tl.base + i;
  for (int a = 0; a < 3; ++a)
    out[(size_t)a * NT + g] = a < dim ? cell_index(s[(size_t)a * NT + g], tm ? tm[tl.t * 3 + a] : 1) : 0;
}

template <int DIM>
__global__ void k_dbg_bins(Params p, const uint64_t *__restrict__ meta, const unsigned long long *__restrict__ acc,
                           const uint32_t *__restrict__ seg_key, const uint32_t *__restrict__ kbase,
                           const int32_t *__restrict__ bbox_cur, int what, void *__restrict__ out,
                           const double *__restrict__ wacc, const int32_t *__restrict__ tuni) {
  constexpr int D = 2 * DIM + 1;
  const uint32_t B = (uint32_t)meta[META_B];
  const uint32_t NT = p.NT;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < B; s += gridDim.x * blockDim.x) {
    int t;
    int32_t cell[3];
    decode_key<DIM>(seg_key[s], p.T, kbase, bbox_cur, t, cell);
    const double n = (double)(long long)acc[s];
    if (what == 3) ((int32_t *)out)[s] = t;
    if (what == 4)
      for (int a = 0; a < 3; ++a) ((int32_t *)out)[(size_t)a * B + s] = cell[a];
    if (what == 5) ((long long *)out)[s] = (long long)acc[s];
    if (what == 6 && wacc && !tuni[t] && wacc[s] > 0.0) {
      // kept weights: the weighted mean the dummy was formed from
      double *o = (double *)out;
      const double ws = wacc[s];
      for (int a = 0; a < DIM; ++a)
        o[(size_t)a * B + s] = (double)floor_div(cell[a], p.tm[t * 3 + a]) + wacc[(size_t)(1 + a) * NT + s] / ws;
      for (int d = DIM; d < D; ++d) o[(size_t)d * B + s] = wacc[(size_t)(1 + d) * NT + s] / ws;
    } else if (what == 6) {
      double *o = (double *)out;
      for (int a = 0; a < DIM; ++a) {
        const double c0 = (double)floor_div(cell[a], p.tm[t * 3 + a]);
        o[(size_t)a * B + s] = c0 + (double)(long long)acc[(size_t)(1 + a) * NT + s] / (double)FX_POS / n;
      }
      for (int a = 0; a < DIM; ++a)
        o[(size_t)(DIM + a) * B + s] = (double)(long long)acc[(size_t)(1 + DIM + a) * NT + s] / (double)FX_VEL / n;
      o[(size_t)(2 * DIM) * B + s] = (double)(long long)acc[(size_t)(1 + 2 * DIM) * NT + s] / (double)FX_INT / n;
    }
  }
}

// Normalised weights of the last step. A target that kept its weights
// (tuni_next 0) already holds log w in lw, in place of the step's input.
template <bool SIR>
__global__ __launch_bounds__(TPB) void k_dbg_weights(const Tile *__restrict__ tiles, const uint32_t *__restrict__ off,
                                                     WeightSrc ws, const int32_t *__restrict__ tuni_next,
                                                     double *__restrict__ out) {
  const Tile tl = tiles[blockIdx.x];
  const uint32_t base = tl.base, n = tl.n;
  const uint32_t i = tl.i0 + threadIdx.x;
  if (i >= n) return;
  out[base + i] = (ws.lw && !tuni_next[tl.t]) ? exp(ws.lw[base + i]) : particle_weight<SIR>(ws, tl.t, base + i);
}

// Log-weight each particle carries into the next frame (uniform targets: -log N_t).
__global__ __launch_bounds__(TPB) void k_dbg_logw(const Tile *__restrict__ tiles, const uint32_t *__restrict__ off,
                                                  const double *__restrict__ lw, const int32_t *__restrict__ tuni,
                                                  double *__restrict__ out) {
  const Tile tl = tiles[blockIdx.x];
  const uint32_t base = tl.base, n = tl.n;
  const uint32_t i = tl.i0 + threadIdx.x;
  if (i >= n) return;
  out[base + i] = (!lw || tuni[tl.t]) ? -log((double)n) : lw[base + i];
}

}  // namespace pcsir
