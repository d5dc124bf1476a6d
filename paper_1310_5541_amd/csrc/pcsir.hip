// Host side of the pcSIR library: workspace planning, tile tables, launch
// sequences of one SIR / pcSIR frame, and the C ABI declared in pcsir.h.
// The library never allocates device memory: every buffer is carved out of
// the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pcsir.h"
#include "kernels.h"
#include "surrogate.h"
#include "../../include/pcsir_mlp.h"

using namespace pcsir;

namespace {

constexpr size_t ALIGN = 256;

struct Layout {
  size_t S0, S1, anc, key, kA, kB, hist, dtot, chunk_heads, acc, seg_key, seg_t, segid, dpix, doff, dint, dlo,
      ll, ll9, wbin, lw, wacc, tuni, tuni_next, desc, dvel, surr, tfb, tmax, tsse, tcnt, tcount, lut, seg_first, bm,
      bbox_part, mom_part, tm, range, bbox_cur, kbase, meta, tgt, est, tflag, part, tile_sum, tile_pre, cdf, rs_work, rs_count,
      tiles256, tilesS, tilesR, tilesB, tilesK, tile_last, tfirst, tfirstR, t256_first, off;
  size_t total;
  uint32_t G;    // workgroups of the sort and segment passes over the key list
  uint32_t n256; // propagate tiles
  uint64_t lut_cap;  // entries of the cell -> bin table
  uint32_t nS;   // scan tiles
  uint32_t nR;   // resampling search tiles
  uint32_t nW;   // capacity of the resampling work list (search tile, heavy scan tile)
  uint32_t nB;   // bin-sum tiles
  uint32_t nK;   // key tiles
};

struct Tables {
  std::vector<Tile> t256, tS, tR;
  std::vector<BinTile> tB, tK;
  std::vector<uint32_t> tile_last, tfirst, tfirstR, t256_first, off;
};

bool valid_config(const pcsir_config *c, std::string *why) {
  auto bad = [&](const char *m) {
    if (why) *why = m;
    return false;
  };
  if (!c) return bad("config is NULL");
  if (c->abi_version != PCSIR_ABI_VERSION) return bad("abi_version mismatch");
  if (c->dim != 2 && c->dim != 3) return bad("dim must be 2 or 3");
  if (c->n_targets < 1) return bad("n_targets must be >= 1");
  if (!c->n_particles) return bad("n_particles is NULL");
  long long sum = 0;
  for (int t = 0; t < c->n_targets; ++t) {
    if (c->n_particles[t] < 1) return bad("every n_particles[t] must be >= 1");
    sum += c->n_particles[t];
    if (sum >= (1LL << 31)) return bad("sum of n_particles must be < 2^31");
  }
  for (int a = 0; a < c->dim; ++a)
    if (c->bins_per_px[a] < 1 || c->bins_per_px[a] > 4096) return bad("bins_per_px must lie in [1, 4096]");
  if (c->patch < 1 || c->patch > 127 || (c->patch % 2) == 0) return bad("patch must be odd and in [1, 127]");
  if (c->quad < 1 || c->quad > 16) return bad("quad must lie in [1, 16]");
  if (c->psf != PCSIR_PSF_GAUSS2D && c->psf != PCSIR_PSF_ASTIG3D) return bad("unknown psf");
  if (c->psf == PCSIR_PSF_ASTIG3D && c->dim != 3) return bad("astigmatic PSF needs dim == 3");
  if (c->dummy_mode != PCSIR_DUMMY_COM && c->dummy_mode != PCSIR_DUMMY_COC && c->dummy_mode != PCSIR_DUMMY_COM2)
    return bad("unknown dummy_mode");
  if (c->lik_mode < PCSIR_LIK_DIRECT || c->lik_mode > PCSIR_LIK_SURR_FP8) return bad("unknown lik_mode");
  if (c->lik_mode >= PCSIR_LIK_SURR_BF16 && c->patch * c->patch + 2 * c->dim + 1 > MLP_F)
    return bad("surrogate features (patch^2 + 2 dim + 1) exceed 256");
  if (c->frame_h < 1 || c->frame_w < 1) return bad("frame_h and frame_w must be >= 1");
  if (!(c->sigma_psf > 0.0f) || !(c->sigma_xi > 0.0f)) return bad("sigma_psf and sigma_xi must be > 0");
  if (c->psf == PCSIR_PSF_ASTIG3D && !(c->astig_d > 0.0f)) return bad("astig_d must be > 0");
  for (int d = 0; d < 2 * c->dim + 1; ++d)
    if (!(c->proc_sigma[d] >= 0.0f)) return bad("proc_sigma must be >= 0");
  if (!(c->neff_threshold >= 0.0)) return bad("neff_threshold must be >= 0 (above 1: resample every frame)");
  if (c->dummy_mode == PCSIR_DUMMY_COM2 &&
      (c->dim != 2 || c->lik_mode > PCSIR_LIK_SEPARABLE || c->neff_threshold <= 1.0))
    return bad("second-order dummies need dim 2, an exact likelihood and resampling every frame");
  if (!(c->bins_per_sigma >= 0.0) || !std::isfinite(c->bins_per_sigma))
    return bad("bins_per_sigma must be finite and >= 0 (0: the fixed bins_per_px)");
  if (c->bins_per_sigma > 0.0 && (c->bins_max < 1 || c->bins_max > 4096)) return bad("bins_max must lie in [1, 4096]");
  return true;
}

constexpr int BIN_TILE_MIN = 1024;

void build_bin_tiles(const pcsir_config *c, uint32_t tile, std::vector<BinTile> &tB) {
  tB.clear();
  uint32_t base = 0;
  for (int t = 0; t < c->n_targets; ++t) {
    const uint32_t n = (uint32_t)c->n_particles[t];
    for (uint32_t i0 = 0; i0 < n; i0 += tile) tB.push_back(BinTile{t, i0, std::min<uint32_t>(n, i0 + tile), base});
    base += n;
  }
}

void build_tables(const pcsir_config *c, Tables &tb) {
  const int T = c->n_targets;
  tb.off.assign(T + 1, 0);
  tb.tfirst.assign(T + 1, 0);
  tb.tfirstR.assign(T + 1, 0);
  tb.tR.clear();
  tb.t256_first.assign(T + 1, 0);
  tb.t256.clear();
  tb.tS.clear();
  tb.tile_last.clear();
  tb.tB.clear();
  for (int t = 0; t < T; ++t) {
    const uint32_t n = (uint32_t)c->n_particles[t];
    tb.off[t + 1] = tb.off[t] + n;
    tb.t256_first[t] = (uint32_t)tb.t256.size();
    for (uint32_t i0 = 0; i0 < n; i0 += TPB) tb.t256.push_back(Tile{t, i0, tb.off[t], n});
    tb.tfirst[t] = (uint32_t)tb.tS.size();
    for (uint32_t i0 = 0; i0 < n; i0 += SCAN_TILE) {
      tb.tS.push_back(Tile{t, i0, tb.off[t], n});
      tb.tile_last.push_back(i0 + SCAN_TILE >= n ? 1u : 0u);
    }
    tb.tfirstR[t] = (uint32_t)tb.tR.size();
    for (uint32_t i0 = 0; i0 < n; i0 += RS_TILE) tb.tR.push_back(Tile{t, i0, tb.off[t], n});
  }
  build_bin_tiles(c, BIN_TILE_MAX, tb.tB);
  build_bin_tiles(c, KEYS_TILE, tb.tK);
  tb.tfirst[T] = (uint32_t)tb.tS.size();
  tb.tfirstR[T] = (uint32_t)tb.tR.size();
  tb.t256_first[T] = (uint32_t)tb.t256.size();
}


// A resampling threshold in [0, 1] keeps weights across frames.
bool keeps_weights(const pcsir_config *c) { return c->neff_threshold <= 1.0; }

Layout plan(const pcsir_config *c, const Tables &tb) {
  Layout L{};
  const size_t NT = tb.off.back();
  const size_t T = c->n_targets;
  const size_t dim = c->dim, D = 2 * dim + 1;
  L.G = (uint32_t)std::max<size_t>(1, std::min<size_t>(LIST_BLOCKS_MAX, (NT + TPB - 1) / TPB));
  L.n256 = (uint32_t)tb.t256.size();
  L.nS = (uint32_t)tb.tS.size();
  L.nR = (uint32_t)tb.tR.size();
  {
    // bin-tile table sized for the smallest tile the tuning allows
    std::vector<BinTile> most;
    build_bin_tiles(c, BIN_TILE_MIN, most);
    L.nB = (uint32_t)most.size();
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + ALIGN - 1) / ALIGN * ALIGN;
    return at;
  };
  L.S0 = take(4 * D * NT);
  L.S1 = take(4 * D * NT);
  L.anc = take(4 * NT);
  L.key = take(4 * NT);
  L.kA = take(4 * NT);
  L.kB = take(4 * NT);
  L.hist = take(4 * (size_t)MAX_BUCKETS * (size_t)L.G);
  L.dtot = take(4 * (size_t)MAX_BUCKETS);
  L.chunk_heads = take(4 * (size_t)L.G);
  const size_t acc_rows = 1 + D + (c->dummy_mode == PCSIR_DUMMY_COM2 ? 3 : 0);
  L.acc = take(8 * acc_rows * NT);
  L.ll9 = c->dummy_mode == PCSIR_DUMMY_COM2 ? take(8 * 9 * NT) : 0;
  L.seg_key = take(4 * NT);
  L.seg_t = take(4 * NT);
  L.segid = take(4 * NT);
  L.dpix = take(4 * dim * NT);
  L.doff = take(4 * dim * NT);
  L.dint = take(4 * NT);
  L.dlo = take(4 * (dim + 1) * NT);
  L.dvel = take(4 * dim * NT);
  L.ll = take(8 * NT);
  L.wbin = take(8 * NT);
  if (keeps_weights(c)) {
    L.lw = take(8 * NT);
    L.wacc = take(8 * (2 + D) * NT);
    L.tuni = take(4 * T);
    L.tuni_next = take(4 * T);
  }
  L.desc = take(sizeof(StepDesc));
  L.surr = c->lik_mode >= PCSIR_LIK_SURR_BF16 ? take(SURR_BYTES) : 0;  // surrogate weights
  L.tfb = take(4 * T);
  L.tmax = take(8 * T);
  L.tsse = take(8 * T);
  L.tcnt = take(4 * T);
  L.seg_first = take(4 * (T + 1));
  L.bbox_part = take(4 * 6 * (size_t)L.n256);
  L.mom_part = take(8 * 6 * (size_t)L.n256);
  L.tm = take(4 * 3 * T);
  L.range = take(8 * T);
  L.bbox_cur = take(4 * 6 * T);
  L.kbase = take(4 * (T + 1));
  L.meta = take(8 * META_N);
  L.tgt = take(8 * 4 * T);
  L.est = take(8 * D * T);
  L.tflag = take(4 * T);
  L.part = take(8 * (3 + D) * (size_t)L.nS);
  L.tile_sum = take(8 * (size_t)L.nS);
  L.tile_pre = take(8 * (size_t)L.nS);
  L.cdf = take(8 * NT);
  // a heavy scan tile with M offspring touches at most M / RS_TILE + 2 search tiles
  L.nW = L.nR + 2 * L.nS;
  L.rs_work = take(8 * (size_t)L.nW);
  L.rs_count = take(4);
  L.tiles256 = take(sizeof(Tile) * (size_t)L.n256);
  L.tilesS = take(sizeof(Tile) * (size_t)L.nS);
  L.tilesR = take(sizeof(Tile) * (size_t)L.nR);
  L.tilesB = take(sizeof(BinTile) * (size_t)L.nB);
  L.nK = (uint32_t)tb.tK.size();
  L.tilesK = take(sizeof(BinTile) * (size_t)L.nK);
  L.tcount = take(4 * (size_t)L.nK);
  // cell -> bin table: 8 entries per particle, between 2^16 and 2^25 (128 MB)
  L.lut_cap = 1ull << 16;
  while (L.lut_cap < 8 * NT && L.lut_cap < (1ull << 25)) L.lut_cap <<= 1;
  L.lut = take(4 * L.lut_cap);
  // cell-occupancy bitmap over every 32-bit key, with each word's first bin (1 GB)
  L.bm = take(sizeof(BmWord) * BM_WORDS);
  L.tile_last = take(4 * (size_t)L.nS);
  L.tfirst = take(4 * (T + 1));
  L.tfirstR = take(4 * (T + 1));
  L.t256_first = take(4 * (T + 1));
  L.off = take(4 * (T + 1));
  L.total = o;
  return L;
}

}  // namespace

struct pcsir_ctx {
  pcsir_config cfg;
  std::vector<int64_t> n;
  Tables tb;
  Layout L;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  Params p;
  uint32_t NT = 0;
  int cur = 0;       // state buffer holding the current particles (0: S0, 1: S1)
  int pending = 0;   // a resampling gather is pending (anc holds s(j))
  int stepped = 0;   // a step has run since init / set_particles
  int last_sir = 0;  // kind of the last step
  int debug = 0;     // keep the per-particle cumulative weights
  int num_cus = 256;
  std::string err;
  // timing
  int timing = 0;
  std::vector<hipEvent_t> ev;
  std::vector<const char *> ev_name;
  int ev_used = 0;
  // captured step graphs, by (sir, buffer parity, pending gather)
  int use_graphs = 1;
  int surr_ready = 0;      // surrogate weights installed
  float surr_fraction = 0.01f, surr_tol = 1.0f;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[2][2][2] = {};
  pcsir_tuning tune{BIN_TILE_MAX, 1024, MAX_DIGIT_BITS, 32, RS_LIGHT_DEFAULT, 0};
  uint32_t nB = 0;  // bin tiles of the current tile size

  template <typename T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
  float *state(int which) const { return at<float>(which ? L.S1 : L.S0); }
};

namespace {

pcsir_status fail(pcsir_ctx *c, pcsir_status s, const std::string &m) {
  if (c) c->err = m;
  return s;
}

pcsir_status check_hip(pcsir_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return PCSIR_OK;
  return fail(c, PCSIR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void mark(pcsir_ctx *c, const char *name) {
  if (!c->timing) return;
  if (c->ev_used >= (int)c->ev.size()) return;
  (void)hipEventRecord(c->ev[c->ev_used], c->stream);
  c->ev_name[c->ev_used] = name;
  ++c->ev_used;
}

Params make_params(const pcsir_config *c, uint32_t NT) {
  Params p;
  memset(&p, 0, sizeof(p));
  p.dim = c->dim;
  p.D = 2 * c->dim + 1;
  p.T = c->n_targets;
  p.NT = NT;
  for (int a = 0; a < 3; ++a) p.m[a] = a < c->dim ? c->bins_per_px[a] : 1;
  p.bins_per_sigma = c->bins_per_sigma;
  p.acc_rows = 1 + p.D + (c->dummy_mode == PCSIR_DUMMY_COM2 ? 3 : 0);
  p.bins_max = c->bins_max;
  p.P = c->patch;
  p.R = (c->patch - 1) / 2;
  p.q = c->quad;
  p.psf = c->psf;
  p.dummy_mode = c->dummy_mode;
  p.per_target_frames = c->per_target_frames;
  p.H = c->frame_h;
  p.W = c->frame_w;
  p.sigma_psf = c->sigma_psf;
  p.astig_gamma = c->astig_gamma;
  p.astig_d = c->astig_d;
  p.i_bg = c->i_bg;
  p.inv2sxi2 = 1.0 / (2.0 * (double)c->sigma_xi * (double)c->sigma_xi);
  for (int d = 0; d < 7; ++d) p.proc_sigma[d] = c->proc_sigma[d];
  p.seed = c->seed;
  return p;
}

SortBufs sort_bufs(const pcsir_ctx *c) {
  SortBufs sb;
  sb.key_store = c->at<uint32_t>(c->L.key);
  sb.kA = c->at<uint32_t>(c->L.kA);
  sb.kB = c->at<uint32_t>(c->L.kB);
  return sb;
}

WeightSrc weight_src(const pcsir_ctx *c) {
  WeightSrc w;
  w.segid = c->at<uint32_t>(c->L.segid);
  w.wbin = c->at<double>(c->L.wbin);
  w.ll = c->at<double>(c->L.ll);
  w.tgt = c->at<double>(c->L.tgt);
  const bool keep = keeps_weights(&c->cfg);
  w.lw = keep ? c->at<double>(c->L.lw) : nullptr;
  w.tuni = keep ? c->at<int32_t>(c->L.tuni) : nullptr;
  return w;
}

uint32_t grid_stride_blocks(const pcsir_ctx *c, uint32_t work, uint32_t per_block) {
  const uint32_t need = (work + per_block - 1) / per_block;
  const uint32_t cap = (uint32_t)c->num_cus * (uint32_t)c->tune.grid_per_cu;
  return std::max(1u, std::min(need, cap));
}

template <int DIM, bool SIR, bool SEP>
void launch_lik(pcsir_ctx *c, const LikInput &in, hipStream_t st) {
  const uint32_t grid = grid_stride_blocks(c, c->p.NT, LIK_WAVES);
  const uint64_t *meta = c->at<uint64_t>(c->L.meta);
  double *ll = c->at<double>(c->L.ll);
  const StepDesc *desc = c->at<StepDesc>(c->L.desc);
  if (SEP) {
    // the common window (15 x 15 pixels, 8 x 8 sub-samples) with constant loop counts
    if (c->p.P == 15 && c->p.q == 8)
      k_lik<DIM, SIR, true, 8, LIK_ALL, 15><<<grid, TPB, 0, st>>>(c->p, in, meta, desc, ll);
    else
      k_lik<DIM, SIR, true, 0><<<grid, TPB, 0, st>>>(c->p, in, meta, desc, ll);
    return;
  }
  switch (c->p.q) {
    case 2: k_lik<DIM, SIR, false, 2><<<grid, TPB, 0, st>>>(c->p, in, meta, desc, ll); break;
    case 4: k_lik<DIM, SIR, false, 4><<<grid, TPB, 0, st>>>(c->p, in, meta, desc, ll); break;
    case 8: k_lik<DIM, SIR, false, 8><<<grid, TPB, 0, st>>>(c->p, in, meta, desc, ll); break;
    default: k_lik<DIM, SIR, false, 0><<<grid, TPB, 0, st>>>(c->p, in, meta, desc, ll); break;
  }
}

SurrWeights surr_weights(const pcsir_ctx *c) { return surr_view(c->at<char>(c->L.surr)); }

// Surrogate log-likelihood of every dummy, then the exact check of a random
// share of dummies and the exact recomputation of targets that failed it.
template <int DIM>
void launch_surrogate(pcsir_ctx *c, const LikInput &in, hipStream_t st) {
  const Layout &L = c->L;
  DummyView dv;
  dv.dpix = in.dpix;
  dv.doff = in.doff;
  dv.dvel = c->at<float>(L.dvel);
  dv.dint = in.dint;
  dv.seg_t = in.seg_t;
  const uint64_t *meta = c->at<uint64_t>(L.meta);
  const StepDesc *desc = c->at<StepDesc>(L.desc);
  double *ll = c->at<double>(L.ll);
  const bool fp8 = c->cfg.lik_mode == PCSIR_LIK_SURR_FP8;
  const uint32_t grid = grid_stride_blocks(c, c->p.NT, SURR_ROWS);
  unsigned long long *tmax = c->at<unsigned long long>(L.tmax);
  k_clear_u64<<<(c->p.T + TPB - 1) / TPB, TPB, 0, st>>>(tmax, (uint32_t)c->p.T);
  if (c->cfg.lik_mode == PCSIR_LIK_SURR_FP8)
    if (c->p.P == 15)
      k_surr_infer<DIM, true, 15><<<grid, SURR_TPB, 0, st>>>(c->p, dv, meta, desc, surr_weights(c), ll, tmax);
    else
      k_surr_infer<DIM, true><<<grid, SURR_TPB, 0, st>>>(c->p, dv, meta, desc, surr_weights(c), ll, tmax);
  else
    if (c->p.P == 15)
      k_surr_infer<DIM, false, 15><<<grid, SURR_TPB, 0, st>>>(c->p, dv, meta, desc, surr_weights(c), ll, tmax);
    else
      k_surr_infer<DIM, false><<<grid, SURR_TPB, 0, st>>>(c->p, dv, meta, desc, surr_weights(c), ll, tmax);
  // exact check of the picked dummies, then exact recomputation of the targets
  // that failed it; the lists reuse the sort buffers, free at this point
  uint32_t *list_chk = c->at<uint32_t>(L.kA), *list_fb = c->at<uint32_t>(L.kB);
  uint64_t *meta_w = c->at<uint64_t>(L.meta);
  int32_t *tfb = c->at<int32_t>(L.tfb);
  // list kernels: about two workgroups per compute unit, each flushing its
  // staged list once or a few times
  const uint32_t pg = std::min(grid_stride_blocks(c, c->p.NT, TPB), 2u * (uint32_t)c->num_cus);
  SurrCheck chk;
  chk.fraction = c->surr_fraction;
  chk.tol = c->surr_tol;
  chk.tfallback = tfb;
  chk.list = list_chk;
  chk.tmax = tmax;
  chk.err = (float *)c->at<double>(L.wbin);  // bin weights are formed after the check
  chk.tsse = c->at<unsigned long long>(L.tsse);
  chk.tcnt = c->at<unsigned int>(L.tcnt);
  const uint32_t lg = grid_stride_blocks(c, c->p.NT, LIK_WAVES);
  const Params &p = c->p;
  mark(c, "surr_check");
  k_surr_pick<<<pg, TPB, 0, st>>>(p, meta, desc, in.seg_t, c->surr_fraction, list_chk, meta_w + META_NCHK);
  const bool common = p.P == 15 && p.q == 8;  // the window compiled with constant loop counts
  if (common)
    k_lik<DIM, false, true, 8, LIK_CHECK, 15><<<lg, TPB, 0, st>>>(p, in, meta, desc, ll, chk, meta_w);
  else
    k_lik<DIM, false, true, 0, LIK_CHECK><<<lg, TPB, 0, st>>>(p, in, meta, desc, ll, chk, meta_w);
  k_surr_stats<<<1, TPB, 0, st>>>(chk.err, meta_w);
  k_surr_decide<<<(p.T + TPB - 1) / TPB, TPB, 0, st>>>(p.T, chk.tol, chk.tsse, chk.tcnt, tfb);
  mark(c, "surr_fallback");
  k_surr_fallback_list<<<pg, TPB, 0, st>>>(meta, in.seg_t, tfb, list_fb, meta_w + META_NFB);
  chk.list = list_fb;
  if (common)
    k_lik<DIM, false, true, 8, LIK_FALLBACK, 15><<<lg, TPB, 0, st>>>(p, in, meta, desc, ll, chk, meta_w);
  else
    k_lik<DIM, false, true, 0, LIK_FALLBACK><<<lg, TPB, 0, st>>>(p, in, meta, desc, ll, chk, meta_w);
}

template <int DIM, bool SEP>
void launch_pcsir(pcsir_ctx *c, hipStream_t st) {
  const Layout &L = c->L;
  const Params &p = c->p;
  const StepDesc *desc = c->at<StepDesc>(L.desc);
  const Tile *t256 = c->at<Tile>(L.tiles256);
  const Tile *tS = c->at<Tile>(L.tilesS);
  const uint32_t *off = c->at<uint32_t>(L.off);
  float *sin = c->state(c->cur);
  float *sout = c->state(1 - c->cur);
  uint32_t *anc = c->at<uint32_t>(L.anc);
  uint64_t *meta = c->at<uint64_t>(L.meta);
  // bins numbered by the radix sort of the distinct keys, or (default) from the occupancy bitmap
  const bool sort_bins = c->tune.sort_bins != 0;
  BmWord *bm = sort_bins ? nullptr : c->at<BmWord>(L.bm);

  const bool keep = keeps_weights(&c->cfg);
  int32_t *tuni = keep ? c->at<int32_t>(L.tuni) : nullptr;
  double *wacc = keep ? c->at<double>(L.wacc) : nullptr;
  // the previous frame's resampling decisions become this frame's
  if (keep) k_copy_i32<<<(p.T + TPB - 1) / TPB, TPB, 0, st>>>(tuni, c->at<int32_t>(L.tuni_next), (uint32_t)p.T);
  mark(c, "propagate");
  k_propagate<DIM, true><<<(L.n256 + PROP_TILES - 1) / PROP_TILES, TPB, 0, st>>>(
      p, t256, L.n256, off, sin, sout, anc, c->pending, desc, c->at<float>(L.bbox_part), c->at<double>(L.mom_part),
      c->at<unsigned long long>(L.acc), meta, c->at<BmWord>(L.bm));
  mark(c, "bbox");
  k_bbox_reduce<<<p.T, TPB, 0, st>>>(p, c->at<uint32_t>(L.t256_first), off, c->at<float>(L.bbox_part),
                                     c->at<double>(L.mom_part), c->at<int32_t>(L.tm), c->at<int32_t>(L.bbox_cur),
                                     c->at<unsigned long long>(L.range), c->at<int32_t>(L.tfb),
                                     c->at<uint32_t>(L.kbase), meta, sort_bins ? c->tune.digit_bits : 0);
  mark(c, "keys");
  // distinct keys per tile: their bits in the occupancy bitmap, or into the
  // tile's own range of kA, then packed into key (the sort's input)
  k_keys<DIM><<<L.nK, KEYS_TPB, 0, st>>>(p, c->at<BinTile>(L.tilesK), off, sout, c->at<int32_t>(L.bbox_cur),
                                         c->at<uint32_t>(L.kbase), c->at<uint32_t>(L.kA), c->at<uint32_t>(L.tcount),
                                         meta, bm);
  const uint32_t G = std::min<uint32_t>(L.G, (uint32_t)c->tune.list_blocks);
  uint32_t *chunk = c->at<uint32_t>(L.chunk_heads);
  unsigned long long *acc = c->at<unsigned long long>(L.acc);
  if (sort_bins) {
    k_list_compact<<<L.nK, TPB, 0, st>>>(c->at<BinTile>(L.tilesK), off, c->at<uint32_t>(L.tcount), L.nK, meta,
                                          c->at<uint32_t>(L.kA), c->at<uint32_t>(L.key));
    SortBufs sb = sort_bufs(c);
    uint32_t *hist = c->at<uint32_t>(L.hist);
    uint32_t *dtot = c->at<uint32_t>(L.dtot);
    const int max_passes = (32 + c->tune.digit_bits - 1) / c->tune.digit_bits;
    for (int pass = 0; pass < max_passes; ++pass) {
      const uint32_t *kin = pass == 0 ? sb.key_store : ((pass & 1) ? sb.kB : sb.kA);
      uint32_t *kout = (uint32_t *)((pass & 1) ? sb.kA : sb.kB);
      mark(c, "sort_hist");
      k_sort_hist<<<G, TPB, 0, st>>>(pass, kin, hist, G, meta);
      mark(c, "sort_scan");
      k_sort_scan<<<MAX_BUCKETS, TPB, 0, st>>>(pass, hist, G, dtot, meta);
      mark(c, "sort_scatter");
      k_sort_scatter<<<G, TPB, 0, st>>>(pass, kin, kout, hist, G, dtot, meta);
    }
    mark(c, "seg_count");
    k_seg_count<<<G, TPB, 0, st>>>(G, p.T, sb, meta, chunk, c->at<uint32_t>(L.seg_first));
    mark(c, "seg_mark");
    k_seg_mark<<<G, TPB, 0, st>>>(p, G, sb, meta, chunk, c->at<uint32_t>(L.kbase), c->at<uint32_t>(L.seg_key),
                                    c->at<int32_t>(L.seg_t), c->at<uint32_t>(L.lut), L.lut_cap,
                                    c->at<uint32_t>(L.seg_first));
  } else {
    // as many workgroups as the list passes may have: most take one round of TPB words
    mark(c, "map_count");
    k_map_count<<<L.G, TPB, 0, st>>>(L.G, bm, meta, chunk);
    mark(c, "map_rank");
    k_map_rank<<<L.G, TPB, 0, st>>>(p, L.G, meta, chunk, c->at<uint32_t>(L.kbase), bm,
                                    c->at<uint32_t>(L.seg_key), c->at<int32_t>(L.seg_t),
                                    c->at<uint32_t>(L.seg_first));
  }
  mark(c, "bin_sums");
  if constexpr (DIM == 2) {
    if (c->cfg.dummy_mode == PCSIR_DUMMY_COM2)
      k_bin_sums<DIM, true><<<c->nB, BinLds<DIM, true>::NTH, 0, st>>>(p, c->at<BinTile>(L.tilesB), off, sout, c->at<int32_t>(L.bbox_cur),
                                        c->at<uint32_t>(L.kbase), c->at<uint32_t>(L.seg_key),
                                        c->at<uint32_t>(L.seg_first), acc, c->at<uint32_t>(L.segid), meta,
                                        c->at<uint32_t>(L.lut), L.lut_cap, bm);
    else
      k_bin_sums<DIM><<<c->nB, BinLds<DIM>::NTH, 0, st>>>(p, c->at<BinTile>(L.tilesB), off, sout, c->at<int32_t>(L.bbox_cur),
                                        c->at<uint32_t>(L.kbase), c->at<uint32_t>(L.seg_key),
                                        c->at<uint32_t>(L.seg_first), acc, c->at<uint32_t>(L.segid), meta,
                                        c->at<uint32_t>(L.lut), L.lut_cap, bm);
  } else {
    k_bin_sums<DIM><<<c->nB, BinLds<DIM>::NTH, 0, st>>>(p, c->at<BinTile>(L.tilesB), off, sout, c->at<int32_t>(L.bbox_cur),
                                        c->at<uint32_t>(L.kbase), c->at<uint32_t>(L.seg_key),
                                        c->at<uint32_t>(L.seg_first), acc, c->at<uint32_t>(L.segid), meta,
                                        c->at<uint32_t>(L.lut), L.lut_cap, bm);
  }
  if (keep) {
    mark(c, "bin_wsums");
    k_wsum_clear<<<grid_stride_blocks(c, p.NT, TPB), TPB, 0, st>>>(p.NT, p.D, meta, wacc);
    k_bin_wmax<<<L.n256, TPB, 0, st>>>(p, t256, off, c->at<uint32_t>(L.segid), c->at<double>(L.lw), tuni, wacc);
    k_bin_wsums<DIM><<<L.n256, TPB, 0, st>>>(p, t256, off, sout, c->at<uint32_t>(L.segid), c->at<double>(L.lw),
                                             tuni, wacc);
  }
  mark(c, "dummy");
  k_dummy<DIM><<<grid_stride_blocks(c, p.NT, TPB), TPB, 0, st>>>(
      p, meta, acc, c->at<uint32_t>(L.seg_key), c->at<int32_t>(L.seg_t), c->at<uint32_t>(L.kbase),
      c->at<int32_t>(L.bbox_cur), c->at<int32_t>(L.dpix), c->at<float>(L.doff), c->at<float>(L.dint),
      c->at<float>(L.dlo), c->at<float>(L.dvel), wacc, tuni);
  LikInput in;
  in.dpix = c->at<int32_t>(L.dpix);
  in.doff = c->at<float>(L.doff);
  in.dint = c->at<float>(L.dint);
  in.dlo = c->at<float>(L.dlo);
  in.seg_t = c->at<int32_t>(L.seg_t);
  in.state = sout;
  in.off = off;
  mark(c, "likelihood");
  if (c->cfg.lik_mode >= PCSIR_LIK_SURR_BF16) {
    launch_surrogate<DIM>(c, in, st);
  } else {
    if (c->cfg.dummy_mode == PCSIR_DUMMY_COM2) {
      // nine shifted evaluations per dummy, then the second-order combination
      const uint32_t grid = grid_stride_blocks(c, 9 * p.NT, LIK_WAVES);
      double *ll9 = c->at<double>(L.ll9);
      if (SEP)
        k_lik<DIM, false, true, 0, LIK_STENCIL><<<grid, TPB, 0, st>>>(p, in, meta, desc, ll9);
      else
        k_lik<DIM, false, false, 0, LIK_STENCIL><<<grid, TPB, 0, st>>>(p, in, meta, desc, ll9);
      k_second_order<<<grid_stride_blocks(c, p.NT, TPB), TPB, 0, st>>>(p, meta, acc, in.seg_t, ll9,
                                                                      c->at<double>(L.ll));
    } else {
      launch_lik<DIM, false, SEP>(c, in, st);
    }
  }
  mark(c, "normalise");
  WeightSrc ws = weight_src(c);
  const int32_t *tfb = c->cfg.lik_mode >= PCSIR_LIK_SURR_BF16 ? c->at<int32_t>(L.tfb) : nullptr;
  if (keep) {
    // kept weights differ within a bin: normalise over the particles
    k_norm_part<DIM, false><<<L.nS, TPB, 0, st>>>(p, tS, off, ws, sout, c->at<double>(L.part));
    k_norm_comb<DIM><<<p.T, TPB, 0, st>>>(p, c->at<uint32_t>(L.tfirst), c->at<double>(L.part), desc,
                                          c->at<double>(L.tgt), c->at<double>(L.est), c->at<int32_t>(L.tflag), meta,
                                          tfb);
  } else {
    k_norm_bins<DIM><<<p.T, TPB, 0, st>>>(p, c->at<uint32_t>(L.seg_first), c->at<double>(L.ll), acc,
                                          c->at<int32_t>(L.dpix), desc, c->at<double>(L.wbin), c->at<double>(L.tgt),
                                          c->at<double>(L.est), c->at<int32_t>(L.tflag), meta, tfb);
  }
  mark(c, "cdf_sum");
  k_cdf_sum<false><<<(L.nS + CDF_SUM_TILES - 1) / CDF_SUM_TILES, TPB, 0, st>>>(tS, L.nS, off, ws,
                                                                             c->at<double>(L.tile_sum));
  mark(c, "cdf_prefix");
  k_cdf_prefix<<<p.T, TPB, 0, st>>>(c->at<uint32_t>(L.tfirst), c->at<double>(L.tile_sum),
                                    c->at<double>(L.tile_pre), c->at<uint32_t>(L.rs_count));
  mark(c, "cdf_scan");
  k_cdf_scan<false, false><<<L.nS, TPB, 0, st>>>(tS, c->at<uint32_t>(L.tile_last), ws, c->at<double>(L.tile_pre),
                                                 c->at<int32_t>(L.tflag), anc, c->at<double>(L.cdf), c->cfg.neff_threshold,
                                                 keep ? c->at<int32_t>(L.tuni_next) : nullptr, c->at<uint32_t>(L.tfirstR),
                                                 c->at<uint2>(L.rs_work), c->at<uint32_t>(L.rs_count), L.nW,
                                                 (uint32_t)c->tune.resample_light);
  mark(c, "resample");
  k_resample_search<false><<<std::min<uint32_t>(L.nW, RS_SEARCH_BLOCKS), TPB, 0, st>>>(
      c->at<Tile>(L.tilesR), tS, ws, c->at<double>(L.cdf), c->at<double>(L.tile_pre), c->at<uint32_t>(L.tile_last),
      c->at<uint2>(L.rs_work), c->at<uint32_t>(L.rs_count), L.nW, anc);
  mark(c, "end");
}

template <int DIM, bool SEP>
void launch_sir(pcsir_ctx *c, hipStream_t st) {
  const Layout &L = c->L;
  const Params &p = c->p;
  const StepDesc *desc = c->at<StepDesc>(L.desc);
  const Tile *t256 = c->at<Tile>(L.tiles256);
  const Tile *tS = c->at<Tile>(L.tilesS);
  const uint32_t *off = c->at<uint32_t>(L.off);
  float *sin = c->state(c->cur);
  float *sout = c->state(1 - c->cur);
  uint32_t *anc = c->at<uint32_t>(L.anc);
  uint64_t *meta = c->at<uint64_t>(L.meta);
  const bool keep = keeps_weights(&c->cfg);
  if (keep)
    k_copy_i32<<<(p.T + TPB - 1) / TPB, TPB, 0, st>>>(c->at<int32_t>(L.tuni), c->at<int32_t>(L.tuni_next),
                                                      (uint32_t)p.T);
  mark(c, "propagate");
  k_propagate<DIM, false><<<(L.n256 + PROP_TILES - 1) / PROP_TILES, TPB, 0, st>>>(
      p, t256, L.n256, off, sin, sout, anc, c->pending, desc, nullptr, nullptr, nullptr, meta, nullptr);
  LikInput in;
  memset(&in, 0, sizeof(in));
  in.state = sout;
  in.off = off;
  mark(c, "likelihood");
  launch_lik<DIM, true, SEP>(c, in, st);
  WeightSrc ws = weight_src(c);
  mark(c, "normalise");
  k_norm_part<DIM, true><<<L.nS, TPB, 0, st>>>(p, tS, off, ws, sout, c->at<double>(L.part));
  k_norm_comb<DIM><<<p.T, TPB, 0, st>>>(p, c->at<uint32_t>(L.tfirst), c->at<double>(L.part), desc,
                                        c->at<double>(L.tgt), c->at<double>(L.est), c->at<int32_t>(L.tflag), meta,
                                        nullptr);
  mark(c, "cdf_sum");
  k_cdf_sum<true><<<(L.nS + CDF_SUM_TILES - 1) / CDF_SUM_TILES, TPB, 0, st>>>(tS, L.nS, off, ws,
                                                                             c->at<double>(L.tile_sum));
  mark(c, "cdf_prefix");
  k_cdf_prefix<<<p.T, TPB, 0, st>>>(c->at<uint32_t>(L.tfirst), c->at<double>(L.tile_sum),
                                    c->at<double>(L.tile_pre), c->at<uint32_t>(L.rs_count));
  mark(c, "cdf_scan");
  k_cdf_scan<true, false><<<L.nS, TPB, 0, st>>>(tS, c->at<uint32_t>(L.tile_last), ws, c->at<double>(L.tile_pre),
                                                 c->at<int32_t>(L.tflag), anc, c->at<double>(L.cdf), c->cfg.neff_threshold,
                                                 keep ? c->at<int32_t>(L.tuni_next) : nullptr, c->at<uint32_t>(L.tfirstR),
                                                 c->at<uint2>(L.rs_work), c->at<uint32_t>(L.rs_count), L.nW,
                                                 (uint32_t)c->tune.resample_light);
  mark(c, "resample");
  k_resample_search<true><<<std::min<uint32_t>(L.nW, RS_SEARCH_BLOCKS), TPB, 0, st>>>(
      c->at<Tile>(L.tilesR), tS, ws, c->at<double>(L.cdf), c->at<double>(L.tile_pre), c->at<uint32_t>(L.tile_last),
      c->at<uint2>(L.rs_work), c->at<uint32_t>(L.rs_count), L.nW, anc);
  mark(c, "end");
}

void launch_step(pcsir_ctx *c, bool sir, hipStream_t st) {
  // the surrogate modes' exact evaluations (sir_step, check, fallback) use the separable form
  const bool sep = c->cfg.lik_mode != PCSIR_LIK_DIRECT;
  if (sir) {
    if (c->cfg.dim == 2) sep ? launch_sir<2, true>(c, st) : launch_sir<2, false>(c, st);
    else sep ? launch_sir<3, true>(c, st) : launch_sir<3, false>(c, st);
  } else {
    if (c->cfg.dim == 2) sep ? launch_pcsir<2, true>(c, st) : launch_pcsir<2, false>(c, st);
    else sep ? launch_pcsir<3, true>(c, st) : launch_pcsir<3, false>(c, st);
  }
}

// Capture the kernel sequence of one step for the current (kind, buffer
// parity, pending gather) once, on a private stream, and keep the executable.
pcsir_status step_graph(pcsir_ctx *c, bool sir, hipGraphExec_t *out) {
  hipGraphExec_t &ex = c->gexec[sir ? 1 : 0][c->cur][c->pending];
  if (ex) {
    *out = ex;
    return PCSIR_OK;
  }
  hipError_t e = hipSuccess;
  if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return check_hip(c, e, "hipStreamCreate");
  e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return check_hip(c, e, "hipStreamBeginCapture");
  launch_step(c, sir, c->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t el = hipGetLastError();
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (el != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return check_hip(c, el, "kernel launch during capture");
  }
  if (e != hipSuccess) return check_hip(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ex = nullptr;
    return check_hip(c, e, "hipGraphInstantiate");
  }
  *out = ex;
  return PCSIR_OK;
}

pcsir_status run_step(pcsir_ctx *c, const float *frame, int32_t H, int32_t W, int64_t k, bool sir) {
  if (!c) return PCSIR_E_INVAL;
  if (!frame) return fail(c, PCSIR_E_INVAL, "frame_dev is NULL");
  if (H != c->cfg.frame_h || W != c->cfg.frame_w) return fail(c, PCSIR_E_STATE, "frame size differs from the config");
  if (k < 1) return fail(c, PCSIR_E_INVAL, "frame index k must be >= 1");
  if (!sir && c->cfg.lik_mode >= PCSIR_LIK_SURR_BF16 && !c->surr_ready)
    return fail(c, PCSIR_E_STATE, "surrogate mode: call pcsir_set_surrogate before the first step");
  k_set_desc<<<1, 1, 0, c->stream>>>(c->at<StepDesc>(c->L.desc), frame, k);
  if (c->use_graphs && !c->timing) {
    hipGraphExec_t ex = nullptr;
    const pcsir_status s = step_graph(c, sir, &ex);
    if (s != PCSIR_OK) return s;
    const hipError_t e = hipGraphLaunch(ex, c->stream);
    if (e != hipSuccess) return check_hip(c, e, "hipGraphLaunch");
  } else {
    launch_step(c, sir, c->stream);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return check_hip(c, e, "kernel launch");
  c->cur = 1 - c->cur;
  c->pending = 1;
  c->stepped = 1;
  c->last_sir = sir ? 1 : 0;
  return PCSIR_OK;
}

void drop_graphs(pcsir_ctx *c) {
  (void)hipStreamSynchronize(c->stream);
  for (auto &a : c->gexec)
    for (auto &b : a)
      for (auto &x : b)
        if (x) {
          (void)hipGraphExecDestroy(x);
          x = nullptr;
        }
}

// Inference copy of the surrogate's weights (layout of surr_view) from the
// FP32 parameter vector, plus the FP8 input scales of the three layers.
hipError_t surr_prepare(const float *params, const float *act_scale_host, char *block, hipStream_t st) {
  float *sw = (float *)(block + SURR_OFF_SW);
  k_surr_scales<<<3, 256, 0, st>>>(params, sw);
  k_surr_prep<<<768, 256, 0, st>>>(params, sw, (uint16_t *)(block + SURR_OFF_WT), (uint8_t *)(block + SURR_OFF_WT8),
                                   (float *)(block + SURR_OFF_BIAS), (float *)(block + SURR_OFF_W4),
                                   (float *)(block + SURR_OFF_B4));
  hipError_t e = hipGetLastError();
  const float one[3] = {1.0f, 1.0f, 1.0f};
  if (e == hipSuccess)
    e = hipMemcpyAsync(block + SURR_OFF_SX, act_scale_host ? act_scale_host : one, sizeof one, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host scales are read before returning
  return e;
}

bool valid_act_scales(const float *s) {
  if (!s) return true;
  for (int l = 0; l < 3; ++l)
    if (!(s[l] > 0.0f) || !std::isfinite(s[l])) return false;
  return true;
}

// Uniform weights for every target (kept-weight mode): the next step starts
// from the resampled state.
hipError_t reset_weights(pcsir_ctx *c) {
  if (!keeps_weights(&c->cfg)) return hipSuccess;
  const uint32_t T = (uint32_t)c->cfg.n_targets;
  k_fill_i32<<<(T + TPB - 1) / TPB, TPB, 0, c->stream>>>(c->at<int32_t>(c->L.tuni_next), 1, T);
  k_fill_i32<<<(T + TPB - 1) / TPB, TPB, 0, c->stream>>>(c->at<int32_t>(c->L.tuni), 1, T);
  return hipGetLastError();
}

pcsir_status pull_device_status(pcsir_ctx *c) {
  uint64_t meta[META_N];
  hipError_t e = hipMemcpyAsync(meta, c->at<uint64_t>(c->L.meta), sizeof(meta), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "device status");
  if (meta[META_ERR]) {
    std::string m = "device condition:";
    if (meta[META_ERR] & ERR_KEY_RANGE) m += " cell range of all targets exceeds 2^32 cells (clouds spread too far for these bins);";
    if (meta[META_ERR] & ERR_FIXED_SAT) m += " a velocity (|v| >= 128) or intensity (|I| >= 32768) left the bin-sum range;";
    if (meta[META_ERR] & ERR_NONFINITE) m += " a target's normalisation was not finite (its particles were kept, not resampled);";
    uint64_t zero = 0;
    (void)hipMemcpyAsync(c->at<uint64_t>(c->L.meta) + META_ERR, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    return fail(c, PCSIR_E_NUMERIC, m);
  }
  return PCSIR_OK;
}

}  // namespace

extern "C" {

size_t pcsir_workspace_bytes(const pcsir_config *cfg) {
  if (!valid_config(cfg, nullptr)) return 0;
  Tables tb;
  build_tables(cfg, tb);
  return plan(cfg, tb).total;
}

pcsir_status pcsir_init(const pcsir_config *cfg, const float *init_state_dev, void *workspace_dev,
                        size_t workspace_bytes, void *hip_stream, pcsir_ctx **out) {
  if (!out) return PCSIR_E_INVAL;
  *out = nullptr;
  std::string why;
  if (!valid_config(cfg, &why)) {
    fprintf(stderr, "pcsir_init: invalid config: %s\n", why.c_str());
    return PCSIR_E_INVAL;
  }
  if (!init_state_dev || !workspace_dev) return PCSIR_E_INVAL;
  if (((uintptr_t)workspace_dev) % ALIGN) return PCSIR_E_INVAL;
  pcsir_ctx *c = new pcsir_ctx();
  c->cfg = *cfg;
  c->n.assign(cfg->n_particles, cfg->n_particles + cfg->n_targets);
  c->cfg.n_particles = c->n.data();
  build_tables(&c->cfg, c->tb);
  c->L = plan(&c->cfg, c->tb);
  if (workspace_bytes < c->L.total) {
    delete c;
    return PCSIR_E_NOMEM;
  }
  c->ws = (char *)workspace_dev;
  c->stream = (hipStream_t)hip_stream;
  c->NT = c->tb.off.back();
  c->nB = (uint32_t)c->tb.tB.size();
  c->p = make_params(&c->cfg, c->NT);
  c->p.bbox_cur = c->at<int32_t>(c->L.bbox_cur);
  c->p.tm = c->at<int32_t>(c->L.tm);
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      c->num_cus = cus;
  }
  const Layout &L = c->L;
  const int T = c->cfg.n_targets;
  const int D = 2 * c->cfg.dim + 1;
  hipError_t e = hipSuccess;
  auto h2d = [&](size_t off, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  h2d(L.tiles256, c->tb.t256.data(), sizeof(Tile) * c->tb.t256.size());
  h2d(L.tilesS, c->tb.tS.data(), sizeof(Tile) * c->tb.tS.size());
  h2d(L.tilesR, c->tb.tR.data(), sizeof(Tile) * c->tb.tR.size());
  h2d(L.tfirstR, c->tb.tfirstR.data(), 4 * c->tb.tfirstR.size());
  h2d(L.tilesB, c->tb.tB.data(), sizeof(BinTile) * c->tb.tB.size());
  h2d(L.tilesK, c->tb.tK.data(), sizeof(BinTile) * c->tb.tK.size());
  h2d(L.tile_last, c->tb.tile_last.data(), 4 * c->tb.tile_last.size());
  h2d(L.tfirst, c->tb.tfirst.data(), 4 * c->tb.tfirst.size());
  h2d(L.off, c->tb.off.data(), 4 * c->tb.off.size());
  h2d(L.t256_first, c->tb.t256_first.data(), 4 * c->tb.t256_first.size());
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.meta, 0, 8 * META_N, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.tflag, 0, 4 * (size_t)T, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.tsse, 0, 8 * (size_t)T, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.tcnt, 0, 4 * (size_t)T, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.acc, 0, 8 * (size_t)c->p.acc_rows * c->NT, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.bm, 0, sizeof(BmWord) * BM_WORDS, c->stream);  // each step clears what it set
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->state(0), init_state_dev, 4 * (size_t)D * c->NT, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) {
    k_identity<<<L.n256, TPB, 0, c->stream>>>(c->at<Tile>(L.tiles256), c->at<uint32_t>(L.off), c->at<uint32_t>(L.anc));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = reset_weights(c);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    fprintf(stderr, "pcsir_init: %s\n", hipGetErrorString(e));
    delete c;
    return PCSIR_E_HIP;
  }
  *out = c;
  return PCSIR_OK;
}

pcsir_status pcsir_step(pcsir_ctx *ctx, const float *frame_dev, int32_t H, int32_t W, int64_t k) {
  return run_step(ctx, frame_dev, H, W, k, false);
}

pcsir_status sir_step(pcsir_ctx *ctx, const float *frame_dev, int32_t H, int32_t W, int64_t k) {
  return run_step(ctx, frame_dev, H, W, k, true);
}

pcsir_status pcsir_estimate(pcsir_ctx *c, double *est_host, double *neff_host) {
  if (!c || !est_host) return PCSIR_E_INVAL;
  if (!c->stepped) return fail(c, PCSIR_E_STATE, "no step has run since init or set_particles");
  const int T = c->cfg.n_targets, D = 2 * c->cfg.dim + 1;
  hipError_t e = hipMemcpyAsync(est_host, c->at<double>(c->L.est), 8 * (size_t)T * D, hipMemcpyDeviceToHost, c->stream);
  std::vector<double> tg;
  if (neff_host) {
    tg.resize(4 * (size_t)T);
    if (e == hipSuccess) e = hipMemcpyAsync(tg.data(), c->at<double>(c->L.tgt), 8 * tg.size(), hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pcsir_estimate");
  if (neff_host)
    for (int t = 0; t < T; ++t) neff_host[t] = tg[4 * (size_t)t + 2];
  return pull_device_status(c);
}

pcsir_status pcsir_destroy(pcsir_ctx *c) {
  if (!c) return PCSIR_E_INVAL;
  pcsir_status s = PCSIR_OK;
  const hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) s = PCSIR_E_HIP;
  else s = pull_device_status(c);
  for (hipEvent_t ev : c->ev) (void)hipEventDestroy(ev);
  for (auto &a : c->gexec)
    for (auto &b : a)
      for (auto &x : b)
        if (x) (void)hipGraphExecDestroy(x);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return s;
}

const char *pcsir_last_error(const pcsir_ctx *c) { return c ? c->err.c_str() : "context is NULL"; }

pcsir_status pcsir_get_particles(pcsir_ctx *c, float *dst_dev) {
  if (!c || !dst_dev) return PCSIR_E_INVAL;
  k_gather<<<c->L.n256, TPB, 0, c->stream>>>(c->p.D, c->NT, c->at<Tile>(c->L.tiles256), c->at<uint32_t>(c->L.off),
                                             c->state(c->cur), c->at<uint32_t>(c->L.anc), c->pending, dst_dev);
  return check_hip(c, hipGetLastError(), "pcsir_get_particles");
}

pcsir_status pcsir_set_particles(pcsir_ctx *c, const float *src_dev) {
  if (!c || !src_dev) return PCSIR_E_INVAL;
  hipError_t e = hipMemcpyAsync(c->state(c->cur), src_dev, 4 * (size_t)c->p.D * c->NT, hipMemcpyDeviceToDevice,
                                c->stream);
  if (e == hipSuccess) e = reset_weights(c);
  c->pending = 0;
  c->stepped = 0;
  return check_hip(c, e, "pcsir_set_particles");
}

pcsir_status pcsir_set_graphs(pcsir_ctx *c, int32_t on) {
  if (!c) return PCSIR_E_INVAL;
  c->use_graphs = on ? 1 : 0;
  return PCSIR_OK;
}

pcsir_status pcsir_set_debug(pcsir_ctx *c, int32_t on) {
  if (!c) return PCSIR_E_INVAL;
  c->debug = on ? 1 : 0;
  return PCSIR_OK;
}

pcsir_status pcsir_debug_dump(pcsir_ctx *c, int32_t what, void *dst, size_t bytes) {
  if (!c || !dst) return PCSIR_E_INVAL;
  if (!c->stepped) return fail(c, PCSIR_E_STATE, "no step has run since init or set_particles");
  const size_t NT = c->NT, T = c->cfg.n_targets, D = c->p.D;
  const Layout &L = c->L;
  hipStream_t st = c->stream;
  // the propagated states of the last step sit in the current buffer
  const float *prop = c->state(c->cur);
  uint64_t B = 0;
  const bool keep = keeps_weights(&c->cfg);
  if (what >= PCSIR_DUMP_COUNTS && what <= PCSIR_DUMP_BIN_MEAN) {
    uint64_t meta[META_N];
    hipError_t e = hipMemcpyAsync(meta, c->at<uint64_t>(L.meta), sizeof(meta), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(c, e, "debug dump");
    B = c->last_sir ? NT : meta[META_B];
    if (what == PCSIR_DUMP_COUNTS) {
      if (bytes < 16) return fail(c, PCSIR_E_INVAL, "buffer too small");
      const int64_t v[3] = {(int64_t)B, (int64_t)(c->last_sir ? 0 : meta[META_PASSES]),
                            (int64_t)(c->last_sir ? 0 : meta[META_L])};
      return check_hip(c, hipMemcpy(dst, v, bytes >= 24 ? 24 : 16, hipMemcpyHostToDevice), "debug dump");
    }
    if (c->last_sir) return fail(c, PCSIR_E_STATE, "bins exist only after pcsir_step");
  }
  auto need = [&](size_t b) { return bytes >= b; };
  const uint32_t gb = grid_stride_blocks(c, (uint32_t)NT, TPB);
  hipError_t e = hipSuccess;
  switch (what) {
    case PCSIR_DUMP_PROPAGATED:
      if (!need(4 * D * NT)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      e = hipMemcpyAsync(dst, prop, 4 * D * NT, hipMemcpyDeviceToDevice, st);
      break;
    case PCSIR_DUMP_KEYS: {
      if (!need(4 * 3 * NT)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      // SIR: the pixel index (cells with m = 1) that centres each particle's window
      k_dbg_keys<<<L.n256, TPB, 0, st>>>(c->p.dim, (uint32_t)NT, c->at<Tile>(L.tiles256),
                                         c->last_sir ? nullptr : c->at<int32_t>(L.tm), prop, (int32_t *)dst);
      break;
    }
    case PCSIR_DUMP_BINS_PER_PX:
      if (c->last_sir) return fail(c, PCSIR_E_STATE, "bins exist only after pcsir_step");
      if (!need(4 * 3 * T)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      e = hipMemcpyAsync(dst, c->at<int32_t>(L.tm), 4 * 3 * T, hipMemcpyDeviceToDevice, st);
      break;
    case PCSIR_DUMP_BIN_TARGET:
    case PCSIR_DUMP_BIN_KEY:
    case PCSIR_DUMP_BIN_N:
    case PCSIR_DUMP_BIN_MEAN: {
      const size_t per = what == PCSIR_DUMP_BIN_TARGET ? 4 : what == PCSIR_DUMP_BIN_KEY ? 12
                         : what == PCSIR_DUMP_BIN_N ? 8 : 8 * D;
      if (!need(per * B)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      if (c->p.dim == 2)
        k_dbg_bins<2><<<gb, TPB, 0, st>>>(c->p, c->at<uint64_t>(L.meta), c->at<unsigned long long>(L.acc),
                                          c->at<uint32_t>(L.seg_key), c->at<uint32_t>(L.kbase),
                                          c->at<int32_t>(L.bbox_cur), what, dst, keep ? c->at<double>(L.wacc) : nullptr,
                                          keep ? c->at<int32_t>(L.tuni) : nullptr);
      else
        k_dbg_bins<3><<<gb, TPB, 0, st>>>(c->p, c->at<uint64_t>(L.meta), c->at<unsigned long long>(L.acc),
                                          c->at<uint32_t>(L.seg_key), c->at<uint32_t>(L.kbase),
                                          c->at<int32_t>(L.bbox_cur), what, dst, keep ? c->at<double>(L.wacc) : nullptr,
                                          keep ? c->at<int32_t>(L.tuni) : nullptr);
      break;
    }
    case PCSIR_DUMP_LOGLIK: {
      size_t n = NT;
      if (!c->last_sir) {
        uint64_t meta[META_N];
        e = hipMemcpyAsync(meta, c->at<uint64_t>(L.meta), sizeof(meta), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        n = meta[META_B];
      }
      if (!need(8 * n)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      if (e == hipSuccess) e = hipMemcpyAsync(dst, c->at<double>(L.ll), 8 * n, hipMemcpyDeviceToDevice, st);
      break;
    }
    case PCSIR_DUMP_WEIGHTS:
      if (!need(8 * NT)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      if (c->last_sir)
        k_dbg_weights<true><<<L.n256, TPB, 0, st>>>(c->at<Tile>(L.tiles256), c->at<uint32_t>(L.off), weight_src(c),
                                                    keep ? c->at<int32_t>(L.tuni_next) : nullptr, (double *)dst);
      else
        k_dbg_weights<false><<<L.n256, TPB, 0, st>>>(c->at<Tile>(L.tiles256), c->at<uint32_t>(L.off), weight_src(c),
                                                     keep ? c->at<int32_t>(L.tuni_next) : nullptr, (double *)dst);
      break;
    case PCSIR_DUMP_TARGET:
      if (!need(8 * 4 * T)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      e = hipMemcpyAsync(dst, c->at<double>(L.tgt), 8 * 4 * T, hipMemcpyDeviceToDevice, st);
      break;
    case PCSIR_DUMP_CDF:
      if (!c->debug) return fail(c, PCSIR_E_STATE, "the cumulative-weight view needs pcsir_set_debug(ctx, 1)");
      if (!need(8 * NT)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      // the step keeps C on chip where it can; the view forms every
      // resampling target's C again with the step's scan, from the same weights
      if (c->last_sir)
        k_cdf_scan<true, true><<<L.nS, TPB, 0, st>>>(c->at<Tile>(L.tilesS), c->at<uint32_t>(L.tile_last), weight_src(c),
                                                    c->at<double>(L.tile_pre), c->at<int32_t>(L.tflag), nullptr,
                                                    (double *)dst, c->cfg.neff_threshold, nullptr, nullptr, nullptr,
                                                    nullptr, 0u, 0u);
      else
        k_cdf_scan<false, true><<<L.nS, TPB, 0, st>>>(c->at<Tile>(L.tilesS), c->at<uint32_t>(L.tile_last), weight_src(c),
                                                     c->at<double>(L.tile_pre), c->at<int32_t>(L.tflag), nullptr,
                                                     (double *)dst, c->cfg.neff_threshold, nullptr, nullptr, nullptr,
                                                     nullptr, 0u, 0u);
      break;
    case PCSIR_DUMP_RESAMPLE:
      if (!need(4 * NT)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      e = hipMemcpyAsync(dst, c->at<uint32_t>(L.anc), 4 * NT, hipMemcpyDeviceToDevice, st);
      break;
    case PCSIR_DUMP_LOGW:
      if (!need(8 * NT)) return fail(c, PCSIR_E_INVAL, "buffer too small");
      k_dbg_logw<<<L.n256, TPB, 0, st>>>(c->at<Tile>(L.tiles256), c->at<uint32_t>(L.off),
                                         keep ? c->at<double>(L.lw) : nullptr,
                                         keep ? c->at<int32_t>(L.tuni_next) : nullptr, (double *)dst);
      break;
    default:
      return fail(c, PCSIR_E_INVAL, "unknown dump");
  }
  if (e != hipSuccess) return check_hip(c, e, "debug dump");
  return check_hip(c, hipGetLastError(), "debug dump");
}

pcsir_status pcsir_set_timing(pcsir_ctx *c, int32_t on) {
  if (!c) return PCSIR_E_INVAL;
  c->timing = on ? 1 : 0;
  if (c->timing && c->ev.empty()) {
    c->ev.resize(8192);
    c->ev_name.assign(8192, "");
    for (auto &ev : c->ev) {
      const hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return check_hip(c, e, "hipEventCreate");
    }
  }
  c->ev_used = 0;
  return PCSIR_OK;
}

pcsir_status pcsir_kernel_times(pcsir_ctx *c, const char **names, float *ms, int32_t cap, int32_t *count) {
  if (!c || !count) return PCSIR_E_INVAL;
  *count = 0;
  if (!c->timing || c->ev_used < 2) return PCSIR_OK;
  const hipError_t e = hipEventSynchronize(c->ev[c->ev_used - 1]);
  if (e != hipSuccess) return check_hip(c, e, "hipEventSynchronize");
  int n = 0;
  for (int i = 0; i + 1 < c->ev_used && n < cap; ++i) {
    if (strcmp(c->ev_name[i], "end") == 0) continue;  // gap between two steps
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, c->ev[i], c->ev[i + 1]);
    if (names) names[n] = c->ev_name[i];
    if (ms) ms[n] = t;
    ++n;
  }
  *count = n;
  c->ev_used = 0;
  return PCSIR_OK;
}

pcsir_status pcsir_get_tuning(const pcsir_ctx *c, pcsir_tuning *out) {
  if (!c || !out) return PCSIR_E_INVAL;
  *out = c->tune;
  return PCSIR_OK;
}

pcsir_status pcsir_set_tuning(pcsir_ctx *c, const pcsir_tuning *t) {
  if (!c || !t) return PCSIR_E_INVAL;
  if (t->bin_tile != 1024 && t->bin_tile != 2048 && t->bin_tile != BIN_TILE_MAX)
    return fail(c, PCSIR_E_INVAL, "bin_tile must be 1024, 2048 or 4096");
  if (t->list_blocks < 64 || t->list_blocks > LIST_BLOCKS_MAX)
    return fail(c, PCSIR_E_INVAL, "list_blocks must lie in [64, 2048]");
  if (t->digit_bits < MIN_DIGIT_BITS || t->digit_bits > MAX_DIGIT_BITS)
    return fail(c, PCSIR_E_INVAL, "digit_bits must lie in [6, 11]");
  if (t->grid_per_cu < 4 || t->grid_per_cu > 64) return fail(c, PCSIR_E_INVAL, "grid_per_cu must lie in [4, 64]");
  if (t->resample_light < 0 || t->resample_light > RS_LIGHT_MAX)
    return fail(c, PCSIR_E_INVAL, "resample_light must lie in [0, 4096]");
  if (t->sort_bins != 0 && t->sort_bins != 1) return fail(c, PCSIR_E_INVAL, "sort_bins must be 0 or 1");
  drop_graphs(c);  // captured graphs hold the launch shapes
  if (t->bin_tile != c->tune.bin_tile) {
    std::vector<BinTile> tB;
    build_bin_tiles(&c->cfg, (uint32_t)t->bin_tile, tB);
    hipError_t e = hipMemcpyAsync(c->ws + c->L.tilesB, tB.data(), sizeof(BinTile) * tB.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return check_hip(c, e, "pcsir_set_tuning");
    c->nB = (uint32_t)tB.size();
  }
  c->tune = *t;
  return PCSIR_OK;
}

pcsir_status pcsir_autotune(pcsir_ctx *c, const float *frame_dev, int32_t H, int32_t W, int64_t k, int32_t reps,
                            float *state_scratch_dev, pcsir_tuning *best_out, float *best_ms_out,
                            int32_t *trials_out) {
  if (!c) return PCSIR_E_INVAL;
  if (!frame_dev || !state_scratch_dev) return fail(c, PCSIR_E_INVAL, "frame_dev and state_scratch_dev are required");
  if (reps < 1) return fail(c, PCSIR_E_INVAL, "reps must be >= 1");
  if (k < 1) return fail(c, PCSIR_E_INVAL, "frame index k must be >= 1");
  pcsir_status s = pcsir_get_particles(c, state_scratch_dev);
  if (s != PCSIR_OK) return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return check_hip(c, e, "pcsir_autotune");
  int trials = 0;
  auto trial = [&](const pcsir_tuning &t, float *ms) -> pcsir_status {
    pcsir_status r = pcsir_set_tuning(c, &t);
    if (r == PCSIR_OK) r = pcsir_set_particles(c, state_scratch_dev);
    if (r == PCSIR_OK) r = run_step(c, frame_dev, H, W, k, false);  // untimed: graph capture
    if (r == PCSIR_OK) r = pcsir_set_particles(c, state_scratch_dev);
    if (r != PCSIR_OK) return r;
    hipError_t he = hipEventRecord(e0, c->stream);
    for (int i = 0; i < reps && r == PCSIR_OK; ++i) r = run_step(c, frame_dev, H, W, k + i, false);
    if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(ms, e0, e1);
    if (r != PCSIR_OK) return r;
    if (he != hipSuccess) return check_hip(c, he, "pcsir_autotune");
    *ms /= (float)reps;
    ++trials;
    return pull_device_status(c);
  };
  pcsir_tuning best = c->tune;
  float best_ms = 0.0f;
  s = trial(best, &best_ms);
  const int tiles[] = {1024, 2048, BIN_TILE_MAX}, blocks[] = {256, 512, 1024, 2048}, bits[] = {8, 9, 10, 11},
            grids[] = {8, 16, 32, 64}, lights[] = {1024, 2048, 4096}, numbering[] = {0, 1};
  // the bin numbering first, so that the list and sort shapes are tuned for the one chosen
  const int *cands[6] = {numbering, tiles, blocks, bits, grids, lights};
  const int ncand[6] = {2, 3, 4, 4, 4, 3};
  for (int f = 0; f < 6 && s == PCSIR_OK; ++f) {
    if ((f == 2 || f == 3) && !best.sort_bins) continue;  // list blocks and digit width only shape the sort
    for (int i = 0; i < ncand[f] && s == PCSIR_OK; ++i) {
      pcsir_tuning t = best;
      int32_t *field = f == 0 ? &t.sort_bins : f == 1 ? &t.bin_tile : f == 2 ? &t.list_blocks
                     : f == 3 ? &t.digit_bits : f == 4 ? &t.grid_per_cu : &t.resample_light;
      if (*field == cands[f][i]) continue;
      *field = cands[f][i];
      float ms = 0.0f;
      s = trial(t, &ms);
      if (s == PCSIR_OK && ms < best_ms) {
        best = t;
        best_ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != PCSIR_OK) return s;
  s = pcsir_set_tuning(c, &best);
  if (s == PCSIR_OK) s = pcsir_set_particles(c, state_scratch_dev);
  if (s != PCSIR_OK) return s;
  if (best_out) *best_out = best;
  if (best_ms_out) *best_ms_out = best_ms;
  if (trials_out) *trials_out = trials;
  return check_hip(c, hipStreamSynchronize(c->stream), "pcsir_autotune");
}

size_t pcsir_surr_bytes(void) { return SURR_BYTES; }

pcsir_status pcsir_surr_prepare(const float *params_dev, const float *act_scale_host, void *surr_dev, size_t bytes,
                                void *hip_stream) {
  if (!params_dev || !surr_dev || bytes < SURR_BYTES || ((uintptr_t)surr_dev) % ALIGN) return PCSIR_E_INVAL;
  if (!valid_act_scales(act_scale_host)) return PCSIR_E_INVAL;
  return surr_prepare(params_dev, act_scale_host, (char *)surr_dev, (hipStream_t)hip_stream) == hipSuccess
             ? PCSIR_OK
             : PCSIR_E_HIP;
}

pcsir_status pcsir_surr_rows(const void *surr_dev, const uint16_t *X_dev, int32_t n, int32_t fp8, float *f_dev,
                             float *absmax_dev, void *hip_stream) {
  if (!surr_dev || n < 0 || (n > 0 && (!X_dev || !f_dev))) return PCSIR_E_INVAL;
  if (((uintptr_t)surr_dev) % ALIGN || ((uintptr_t)X_dev) % 16) return PCSIR_E_INVAL;
  if (n == 0) return PCSIR_OK;
  const hipStream_t st = (hipStream_t)hip_stream;
  const SurrWeights sw = surr_view((void *)surr_dev);
  const int grid = std::min((n + SURR_ROWS - 1) / SURR_ROWS, 8192);
  if (fp8)
    k_surr_rows<true><<<grid, SURR_TPB, 0, st>>>(n, X_dev, sw, f_dev, (unsigned int *)absmax_dev);
  else
    k_surr_rows<false><<<grid, SURR_TPB, 0, st>>>(n, X_dev, sw, f_dev, (unsigned int *)absmax_dev);
  return hipGetLastError() == hipSuccess ? PCSIR_OK : PCSIR_E_HIP;
}

pcsir_status pcsir_set_surrogate(pcsir_ctx *c, const float *params_dev, const float *act_scale_host,
                                 float check_fraction, float tol_nats) {
  if (!c) return PCSIR_E_INVAL;
  if (c->cfg.lik_mode < PCSIR_LIK_SURR_BF16) return fail(c, PCSIR_E_STATE, "the filter was not made with a surrogate lik_mode");
  if (!params_dev) return fail(c, PCSIR_E_INVAL, "params_dev is NULL");
  if (!(check_fraction >= 0.0f && check_fraction <= 1.0f)) return fail(c, PCSIR_E_INVAL, "check_fraction not in [0, 1]");
  if (!(tol_nats >= 0.0f)) return fail(c, PCSIR_E_INVAL, "tol_nats must be >= 0 (may be +inf)");
  if (!valid_act_scales(act_scale_host)) return fail(c, PCSIR_E_INVAL, "activation scales must be finite and > 0");
  if (c->cfg.lik_mode == PCSIR_LIK_SURR_FP8 && !act_scale_host)
    return fail(c, PCSIR_E_INVAL, "FP8 surrogate needs the activation scales");
  drop_graphs(c);  // captured graphs hold the check fraction and tolerance
  const hipError_t e = surr_prepare(params_dev, act_scale_host, c->at<char>(c->L.surr), c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pcsir_set_surrogate");
  c->surr_fraction = check_fraction;
  c->surr_tol = tol_nats;
  c->surr_ready = 1;
  return PCSIR_OK;
}

pcsir_status pcsir_surrogate_features(pcsir_ctx *c, uint16_t *X_dev, float *y_dev, int32_t cap, int32_t *count) {
  if (!c || !count || cap < 0 || (cap > 0 && (!X_dev || !y_dev))) return PCSIR_E_INVAL;
  *count = 0;
  if (!c->stepped || c->last_sir) return fail(c, PCSIR_E_STATE, "features exist only after pcsir_step");
  uint64_t B = 0;
  hipError_t e = hipMemcpyAsync(&B, c->at<uint64_t>(c->L.meta) + META_B, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pcsir_surrogate_features");
  const Layout &L = c->L;
  DummyView dv;
  dv.dpix = c->at<int32_t>(L.dpix);
  dv.doff = c->at<float>(L.doff);
  dv.dvel = c->at<float>(L.dvel);
  dv.dint = c->at<float>(L.dint);
  dv.seg_t = c->at<int32_t>(L.seg_t);
  const uint64_t n = std::min<uint64_t>(B, (uint64_t)cap);
  if (n) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(n, (uint64_t)c->num_cus * 32);
    if (c->cfg.dim == 2)
      k_surr_features<2><<<grid, 256, 0, c->stream>>>(c->p, dv, c->at<uint64_t>(L.meta), c->at<StepDesc>(L.desc),
                                                      c->at<double>(L.ll), (uint32_t)cap, X_dev, y_dev);
    else
      k_surr_features<3><<<grid, 256, 0, c->stream>>>(c->p, dv, c->at<uint64_t>(L.meta), c->at<StepDesc>(L.desc),
                                                      c->at<double>(L.ll), (uint32_t)cap, X_dev, y_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return check_hip(c, e, "pcsir_surrogate_features");
  }
  *count = (int32_t)B;
  return PCSIR_OK;
}

pcsir_status pcsir_surrogate_stats(pcsir_ctx *c, uint64_t *checked, uint64_t *fallbacks, float *max_err, int32_t reset) {
  if (!c) return PCSIR_E_INVAL;
  uint64_t m[META_N];
  hipError_t e = hipMemcpyAsync(m, c->at<uint64_t>(c->L.meta), sizeof m, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && reset) {
    e = hipMemsetAsync(c->at<uint64_t>(c->L.meta) + META_CHECKED, 0, 8 * 3, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) return check_hip(c, e, "pcsir_surrogate_stats");
  if (checked) *checked = m[META_CHECKED];
  if (fallbacks) *fallbacks = m[META_FALLBACK];
  if (max_err) {
    const uint32_t b = (uint32_t)m[META_MAXERR];
    memcpy(max_err, &b, 4);
  }
  return PCSIR_OK;
}

}  // extern "C"
