/*
 * pcSIR / SIR reference oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of one filter step of classical SIR
 * (paper Sec. 3, Algorithm "SIR") and of piecewise-constant SIR (paper Sec. 4,
 * Algorithm "pcSIR"), with the nearly-constant-velocity dynamics of Sec. 5.1
 * and the Gaussian-PSF sum-of-squared-differences likelihood of Sec. 5.2
 * (Eq. "object" and Eq. "likelihood").
 *
 * It exists only to check the GPU library against: only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it. It shares no
 * code, header, table or constant with the GPU path. Every stage follows the
 * paper's steps in the paper's order; bins are kept in a std::map keyed by
 * the integer cell index, there is no sorting, blocking or fusion.
 *
 * Readings of the paper that the text leaves open (the proposal, the bin
 * grid origin, the window, the resampling scheme, the RNG) are listed in the
 * design notes of the repository and restated at each function below.
 * Parity is pinned for every function here (tests/test_oracle_*.py) except the
 * tracking-RMSE level, which is "parity unpinned" (the paper's data and
 * plotted values are not available).
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

/* ---------------- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ------
 * Counter-based generator. Not from the paper (the paper names no RNG); it
 * is used so that the oracle and the GPU draw the same uniforms from the
 * same (counter, key). Round: two 32x32->64 products of words 0 and 2 with
 * the published multipliers, words permuted and xored with the key; the key
 * is bumped by the published Weyl constants between rounds. */
const uint32_t PHILOX_M0 = 0xD2511F53u;
const uint32_t PHILOX_M1 = 0xCD9E8D57u;
const uint32_t PHILOX_W0 = 0x9E3779B9u;
const uint32_t PHILOX_W1 = 0xBB67AE85u;

void philox4x32_10(const uint32_t in_ctr[4], const uint32_t in_key[2], uint32_t out[4]) {
  uint32_t c0 = in_ctr[0], c1 = in_ctr[1], c2 = in_ctr[2], c3 = in_ctr[3];
  uint32_t k0 = in_key[0], k1 = in_key[1];
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    const uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The key of every draw: the 64-bit seed as (low word, high word). A counter
 * word that holds the frame index k takes k modulo 2^32. */
void philox_draw(uint64_t seed, uint32_t c0, uint64_t k, uint32_t c2, uint32_t c3, uint32_t out[4]) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const uint32_t ctr[4] = {c0, (uint32_t)k, c2, c3};
  philox4x32_10(ctr, key, out);
}

/* Uniform on (0,1) from one word: its top 23 bits plus one half, scaled by
 * 2^-23. The values are dyadic rationals with 24 significant bits, so they
 * are exact in binary32 as well as binary64. */
double uniform23(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }

/* [0, 1) with 53 random bits from two words: (w1 2^32 + w0) >> 11, times 2^-53. */
double uniform53(uint32_t w0, uint32_t w1) {
  return (double)((((uint64_t)w1 << 32) | (uint64_t)w0) >> 11) * 0x1p-53;
}

const double TWO_PI = 6.283185307179586476925286766559;

}  // namespace

extern "C" {

/* Model parameters (paper Sec. 5.1-5.2 and the readings listed in the design notes). */
typedef struct {
  int32_t dim;        /* spatial dimension: 2 -> state (x,y,vx,vy,I0); 3 -> (x,y,z,vx,vy,vz,I0) */
  int32_t m[3];       /* bins per pixel along x, y, z (bin edge length h = 1/m) */
  int32_t patch;      /* P: side of the square likelihood window, odd */
  int32_t quad;       /* q: midpoint sub-samples per pixel axis */
  int32_t psf;        /* 0: Gaussian PSF (Eq. object); 1: astigmatic PSF, sigma_x(z), sigma_y(z) */
  int32_t dummy_mode; /* 0: centre of mass of the bin (pcSIR-CoM); 1: geometric bin centre (CoC);
                         2: CoM with the members' position covariance (second order, 2D) */
  double sigma_psf;   /* PSF sigma in pixels (3D: sigma at focus) */
  double astig_gamma; /* 3D: focal offset of the two axes (pixels) */
  double astig_d;     /* 3D: depth scale (pixels) */
  double i_bg;        /* background intensity I_bg */
  double sigma_xi;    /* likelihood width sigma_xi */
  double proc_sigma[7]; /* per-component process noise std per frame */
  uint64_t seed;      /* Philox key word 0 */
} orc_model;

/* Outputs of the weighting stage of one target. Arrays are caller-owned and
 * sized for N (bins never outnumber particles). */
typedef struct {
  int32_t *keys;      /* [3][N] cell index (kx, ky, kz) of every particle (kz = 0 in 2D) */
  int64_t *bin_of;    /* [N] bin number of every particle (SIR: the particle itself) */
  int32_t *bin_key;   /* [3][N] cell index of every bin, bins in ascending (kz, ky, kx) order */
  int64_t *bin_n;     /* [N] members per bin */
  double *bin_mean;   /* [D][N] dummy state per bin (mean state; CoC: bin centre for positions) */
  double *ll;         /* [N] log-likelihood per bin (pcSIR) or per particle (SIR) */
  double *w;          /* [N] normalised weights, storage order */
  double *scal;       /* [3]: max log-weight M, sum S = sum exp(logw - M), N_eff */
  double *est;        /* [D] posterior-mean estimate sum_i w_i x_i */
} orc_weigh_out;

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox4x32_10(ctr, key, out); }

double orc_uniform(uint32_t w) { return uniform23(w); }

/* Eight standard normals for particle i of target t at frame k: Philox
 * blocks with counters (i, k, t, 0) and (i, k, t, 1); pair p takes
 * (u1, u2) from words 2p and 2p + 1 of their eight words and maps them by
 * Box-Muller, (z_2p, z_2p+1) = sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2). */
void orc_normals(uint64_t seed, uint64_t i, uint64_t k, uint64_t t, double z[8]) {
  uint32_t w[8];
  philox_draw(seed, (uint32_t)i, k, (uint32_t)t, 0, w);
  philox_draw(seed, (uint32_t)i, k, (uint32_t)t, 1, w + 4);
  for (int p = 0; p < 4; ++p) {
    double u1 = uniform23(w[2 * p]);
    double u2 = uniform23(w[2 * p + 1]);
    double r = std::sqrt(-2.0 * std::log(u1));
    z[2 * p] = r * std::cos(TWO_PI * u2);
    z[2 * p + 1] = r * std::sin(TWO_PI * u2);
  }
}

/* The one uniform of systematic resampling for target t at frame k: words 0
 * and 1 of the Philox block with counter (0, k, t, 2), a value in [0, 1). */
double orc_resample_u(uint64_t seed, uint64_t k, uint64_t t) {
  uint32_t w[4];
  philox_draw(seed, 0, k, (uint32_t)t, 2, w);
  return uniform53(w[0], w[1]);
}

/* The draw that picks a dummy for the surrogate's exact check: words 0 and 1
 * of the block with counter (dummy, k, t, 3). */
double orc_check_u(uint64_t seed, uint64_t dummy, uint64_t k, uint64_t t) {
  uint32_t w[4];
  philox_draw(seed, (uint32_t)dummy, k, (uint32_t)t, 3, w);
  return uniform53(w[0], w[1]);
}

/* Cell index of coordinate x on the grid of "B bins of equal size" (Alg.
 * pcSIR, bin creation; Sec. 4.2 takes pixels as cells): bins of edge 1/m whose
 * edges sit at j/m - 1/2, so that pixel c (centre at integer c) is exactly
 * the union of cells c*m ... c*m + m - 1. The index is the exact real
 * floor((x + 1/2) m) of the binary32 input. Non-finite or huge inputs: x is
 * clamped to [-2^24, 2^24] (NaN counts as +2^24) and the index to
 * [-2^30, 2^30]. m must lie in [1, 4096]. */
int32_t orc_bin_key(float xf, int32_t m) {
  const long long KEY_LIM = 1LL << 30;
  double x = (double)xf;
  if (std::isnan(x)) x = 0x1p24;
  if (x > 0x1p24) x = 0x1p24;
  if (x < -0x1p24) x = -0x1p24;
  long long k;
  if (std::fabs(x) < 0x1p-30) {
    /* |x m| < 2^-18 < 1/2: floor(m/2 + x m) is floor(m/2), less one when m is
     * even and x is negative. */
    k = m / 2;
    if ((m % 2) == 0 && x < 0) k -= 1;
  } else {
    /* binary128 holds x + 1/2 (at most 78 significant bits here) and its
     * product with m (at most 13 more) exactly, so the floor is exact. */
    __float128 v = ((__float128)x + (__float128)0.5) * (__float128)m;
    k = (long long)v; /* truncation toward zero */
    if ((__float128)k > v) k -= 1;
  }
  if (k > KEY_LIM) k = KEY_LIM;
  if (k < -KEY_LIM) k = -KEY_LIM;
  return (int32_t)k;
}

/* Floor division of a cell index by m: the pixel that holds the cell. */
static long long floor_div(long long a, long long m) {
  long long q = a / m;
  if ((a % m) != 0 && ((a < 0) != (m < 0))) q -= 1;
  return q;
}

/* Propagation (Alg. SIR / Alg. pcSIR, "draw a sample from pi"), read as the
 * bootstrap proposal pi = p(x_k | x_{k-1}) with the nearly-constant-velocity
 * dynamics of Sec. 5.1 and unit frame interval: each position moves by its
 * (old) velocity plus Gaussian noise, velocity and intensity take Gaussian
 * noise; noise standard deviations per component are model parameters.
 * Computed in binary64 and stored as binary32. State is SoA [D][N]; t is the
 * target index and k the frame index, both part of the RNG counter. */
void orc_propagate(const orc_model *mdl, int64_t N, float *state, int64_t k, int64_t t) {
  const int dim = mdl->dim;
  const int D = 2 * dim + 1;
  for (int64_t i = 0; i < N; ++i) {
    double z[8];
    orc_normals(mdl->seed, (uint64_t)i, (uint64_t)k, (uint64_t)t, z);
    double x[7];
    for (int d = 0; d < D; ++d) x[d] = (double)state[(int64_t)d * N + i];
    double nx[7];
    for (int a = 0; a < dim; ++a) nx[a] = x[a] + x[dim + a] + mdl->proc_sigma[a] * z[a];
    for (int a = 0; a < dim; ++a) nx[dim + a] = x[dim + a] + mdl->proc_sigma[dim + a] * z[dim + a];
    nx[2 * dim] = x[2 * dim] + mdl->proc_sigma[2 * dim] * z[2 * dim];
    for (int d = 0; d < D; ++d) state[(int64_t)d * N + i] = (float)nx[d];
  }
}

/* PSF widths along x and y for a state at depth zpos (Sec. 5.2: Gaussian
 * PSF; the astigmatic 3D form widens each axis away from its own focal
 * plane: sigma_x = s0 sqrt(1 + ((z - g)/d)^2), sigma_y = s0 sqrt(1 + ((z + g)/d)^2)). */
static void psf_sigmas(const orc_model *mdl, double zpos, double *sx, double *sy) {
  if (mdl->psf == 1) {
    double ax = (zpos - mdl->astig_gamma) / mdl->astig_d;
    double ay = (zpos + mdl->astig_gamma) / mdl->astig_d;
    *sx = mdl->sigma_psf * std::sqrt(1.0 + ax * ax);
    *sy = mdl->sigma_psf * std::sqrt(1.0 + ay * ay);
  } else {
    *sx = mdl->sigma_psf;
    *sy = mdl->sigma_psf;
  }
}

/* Log-likelihood of one state against one frame (Eq. likelihood up to its
 * additive constant): minus the sum over the P x P window of pixels around
 * pixel (c0, r0) of the squared difference between the frame and the model
 * image of Eq. object, divided by 2 sigma_xi^2. The model value of a pixel is
 * I_bg + I0 times the Gaussian averaged over q x q midpoint sub-samples of
 * the pixel (q = 1 is Eq. object sampled at the pixel centre). Pixel (c, r)
 * has its centre at integer (c, r), column c along x and row r along y.
 * Pixels outside the frame read as I_bg. */
double orc_loglik(const orc_model *mdl, const float *frame, int32_t H, int32_t W, int64_t c0,
                  int64_t r0, double xh, double yh, double zh, double I0) {
  double sx, sy;
  psf_sigmas(mdl, zh, &sx, &sy);
  const int q = mdl->quad;
  const int R = (mdl->patch - 1) / 2;
  double ssd = 0.0;
  for (int64_t r = r0 - R; r <= r0 + R; ++r) {
    for (int64_t c = c0 - R; c <= c0 + R; ++c) {
      double g = 0.0;
      for (int a = 0; a < q; ++a) {
        for (int b = 0; b < q; ++b) {
          double ox = ((double)c - xh) + ((a + 0.5) / q - 0.5);
          double oy = ((double)r - yh) + ((b + 0.5) / q - 0.5);
          g += std::exp(-(ox * ox / (2.0 * sx * sx) + oy * oy / (2.0 * sy * sy)));
        }
      }
      g /= (double)(q * q);
      double mu = mdl->i_bg + I0 * g;
      double zp = (r >= 0 && r < H && c >= 0 && c < W) ? (double)frame[r * (int64_t)W + c] : mdl->i_bg;
      ssd += (zp - mu) * (zp - mu);
    }
  }
  return -ssd / (2.0 * mdl->sigma_xi * mdl->sigma_xi);
}

/* Weighting stage of one target, from propagated states to normalised
 * weights, N_eff and the posterior-mean estimate.
 *  sir = 1: classical SIR (Alg. SIR): every particle is evaluated.
 *  sir = 0: pcSIR (Alg. pcSIR): particles are assigned to bins; each occupied
 *           bin gets one dummy whose state is the mean state of its members
 *           (CoM; or, with dummy_mode 1, the bin centre for the positions;
 *           dummy_mode 2 adds the second-order term of the members' position
 *           covariance to the dummy's log-likelihood, see below);
 *           the likelihood is evaluated on the dummy only and its value is
 *           copied to every member.
 * The log-weight of particle i is logw_prev[i] + its likelihood term
 * (logw_prev NULL: uniform previous weights, which cancel). With previous
 * weights the dummy is the centre of mass of its members weighted by them
 * (Sec. 4: the dummy's state is formed from the members' states and
 * weights), sum_i w_i x_i / sum_i w_i, w_i = exp(logw_prev[i] - max over the
 * bin); without them, or when they are equal, it is the plain mean of
 * Alg. pcSIR. Normalisation
 * (Alg. SIR, normalise; applied in Alg. pcSIR as well) divides by the sum,
 * after a shift by the maximum log-weight that cancels in exact arithmetic.
 * N_eff = 1 / sum w^2 (both algorithms). The estimate is the posterior mean
 * sum_i w_i x_i over all state components.
 * Only the spatial components (x, y[, z]) are binned. The likelihood window
 * is centred on the pixel that holds the bin (pcSIR) or the particle (SIR).
 * Returns the number of bins B (SIR: N). */
int64_t orc_weigh(const orc_model *mdl, const float *frame, int32_t H, int32_t W, int64_t N,
                  const float *state, const double *logw_prev, int32_t sir, orc_weigh_out *out) {
  const int dim = mdl->dim;
  const int D = 2 * dim + 1;
  const int32_t m1[3] = {1, 1, 1};
  const int32_t *mm = sir ? m1 : mdl->m;
  std::vector<double> cov;  /* second-order dummies: position covariance per bin (xx, yy, xy) */

  for (int64_t i = 0; i < N; ++i) {
    for (int a = 0; a < 3; ++a) {
      int32_t k = 0;
      if (a < dim) k = orc_bin_key(state[(int64_t)a * N + i], mm[a]);
      out->keys[(int64_t)a * N + i] = k;
    }
  }

  int64_t B = 0;
  if (sir) {
    B = N;
    for (int64_t i = 0; i < N; ++i) {
      out->bin_of[i] = i;
      out->bin_n[i] = 1;
      for (int a = 0; a < 3; ++a) out->bin_key[(int64_t)a * N + i] = out->keys[(int64_t)a * N + i];
      for (int d = 0; d < D; ++d) out->bin_mean[(int64_t)d * N + i] = (double)state[(int64_t)d * N + i];
    }
  } else {
    /* Bins ordered by (kz, ky, kx). */
    std::map<std::tuple<int32_t, int32_t, int32_t>, std::vector<int64_t>> bins;
    if (mdl->dummy_mode == 2) cov.assign(3 * (size_t)N, 0.0);
    for (int64_t i = 0; i < N; ++i) {
      auto key = std::make_tuple(out->keys[2 * N + i], out->keys[1 * N + i], out->keys[0 * N + i]);
      bins[key].push_back(i);
    }
    for (auto &kv : bins) {
      const std::vector<int64_t> &mem = kv.second;
      out->bin_key[0 * N + B] = std::get<2>(kv.first);
      out->bin_key[1 * N + B] = std::get<1>(kv.first);
      out->bin_key[2 * N + B] = std::get<0>(kv.first);
      out->bin_n[B] = (int64_t)mem.size();
      if (logw_prev) {
        double mx = -INFINITY;
        for (int64_t i : mem) mx = logw_prev[i] > mx ? logw_prev[i] : mx;
        double ws = 0.0;
        for (int64_t i : mem) ws += std::exp(logw_prev[i] - mx);
        for (int d = 0; d < D; ++d) {
          double s = 0.0;
          for (int64_t i : mem) s += std::exp(logw_prev[i] - mx) * (double)state[(int64_t)d * N + i];
          out->bin_mean[(int64_t)d * N + B] = s / ws;
        }
      } else {
        for (int d = 0; d < D; ++d) {
          double s = 0.0;
          for (int64_t i : mem) s += (double)state[(int64_t)d * N + i];
          out->bin_mean[(int64_t)d * N + B] = s / (double)mem.size();
        }
      }
      if (mdl->dummy_mode == 1) {
        for (int a = 0; a < dim; ++a) {
          double kk = (double)out->bin_key[(int64_t)a * N + B];
          out->bin_mean[(int64_t)a * N + B] = (kk + 0.5) / (double)mdl->m[a] - 0.5;
        }
      }
      if (mdl->dummy_mode == 2) {
        /* covariance of the members' positions about the dummy, weighted
           as the mean is: xx, yy, xy */
        double mx = -INFINITY;
        if (logw_prev)
          for (int64_t i : mem) mx = logw_prev[i] > mx ? logw_prev[i] : mx;
        double ws = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
        const double ux = out->bin_mean[0 * N + B], uy = out->bin_mean[1 * N + B];
        for (int64_t i : mem) {
          const double wi = logw_prev ? std::exp(logw_prev[i] - mx) : 1.0;
          const double ddx = (double)state[0 * N + i] - ux, ddy = (double)state[1 * N + i] - uy;
          ws += wi;
          sxx += wi * ddx * ddx;
          syy += wi * ddy * ddy;
          sxy += wi * ddx * ddy;
        }
        cov[3 * (size_t)B + 0] = sxx / ws;
        cov[3 * (size_t)B + 1] = syy / ws;
        cov[3 * (size_t)B + 2] = sxy / ws;
      }
      for (int64_t i : mem) out->bin_of[i] = B;
      ++B;
    }
  }

  /* Likelihood on dummies (pcSIR) or particles (SIR). */
  for (int64_t b = 0; b < B; ++b) {
    int64_t c0 = floor_div(out->bin_key[0 * N + b], mm[0]);
    int64_t r0 = floor_div(out->bin_key[1 * N + b], mm[1]);
    double zh = dim == 3 ? out->bin_mean[2 * N + b] : 0.0;
    const double ux = out->bin_mean[0 * N + b], uy = out->bin_mean[1 * N + b];
    const double I0 = out->bin_mean[(int64_t)(2 * dim) * N + b];
    out->ll[b] = orc_loglik(mdl, frame, H, W, c0, r0, ux, uy, zh, I0);
    if (!sir && mdl->dummy_mode == 2) {
      /* second order: the bin's log-likelihood is the log of the members'
         mean likelihood to second order in their spread, ell(mu) +
         tr(H S)/2 + g'Sg/2, with g and H the gradient and Hessian of the
         log-likelihood in the bin's (fixed) window, by central differences
         of half a cell */
      const double dx = 0.5 / (double)mm[0], dy = 0.5 / (double)mm[1];
      auto L = [&](double sx, double sy) {
        return orc_loglik(mdl, frame, H, W, c0, r0, ux + sx * dx, uy + sy * dy, zh, I0);
      };
      const double l0 = out->ll[b];
      const double lxp = L(1, 0), lxm = L(-1, 0), lyp = L(0, 1), lym = L(0, -1);
      const double lpp = L(1, 1), lpm = L(1, -1), lmp = L(-1, 1), lmm = L(-1, -1);
      const double gx = (lxp - lxm) / (2.0 * dx), gy = (lyp - lym) / (2.0 * dy);
      const double hxx = (lxp - 2.0 * l0 + lxm) / (dx * dx), hyy = (lyp - 2.0 * l0 + lym) / (dy * dy);
      const double hxy = (lpp - lpm - lmp + lmm) / (4.0 * dx * dy);
      const double sxx = cov[3 * (size_t)b], syy = cov[3 * (size_t)b + 1], sxy = cov[3 * (size_t)b + 2];
      out->ll[b] = l0 + 0.5 * (hxx * sxx + hyy * syy + 2.0 * hxy * sxy) +
                   0.5 * (gx * gx * sxx + gy * gy * syy + 2.0 * gx * gy * sxy);
    }
  }

  /* Weights: copy of the bin's likelihood to every member, then normalise. */
  std::vector<double> lw(N);
  double M = -INFINITY;
  for (int64_t i = 0; i < N; ++i) {
    lw[i] = (logw_prev ? logw_prev[i] : 0.0) + out->ll[out->bin_of[i]];
    if (lw[i] > M) M = lw[i];
  }
  double S = 0.0;
  for (int64_t i = 0; i < N; ++i) S += std::exp(lw[i] - M);
  double sq = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    out->w[i] = std::exp(lw[i] - M) / S;
    sq += out->w[i] * out->w[i];
  }
  out->scal[0] = M;
  out->scal[1] = S;
  out->scal[2] = 1.0 / sq;
  for (int d = 0; d < D; ++d) {
    double e = 0.0;
    for (int64_t i = 0; i < N; ++i) e += out->w[i] * (double)state[(int64_t)d * N + i];
    out->est[d] = e;
  }
  return B;
}

/* Resampling (Alg. SIR / Alg. pcSIR, resampling step) by the systematic
 * scheme: cumulative weights C_l = w_0 + ... + w_l in storage order, one
 * uniform u in [0,1), thresholds theta_j = (j + u) / N, and
 * s(j) = min { l : C_l > theta_j }, taken as N-1 if rounding leaves no such l.
 * Each l then has Pr[s(j) = l] = w_l for a uniformly chosen j. cdf may be NULL. */
void orc_resample(int64_t N, const double *w, double u, double *cdf, int64_t *s) {
  std::vector<double> C(N);
  double acc = 0.0;
  for (int64_t l = 0; l < N; ++l) {
    acc += w[l];
    C[l] = acc;
  }
  if (cdf)
    for (int64_t l = 0; l < N; ++l) cdf[l] = C[l];
  int64_t l = 0;
  for (int64_t j = 0; j < N; ++j) {
    double theta = ((double)j + u) / (double)N;
    while (l < N - 1 && !(C[l] > theta)) ++l;
    s[j] = l;
  }
}

/* One complete step of one target: propagate, weigh, estimate, resample
 * (every frame: the resampling threshold is taken as infinite), and replace
 * the particle set by the resampled one. state is updated in place; est [D]
 * and neff receive the estimate and N_eff of this frame. */
void orc_step(const orc_model *mdl, const float *frame, int32_t H, int32_t W, int64_t N, float *state,
              int64_t k, int64_t t, int32_t sir, double *est, double *neff) {
  const int D = 2 * mdl->dim + 1;
  orc_propagate(mdl, N, state, k, t);
  std::vector<int32_t> keys(3 * N), bin_key(3 * N);
  std::vector<int64_t> bin_of(N), bin_n(N), s(N);
  std::vector<double> bin_mean((size_t)D * N), ll(N), w(N);
  double scal[3];
  orc_weigh_out o = {keys.data(), bin_of.data(), bin_key.data(), bin_n.data(), bin_mean.data(),
                     ll.data(),   w.data(),      scal,           est};
  orc_weigh(mdl, frame, H, W, N, state, nullptr, sir, &o);
  *neff = scal[2];
  double u = orc_resample_u(mdl->seed, (uint64_t)k, (uint64_t)t);
  orc_resample(N, w.data(), u, nullptr, s.data());
  std::vector<float> old(state, state + (size_t)D * N);
  for (int d = 0; d < D; ++d)
    for (int64_t j = 0; j < N; ++j) state[(int64_t)d * N + j] = old[(int64_t)d * N + s[j]];
}

/* One step of one target with a resampling threshold (Alg. SIR / Alg.
 * pcSIR: resample only when N_eff falls below it). logw [N] holds the
 * normalised log-weights kept from the previous frame; *uniform != 0 means
 * they are all equal (after resampling or at the start), which is weighed
 * exactly as without previous weights. The target resamples when
 * N_eff < neff_frac * N; it then takes the resampled set and *uniform = 1.
 * Otherwise the propagated particles stay in place, logw[i] = log w_i,
 * formed in the log domain (previous logw_i + l_i - M - log S) so that it
 * stays finite where w_i underflows binary64, and *uniform = 0. *resampled reports which happened. neff_frac = +inf gives
 * orc_step. */
void orc_step_thr(const orc_model *mdl, const float *frame, int32_t H, int32_t W, int64_t N, float *state,
                  double *logw, int32_t *uniform, int64_t k, int64_t t, int32_t sir, double neff_frac, double *est,
                  double *neff, int32_t *resampled) {
  const int D = 2 * mdl->dim + 1;
  orc_propagate(mdl, N, state, k, t);
  std::vector<int32_t> keys(3 * N), bin_key(3 * N);
  std::vector<int64_t> bin_of(N), bin_n(N), s(N);
  std::vector<double> bin_mean((size_t)D * N), ll(N), w(N);
  double scal[3];
  orc_weigh_out o = {keys.data(), bin_of.data(), bin_key.data(), bin_n.data(), bin_mean.data(),
                     ll.data(),   w.data(),      scal,           est};
  orc_weigh(mdl, frame, H, W, N, state, *uniform ? nullptr : logw, sir, &o);
  *neff = scal[2];
  if (scal[2] < neff_frac * (double)N) {
    double u = orc_resample_u(mdl->seed, (uint64_t)k, (uint64_t)t);
    orc_resample(N, w.data(), u, nullptr, s.data());
    std::vector<float> old(state, state + (size_t)D * N);
    for (int d = 0; d < D; ++d)
      for (int64_t j = 0; j < N; ++j) state[(int64_t)d * N + j] = old[(int64_t)d * N + s[j]];
    *uniform = 1;
    *resampled = 1;
  } else {
    /* normalised log-weights, kept in the log domain: log w_i = logw_i - M - log S,
       finite even where w_i itself underflows binary64 */
    const double lnorm = scal[0] + std::log(scal[1]);
    for (int64_t i = 0; i < N; ++i) logw[i] = (*uniform ? 0.0 : logw[i]) + ll[bin_of[i]] - lnorm;
    *uniform = 0;
    *resampled = 0;
  }
}

/* Several targets over several frames: targets t = 0..T-1 with particle
 * counts n[t], stored one after another in a SoA array [D][sum n]; frames
 * k = k0 .. k0+K-1 read frame index k - k0 from frames (shared by all
 * targets, [K][H][W]) or, with per_target != 0, from [K][T][H][W]. Writes the
 * per-frame estimates [K][T][D] and N_eff [K][T]. Targets are independent
 * (every step of both algorithms is per target), so within a frame they run
 * on the OpenMP threads that orc_set_threads chose, each on its own copy of
 * its particles; the results do not depend on the thread count. */
void orc_track(const orc_model *mdl, const float *frames, int32_t H, int32_t W, int32_t per_target,
               int64_t T, const int64_t *n, float *state, int64_t k0, int64_t K, int32_t sir, double *est,
               double *neff) {
  const int D = 2 * mdl->dim + 1;
  std::vector<int64_t> off((size_t)T + 1, 0);
  for (int64_t t = 0; t < T; ++t) off[(size_t)t + 1] = off[(size_t)t] + n[t];
  const int64_t total = off[(size_t)T];
  for (int64_t kk = 0; kk < K; ++kk) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < T; ++t) {
      const int64_t Nt = n[t], o = off[(size_t)t];
      std::vector<float> tmp((size_t)D * Nt);
      for (int d = 0; d < D; ++d)
        for (int64_t i = 0; i < Nt; ++i) tmp[(size_t)d * Nt + i] = state[(int64_t)d * total + o + i];
      const float *fr = per_target ? frames + ((kk * T + t) * (int64_t)H * W) : frames + kk * (int64_t)H * W;
      orc_step(mdl, fr, H, W, Nt, tmp.data(), k0 + kk, t, sir, est + (kk * T + t) * D, neff + kk * T + t);
      for (int d = 0; d < D; ++d)
        for (int64_t i = 0; i < Nt; ++i) state[(int64_t)d * total + o + i] = tmp[(size_t)d * Nt + i];
    }
  }
}

/* Threads of orc_track (1 = the paper's single-core setting); returns the
 * count now in effect. n <= 0 leaves it unchanged. */
int32_t orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return (int32_t)omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

}  /* extern "C" */
