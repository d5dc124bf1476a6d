/*
 * pcsir.h — C ABI of the MI355X (gfx950) piecewise-constant SIR particle filter.
 *
 * The library advances T independent targets, each a set of N_t weighted
 * particles, through one frame of classical SIR (paper Sec. 3, Algorithm
 * "SIR") or of piecewise-constant SIR (paper Sec. 4, Algorithm "pcSIR"). The
 * objects follow the problem statement of Sec. 3: a measurement per time step
 * (a frame), the dynamics density (nearly-constant velocity, Sec. 5.1), the
 * likelihood (Gaussian-PSF sum of squared differences, Sec. 5.2, Eq. object
 * and Eq. likelihood), and a weighted particle set whose posterior mean is
 * the state estimate.
 *
 * Conventions
 *  - C99, plain pointers and sizes. "_dev" pointers are device (HBM) memory,
 *    "_host" pointers are host memory. Nothing here allocates device memory:
 *    the caller provides one workspace of pcsir_workspace_bytes() bytes.
 *  - Every function returns a pcsir_status; PCSIR_OK is 0, errors are
 *    negative. A failing call leaves a message in pcsir_last_error(ctx).
 *  - All device work is enqueued on the stream given to pcsir_init, in call
 *    order. pcsir_step / sir_step return without synchronising; device-side
 *    conditions (bin range overflow, non-finite normalisation) are reported
 *    by the next pcsir_estimate or pcsir_destroy.
 *  - A context is not thread-safe; separate contexts may run on separate
 *    streams. Outputs are bit-reproducible for equal inputs (config, initial
 *    state, frames and frame indices k): no floating-point atomics are used.
 *  - State layout is SoA: component d of particle i of target t sits at
 *    [d * sum_N + off_t + i], off_t = n_0 + ... + n_{t-1}. Components are
 *    (x, y, vx, vy, I0) in 2D and (x, y, z, vx, vy, vz, I0) in 3D; positions
 *    are in pixels, pixel (c, r) has its centre at integer (c, r), x runs
 *    along columns and y along rows.
 */
#ifndef PCSIR_H
#define PCSIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCSIR_ABI_VERSION 3

typedef struct pcsir_ctx pcsir_ctx; /* opaque; host memory owned by the library */

typedef enum {
  PCSIR_OK = 0,
  PCSIR_E_INVAL = -1,       /* argument or config field out of range, null pointer */
  PCSIR_E_NOMEM = -2,       /* workspace smaller than pcsir_workspace_bytes() */
  PCSIR_E_HIP = -3,         /* a HIP runtime call failed (message in pcsir_last_error) */
  PCSIR_E_STATE = -4,       /* call out of order, or frame size differs from the config */
  PCSIR_E_NUMERIC = -5,     /* device-side condition: see pcsir_last_error */
  PCSIR_E_UNSUPPORTED = -6  /* feature not available on this device or build */
} pcsir_status;

/* How the likelihood of Eq. likelihood is evaluated. Both exact modes compute
 * the same value (the model image of Eq. object averaged over q x q midpoint
 * sub-samples per pixel); they differ only in floating-point rounding.
 *  DIRECT:    one exponential per sub-sample and pixel (P^2 q^2 per evaluation),
 *             the image-formation simulation written out, in binary32: its
 *             log-likelihood errs by up to about 3e-7 of |l| (the rounding of
 *             each model value to one binary32 word);
 *  SEPARABLE: the Gaussian factorises over x and y, so 2 P q exponentials per
 *             evaluation suffice; the per-axis sums, the model image and the
 *             residuals are carried as binary32 pairs (about 48 bits), and the
 *             log-likelihood errs by about 1e-8 absolute. */
typedef enum {
  PCSIR_LIK_DIRECT = 0,
  PCSIR_LIK_SEPARABLE = 1,
  /* Learned surrogate of the dummies' log-likelihood (pcsir_mlp.h), BF16 or
   * FP8 matrix-core inference, with an exact check of a random share of the
   * dummies each frame and exact recomputation (SEPARABLE) of every target
   * whose check fails. pcsir_step only; sir_step stays exact (SEPARABLE). */
  PCSIR_LIK_SURR_BF16 = 2,
  PCSIR_LIK_SURR_FP8 = 3
} pcsir_lik_mode;

typedef enum { PCSIR_PSF_GAUSS2D = 0, PCSIR_PSF_ASTIG3D = 1 } pcsir_psf;

/* Dummy particle of a bin (Alg. pcSIR: mean state of the members; Sec. 5.5
 * also uses the geometric cell centre, "CoC", for the positions).
 * COM2: the CoM dummy also carries its members' position covariance S (Sec. 4
 * notes that a dummy could store higher moments): the bin's log-likelihood
 * is ell(mu) + tr(H S)/2 + g'S g/2, the log of the members' mean likelihood
 * to second order in their spread, with g and H from nine evaluations of
 * the dummy's window at shifts of half a cell (central differences). 2D,
 * exact likelihood modes and every-frame resampling only. */
typedef enum { PCSIR_DUMMY_COM = 0, PCSIR_DUMMY_COC = 1, PCSIR_DUMMY_COM2 = 2 } pcsir_dummy;

typedef struct {
  uint32_t abi_version;        /* must equal PCSIR_ABI_VERSION */
  int32_t dim;                 /* spatial dimension: 2 (D = 5) or 3 (D = 7) */
  int32_t n_targets;           /* T >= 1 */
  const int64_t *n_particles;  /* host [T], each >= 1; sum < 2^31. Read during pcsir_init only. */
  int32_t bins_per_px[3];      /* m_x, m_y, m_z in [1, 4096]: cells of edge h = 1/m, edges at
                                  j/m - 1/2, so every pixel is a union of cells (Sec. 4.2:
                                  m = 1 is pcSIR-1x1, m = 2 is pcSIR-2x2). m_z used in 3D only. */
  int32_t patch;               /* P: side of the likelihood window, odd, 1..127 (65 for the
                                  large-object support of Sec. 5) */
  int32_t quad;                /* q: midpoint sub-samples per pixel axis, 1..16 */
  int32_t psf;                 /* pcsir_psf; ASTIG3D requires dim == 3 */
  int32_t dummy_mode;          /* pcsir_dummy */
  int32_t lik_mode;            /* pcsir_lik_mode */
  int32_t per_target_frames;   /* 0: one H x W frame for all targets; 1: a [T][H][W] stack */
  int32_t frame_h, frame_w;    /* H, W >= 1: size of every frame */
  float sigma_psf;             /* PSF sigma (pixels); 3D: sigma at focus */
  float astig_gamma, astig_d;  /* 3D: sigma_x = s0 sqrt(1+((z-g)/d)^2), sigma_y = s0 sqrt(1+((z+g)/d)^2) */
  float i_bg;                  /* background intensity; also the value of pixels outside the frame */
  float sigma_xi;              /* likelihood width sigma_xi > 0 */
  float proc_sigma[7];         /* process-noise standard deviation per state component and frame */
  uint64_t seed;               /* Philox4x32-10 key: (low 32 bits, high 32 bits) */
  double neff_threshold;       /* resampling threshold as a fraction of N_t (Alg. SIR and Alg. pcSIR
                                  resample when N_eff falls below a threshold). Above 1 (e.g.
                                  +inf): resample every frame, the default. In [0, 1]: a target
                                  resamples only when N_eff < neff_threshold * N_t; otherwise its
                                  particles stay and carry their normalised log-weights into the
                                  next frame, where each pcSIR dummy is the centre of mass of its
                                  members weighted by them (Sec. 4). Weighted sums use float64
                                  atomics, so results with kept weights are reproducible to
                                  rounding, not bit for bit. NaN or < 0: invalid. */
  double bins_per_sigma;       /* 0: every target uses bins_per_px. > 0: adaptive bin size (the paper
                                  names adaptive bins as future work): per frame, target and spatial
                                  axis, m = ceil(bins_per_sigma / sd) cells per pixel, clamped to
                                  [1, bins_max], where sd is the standard deviation of the target's
                                  propagated positions on that axis (population variance
                                  S2/n - (S1/n)^2 in binary64; bins_max when sd = 0). Cells keep
                                  their edges at j/m - 1/2. Must be finite. */
  int32_t bins_max;            /* adaptive bins: largest m, 1..4096 */
} pcsir_config;

/* Bytes of device workspace that a context with this config needs (0 if the
 * config is invalid): a fixed 1 GiB for the cell-occupancy bitmap (one bit
 * per 32-bit cell key, each 64-bit word in a 16-byte entry with the number of
 * its first bin), plus a part that grows linearly with sum N_t (about 175 B
 * per particle in 2D) and with T. */
size_t pcsir_workspace_bytes(const pcsir_config *cfg);

/* Create a context. init_state_dev: SoA [D][sum N] float32, copied into the
 * workspace (Alg. SIR / Alg. pcSIR initialisation: weights 1/N). workspace_dev:
 * caller-owned device memory of workspace_bytes bytes, 256-byte aligned, kept
 * alive and untouched until pcsir_destroy. hip_stream: the hipStream_t all work
 * goes to (NULL: the legacy default stream). Synchronises the stream once. */
pcsir_status pcsir_init(const pcsir_config *cfg, const float *init_state_dev, void *workspace_dev,
                        size_t workspace_bytes, void *hip_stream, pcsir_ctx **out);

/* One frame of pcSIR (Alg. pcSIR) for every target: propagate, assign to
 * cells, form one dummy per occupied cell, evaluate the likelihood on the
 * dummies, copy each dummy's weight to its members, normalise, compute N_eff
 * and the posterior-mean estimate, and resample (systematic scheme, every
 * frame). frame_dev: float32 [H][W], or [T][H][W] with per_target_frames;
 * it must stay valid until the stream has passed this step. k >= 1 is the
 * frame index; it is part of the random-number counter. With neff_threshold
 * in [0, 1] a target resamples only when its N_eff is below the threshold.
 * Asynchronous. */
pcsir_status pcsir_step(pcsir_ctx *ctx, const float *frame_dev, int32_t H, int32_t W, int64_t k);

/* One frame of classical SIR (Alg. SIR): as pcsir_step, but the likelihood
 * is evaluated for every particle. Asynchronous. */
pcsir_status sir_step(pcsir_ctx *ctx, const float *frame_dev, int32_t H, int32_t W, int64_t k);

/* Copy the estimates of the last step to the host: est_host [T][D] float64
 * (posterior mean, taken after weighting and before resampling) and, if not
 * NULL, neff_host [T] float64 (N_eff = 1 / sum w^2). Synchronises the stream.
 * Returns PCSIR_E_NUMERIC if a device-side condition was raised since the
 * last call (the flag is then cleared; pcsir_last_error names it): a
 * target's normalisation not finite (its particles are kept), a velocity or
 * intensity outside the bin sums' fixed-point range, or all targets' cell
 * boxes together above 2^32 cells (the frame then gets no bins, so its
 * targets keep their particles). */
pcsir_status pcsir_estimate(pcsir_ctx *ctx, double *est_host, double *neff_host);

/* Synchronise the stream and free the host context. The workspace may be
 * freed by the caller afterwards. Returns the pending device-side status. */
pcsir_status pcsir_destroy(pcsir_ctx *ctx);

/* Last error message of this context (empty if none). Owned by ctx. */
const char *pcsir_last_error(const pcsir_ctx *ctx);

/* Current particle set (after the last resampling) into dst_dev, SoA
 * [D][sum N] float32. Asynchronous. */
pcsir_status pcsir_get_particles(pcsir_ctx *ctx, float *dst_dev);

/* Replace the particle set by src_dev (SoA [D][sum N] float32), with uniform
 * weights. Asynchronous. Used to resume from a checkpoint and by tests. */
pcsir_status pcsir_set_particles(pcsir_ctx *ctx, const float *src_dev);

/* Debug and parity views of the last step, copied into dst_dev (device
 * memory of at least `bytes` bytes; PCSIR_E_INVAL if too small). Asynchronous
 * except PCSIR_DUMP_COUNTS, which synchronises. Layouts:
 *  PROPAGATED  float32 [D][sum N]   propagated states x~_k (before resampling)
 *  KEYS        int32   [3][sum N]   cell index (kx, ky, kz) of every particle; SIR: pixel index
 *  COUNTS      int64   [2] or [3]   (bins B over all targets, passes of the sort (0 with bins from the
 *                                   occupancy bitmap), number of distinct per-tile cell keys); the
 *                                   third when bytes >= 24
 *  BIN_TARGET  int32   [B]          target of every bin; bins in ascending (target, kz, ky, kx)
 *  BIN_KEY     int32   [3][B]       cell index of every bin
 *  BIN_N       int64   [B]          members per bin
 *  BIN_MEAN    float64 [D][B]       mean state of the members of every bin (exact sums); with kept
 *                                   weights, the weighted mean the dummy used (CoM positions)
 *  LOGLIK      float64 [B] (pcSIR) or [sum N] (SIR)  log-likelihood per bin or particle
 *  WEIGHTS     float64 [sum N]      normalised weights, storage order
 *  TARGET      float64 [T][4]       per target: max log-weight M, S = sum exp(logw - M),
 *                                   N_eff, resampling uniform u
 *  CDF         float64 [sum N]      cumulative weights per target, storage order (targets that
 *                                   resampled; needs pcsir_set_debug)
 *  RESAMPLE    int32   [sum N]      s(j): parent of new particle j, index within its target
 *                                   (the identity for a target that did not resample)
 *  BINS_PER_PX int32   [T][3]       cells per pixel m of every target and axis in the last pcsir_step
 *  LOGW        float64 [sum N]      log-weight every current particle carries into the next frame:
 *                                   -log N_t for a target that resampled (or always, with
 *                                   neff_threshold above 1), else its normalised log-weight */
typedef enum {
  PCSIR_DUMP_PROPAGATED = 0,
  PCSIR_DUMP_KEYS = 1,
  PCSIR_DUMP_COUNTS = 2,
  PCSIR_DUMP_BIN_TARGET = 3,
  PCSIR_DUMP_BIN_KEY = 4,
  PCSIR_DUMP_BIN_N = 5,
  PCSIR_DUMP_BIN_MEAN = 6,
  PCSIR_DUMP_LOGLIK = 7,
  PCSIR_DUMP_WEIGHTS = 8,
  PCSIR_DUMP_TARGET = 9,
  PCSIR_DUMP_CDF = 10,
  PCSIR_DUMP_RESAMPLE = 11,
  PCSIR_DUMP_LOGW = 12,
  PCSIR_DUMP_BINS_PER_PX = 13
} pcsir_dump;

pcsir_status pcsir_debug_dump(pcsir_ctx *ctx, int32_t what, void *dst_dev, size_t bytes);

/* Replay each step as a captured HIP graph (on != 0, the default) or launch
 * its kernels one by one. The graph of a step kind is captured on its first
 * use (on a private stream; nothing runs during capture) and launched on the
 * context's stream; per-step values (frame pointer, frame index) are passed
 * through device memory, so replays need no parameter updates. Steps launch
 * kernels one by one while timing is on. */
pcsir_status pcsir_set_graphs(pcsir_ctx *ctx, int32_t on);

/* Allow PCSIR_DUMP_CDF (on != 0; off by default). The step keeps the
 * per-particle cumulative weights on chip except in tiles with many offspring;
 * the view forms them again, for every target that resampled, with the step's
 * own scan over the last step's weights. */
pcsir_status pcsir_set_debug(pcsir_ctx *ctx, int32_t on);

/* Per-kernel times, in milliseconds, of every launch since timing was turned
 * on (pcsir_set_timing) or since the previous pcsir_kernel_times call, taken
 * with HIP events recorded on the context's stream between the launches (up
 * to 8191 launches are kept). names/ms: host arrays of capacity `cap`; the
 * number of entries written goes to *count. Synchronises and clears the log. */
pcsir_status pcsir_set_timing(pcsir_ctx *ctx, int32_t on);
pcsir_status pcsir_kernel_times(pcsir_ctx *ctx, const char **names, float *ms, int32_t cap, int32_t *count);

/* Launch shapes of the pcSIR step. None of them changes any result: bins
 * are the sorted distinct cell keys whatever the tile size, bin sums are exact
 * integers, no reduction depends on the grid, and a scan tile's offspring get
 * the same parents whichever resampling path resolves them. */
typedef struct {
  int32_t bin_tile;     /* particles per work item of the bin sums: 1024, 2048 or 4096
                           (default 4096); the key deduplication takes 8192 */
  int32_t list_blocks;  /* workgroups of the sort and segment passes over the list of
                           distinct keys (sort_bins = 1): 64 .. 2048 (default 1024) */
  int32_t digit_bits;   /* widest digit of the radix sort, 6 .. 11 (default 11); the
                           width actually used is the narrowest that keeps the fewest passes */
  int32_t grid_per_cu;  /* workgroups per compute unit of the grid-stride kernels
                           (likelihood, surrogate, dummies): 4 .. 64 (default 32) */
  int32_t resample_light; /* most new particles that one 2048-particle tile of the weight
                           scan resolves itself, from its cumulative weights on chip:
                           0 .. 4096 (default 4096); a tile with more offspring stores its
                           cumulative weights, and blocks of 1024 new particles resolve them */
  int32_t sort_bins;    /* how the bins are numbered (the same bins either way: the occupied
                           cells in ascending key order): 0 (default) from a bitmap of the
                           occupied cells, one bit per cell key, and a popcount scan over its
                           words; 1 by a radix sort of the list of distinct per-tile keys */
} pcsir_tuning;

/* Current launch shapes. */
pcsir_status pcsir_get_tuning(const pcsir_ctx *ctx, pcsir_tuning *out);

/* Set the launch shapes (validated; E_INVAL when out of range). Synchronises the
 * context's stream and drops captured graphs, which are captured again on the
 * next step. */
pcsir_status pcsir_set_tuning(pcsir_ctx *ctx, const pcsir_tuning *tuning);

/* Self-tuning of the launch shapes on the caller's data: a coordinate search,
 * one field at a time, over sort_bins {0, 1} first, then in the order above
 * bin_tile {1024, 2048, 4096}, list_blocks {256, 512, 1024, 2048} and
 * digit_bits {8, 9, 10, 11} (these two only when the sort numbers the bins),
 * grid_per_cu {8, 16, 32, 64} and resample_light {1024, 2048, 4096},
 * keeping the best setting of each field before moving to the next. A trial
 * restores the particles, runs one untimed pcsir_step on `frame_dev` with
 * frame index k (graph capture), restores them again and times `reps` steps with HIP events on the context's stream.
 * state_scratch_dev: caller buffer of D * sum(N_t) floats that receives the
 * current particles first; the particles are restored from it at the end
 * (no step has then run: pcsir_estimate needs a new step). The best setting is
 * applied to ctx and written to *best (may be NULL), its time per step in ms to
 * *best_ms (may be NULL), the number of trials to *trials (may be NULL). */
pcsir_status pcsir_autotune(pcsir_ctx *ctx, const float *frame_dev, int32_t H, int32_t W, int64_t k, int32_t reps,
                            float *state_scratch_dev, pcsir_tuning *best, float *best_ms, int32_t *trials);

#ifdef __cplusplus
}
#endif
#endif /* PCSIR_H */
