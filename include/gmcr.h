/*
 * gmcr.h -- C ABI of libgmcr.so: Gaussian-mixture checkpoint-restart of
 * particle-in-cell velocity data on AMD Instinct MI355X (gfx950).
 *
 * Method: Chen, Chacon & Nguyen, "Gaussian-mixture checkpoint-restart for
 * particle-in-cell" (arXiv:2007.12273).
 *
 *   gm_compress     per spatial cell, fit the particle-weighted velocity
 *                   distribution with a Gaussian mixture by component-wise
 *                   adaptive EM under the minimum-message-length penalty
 *                   (Sec. 2.1-2.3, eqs. lnL-GM, responsibility, muk, sigmak,
 *                   omegak), then one unpenalised joint EM step (eq.
 *                   omegak-mle, Sec. 2.3.1) that makes the mixture's mass,
 *                   mean and second-moment tensor equal the particles'.
 *   gm_reconstruct  per cell, draw particles from the mixture by ancestral
 *                   sampling with equal weights and uniform positions
 *                   (Sec. 2.4, eq. mix-dist-1), then apply Lemons'
 *                   moment-matching projection (Sec. 2.4.2, eqs. alpha/beta)
 *                   so the sample's momentum and energy equal the targets.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller.  The library
 *     never frees caller memory.  Scratch memory is a caller-supplied
 *     workspace whose size is queried first.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t, NULL for
 *     the default stream).  Only host-side argument checks are synchronous.
 *   - Return value: GM_OK (0) or a negative error code (gm_strerror()).  An
 *     error return means nothing was enqueued.
 *   - Per-cell outcomes are reported in a status bitmask array (GM_ST_*);
 *     they are not errors.
 *   - Mixture records are padded to kmax components; slots >= K hold zeros.
 *   - Covariances are stored as the packed upper triangle, row-major:
 *     D = 3 -> (xx, xy, xz, yy, yz, zz); D = 1 -> (xx).
 *   - Limits: D in {1, 3}; 1 <= kmax <= 16; at most 8192 particles per
 *     cell (larger cells get K = 0 and GM_ST_DEGENERATE); reconstruct
 *     position dimensions 0 <= dx <= 3.
 */
#ifndef GMCR_H
#define GMCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define GM_OK 0
#define GM_EINVAL (-1)    /* bad scalar argument or NULL required pointer */
#define GM_EHIP (-2)      /* a HIP runtime call failed */
#define GM_ENOMEM (-3)    /* workspace missing or smaller than required */
#define GM_ENOTIMPL (-4)  /* combination not built into this library */

/* ---- per-cell status bits ---- */
#define GM_ST_SMALL_CELL_K1 (1 << 0)   /* n <= n_min: single Gaussian with the cell's moments */
#define GM_ST_K0_CAPPED (1 << 1)       /* initial K limited to floor(N/T) so N - T K / 2 > 0 */
#define GM_ST_COV_FLOOR (1 << 2)       /* a covariance needed eps*I to factor during EM */
#define GM_ST_MAXSWEEPS (1 << 3)       /* stopped at max_sweeps before the tolerance was met */
#define GM_ST_NEAR_TIE (1 << 4)        /* some N_k came within 1e-5*T/2 of the annihilation threshold */
#define GM_ST_WARM_FALLBACK (1 << 5)   /* warm start rejected; result is the cold-start fit */
#define GM_ST_NONFINITE_INPUT (1 << 6) /* non-finite velocity or non-positive/non-finite weight */
#define GM_ST_LEMONS_SKIPPED (1 << 7)  /* projection had no real solution; sample left as drawn */
#define GM_ST_DEGENERATE (1 << 8)      /* empty/oversized cell or singular covariance */

/* ---- options ---- */
typedef struct gm_opts {
    int32_t D;            /* velocity dimensions: 1 or 3 */
    int32_t kmax;         /* initial / maximum number of components, <= 16 */
    int32_t n_min;        /* cells with n <= n_min get the K = 1 closed form (default 10) */
    int32_t max_sweeps;   /* cap on EM sweeps (default 1000) */
    double tol_rel;       /* stop when |L_s - L_{s-1}| <= tol_rel |L_s| after a sweep
                             without annihilation (default 1e-7) */
    uint64_t seed;        /* seed of the cold-start particle choice */
    int32_t estep_fp64;   /* 0: EM iterations in FP32 (default); 1: in FP64 */
    int32_t reserved;     /* must be 0 */
} gm_opts;

/* Fill *o with the defaults above for the given D and kmax. */
void gm_opts_default(gm_opts* o, int32_t D, int32_t kmax);

/* Output record of gm_compress: caller-allocated device arrays.
 * M = 1 + D + D(D+1)/2 preserved-moment entries per cell: W = sum alpha,
 * P = sum alpha v (D), S = sum alpha v v^T (packed upper triangle). */
typedef struct gm_mix {
    int32_t* K;        /* [n_cells] live components */
    double* omega;     /* [n_cells * kmax] mixing weights, sum 1 over the first K */
    double* mu;        /* [n_cells * kmax * D] means */
    double* sigma;     /* [n_cells * kmax * D(D+1)/2] covariances, packed */
    double* moments;   /* [n_cells * M] W, P, S of the input particles */
    double* L_pen;     /* [n_cells] penalised log-likelihood at the converged penalised state */
    double* L_final;   /* [n_cells] penalised log-likelihood of the output mixture */
    int32_t* sweeps;   /* [n_cells] EM sweeps performed */
    int32_t* status;   /* [n_cells] GM_ST_* bits */
    int64_t* visits;   /* [n_cells] component updates performed (E-step + M-step pairs) */
} gm_mix;

/* Optional initial mixtures (learned warm start).  Cells with K[c] > 0
 * start from them instead of the random cold start; mu in the same
 * coordinates as v.  Same layout as gm_mix. */
typedef struct gm_init {
    const int32_t* K;
    const double* omega;
    const double* mu;
    const double* sigma;
} gm_init;

/* Bytes of workspace gm_compress needs for n_cells cells. */
size_t gm_compress_workspace(int64_t n_cells, const gm_opts* o);

/*
 * gm_compress -- per-cell adaptive EM-GM with the exact-moment finish.
 *
 *   v         [n_tot * D] FP64 velocities, row-major, cells contiguous
 *   alpha     [n_tot] FP64 particle weights (> 0)
 *   cell_off  [n_cells + 1] int64 exclusive prefix: cell c owns particles
 *             cell_off[c] .. cell_off[c+1]-1; must be non-decreasing
 *   fixed_sweeps  nullable [n_cells] int32: > 0 runs exactly that many
 *             sweeps in that cell (replay mode), <= 0 runs to convergence
 *   init      nullable: warm-start mixtures (see gm_init)
 *   out       output arrays, every pointer required
 *   ws        device workspace of at least gm_compress_workspace() bytes
 *
 * Per cell (Sec. 2.3): moments in FP64; cold start with min(kmax, n,
 * floor(N/T)) components whose means are distinct particles chosen by a
 * Philox4x64-10 partial Fisher-Yates draw (key (seed, "INIT"), counter
 * (j, cell, 0, 0)), covariances equal to the cell covariance and equal
 * weights; component-wise sweeps (E-step, M-step, annihilation when
 * N_k <= T/2, renormalisation) with T = D(D+3)/2; stop on the relative
 * change of eq. (lnL-GM); then the unpenalised joint FP64 step.
 */
int gm_compress(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                const gm_opts* o, const int32_t* fixed_sweeps, const gm_init* init, const gm_mix* out,
                void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace gm_reconstruct needs (currently 0; pass NULL). */
size_t gm_reconstruct_workspace(int64_t n_cells, int32_t D);

/*
 * gm_reconstruct -- per-cell ancestral sampling plus Lemons projection.
 *
 *   K, omega, mu, sigma  mixtures as produced by gm_compress (kmax slots)
 *   out_off   [n_cells + 1] int64 exclusive prefix of the number of
 *             particles n'_c to draw per cell
 *   target    [n_cells * M] FP64 per cell, the moments record layout of
 *             gm_compress (M = 1 + D + D(D+1)/2): W (mass), P (momentum,
 *             sum alpha v), S (packed sum alpha v v^T); the energy target is
 *             E = tr(S) / 2
 *   seed      Philox key (seed, "RECO"); particle i of cell c uses counters
 *             (i, c, b, 0), b = 0, 1; uniform j of the particle is word
 *             j % 4 of block j / 4, mapped to [0,1) from its top 53 bits.
 *             Uniform 0 picks the component (inverse CDF over cumulative
 *             omega), then ceil(D/2) Box-Muller pairs, then dx positions.
 *   v_out     [n'_tot * D] FP64, w_out [n'_tot] FP64 (= W / n'_c),
 *   x_out     [n'_tot * dx] FP64 in [0,1)^dx (cell-local), NULL if dx == 0
 *   status    [n_cells] int32 GM_ST_* bits
 *
 * The projection v' = a (v + beta) uses a = sqrt((2 E N' - |P|^2) /
 * (2 E' N' - |p'|^2)), beta = (P - a p') / (a N') with N', p', E' the
 * sample's moments; when either bracket is not above 1e-12 of its leading
 * term (2 E N' or 2 E' N', i.e. zero to rounding, as for n' = 1) the sample
 * is left as drawn and GM_ST_LEMONS_SKIPPED is set.
 */
int gm_reconstruct(const int32_t* K, const double* omega, const double* mu, const double* sigma, int32_t kmax,
                   const int64_t* out_off, const double* target, int64_t n_cells, int32_t D, int32_t dx,
                   uint64_t seed, double* v_out, double* w_out, double* x_out, int32_t* status, void* ws,
                   size_t ws_bytes, void* stream);

/* ---- diagnostics ----
 * Phase timing for benchmarks.  While enabled, gm_compress records HIP
 * events on its stream before the moment/plan kernels, before and after the
 * EM kernels and after the finish; gm_reconstruct records events around its
 * launch.  gm_profile_read waits for the last recorded events and writes the
 * durations in milliseconds of the most recent calls: ms[0] moments and
 * plan, ms[1] EM sweeps (all length buckets), ms[2] FP64 finish, ms[3]
 * reconstruct (-1 where nothing was recorded); n must be >= 4.  The events
 * are process-global: do not enable while calls run on several streams or
 * threads at once, nor during stream capture. */
void gm_profile_enable(int on);
int gm_profile_read(double* ms, int n);

/* Human-readable text for a return code. */
const char* gm_strerror(int code);

/* Library version as 10000*major + 100*minor + patch. */
int gm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GMCR_H */
