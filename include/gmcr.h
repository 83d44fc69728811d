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
 *   - Limits: D in {1, 3}; 1 <= kmax <= 16; reconstruct position
 *     dimensions 0 <= dx <= 3.  Cells of up to 8192 particles run in the
 *     register-resident EM launches; larger cells in a launch that re-reads
 *     their particles on every pass (same results, slower per particle).
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
#define GM_ENOCONV (-5)   /* iterative solve stopped above its tolerance */
#define GM_EIO (-6)       /* a file could not be opened, read or written */
#define GM_ETOOBIG (-7)   /* input larger than a fixed limit of the entry point */

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
                             without annihilation (default 1e-7); FP32
                             iterations, which resolve L only to about 1e-7 n,
                             also stop after such a sweep with |L_s - L_{s-1}|
                             <= tol_rel n or L_s < L_{s-1} (the component
                             updates do not lower L) */
    uint64_t seed;        /* seed of the cold-start particle choice */
    int32_t estep_fp64;   /* 0: EM iterations in FP32 (default); 1: in FP64 */
    int32_t outer_k;      /* 0: one run of the sweeps (the paper's algorithm, default);
                             1: outer search over K: after every converged run keep
                             the state if its penalised L is the best so far, remove
                             the least probable component (smallest weight, lowest
                             slot on ties) and run again, down to K = 1; the best
                             state is the result (the component-wise algorithm the
                             paper cites for its penalised likelihood, Sec. 1).
                             Every run counts its own sweeps for the stop test and
                             the cap; sweeps and visits report the totals.  Ignored
                             in replay mode (fixed_sweeps > 0). */
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
 * coordinates as v.  Same layout as gm_mix; the first min(K[c], kmax) slots
 * are used, their weights renormalised.  A start for which eq. (omegak) is
 * undefined -- N - T K / 2 <= 0, or N w_k <= T/2 for a supplied component
 * (N the cell's particle count, T = D(D+3)/2) -- is not used: the cell
 * starts cold and is flagged GM_ST_WARM_FALLBACK (gm_warm_decode never
 * produces one).  When running to convergence, a cell whose warm-started penalised
 * likelihood ends below that of the single Gaussian with its moments, less
 * 1e-5 of its magnitude, is fitted again from the cold start and flagged
 * GM_ST_WARM_FALLBACK (its other flags are the cold fit's; visits count
 * both fits). */
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

/*
 * gm_compress_noalloc -- gm_compress for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * gm_compress, without the workspace: the library keeps the workspace in a
 * fixed device array of its own, one per GPU, held until the process ends
 * (about 11 MB: n_cells <= GM_NOALLOC_MAX_CELLS; larger batches return
 * GM_ETOOBIG and enqueue nothing).  The first call on a device looks up that
 * device's array and creates the library's stream set for it (no memory
 * allocation); later calls only enqueue kernels.  The array starts every call
 * from kernels that rewrite what they read, so a call does not depend on the
 * previous one.  Calls that overlap on one GPU (two host threads, or two
 * streams without ordering between them) share the array and race: order
 * them on one stream or serialise them.  Callers that can allocate should
 * use gm_compress with their own workspace.
 */
#define GM_NOALLOC_MAX_CELLS 65536
int gm_compress_noalloc(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                        const gm_opts* o, const int32_t* fixed_sweeps, const gm_init* init, const gm_mix* out,
                        void* stream);

/* ---- launch-plan autotuner ----
 * gm_compress runs the EM iterations in twelve length buckets (largest
 * cells: 64, 128, 256, 512, 1024, 1536, 2048, 2560, 3072, 3584, 4096, 8192
 * particles at kmax <= 8; 128, 256, 512, 768, 1024, 1280, 1536, 1792, 2048,
 * 2560, 4096, 8192 at kmax > 8), each a
 * persistent launch whose workgroups take cells from a queue, each on a
 * library stream of its own (cells of more than 8192 particles run on the
 * caller's stream), so that all thirteen launches run concurrently.  The
 * launches of buckets whose workgroups fill a compute unit's register file
 * (eight or more waves of a standard build, sixteen of a lean one) are
 * released first and the others about 40 us later, after a one-wave wait
 * kernel on the caller's stream that ends at once when those buckets hold
 * no cell.  HIP
 * maps streams onto GPU_MAX_HW_QUEUES hardware queues per process (default
 * 4): run with GPU_MAX_HW_QUEUES >= 13 (set before the HIP runtime starts)
 * for them to overlap; with fewer, launches sharing a queue run one after
 * another (same results, longer EM phase).  The same holds for a captured
 * compress: a HIP graph replay runs the graph's parallel launches on the
 * few streams of the runtime's graph executor (three or four hardware
 * queues measured), so a replayed EM phase is several times longer than
 * an eager one (same results).  A bucket can run with
 * several launch variants: particles per thread (1, 2, 4, 5, 6, 7, 8, 16), the
 * matching number of 64-lane waves per workgroup, density terms kept in
 * registers or recomputed, and the standard build (up to 8 waves per
 * workgroup, up to 256 VGPRs per lane) or, for FP32 iterations, the lean
 * build (up to 16 waves, at most 128 VGPRs: twice the waves per SIMD).
 * With FP32 iterations at kmax 16 the buckets of cells above 2048
 * particles hold few cells, and a single long fit there can set the
 * phase's length: they run by default with a lean build of more than 8
 * waves (4 or 8 recomputed particles per thread), and in 3V the cells of
 * 2049-4096 particles with eight waves of 5 and 8 register-resident
 * particles per thread instead; the tuner chooses only among these
 * builds there.  The cells of 1025-1792 particles run by default as four
 * waves of 5, 6 or 7 register-resident particles per thread.  gm_autotune measures, on the caller's batch,
 * every non-empty bucket alone under each variant, keeps the fastest per
 * bucket (and, as a second plan, the fastest lean build where there is
 * one), gives each bucket a library stream of its own, longest first, times
 * the concurrent EM phase of these plans and of the built-in plan (the
 * median of three runs each, the plans in turn), and installs the fastest
 * for this device,
 * D, kmax class (<= 8 or <= 16), precision and kind of start (warm when
 * init supplies mixtures).  Later gm_compress calls of that kind use it.
 * Arguments as for gm_compress (converged mode, no fixed sweeps); `out`
 * holds a complete compress result afterwards.  Synchronous on `stream`;
 * it must not run while other host threads call gm_compress on the device,
 * nor with gm_profile enabled (GM_EINVAL).
 * report: nullable, at least GM_TUNE_REPORT_LEN doubles: [0] EM phase of
 * the built-in plan (ms), [1] of the tuned plan, [2 + b] bucket b's
 * fastest standalone time (0 when empty), [14 + b] the installed variant of
 * bucket b as per_thread * 1000 + waves * 10 + mode, mode = (1 if
 * register-resident) + (2 if lean), [26 + b] its stream (0-11 library
 * streams, 12 the caller's, which also carries the cells larger than the
 * buckets hold). */
#define GM_TUNE_REPORT_LEN 38
int gm_autotune(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                const gm_opts* o, const gm_init* init, const gm_mix* out, void* ws, size_t ws_bytes,
                void* stream, double* report, int32_t report_len);

/* Install a plan by hand for (D, kmax class, fp64, warm): variant[b] and
 * (nullable) lane[b] for the twelve buckets, coded as in the report; a
 * variant must be built (see above) and cover the bucket: 64 * per_thread *
 * waves >= the bucket's largest cell, waves <= 8 (16 for lean builds).
 * Built: standard 1, 2, 4, 8 register-resident (8 for FP32 only at kmax
 * > 8; 5, 6, 7 for FP32 at kmax > 8) and 8, 16 recomputed; lean (FP32
 * only) 1, 2 register-resident and 4, 8 recomputed.
 * GM_EINVAL otherwise. */
int gm_autotune_set(int32_t D, int32_t kmax, int32_t fp64, int32_t warm, const int32_t* variant,
                    const int32_t* lane);

/* Forget every tuned plan; gm_compress returns to the built-in plans. */
int gm_autotune_reset(void);

/* The plan gm_compress uses on the current device for (D, kmax class,
 * fp64, warm): variant[b] coded as in the report, and (nullable) lane[b]
 * and order[b] (launch order, 0 first) for the twelve buckets, caller-owned
 * arrays of 12.  Returns 1 for a plan installed by gm_autotune (also where
 * it kept the built-in plan), gm_autotune_set or gm_autotune_load, 0 where
 * none is installed (the built-in plan; also when no device is visible),
 * GM_EINVAL for bad arguments. */
int gm_autotune_get(int32_t D, int32_t kmax, int32_t fp64, int32_t warm, int32_t* variant, int32_t* lane,
                    int32_t* order);

/* Launch-plan cache file (plain text, one plan per line:
 *   gmcr-plan 1 <arch> <CUs> <D> <kmax class 8|16> <fp64> <warm>
 *   variant[12] lane[12] order[12]),
 * keyed by the device (architecture name and CU count), D, kmax class,
 * precision and kind of start, with the variant, stream and launch order of
 * every length bucket.  gm_autotune_save writes the current device's
 * installed plans (those gm_autotune_get reports as 1) to `path`, keeping the lines of other devices already in the file;
 * GM_EINVAL (NULL or empty path), GM_EHIP (no device), GM_EIO.
 * gm_autotune_load reads `path` and installs the plans whose device key is
 * the current device's, each checked as by gm_autotune_set (and the order a
 * permutation of the buckets); blank lines and lines starting with '#' are
 * skipped.  A malformed or invalid line rejects the whole file before any
 * plan is installed (GM_EINVAL); GM_EIO if the file cannot be read.
 * Returns the number of plans installed.  Not safe against concurrent
 * gm_compress or gm_autotune calls. */
int gm_autotune_save(const char* path);
int gm_autotune_load(const char* path);

/* ---- standard EM with K-means start and Anderson acceleration ----
 * The non-adaptive EM of Sec. 3.4 (fixed K, joint E-step, weights N_k / N),
 * as the paper uses to study faster convergence.  Per cell, K0 = min(K, n)
 * components start at the cold-start particles of gm_compress (the same
 * Philox draw, without the floor(N/T) cap) with the cell covariance and
 * equal weights, or (kmeans = 1) at the mixture of a K-means clustering
 * started from those particles (Lloyd's algorithm in FP64 on the centred
 * velocities, Euclidean distance, ties to the lowest slot, weighted
 * centroids, an emptied centre stays put, at most 100 passes; weights W_k /
 * N, centroids, cluster covariances).  Iterations apply the EM map G (FP32
 * E-step and sums) to theta = (w_k, mu_k, M2_k = Sigma_k + mu_k mu_k^T) and,
 * with aa_memory = m > 0, mix it by Anderson acceleration in FP64
 * (theta_{i+1} = G(theta_i) - dG gamma, gamma the least-squares
 * coefficients of f_i = G(theta_i) - theta_i on the last min(m, i)
 * differences of f, by modified Gram-Schmidt).  A mixed iterate with a
 * negative weight or an indefinite Sigma, or a numerically dependent
 * difference, resets the history and takes G(theta_i); a mixed iterate
 * whose log-likelihood is below the last accepted one's is replaced by G of
 * that iterate.  Stop when the log-likelihood changes by at most tol_rel
 * (relative) between accepted iterates or after max_sweeps evaluations of
 * G; the unpenalised joint FP64 step of gm_compress then follows (it is the
 * standard EM step after the iteration and restores the moments exactly).
 *
 * Output record as gm_compress, with: K the components left with weight;
 * L_pen the log-likelihood sum_p a_p ln sum_k w_k f_k(v_p) at the last
 * iterate (a normalised to sum n); L_final the penalised likelihood of the
 * output; sweeps the evaluations of G; visits sweeps * K0; MAXSWEEPS when
 * the cap was reached.  resets [n_cells] (Anderson resets and rejections),
 * kmeans_passes [n_cells] and ll_trace [n_cells * max_sweeps] (the
 * log-likelihood at every evaluation; untouched after the last) are
 * nullable device arrays.  n_tot = cell_off[n_cells] (a cell reaching
 * beyond n_tot is not fitted: K = 0, GM_ST_DEGENERATE).  Options: as
 * gm_compress, estep_fp64 = 0 (else GM_ENOTIMPL), outer_k = 0; 1 <= K <=
 * kmax; 0 <= aa_memory <= 5. */
size_t gm_compress_standard_workspace(int64_t n_cells, int64_t n_tot, const gm_opts* o);
int gm_compress_standard(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                         int64_t n_tot, const gm_opts* o, int32_t K, int32_t kmeans, int32_t aa_memory,
                         const gm_mix* out, int32_t* resets, int32_t* kmeans_passes, double* ll_trace, void* ws,
                         size_t ws_bytes, void* stream);

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

/* ---- learned warm start ----
 * The paper starts every cell's EM from random particles (Sec. 2.3) and
 * notes that the iteration converges slowly from poor starting points while
 * better ones speed it up (Sec. 3.4).  The warm start maps per-cell features
 * of the velocity distribution to an initial mixture (a gm_init record) with
 * a 105 -> 256 -> 256 -> 160 perceptron (ReLU hidden layers) whose products
 * run on BF16 matrix cores with FP32 accumulation.  gm_compress keeps a warm
 * start only if its converged penalised likelihood is at least that of the
 * single Gaussian with the cell's moments; otherwise it refits the cell from
 * the cold start and sets GM_ST_WARM_FALLBACK.  Only D = 3 is built.
 *
 * Features (105 per cell, stored as BF16 bit patterns in rows of 128, the
 * last 23 zero): with m, C the cell's weighted mean and covariance and
 * C = L_C L_C^T, the whitened velocities u = L_C^-1 (v - m); three 32-bin
 * histograms of u_x, u_y, u_z over [-4, 4) (bin width 1/4, values outside
 * clamped to the end bins) weighted by alpha/W; E[u_d^3] (3); E[u_d^4] - 3
 * (3); E[u_x^2 u_y^2] - 1, E[u_x^2 u_z^2] - 1, E[u_y^2 u_z^2] - 1, all
 * expectations weighted by alpha/W.  The frame record (9 doubles per cell)
 * is m (3) and L_C packed lower row-major (00, 10, 11, 20, 21, 22); a cell
 * that is empty or has a singular covariance gets zero features and a zero
 * factor, and decodes to K = 0 (cold start).
 *
 * Network output (160 FP32 per cell): 16 slots of (logit, mu_hat[3],
 * ln l00, l10, ln l11, l20, l21, ln l22) in the whitened frame.  Decode:
 * w = softmax(logits); keep, in slot order, the slots with n w > T/2 (at most
 * kmax; if none, the most probable), renormalise their weights; mu = m +
 * L_C mu_hat; Sigma = (L_C L_hat)(L_C L_hat)^T.
 *
 * Training targets (160 FP32 per cell): a fitted mixture in the same frame
 * and slot layout (weight in place of the logit), slots sorted by weight
 * descending (ties by mu_hat_x ascending), unused slots zero.  Loss per
 * batch of B cells: (1/B) sum over cells of the soft cross-entropy
 * -sum_j w_t,j ln softmax_j plus lambda sum_j w_t,j (|mu_hat_j - mu_t,j|^2 +
 * |l_j - l_t,j|^2) over the 9 non-logit slot entries.  Optimiser: Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights; the products
 * use BF16 copies refreshed after every step.
 *
 * Parameters (gm_warm_param_count() FP32 values, the layout of get/set):
 * W1 [128][256] (rows 105..127 unused), b1 [256], W2 [256][256], b2 [256],
 * W3 [256][160], b3 [160]; weight matrices row-major [in][out].
 */
typedef struct gm_warm gm_warm;

size_t gm_warm_param_count(void);

/* Create a model with Glorot-uniform weights drawn from Philox4x64-10
 * (key (seed, "WARM"), counter (index, tensor, 0, 0)) and zero biases, and
 * training buffers for batches of `batch` cells (1 <= batch <= 2^20).
 * Allocates device memory on the current device; D must be 3. */
int gm_warm_create(gm_warm** model, int32_t D, int32_t kmax, int32_t batch, uint64_t seed, void* stream);
/* Free the model (waits for the device). */
void gm_warm_destroy(gm_warm* model);
/* Copy the FP32 parameters to / from HOST memory of gm_warm_param_count()
 * floats (synchronous).  set_params also resets the Adam state. */
int gm_warm_get_params(const gm_warm* model, float* host);
int gm_warm_set_params(gm_warm* model, const float* host);
/* Write the model's FP32 parameters to a file (synchronous): the 8 bytes
 * "GMCRWRM1", int32 D, int32 kmax, uint64 gm_warm_param_count(), then the
 * parameters in the get/set layout, host byte order.  The Adam state and
 * step count are not stored.  GM_EIO if the file cannot be written. */
int gm_warm_save(const gm_warm* model, const char* path);
/* Create a model from a file written by gm_warm_save, with training buffers
 * for batches of `batch` cells (as gm_warm_create; fresh Adam state).  The
 * file is read and checked before any device memory is allocated: GM_EIO if
 * it cannot be opened, is truncated or has trailing bytes, GM_EINVAL if it
 * is not a model file of this layout (magic, D = 3, kmax 1..16, parameter
 * count). */
int gm_warm_load(gm_warm** model, const char* path, int32_t batch, void* stream);
/* Copy the gradient of the last gm_warm_train_step to HOST memory
 * (synchronous; same layout as the parameters). */
int gm_warm_gradients(const gm_warm* model, float* host);

/* Features and frames of n_cells D = 3 cells (device arrays):
 *   v, alpha, cell_off  as for gm_compress
 *   feats  [n_cells * 128] uint16 BF16 bit patterns
 *   frame  [n_cells * 9] FP64 */
int gm_warm_features(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells, int32_t D,
                     uint16_t* feats, double* frame, void* stream);

/* Network outputs Y [n_rows * 160] FP32 for features [n_rows * 128] BF16;
 * ws: device workspace of at least gm_warm_forward_workspace(n_rows) bytes. */
size_t gm_warm_forward_workspace(int64_t n_rows);
int gm_warm_forward(const gm_warm* model, const uint16_t* feats, int64_t n_rows, float* Y, void* ws,
                    size_t ws_bytes, void* stream);

/* Decode Y into initial mixtures (gm_init layout, kmax slots; K = 0 where
 * the frame has no factor).  cell_off gives the cell sizes n. */
int gm_warm_decode(const float* Y, const double* frame, const int64_t* cell_off, int64_t n_cells, int32_t kmax,
                   int32_t* K, double* omega, double* mu, double* sigma, void* stream);

/* kmax of a model (the number of component slots it predicts); 0 for NULL. */
int gm_warm_model_kmax(const gm_warm* model);

/*
 * gm_compress_warm -- the learned warm start and the compress in one call
 * (the warm path of the compress entry point: gm_compress with a model
 * handle).  Enqueues on `stream`: features of every cell (gm_warm_features),
 * the network and the decode into initial mixtures (gm_warm_infer), then
 * gm_compress from those mixtures (converged mode;
 * a cell whose warm fit ends below the single Gaussian is refitted from the
 * cold start and flagged GM_ST_WARM_FALLBACK, see gm_init).  The result is
 * the one gm_compress gives for the decoded mixtures.  Arguments as for
 * gm_compress; o->D must be 3 and o->kmax the model's kmax (GM_EINVAL
 * otherwise).  ws: device workspace of at least
 * gm_compress_warm_workspace(n_cells, o) bytes holding the compress
 * workspace, the features, frames and decoded mixtures.
 * The model is only read (its weights); calls on one model may overlap.
 */
size_t gm_compress_warm_workspace(int64_t n_cells, const gm_opts* o);
int gm_compress_warm(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                     const gm_opts* o, const gm_warm* model, const gm_mix* out, void* ws, size_t ws_bytes,
                     void* stream);

/* Network and decode fused (one launch, 32 cells per workgroup, the
 * activations in LDS): the initial mixtures gm_warm_forward followed by
 * gm_warm_decode give, bit for bit, without the FP32 network outputs
 * leaving the chip.  Arguments as for those two calls. */
int gm_warm_infer(const gm_warm* model, const uint16_t* feats, const double* frame, const int64_t* cell_off,
                  int64_t n_cells, int32_t kmax, int32_t* K, double* omega, double* mu, double* sigma, void* stream);

/* Training targets [n_cells * 160] FP32 from fitted mixtures (gm_mix
 * layout, kmax slots) and frames.  A component whose whitened covariance
 * does not factor gets L_hat = 1e-3 I. */
int gm_warm_targets(const int32_t* K, const double* omega, const double* mu, const double* sigma, int32_t kmax,
                    const double* frame, int64_t n_cells, float* targets, void* stream);

/* One Adam step on the rows idx[0..batch-1] (device int32) of feats
 * [n_rows * 128] BF16 and targets [n_rows * 160] FP32, learning rate lr > 0,
 * loss weight lambda >= 0.  An index outside [0, n_rows) contributes a zero
 * row (no loss, no gradient).  loss_rows: nullable device [batch] FP32
 * receiving each row's loss term (the batch loss is their sum divided by
 * batch).  Calls on one model must not overlap. */
int gm_warm_train_step(gm_warm* model, const uint16_t* feats, const float* targets, int64_t n_rows,
                       const int32_t* idx, float lr, float lambda, float* loss_rows, void* stream);

/* Training loop: `epochs` passes over the n_rows rows of feats / targets (as
 * for gm_warm_train_step), each in floor(n_rows / batch) Adam steps on
 * shuffled rows (the last partial batch is dropped).  The shuffle of epoch
 * e is a Fisher-Yates permutation (top index down; j = high 64 bits of
 * draw * (i + 1)) driven by splitmix64 from seed ^ (0xD1B54A32D192ED03 *
 * (e + 1)), so the loop equals gm_warm_train_step calls on those rows.
 * ws: device workspace of gm_warm_train_workspace(n_rows, batch) bytes
 * (the permutation and the per-row losses).  epoch_loss: nullable HOST
 * [epochs] receiving each epoch's mean row loss.  Synchronises the stream
 * once per epoch.  GM_EINVAL if n_rows < batch. */
size_t gm_warm_train_workspace(int64_t n_rows, int32_t batch);
int gm_warm_train(gm_warm* model, const uint16_t* feats, const float* targets, int64_t n_rows, int32_t epochs,
                  float lr, float lambda, uint64_t seed, void* ws, size_t ws_bytes, float* epoch_loss, void* stream);

/*
 * gm_reconstruct_tensor -- as gm_reconstruct, with a projection that matches
 * the whole second-moment tensor of the target, not only its trace.  With
 * the sample's N', p', S' (sums over the drawn particles) and the target's
 * W, P, S:
 *     v' = P / W + A (v - p' / N'),   A = L_t L_s^-1,
 *     L_t L_t^T = S - P P^T / W,      L_s L_s^T = S' - p' p'^T / N',
 * so the projected sample has mass W, momentum P and second moment S (the
 * whole pressure tensor, which the exact-moment step of Sec. 2.3.1 conserves
 * in the mixture; Lemons' scalar projection of Sec. 2.4.2 matches its trace
 * only).  In 1V the two projections coincide.  When either centred tensor
 * has a pivot^2 not above 1e-12 of its mean diagonal (n' <= D, or a
 * degenerate target) the sample is left as drawn and GM_ST_LEMONS_SKIPPED
 * is set.  Arguments, layouts and sampling as for gm_reconstruct.
 */
int gm_reconstruct_tensor(const int32_t* K, const double* omega, const double* mu, const double* sigma,
                          int32_t kmax, const int64_t* out_off, const double* target, int64_t n_cells, int32_t D,
                          int32_t dx, uint64_t seed, double* v_out, double* w_out, double* x_out, int32_t* status,
                          void* ws, size_t ws_bytes, void* stream);

/*
 * gm_project -- the projection of gm_reconstruct (tensor = 0, Lemons'
 * scalar form) or of gm_reconstruct_tensor (tensor = 1) applied to given
 * particles: v [n_tot * D] and w [n_tot] FP64 grouped by cell_off [n_cells
 * + 1], towards the moments record `moments` [n_cells * (1 + D + D(D+1)/2)]
 * (W, P, S packed) of each cell.  N', p' and S' (or E') are the sums over
 * the given weights, so after a change of the weights (the Gauss'-law
 * correction below) the projected particles carry momentum P and second
 * moment S (or energy tr(S) / 2) with the new mass N'.  v_out [n_tot * D]
 * may equal v (in place).  Status bits as gm_reconstruct (0 or
 * GM_ST_LEMONS_SKIPPED; empty cells 0).  D in {1, 3}.
 */
int gm_project(const double* v, const double* w, const int64_t* cell_off, const double* moments, int64_t n_cells,
               int32_t D, int32_t tensor, double* v_out, int32_t* status, void* stream);

/* ---- Gauss'-law weight correction (Sec. 2.4.1) ----
 * The resampled particles must deposit the charge density the original
 * ones did.  The mesh is periodic with unit cells: dx = 1, n_cells cells in
 * a row (nx = n_cells, or nx <= 0); dx = 2, nx * (n_cells / nx) cells, cell c
 * at (c % nx, c / nx).  Cell i has centre X_i = i + 1/2 (per axis); a
 * particle of cell c with cell-local position x in [0,1)^dx (the x_out of
 * gm_reconstruct) sits at X = (cell coordinates) + x.  Charge goes to the
 * mesh with the quadratic B-spline S2 (3 cells per axis):
 *     D_i = sum_p w_p S2(X_i - X_p)        (unit charge; rho_i times volume)
 * The per-cell corrections dA solve M dA = D_target - D(w) with
 * M_ij = sum_{p in cell j} S2(X_i - X_p) (the top-hat S0 selects the
 * particles of cell j, eq. p-weight-correction), and w'_p = w_p +
 * dA_{cell(p)} (eq. new-p-weight).  Sums are FP64 in a fixed order.
 *
 * Workspace (device, caller-owned, for both calls) of gm_gauss_workspace
 * bytes: 2 * 9 (2D; 3 in 1D) + 9 doubles per cell plus 16 bytes per 256
 * cells and the solver state, 256-byte aligned pieces.  Returns 0 for bad
 * arguments (dx not 1 or 2, n_cells < 1).
 */
size_t gm_gauss_workspace(int64_t n_cells, int32_t dx);

/* gm_deposit -- D_i of the particles x [n_tot * dx], w [n_tot] grouped by
 * cell_off into dep [n_cells] (FP64, device).  Enqueued on stream. */
int gm_deposit(const double* x, const double* w, const int64_t* cell_off, int64_t n_cells, int32_t dx, int32_t nx,
               double* dep, void* ws, size_t ws_bytes, void* stream);

/* gm_gauss_correct -- weights w [n_tot] (in place) corrected so that the
 * deposit of (x, w) equals dep_target [n_cells].  M dA = b is solved by
 * BiCGSTAB with the preconditioner diag(M) on the right, from dA = 0, until
 * the true residual |b - M dA| is at most tol |b| (0 < tol < 1), within
 * max_iter iterations in all (restarts from the true residual included).
 * Every cell must hold at least one particle (else GM_EINVAL, weights
 * untouched).  In 1D, M is then strictly diagonally dominant by columns
 * (each particle puts at least half its spline on its own cell, more unless
 * it sits on the cell's edge) and nonsingular; in 2D it is not dominant but
 * nonsingular for generic positions.  The iteration's scalars stay on the
 * device; the call reads them back once per 8 iterations and per restart,
 * so it synchronises `stream` and cannot be captured in a graph; the empty
 * cell check and GM_ENOCONV come from those reads, after kernels on the
 * workspace were enqueued.  iters_out (iterations) and resid_out (final
 * true relative residual) are host pointers, may be NULL.  Returns
 * GM_ENOCONV, with the weights corrected by the last iterate, when the
 * tolerance was not reached. */
int gm_gauss_correct(const double* x, double* w, const int64_t* cell_off, int64_t n_cells, int32_t dx, int32_t nx,
                     const double* dep_target, double tol, int32_t max_iter, void* ws, size_t ws_bytes, void* stream,
                     int32_t* iters_out, double* resid_out);

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
