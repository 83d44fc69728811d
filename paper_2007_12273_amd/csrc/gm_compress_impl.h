// gm_compress_impl.h -- per-cell adaptive EM-GM for gfx950.
//
// Three kernels per compress call (plus the length-bucket plan):
//   k_moments  one wave per cell, FP64: W = sum alpha, P = sum alpha v,
//              S = sum alpha v v^T, mean m = P / W, covariance C about m (two
//              passes); classifies the cell (invalid / empty / small or
//              singular -> closed form / EM) and bins EM cells by length.
//   k_em       the hot loop.  Persistent workgroups pull cells of one length
//              bucket from a queue.  Centred FP32 velocities, normalised
//              weights and every (particle, component) density term stay in
//              VGPRs for the whole fit; LDS carries only the component
//              parameters and the cross-wave partial sums.  Writes the
//              converged penalised mixture into the output record.
//   k_finish   one wave (up to 512 particles) or one workgroup per cell, FP64:
//              the unpenalised joint EM step
//              (Sec. 2.3.1) or the single-Gaussian closed form, then the
//              penalised log-likelihood of the output mixture.
//
// EM arithmetic per cell (Sec. 2.3 of the paper):
//   start   cold: min(kmax, n, floor(N/T)) distinct particles (Philox partial
//           Fisher-Yates) as means, C as covariances, equal weights; or a
//           supplied warm-start mixture
//   sweep   for each live component k in slot order:
//             E-step  gamma_pk = a_p e_pk / sum_j e_pj            (eq. responsibility)
//             M-step  N_k, mu_k, Sigma_k about the new mean       (eqs. muk, sigmak)
//             remove k if N_k - T/2 <= 0                          (eq. omegak)
//             else w_k = (N_k - T/2)/(N - T K/2), renormalise     (eq. omegak, step 3)
//           then the penalised log-likelihood (eq. lnL-GM) and the stop test
//
// Density terms are kept relative to a per-particle reference in base 2:
//   e_pj = 2^(c_j - |A_j (x_p - mu_j)|^2 - ref_p),
//   c_j  = log2 u_j - D/2 log2(2 pi) - log2 sqrt(det Sigma_j),
//   A_j  = sqrt(log2(e)/2) L_j^{-1},   Sigma_j = L_j L_j^T,
// with u_j unnormalised weights (G = sum u_j).  A component update costs one
// exp2 per particle; the denominator sum_j e_pj is updated by the change of
// the one term and re-summed exactly where most of it cancelled.  At the end
// of a sweep ref_p + log2(sum_j e_pj) - log2 G is the particle's log2
// mixture density, the per-particle term of eq. (lnL-GM); the sum is exact
// there (from the stored terms in the register-resident buckets, recomputed
// every fourth sweep and after an annihilation in the others, which close
// the remaining sweeps with the running sum, accurate to a few FP32 ulps of
// the particle's density).  A particle
// whose sum underflows, or whose new term overflows the reference, is
// rebased: its terms are recomputed about their own maximum (a log2-space
// log-sum-exp).
#pragma once

#include "gm_device.h"
#include "gm_launch.h"

namespace gm {

// per-cell record written by k_moments, read by k_em and k_finish
template <int D>
struct CellInfo {
    double m[D];        // mean
    double C[ntri(D)];  // covariance about the mean (packed)
    double trC;
    double W;           // sum of weights
    int32_t kind;       // CELL_*
    int32_t n;
};

// CELL_BIG: more particles than the register-resident EM launches hold
// (kMaxCellParticles), fitted by k_em_big; CELL_OVERSIZE: a cell the
// standard EM's staging buffers do not reach (no mixture)
enum { CELL_EM = 0, CELL_CLOSED = 1, CELL_INVALID = 2, CELL_EMPTY = 3, CELL_OVERSIZE = 4, CELL_BIG = 5 };

struct CompressArgs {
    const double* v;
    const double* alpha;
    const int64_t* off;
    int64_t n_cells;
    void* cells;             // CellInfo<D>[n_cells]
    int32_t* list;           // bucketed EM cells
    int32_t* init_idx;       // [n_cells * kInitSlots] cold-start particle indices
    int32_t* plan;           // PLAN_* layout
    int32_t bucket;
    int32_t nwaves;
    int32_t kmax, n_min, max_sweeps;
    int32_t outer;           // 1: outer search over K (gm_opts.outer_k)
    int32_t std_K;           // > 0: standard EM with this K (start of min(K, n) particles, no cap)
    double tol;
    uint64_t seed;
    const int32_t* fixed;    // nullable
    gm_init init;            // init.K == nullptr: cold start
    gm_mix out;
};

// PLAN_LEVEL: per bucket, kPlanLevels counters of its cells by size level
// (counts in k_moments, turned into list positions by k_plan_scan)
constexpr int kPlanLevels = 16;
enum { PLAN_COUNT = 0, PLAN_BASE = 16, PLAN_QUEUE = 32, PLAN_LEVEL = 48, PLAN_SIZE = 48 + 16 * kPlanLevels };

// standard EM (gm_std.hip)
constexpr int kStdAaMax = 5;  // largest Anderson memory
struct StdArgs {
    CompressArgs a;
    int64_t n_tot;        // particles the staging buffers hold
    float* xa_w;          // [n_tot * (D + 1)] centred FP32 velocities and weights a_p (sum N)
    int32_t* assign;      // [n_tot] K-means labels
    int32_t K;            // components requested (<= kmax)
    int32_t kmeans;       // 1: K-means start
    int32_t aa_m;         // Anderson memory, 0 = plain EM
    int32_t* resets;      // nullable [n_cells]
    int32_t* kmeans_passes;  // nullable [n_cells]
    double* ll_trace;     // nullable [n_cells * max_sweeps]
};
constexpr int kInitSlots = 16;

constexpr double kSqrtHalfLog2e = 0.84932180028801904272;  // sqrt(log2(e) / 2)
constexpr double kLog2TwoPi = 2.6514961294723187980;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLnTwoPi = 1.8378770664093454836;

__host__ __device__ inline int bucket_of(int kmax_tpl, int n)
{
    for (int b = 0; b < kNumBuckets; ++b)
        if (n <= bucket_cfg(kmax_tpl, b).max_n) return b;
    return -1;
}

// Size level of an n-particle cell within its bucket's range: 0 for the
// largest cells, kPlanLevels - 1 for the smallest.  A bucket's queue hands
// out its cells level by level, largest first: the fit's cost grows with
// the cell's size (more particles per update and, on these inputs, more
// sweeps), so the longest fits start first and do not trail the phase.
__host__ __device__ inline int size_level(int kmax_tpl, int b, int n)
{
    if (b < 0 || b >= kNumBuckets) return 0;
    const int hi = bucket_cfg(kmax_tpl, b).max_n;
    const int lo = b == 0 ? 1 : bucket_cfg(kmax_tpl, b - 1).max_n + 1;
    const int l = (int)((int64_t)(hi - n) * kPlanLevels / (hi - lo + 1));
    return l < 0 ? 0 : (l >= kPlanLevels ? kPlanLevels - 1 : l);
}

// ===========================================================================
// k_moments: one wave per cell (kMomCellsPerBlock cells per workgroup), no
// workgroup barrier; fixed-order DPP wave sums
// ===========================================================================
constexpr int kMomCellsPerBlock = 4;

template <int D>
__global__ __launch_bounds__(64 * kMomCellsPerBlock) void k_moments(CompressArgs A)
{
    constexpr int NT = ntri(D);
    constexpr int NM = nmom(D);
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * kMomCellsPerBlock + (threadIdx.x >> 6);
    if (c >= A.n_cells) return;  // whole waves leave
    const int64_t o0 = A.off[c];
    const int64_t n64 = A.off[c + 1] - o0;
    CellInfo<D>* ci = static_cast<CellInfo<D>*>(A.cells) + c;
    double* mom = A.out.moments + (size_t)c * NM;
    if (n64 <= 0 || n64 > 0x7fffffff) {
        if (lane < NM) mom[lane] = 0.0;
        if (lane == 0) {
            ci->kind = n64 == 0 ? CELL_EMPTY : CELL_OVERSIZE;
            ci->n = 0;
        }
        return;
    }
    const int n = (int)n64;
    const double* vc = A.v + o0 * D;
    const double* ac = A.alpha + o0;
    double acc[NM + 1];
#pragma unroll
    for (int t = 0; t < NM + 1; ++t) acc[t] = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double al = ac[i];
        double x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = vc[(size_t)i * D + d];
        bool bad = !isfinite(al) || !(al > 0.0);
#pragma unroll
        for (int d = 0; d < D; ++d) bad |= !isfinite(x[d]);
        acc[NM] += bad ? 1.0 : 0.0;
        acc[0] += al;
#pragma unroll
        for (int d = 0; d < D; ++d) acc[1 + d] += al * x[d];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b) acc[1 + D + tri_idx<D>(a, b)] += al * x[a] * x[b];
    }
#pragma unroll
    for (int t = 0; t < NM + 1; ++t) acc[t] = wave_sum(acc[t]);
    if (acc[NM] > 0.0) {
        if (lane < NM) mom[lane] = 0.0;
        if (lane == 0) {
            ci->kind = CELL_INVALID;
            ci->n = n;
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < NM; ++t)
        if (lane == t) mom[t] = acc[t];
    const double W = acc[0];
    double m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = acc[1 + d] / W;
    double cov[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) cov[t] = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double al = ac[i];
        double x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = vc[(size_t)i * D + d] - m[d];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b) cov[tri_idx<D>(a, b)] += al * x[a] * x[b];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) cov[t] = wave_sum(cov[t]);
    double C[NT], L[NT], tr = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) C[t] = cov[t] / W;
#pragma unroll
    for (int d = 0; d < D; ++d) tr += C[tri_idx<D>(d, d)];
    const bool spd = chol<D, double>(C, L);
    const bool closed = n <= A.n_min || !spd;
    if (lane == 0) {
        for (int d = 0; d < D; ++d) ci->m[d] = m[d];
        for (int t = 0; t < NT; ++t) ci->C[t] = C[t];
        ci->trC = tr;
        ci->W = W;
        ci->n = n;
        const bool big = n > kMaxCellParticles;
        ci->kind = closed ? CELL_CLOSED : (big ? CELL_BIG : CELL_EM);
        if (!closed) {
            const int kt = A.kmax <= 8 ? 8 : 16;
            const int b = big ? kNumBuckets : bucket_of(kt, n);
            atomicAdd(&A.plan[PLAN_COUNT + b], 1);
            atomicAdd(&A.plan[PLAN_LEVEL + b * kPlanLevels + size_level(kt, b, n)], 1);
        }
    }
    if (closed) return;
    // cold start: min(kmax, n, floor(N/T)) distinct particles by a partial
    // Fisher-Yates draw; draw j swaps positions j and j + floor(x (n - j) /
    // 2^64), x the first word of Philox with key (seed, "INIT") and counter
    // (j, cell, 0, 0).  Lane j computes draw j; the swaps then run in order
    // on every lane alike, the permutation kept as a sparse record of the
    // swapped positions.
    const double T = 0.5 * D * (D + 3);
    int K = min(A.std_K > 0 ? A.std_K : A.kmax, n);
    const int cap = max(1, (int)floor((double)n / T));
    if (A.std_K == 0 && K > cap) K = cap;
    int my_rr = 0;
    if (lane < K) {
        const u64x4 r = philox4x64_10((uint64_t)lane, (uint64_t)c, 0, 0, A.seed, kTagInit);
        my_rr = lane + (int)__umul64hi(r.x, (uint64_t)(n - lane));
    }
    int pos[2 * kInitSlots], val[2 * kInitSlots], nrec = 0;
    for (int j = 0; j < K; ++j) {
        const int rr = __builtin_amdgcn_readlane(my_rr, j);
        int vr = rr, vj = j, trr = -1, tj = -1;
        for (int t = 0; t < nrec; ++t) {
            if (pos[t] == rr) {
                vr = val[t];
                trr = t;
            }
            if (pos[t] == j) {
                vj = val[t];
                tj = t;
            }
        }
        if (tj < 0) {
            tj = nrec++;
            pos[tj] = j;
        }
        val[tj] = vr;
        if (rr != j) {
            if (trr < 0) {
                trr = nrec++;
                pos[trr] = rr;
            }
            val[trr] = vj;
        }
        if (lane == 0) A.init_idx[(size_t)c * kInitSlots + j] = vr;
    }
}

// bucket bases and queue resets (one thread); slot kNumBuckets lists the
// cells larger than the buckets hold
static __global__ void k_plan_scan(int32_t* plan)
{
    int base = 0;
    for (int b = 0; b <= kNumBuckets; ++b) {
        plan[PLAN_BASE + b] = base;
        plan[PLAN_QUEUE + b] = 0;
        // level counts -> first list position of each level
        int pos = base;
        for (int l = 0; l < kPlanLevels; ++l) {
            const int cnt = plan[PLAN_LEVEL + b * kPlanLevels + l];
            plan[PLAN_LEVEL + b * kPlanLevels + l] = pos;
            pos += cnt;
        }
        base += plan[PLAN_COUNT + b];
    }
}

// EM cells into their buckets, level by level: per wave, one atomic per
// distinct (bucket, size level) among its lanes (an add of the group's size
// to that level's list position), and each lane's slot is its rank within
// the group
template <int D>
__global__ void k_plan_scatter(CompressArgs A)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int key = -1;
    if (c < A.n_cells) {
        const CellInfo<D>* ci = static_cast<const CellInfo<D>*>(A.cells) + c;
        const int kt = A.kmax <= 8 ? 8 : 16;
        int b = -1;
        if (ci->kind == CELL_EM) b = bucket_of(kt, ci->n);
        else if (ci->kind == CELL_BIG) b = kNumBuckets;
        if (b >= 0) key = b * kPlanLevels + size_level(kt, b, ci->n);
    }
    uint64_t todo = __builtin_amdgcn_ballot_w64(key >= 0);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int kl = __builtin_amdgcn_readlane(key, leader);
        const uint64_t group = __builtin_amdgcn_ballot_w64(key == kl);
        int first = 0;
        if (lane == leader) first = atomicAdd(&A.plan[PLAN_LEVEL + kl], __builtin_popcountll(group));
        first = __builtin_amdgcn_readlane(first, leader);
        if (key == kl) A.list[first + __builtin_popcountll(group & below)] = (int32_t)c;
        todo &= ~group;
    }
}

static __global__ void k_plan_reset(int32_t* plan)
{
    for (int i = threadIdx.x; i < PLAN_SIZE; i += blockDim.x) plan[i] = 0;
}

// rewind every bucket's work queue (the autotuner reruns the EM launches)
static __global__ void k_plan_requeue(int32_t* plan)
{
    if (threadIdx.x <= kNumBuckets) plan[PLAN_QUEUE + threadIdx.x] = 0;
}

template <int D>
int launch_requeue_dr(const CompressArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_plan_requeue, dim3(1), dim3(64), 0, st, a.plan);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ===========================================================================
// k_em
// ===========================================================================
template <typename R, int D>
struct CompState {
    R mu[D];
    R A[ntri(D)];   // sqrt(log2(e)/2) * inverse Cholesky factor, packed lower
    R c2;           // log2 u + log2 sqrt det C - log2 sqrt det Sigma (C: cell covariance)
    R S[ntri(D)];   // covariance (packed)
    R u;            // unnormalised mixing weight
};

// Reciprocal and square root for the FP32 M-step: the hardware instructions
// (about 1 ulp); FP64 keeps the correctly rounded operations.
template <typename R>
__device__ __forceinline__ R m_rcp(R x)
{
    if constexpr (std::is_same<R, float>::value)
        return __builtin_amdgcn_rcpf(x);
    else
        return R(1) / x;
}

template <typename R>
__device__ __forceinline__ R m_sqrt(R x)
{
    if constexpr (std::is_same<R, float>::value)
        return __builtin_amdgcn_sqrtf(x);
    else
        return sqrt(x);
}

// Cholesky factor of a packed 1x1 / 3x3 covariance and the parameters of the
// density term: A = sqrt(log2(e)/2) L^-1 and
//   c2 = log2 u + log2 sqrt det C - log2 sqrt det Sigma
// i.e. the log2 weighted density relative to the cell's own scale (C the
// cell covariance, sdc = sqrt det C), so that exponent arguments stay O(1)
// in FP32.  Returns false if S is not numerically positive definite.
template <typename R, int D>
__device__ __forceinline__ bool density_params(const R (&S)[ntri(D)], R u, R sdc, R (&Aout)[ntri(D)], R& c2)
{
    const R k = (R)kSqrtHalfLog2e;
    if constexpr (D == 1) {
        if (!(S[0] > R(0)) || !isfinite(S[0])) return false;
        const R l00 = m_sqrt(S[0]);
        const R i00 = m_rcp(l00);
        Aout[0] = k * i00;
        c2 = fast_log2(u * sdc * i00);
        return true;
    } else {
        if (!(S[0] > R(0)) || !isfinite(S[0])) return false;
        const R l00 = m_sqrt(S[0]);
        const R i00 = m_rcp(l00);
        const R l10 = S[1] * i00, l20 = S[2] * i00;
        const R t11 = S[3] - l10 * l10;
        if (!(t11 > R(0)) || !isfinite(t11)) return false;
        const R l11 = m_sqrt(t11);
        const R i11 = m_rcp(l11);
        const R l21 = (S[4] - l20 * l10) * i11;
        const R t22 = S[5] - l20 * l20 - l21 * l21;
        if (!(t22 > R(0)) || !isfinite(t22)) return false;
        const R l22 = m_sqrt(t22);
        const R i22 = m_rcp(l22);
        // inverse of the lower factor
        const R m10 = -l10 * i00 * i11;
        const R m21 = -l21 * i11 * i22;
        const R m20 = -(l20 * i00 + l21 * m10) * i22;
        Aout[0] = k * i00;
        Aout[1] = k * m10;
        Aout[2] = k * m20;
        Aout[3] = k * i11;
        Aout[4] = k * m21;
        Aout[5] = k * i22;
        c2 = fast_log2(u * (sdc * i00) * (i11 * i22));
        return true;
    }
}

// Factor a component, with the floor used when it fails (eps I, eps =
// 1e-12 tr(C)/D, growing tenfold).  Returns true if the floor was needed.
template <typename R, int D>
__device__ __forceinline__ bool factor_comp(CompState<R, D>& cs, double trC, R sdc)
{
    if (density_params<R, D>(cs.S, cs.u, sdc, cs.A, cs.c2)) return false;
    double eps = 1e-12 * trC / D;
    for (int it = 0; it < 40; ++it) {
#pragma unroll
        for (int i = 0; i < D; ++i) cs.S[tri_idx<D>(i, i)] += (R)eps;
        if (density_params<R, D>(cs.S, cs.u, sdc, cs.A, cs.c2)) break;
        eps *= 10.0;
    }
    return true;
}

template <typename R, int D>
__device__ __forceinline__ R log2_term(const CompState<R, D>& cs, const R (&x)[D])
{
    R d[D];
#pragma unroll
    for (int i = 0; i < D; ++i) d[i] = x[i] - cs.mu[i];
    return cs.c2 - tri_quad<D, R>(cs.A, d);
}

// recomputed-density buckets re-sum every particle's density terms exactly
// every kResumSweeps sweeps (and after a sweep with an annihilation); in the
// other sweeps the running sums close the sweep
constexpr int kResumSweeps = 4;
// largest finite value of the iteration precision
template <typename R>
constexpr double kBigFinite = std::is_same<R, float>::value ? 3.4028234663852886e38 : 1.7976931348623157e308;

template <int CTRL, int ROW_MASK = 0xf, typename T>
__device__ __forceinline__ T dpp_get(T x)
{
    if constexpr (std::is_same<T, float>::value)
        return __int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(x)));
    else
        return dpp_d<CTRL, ROW_MASK>(x);
}

// Wave sums of NV FP32 values, transposed: values are paired so that each
// step halves the registers still to be reduced.  A lane-half swap
// (v_permlane32_swap) of x[2i] and x[2i+1] plus one add leaves x[2i]'s sums
// over lane pairs (l, l + 32) in lanes 0-31 and x[2i+1]'s in lanes 32-63; a
// row swap (v_permlane16_swap) of two such registers plus one add leaves
// four values' 4-lane partial sums, one per 16-lane row; four in-row DPP
// levels then give every lane its row's total.  Value v ends in register
// v / 4, in row tv_row(v): about 28 VALU instructions for ten values
// against 60 for ten separate 64-lane trees.
// An unpaired last value is swapped with itself (both halves, or both rows,
// then hold it).
constexpr int tv_row(int v) { return 2 * (v & 1) + ((v >> 1) & 1); }

template <int NV>
__device__ __forceinline__ void wave_sums_transposed(const float (&x)[NV], float (&b)[(NV + 3) / 4])
{
    constexpr int NA = (NV + 1) / 2, NB = (NV + 3) / 4;
    float a[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const unsigned lo = __float_as_uint(x[2 * i]);
        const unsigned hi = __float_as_uint(x[2 * i + 1 < NV ? 2 * i + 1 : 2 * i]);
        const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
        a[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const unsigned f = __float_as_uint(a[2 * j]);
        const unsigned g = __float_as_uint(a[2 * j + 1 < NA ? 2 * j + 1 : 2 * j]);
        const auto r = __builtin_amdgcn_permlane16_swap(f, g, false, false);
        b[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] += dpp_get<0xB1>(b[j]);   // quad_perm [1,0,3,2]
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] += dpp_get<0x4E>(b[j]);   // quad_perm [2,3,0,1]
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] += dpp_get<0x141>(b[j]);  // row_half_mirror
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] += dpp_get<0x140>(b[j]);  // row_mirror
}

// Workgroup sum of the NV M-step sums of one component update, delivered to
// every thread.  FP32: the transposed wave sums above; lane 15 of each row
// publishes the values its row holds.  FP64: the 64-lane tree of wave_sum
// applied to all NV values one level at a time (the independent DPP
// operations fill each other's wait states); lane 63, where the tree ends,
// publishes.  After one barrier lane v < NV adds value v over all MAXW
// slots in wave order: slots of absent waves hold zeros (the buffer is
// cleared when the kernel starts and only present waves write), so no
// per-wave test is needed.
template <int NVMAX, int MAXW, typename T, int NV>
__device__ __forceinline__ void em_block_sum(T (&x)[NV], T* buf, int& parity, int nwaves)
{
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T* bb = buf + parity * (MAXW * NVMAX);
    if constexpr (std::is_same<T, float>::value) {
        constexpr int NB = (NV + 3) / 4;
        float b[NB];
        wave_sums_transposed<NV>(x, b);
        if (nwaves == 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) x[v] = lane_bcast(b[v / 4], 16 * tv_row(v) + 15);
            return;
        }
        if ((lane & 15) == 15) {
            const int r = lane >> 4;
            const int off = 2 * (r & 1) + (r >> 1);  // value index within each group of four
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (4 * j + off < NV) bb[wid * NVMAX + 4 * j + off] = b[j];
        }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] += dpp_get<0xB1>(x[v]);   // quad_perm [1,0,3,2]
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] += dpp_get<0x4E>(x[v]);   // quad_perm [2,3,0,1]
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] += dpp_get<0x141>(x[v]);  // row_half_mirror
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] += dpp_get<0x140>(x[v]);  // row_mirror
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] += dpp_get<0x142>(x[v]);  // row_bcast:15
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] += dpp_get<0x143>(x[v]);  // row_bcast:31
        if (nwaves == 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) x[v] = lane_bcast(x[v], 63);
            return;
        }
        if (lane == 63) {
#pragma unroll
            for (int v = 0; v < NV; ++v) bb[wid * NVMAX + v] = x[v];
        }
    }
    __syncthreads();
    T t = T(0);
    if (lane < NV) {
        T part[MAXW];
#pragma unroll
        for (int w = 0; w < MAXW; ++w) part[w] = bb[w * NVMAX + lane];
        t = part[0];
#pragma unroll
        for (int w = 1; w < MAXW; ++w) t += part[w];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = lane_bcast(t, v);
    parity ^= 1;
}

// sum of all slots of a density-term vector (unused and dead slots hold 0)
template <typename V>
__device__ __forceinline__ auto resum(const V& v) -> decltype(v[0] + v[0])
{
    constexpr int n = sizeof(V) / sizeof(v[0]);
    auto s = v[0];
#pragma unroll
    for (int j = 1; j < n; ++j) s += v[j];
    return s;
}

template <int D>
__device__ __forceinline__ double sqrt_det(const double* C)
{
    if constexpr (D == 1) {
        return sqrt(C[0]);
    } else {
        const double det = C[0] * (C[3] * C[5] - C[4] * C[4]) - C[1] * (C[1] * C[5] - C[4] * C[2]) +
                           C[2] * (C[1] * C[4] - C[3] * C[2]);
        return sqrt(det);
    }
}

// P: particles per thread held in registers.  STORE_E: keep e_pj for every
// (particle, slot) in registers; otherwise recompute the old term of the
// updated component and track the denominator incrementally (large cells).
//
// Every wave keeps its own copy of the component parameters in LDS: all
// threads compute the identical M-step, so a wave can publish an update to
// its copy without waiting for the others.  The only workgroup barrier per
// component update is the one inside the cross-wave reduction.
// The standard FP32 build with one register-resident particle per thread is
// held to three waves per SIMD (at most 168 VGPRs, which it fits without
// spilling): more of its small cells per CU.  The other builds keep the
// register file they need: held to 168 VGPRs they spill inside the update
// loop (measured: 4x the EM phase's algorithmic HBM bytes).
template <typename R, bool LEAN, int P, bool STORE_E>
constexpr int em_min_waves_per_simd()
{
    return (!LEAN && std::is_same<R, float>::value && STORE_E && P == 1) ? 3 : 1;
}

template <int D, int KMAX, int P, bool STORE_E, typename R, bool LEAN>
__global__ __launch_bounds__(LEAN ? kEmLeanThreads : kEmMaxThreads, (em_min_waves_per_simd<R, LEAN, P, STORE_E>()))
void k_em(CompressArgs A_in)
{
    constexpr int MAXW = em_max_waves(LEAN);
    constexpr int NT = ntri(D);
    constexpr int NS = 1 + D + NT;
    const int nthreads = blockDim.x;
    const int tid = threadIdx.x;
    const int wid = tid >> 6, lane = tid & 63;
    const double T = 0.5 * D * (D + 3);
    const double halfT = 0.5 * T;

    __shared__ CompressArgs A;   // arguments read where they are used, not pinned in SGPRs
    __shared__ CompState<R, D> compw[MAXW][KMAX];
    __shared__ CompState<R, D> bestc[KMAX];  // best state of the outer search over K
    __shared__ double red_d[2 * kMaxWaves * 2];
    __shared__ R red_r[2 * MAXW * NS];  // zero where no wave writes (em_block_sum)
    __shared__ int s_idx;
    __shared__ int s_flag;

    if (tid == 0) A = A_in;
    for (int t = tid; t < 2 * MAXW * NS; t += blockDim.x) red_r[t] = R(0);
    __syncthreads();
    const int nwaves = A.nwaves;
    const int bucket = A.bucket;
    const int count = A.plan[PLAN_COUNT + bucket];
    const int base = A.plan[PLAN_BASE + bucket];
    int par_d = 0, par_r = 0;
    CompState<R, D>* comp = compw[wid];

    // The first cell is claimed before the loop: a workgroup that finds the
    // queue empty leaves before the loop's invariants are set up (a build
    // that fills the register file spills them to scratch, a write per lane
    // of every workgroup of the persistent grid).
    if (tid == 0) s_idx = atomicAdd(&A.plan[PLAN_QUEUE + bucket], 1);
    __syncthreads();
    int idx = s_idx;
    __syncthreads();
    if (idx >= count) return;
    for (;;) {
        const int c = A.list[base + idx];
        const CellInfo<D>* ci = static_cast<const CellInfo<D>*>(A.cells) + c;
        const int n = ci->n;
        const double trC = ci->trC;
        // sqrt det C: densities are kept relative to the cell's own scale
        const double sdc64 = sqrt_det<D>(ci->C);
        const R sdc = (R)sdc64;
        const double lnc0 = -0.5 * D * kLnTwoPi - log(sdc64);
        const double lnN = log((double)n);
        R inv_den = R(0);  // 1 / (N - T K / 2) of eq. omegak, set whenever K changes
        const int64_t o0 = A.off[c];
        const double* vc = A.v + o0 * D;
        const int kmax = A.kmax;
        const double N = (double)n;
        int32_t status = 0;

        // ---------------- particles into registers --------------------------
        R x[P][D], a[P], ref[P];
        // density terms: one KMAX-vector per particle, indexed with the
        // uniform slot number (register-indexed moves, no code per slot)
        typedef R VecK __attribute__((ext_vector_type(KMAX)));
        [[maybe_unused]] VecK e[STORE_E ? P : 1];
        R Sden[P];  // sum_j e_pj, tracked incrementally and re-summed every sweep
        {
            const double wscale = N / ci->W;
            double m[D];
#pragma unroll
            for (int d = 0; d < D; ++d) m[d] = ci->m[d];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int i = tid + j * nthreads;
                if (i < n) {
#pragma unroll
                    for (int d = 0; d < D; ++d) x[j][d] = (R)(vc[(size_t)i * D + d] - m[d]);
                    a[j] = (R)(A.alpha[o0 + i] * wscale);
                } else {
#pragma unroll
                    for (int d = 0; d < D; ++d) x[j][d] = R(0);
                    a[j] = R(0);
                }
                ref[j] = R(0);
            }
        }

        // A warm start is kept when its converged penalised likelihood is at
        // least that of the single Gaussian with the cell's own moments,
        // sum_p a_p ln N(x_p; 0, C) - (T/2) ln N = N (lnc0 - D/2) - (T/2) ln N
        // (sum_p a_p x_p x_p^T = N C), less 1e-5 of its magnitude; otherwise
        // the cell is fitted again from the cold start.  Replay mode (fixed sweep counts) never restarts.
        const int fixed = A.fixed ? A.fixed[c] : 0;
        const double L_one = N * (lnc0 - 0.5 * D) - halfT * log(N);
        bool warm = A.init.K != nullptr && A.init.K[c] > 0;
        // A supplied start is used only if eq. (omegak) is defined for it:
        // N - T K / 2 > 0 and N w_k > T/2 for every supplied component
        // (weights renormalised over the K used); otherwise the cell starts
        // cold, flagged as a rejected warm start.
        if (warm) {
            const int Kw = min(A.init.K[c], kmax);
            const size_t s0 = (size_t)c * kmax;
            double wsum = 0.0;
            for (int j = 0; j < Kw; ++j) wsum += A.init.omega[s0 + j];
            bool usable = N - halfT * Kw > 0.0 && wsum > 0.0 && isfinite(wsum);
            for (int j = 0; j < Kw; ++j) usable &= N * (A.init.omega[s0 + j] / wsum) > halfT;
            if (!usable) {
                warm = false;
                status = GM_ST_WARM_FALLBACK;
            }
        }
        long long visits = 0;
        double L_s = 0.0;
        int s = 0;
        int K = 0;
        R G = R(0);
        for (;;) {
            // ---------------- initial mixture ------------------------------------
            if (tid == 0) s_flag = 0;
            if (warm) {
                K = min(A.init.K[c], kmax);
            } else {
                K = min(kmax, n);
                const int cap = max(1, (int)floor(N / T));
                if (K > cap) {
                    K = cap;
                    status |= GM_ST_K0_CAPPED;
                }
            }
            __syncthreads();
            if (tid < K) {
                CompState<R, D> cs;
                if (warm) {
                    const size_t s0 = (size_t)c * kmax;
                    double wsum = 0.0;
                    for (int j = 0; j < K; ++j) wsum += A.init.omega[s0 + j];
                    const size_t sk = s0 + tid;
#pragma unroll
                    for (int d = 0; d < D; ++d) cs.mu[d] = (R)(A.init.mu[sk * D + d] - ci->m[d]);
#pragma unroll
                    for (int q = 0; q < NT; ++q) cs.S[q] = (R)A.init.sigma[sk * NT + q];
                    cs.u = (R)(A.init.omega[sk] / wsum);
                } else {
                    const int ip = A.init_idx[(size_t)c * kInitSlots + tid];
#pragma unroll
                    for (int d = 0; d < D; ++d) cs.mu[d] = (R)(vc[(size_t)ip * D + d] - ci->m[d]);
#pragma unroll
                    for (int q = 0; q < NT; ++q) cs.S[q] = (R)ci->C[q];
                    cs.u = (R)(1.0 / K);
                }
                if (factor_comp<R, D>(cs, trC, sdc)) s_flag = 1;
                for (int w = 0; w < nwaves; ++w) compw[w][tid] = cs;
            }
            __syncthreads();
            if (s_flag) status |= GM_ST_COV_FLOOR;
            G = R(0);
            for (int j = 0; j < K; ++j) G += comp[j].u;

            // Runs of the outer search over K (a single run unless A.outer):
            // after every converged run the state is kept if its penalised L
            // is the best so far, the least probable component is removed
            // and the sweeps run again, down to K = 1.
            const bool outer = A.outer != 0 && fixed <= 0;
            double L_best = -INFINITY;
            int K_best = 0, s_total = 0;
            R G_best = R(0);
            for (;;) {
                inv_den = m_rcp((R)(N - halfT * K));
                // ---------------- initial density terms ------------------------------
                if constexpr (STORE_E) {
                    for (int j = 0; j < K; ++j) {
                        const CompState<R, D> cj = comp[j];
#pragma unroll
                        for (int p = 0; p < P; ++p) e[p][j] = log2_term<R, D>(cj, x[p]);
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        R mx = e[p][0];
#pragma unroll
                        for (int j = 1; j < KMAX; ++j)
                            if (j < K) mx = fmax(mx, e[p][j]);
                        ref[p] = mx;
#pragma unroll
                        for (int j = 0; j < KMAX; ++j) e[p][j] = (j < K) ? fast_exp2(e[p][j] - mx) : R(0);
                        Sden[p] = resum(e[p]);
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        R mx = R(-1e30);
                        for (int j = 0; j < K; ++j) mx = fmax(mx, log2_term<R, D>(comp[j], x[p]));
                        R s = R(0);
                        for (int j = 0; j < K; ++j) s += fast_exp2(log2_term<R, D>(comp[j], x[p]) - mx);
                        ref[p] = mx;
                        Sden[p] = s;
                    }
                }

                // ---------------- sweeps ---------------------------------------------
                const int max_sweeps = A.max_sweeps;
                const double tol = A.tol;
                const int cap_sweeps = fixed > 0 ? fixed : max_sweeps;
                int Kslots = K;  // slots 0..Kslots-1 hold components; some may die within a sweep
                uint32_t alive = (1u << K) - 1u;
                // A particle whose density sum falls far below its reference (every
                // live component now far from it, e.g. after the one that covered
                // it was annihilated or moved away) gets its terms recomputed in
                // log2 space about their own maximum, as a log-sum-exp would, so
                // that no term underflows to zero.
                const R rebase_below = R(9.094947017729282e-13);  // 2^-40
                auto rebase_store = [&](VecK& ep, const R (&xp)[D], R& refp) -> R {
                    R mx = R(-INFINITY);
#pragma unroll
                    for (int j = 0; j < KMAX; ++j) {
                        const bool live = j < Kslots && ((alive >> j) & 1u);
                        const R t = live ? log2_term<R, D>(comp[j], xp) : R(-INFINITY);
                        ep[j] = t;
                        mx = fmax(mx, t);
                    }
                    if (!(mx > R(-INFINITY))) return R(0);
#pragma unroll
                    for (int j = 0; j < KMAX; ++j)
                        ep[j] = (j < Kslots && ((alive >> j) & 1u)) ? fast_exp2(ep[j] - mx) : R(0);
                    refp = mx;
                    return resum(ep);
                };
                auto rebase_sum = [&](const R (&xp)[D], R& refp) -> R {
                    R mx = R(-INFINITY);
                    for (int j = 0; j < Kslots; ++j)
                        if ((alive >> j) & 1u) mx = fmax(mx, log2_term<R, D>(comp[j], xp));
                    if (!(mx > R(-INFINITY))) return R(0);
                    R sum = R(0);
                    for (int j = 0; j < Kslots; ++j)
                        if ((alive >> j) & 1u) sum += fast_exp2(log2_term<R, D>(comp[j], xp) - mx);
                    refp = mx;
                    return sum;
                };
                // Particles flagged in `low` lost most of their density in an
                // update (the running sum may have cancelled): re-sum their terms
                // exactly, and rebase those whose sum is still tiny.  Particles
                // flagged in `big` got a term more than 2^64 above their reference
                // (a component moved onto a particle that had been rebased far
                // down): rebase them.  The branch is wave-uniform and rarely taken.
                // The flags are per-particle lane masks (SALU), not VGPR bit sets.
                auto repair_store = [&](bool any, const bool (&low)[P], const bool (&big)[P]) {
                    if constexpr (STORE_E) {
                        if (__builtin_amdgcn_ballot_w64(any) == 0) return;
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            if (big[p]) {
                                Sden[p] = rebase_store(e[p], x[p], ref[p]);
                            } else if (low[p]) {
                                Sden[p] = resum(e[p]);
                                if (!(Sden[p] > rebase_below)) Sden[p] = rebase_store(e[p], x[p], ref[p]);
                            }
                        }
                    }
                };

                double L_prev = 0.0;
                for (s = 1; s <= cap_sweeps; ++s) {
                    bool annihilated = false;
                    for (int k = 0; k < Kslots; ++k) {
                        if (!((alive >> k) & 1u)) continue;
                        ++visits;
                        R ckmu[D];
#pragma unroll
                        for (int i = 0; i < D; ++i) ckmu[i] = comp[k].mu[i];
                        const R cku = comp[k].u;
                        // E-step of k with the current parameters of every component,
                        // and the M-step sums about the current mean of k
                        R sums[NS];
#pragma unroll
                        for (int t = 0; t < NS; ++t) sums[t] = R(0);
                        [[maybe_unused]] R eold[STORE_E ? 1 : P];
                        auto accumulate = [&](int p, R ek, R den) {
                            // den > 0 for every particle of a fitted cell (the rebase keeps
                            // it above 2^-40); the clamp keeps a zero from turning a
                            // zero-weight padding particle's 0 * inf into NaN
                            const R inv = fmin(fast_rcp(den), R(kBigFinite<R>));
                            const R g = a[p] * ek * inv;
                            R d[D];
#pragma unroll
                            for (int i = 0; i < D; ++i) d[i] = x[p][i] - ckmu[i];
                            sums[0] += g;
#pragma unroll
                            for (int i = 0; i < D; ++i) {
                                const R gd = g * d[i];
                                sums[1 + i] += gd;
#pragma unroll
                                for (int j = i; j < D; ++j) sums[1 + D + tri_idx<D>(i, j)] += gd * d[j];
                            }
                        };
                        if constexpr (STORE_E) {
#pragma unroll
                            for (int p = 0; p < P; ++p) accumulate(p, e[p][k], Sden[p]);
                        } else {
                            const CompState<R, D> ck = comp[k];
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                eold[p] = fast_exp2(fmin(log2_term<R, D>(ck, x[p]) - ref[p], R(64)));
                                accumulate(p, eold[p], Sden[p]);
                            }
                        }
                        em_block_sum<NS, MAXW>(sums, red_r, par_r, nwaves);
                        const R Nk = sums[0];
                        const R NkT = Nk - (R)halfT;
                        if (fabs(NkT) < (R)(1e-5 * halfT)) status |= GM_ST_NEAR_TIE;
                        if (NkT <= R(0)) {
                            // annihilate k (eq. omegak); the weights renormalise through G
                            alive &= ~(1u << k);
                            G -= cku;
                            --K;
                            inv_den = m_rcp((R)(N - halfT * K));
                            annihilated = true;
                            if constexpr (STORE_E) {
                                bool low[P], big[P], any = false;
#pragma unroll
                                for (int p = 0; p < P; ++p) {
                                    const R s_old = Sden[p];
                                    const R s_new = s_old - e[p][k];
                                    e[p][k] = R(0);
                                    Sden[p] = s_new;
                                    low[p] = !(s_new > R(1e-3) * s_old);
                                    big[p] = false;
                                    any |= low[p];
                                }
                                repair_store(any, low, big);
                            } else {
#pragma unroll
                                for (int p = 0; p < P; ++p) {
                                    const R s_old = Sden[p];
                                    R s_new = s_old - eold[p];
                                    if (!(s_new > R(1e-4) * s_old)) {
                                        s_new = R(0);
                                        for (int j = 0; j < Kslots; ++j)
                                            if ((alive >> j) & 1u)
                                                s_new += fast_exp2(fmin(log2_term<R, D>(comp[j], x[p]) - ref[p], R(64)));
                                    }
                                    Sden[p] = (s_new > rebase_below) ? s_new : rebase_sum(x[p], ref[p]);
                                }
                            }
                            continue;
                        }
                        // M-step (eqs. muk, sigmak about the new mean; eq. omegak)
                        CompState<R, D> cn;
                        const R invN = m_rcp(Nk);
                        R dl[D];
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            dl[i] = sums[1 + i] * invN;
                            cn.mu[i] = ckmu[i] + dl[i];
                        }
#pragma unroll
                        for (int i = 0; i < D; ++i)
#pragma unroll
                            for (int j = i; j < D; ++j)
                                cn.S[tri_idx<D>(i, j)] = sums[1 + D + tri_idx<D>(i, j)] * invN - dl[i] * dl[j];
                        const R wk = NkT * inv_den;
                        const R unew = wk * G;
                        G = G - cku + unew;
                        cn.u = unew;
                        if (factor_comp<R, D>(cn, trC, sdc)) status |= GM_ST_COV_FLOOR;
                        if (lane == 0) comp[k] = cn;  // this wave's copy; read back only by this wave
                        if constexpr (STORE_E) {
                            bool low[P], big[P], any = false;
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const R dt = log2_term<R, D>(cn, x[p]) - ref[p];
                                const R enew = fast_exp2(fmin(dt, R(64)));
                                const R s_old = Sden[p];
                                const R s_new = s_old - e[p][k] + enew;
                                e[p][k] = enew;
                                Sden[p] = s_new;
                                low[p] = !(s_new > R(1e-3) * s_old);
                                big[p] = dt > R(64);
                                any |= low[p] | big[p];
                            }
                            repair_store(any, low, big);
                        } else {
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const R dt = log2_term<R, D>(cn, x[p]) - ref[p];
                                const R enew = fast_exp2(fmin(dt, R(64)));
                                const R s_old = Sden[p];
                                R s_new = s_old - eold[p] + enew;
                                if (!(s_new > R(1e-4) * s_old)) {
                                    // the particle lost most of its density: re-sum exactly
                                    s_new = enew;
                                    for (int j = 0; j < Kslots; ++j)
                                        if (j != k && ((alive >> j) & 1u))
                                            s_new += fast_exp2(fmin(log2_term<R, D>(comp[j], x[p]) - ref[p], R(64)));
                                }
                                Sden[p] = (s_new > rebase_below && !(dt > R(64))) ? s_new : rebase_sum(x[p], ref[p]);
                            }
                        }
                    }

                    // ---- end of sweep: per-particle mixture density, eq. (lnL-GM) ----
                    const R lg2G = fast_log2(G);
                    double lsum[1] = {0.0};
                    R dens[P];
                    uint32_t low = 0;
                    if constexpr (STORE_E) {
#pragma unroll
                        for (int p = 0; p < P; ++p) dens[p] = resum(e[p]);
                    } else if (s % kResumSweeps != 0 && !annihilated) {
                        // the running sums, kept through the sweep's updates
                        // (each re-summed exactly where it had cancelled)
#pragma unroll
                        for (int p = 0; p < P; ++p) dens[p] = Sden[p];
                    } else {
                        // exact re-sum every kResumSweeps sweeps and after an
                        // annihilation: component outer, particles inner, each
                        // component's parameters read from LDS once
#pragma unroll
                        for (int p = 0; p < P; ++p) dens[p] = R(0);
                        for (int j = 0; j < Kslots; ++j) {
                            if (!((alive >> j) & 1u)) continue;
                            const CompState<R, D> cj = comp[j];
#pragma unroll
                            for (int p = 0; p < P; ++p)
                                dens[p] += fast_exp2(fmin(log2_term<R, D>(cj, x[p]) - ref[p], R(64)));
                        }
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) low |= (uint32_t)!(dens[p] > rebase_below) << p;
                    if (__builtin_amdgcn_ballot_w64(low != 0) != 0) {
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            if ((low >> p) & 1u) {
                                if constexpr (STORE_E)
                                    dens[p] = rebase_store(e[p], x[p], ref[p]);
                                else
                                    dens[p] = rebase_sum(x[p], ref[p]);
                            }
                        }
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const R den = dens[p];
                        const R lg = fast_log2(den);
                        if constexpr (STORE_E) {
                            // the weights are normalised below (u_j / G, c_j - log2 G):
                            // lowering the reference by log2 G keeps every stored term
                            ref[p] = ref[p] - lg2G;
                            lsum[0] += (double)a[p] * (double)(ref[p] + lg);  // log2 mixture density at x_p
                            Sden[p] = den;
                        } else {
                            ref[p] = ref[p] + lg - lg2G;  // log2 of the normalised mixture density at x_p
                            lsum[0] += (double)a[p] * (double)ref[p];
                            Sden[p] = R(1);
                        }
                    }
                    block_sum<2, MAXW>(lsum, red_d, par_d, nwaves);
                    // normalise the weights in this wave's copy: u_j /= G, c2_j -= log2 G
                    if (lane < Kslots && ((alive >> lane) & 1u)) {
                        comp[lane].u = comp[lane].u * m_rcp(G);
                        comp[lane].c2 = comp[lane].c2 - lg2G;
                    }
                    // G = sum_j u_j and sum_j log2(u_j / G) over the live slots, lane j
                    // holding slot j (a 16-lane tree, then broadcast from lane 0)
                    const bool live_lane = lane < Kslots && ((alive >> lane) & 1u);
                    R uj = live_lane ? comp[lane].u : R(0);
                    R Gn = uj;
                    Gn += dpp_get<0xB1>(Gn);
                    Gn += dpp_get<0x4E>(Gn);
                    Gn += dpp_get<0x141>(Gn);
                    Gn += dpp_get<0x140>(Gn);
                    Gn = lane_bcast(Gn, 0);
                    double pl = live_lane ? (double)fast_log2(uj * m_rcp(Gn)) : 0.0;
                    pl += dpp_get<0xB1>(pl);
                    pl += dpp_get<0x4E>(pl);
                    pl += dpp_get<0x141>(pl);
                    pl += dpp_get<0x140>(pl);
                    const double pen = lane_bcast(pl, 0);
                    G = Gn;
                    const double dpar = K * T + K - 1;
                    // ref_p is log2 of the mixture density relative to (2 pi)^(-D/2) / sqrt det C
                    L_s = kLn2 * (lsum[0] - 0.5 * T * pen) + N * lnc0 - 0.5 * dpar * lnN;

                    // ---- compaction of dead slots (rare) ----
                    if (annihilated) {
                        for (int k = Kslots - 1; k >= 0; --k) {
                            if ((alive >> k) & 1u) continue;
                            if (lane == 0)
                                for (int j = k; j + 1 < Kslots; ++j) comp[j] = comp[j + 1];
                            if constexpr (STORE_E) {
#pragma unroll
                                for (int j = 0; j + 1 < KMAX; ++j)
                                    if (j >= k) {
#pragma unroll
                                        for (int p = 0; p < P; ++p) e[p][j] = e[p][j + 1];
                                    }
#pragma unroll
                                for (int p = 0; p < P; ++p) e[p][KMAX - 1] = R(0);
                            }
                            const uint32_t low = alive & ((1u << k) - 1u);
                            const uint32_t high = (alive >> (k + 1)) << k;
                            alive = low | high;
                            --Kslots;
                        }
                    }

                    if (fixed > 0) {
                        if (s == fixed) break;
                        L_prev = L_s;
                        continue;
                    }
                    if (!isfinite(L_s)) break;  // the objective is undefined: no further sweep can help
                    if (s >= 2 && !annihilated && fabs(L_s - L_prev) <= tol * fabs(L_s)) break;
                    // FP32 resolves L only to the rounding of the per-particle
                    // log-densities it sums, about 1e-7 of N: a change of L within
                    // tol N, or a lower L (the iteration does not lower L between
                    // sweeps without an annihilation), is below that, and the fit
                    // stops as converged
                    if constexpr (std::is_same<R, float>::value)
                        if (s >= 2 && !annihilated && (L_s < L_prev || fabs(L_s - L_prev) <= tol * N)) break;
                    if (s == max_sweeps) {
                        status |= GM_ST_MAXSWEEPS;
                        break;
                    }
                    L_prev = L_s;
                }
                if (s > cap_sweeps) s = cap_sweeps;
                s_total += s;
                if (!outer) break;
                if (K_best == 0 || L_s > L_best) {
                    if (wid == 0 && lane < K) bestc[lane] = comp[lane];
                    L_best = L_s;
                    K_best = K;
                    G_best = G;
                }
                if (K <= 1 || !isfinite(L_s)) break;
                // remove the least probable component (smallest weight, lowest
                // slot on ties); the others keep their parameters and the
                // weights renormalise through G
                int kmin = 0;
                R umin = comp[0].u;
                for (int j = 1; j < K; ++j) {
                    const R uj = comp[j].u;
                    if (uj < umin) {
                        umin = uj;
                        kmin = j;
                    }
                }
                if (lane == 0)
                    for (int j = kmin; j + 1 < K; ++j) comp[j] = comp[j + 1];
                G -= umin;
                --K;
            }
            if (outer && K_best > 0) {
                __syncthreads();  // the best state, written by wave 0, into every wave's copy
                if (lane < K_best) comp[lane] = bestc[lane];
                K = K_best;
                G = G_best;
                L_s = L_best;
            }
            s = s_total;
            if (!warm || fixed > 0 || L_s >= L_one - 1e-5 * fabs(L_one)) break;
            // rejected warm start: cold start, flags of the cold fit only
            warm = false;
            status = GM_ST_WARM_FALLBACK;
            __syncthreads();
        }

        // ---------------- penalised state into the output record -------------
        // (centred coordinates; k_finish turns it into the final mixture)
        if (tid < K) {
            const size_t sk = (size_t)c * kmax + tid;
            const CompState<R, D> cs = compw[0][tid];
            A.out.omega[sk] = (double)cs.u / (double)G;
            for (int d = 0; d < D; ++d) A.out.mu[sk * D + d] = (double)cs.mu[d];
            for (int q = 0; q < NT; ++q) A.out.sigma[sk * NT + q] = (double)cs.S[q];
        }
        if (tid == 0) {
            A.out.K[c] = K;
            A.out.L_pen[c] = L_s;
            A.out.sweeps[c] = s;
            A.out.visits[c] = visits;
            A.out.status[c] = status;
        }
        __syncthreads();
        if (tid == 0) s_idx = atomicAdd(&A.plan[PLAN_QUEUE + bucket], 1);
        __syncthreads();
        idx = s_idx;
        __syncthreads();
        if (idx >= count) break;
    }
}

// ===========================================================================
// k_em_big: the sweeps of cells larger than the register-resident launches
// hold (n > kMaxCellParticles).  Persistent 1024-thread workgroups take cells
// from the big-cell queue.  No per-particle state is kept: every pass reads
// the cell's particles from the input, and every E-step forms each
// particle's mixture denominator from all live components by a base-2
// log-sum-exp, so the cost per component update grows with K, which these
// rare cells can afford.  Start, M-step, annihilation, weights, objective,
// stop test, warm-start acceptance and the outer search over K are those of
// k_em; the penalised state goes into the record for k_finish.
// ===========================================================================
constexpr int kBigBucket = kNumBuckets;  // plan slot of the big cells
constexpr int kBigThreads = 1024;

template <int D, int KMAX, typename R>
__global__ __launch_bounds__(kBigThreads) void k_em_big(CompressArgs A)
{
    constexpr int NT = ntri(D);
    constexpr int NS = 1 + D + NT;
    constexpr int NW = kBigThreads / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const double T = 0.5 * D * (D + 3);
    const double halfT = 0.5 * T;
    __shared__ CompState<R, D> comp[KMAX];
    __shared__ CompState<R, D> bestc[KMAX];
    __shared__ R red_r[2 * kMaxWaves * 16];
    __shared__ double red_d[2 * kMaxWaves * 2];
    __shared__ int s_idx, s_flag;
    int par_r = 0, par_d = 0;
    const int count = A.plan[PLAN_COUNT + kBigBucket];
    const int base = A.plan[PLAN_BASE + kBigBucket];

    for (;;) {
        if (tid == 0) s_idx = atomicAdd(&A.plan[PLAN_QUEUE + kBigBucket], 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= count) break;
        const int c = A.list[base + idx];
        const CellInfo<D>* ci = static_cast<const CellInfo<D>*>(A.cells) + c;
        const int n = ci->n;
        const double trC = ci->trC;
        const double sdc64 = sqrt_det<D>(ci->C);
        const R sdc = (R)sdc64;
        const double lnc0 = -0.5 * D * kLnTwoPi - log(sdc64);
        const double lnN = log((double)n);
        const double N = (double)n;
        const double wscale = N / ci->W;
        const int64_t o0 = A.off[c];
        const double* vc = A.v + o0 * D;
        const double* ac = A.alpha + o0;
        const int kmax = A.kmax;
        double m[D];
#pragma unroll
        for (int d = 0; d < D; ++d) m[d] = ci->m[d];
        // particle i: centred velocity and normalised weight in R
        auto load = [&](int i, R (&x)[D], R& a) {
#pragma unroll
            for (int d = 0; d < D; ++d) x[d] = (R)(vc[(size_t)i * D + d] - m[d]);
            a = (R)(ac[i] * wscale);
        };
        int32_t status = 0;
        const int fixed = A.fixed ? A.fixed[c] : 0;
        const double L_one = N * (lnc0 - 0.5 * D) - halfT * log(N);
        bool warm = A.init.K != nullptr && A.init.K[c] > 0;
        // A supplied start is used only if eq. (omegak) is defined for it:
        // N - T K / 2 > 0 and N w_k > T/2 for every supplied component
        // (weights renormalised over the K used); otherwise the cell starts
        // cold, flagged as a rejected warm start.
        if (warm) {
            const int Kw = min(A.init.K[c], kmax);
            const size_t s0 = (size_t)c * kmax;
            double wsum = 0.0;
            for (int j = 0; j < Kw; ++j) wsum += A.init.omega[s0 + j];
            bool usable = N - halfT * Kw > 0.0 && wsum > 0.0 && isfinite(wsum);
            for (int j = 0; j < Kw; ++j) usable &= N * (A.init.omega[s0 + j] / wsum) > halfT;
            if (!usable) {
                warm = false;
                status = GM_ST_WARM_FALLBACK;
            }
        }
        long long visits = 0;
        double L_s = 0.0;
        int s = 0, K = 0;
        R G = R(0);
        for (;;) {
            // ---------------- initial mixture (as in k_em) ------------------
            if (tid == 0) s_flag = 0;
            if (warm) {
                K = min(A.init.K[c], kmax);
            } else {
                K = min(kmax, n);
                const int cap = max(1, (int)floor(N / T));
                if (K > cap) {
                    K = cap;
                    status |= GM_ST_K0_CAPPED;
                }
            }
            __syncthreads();
            if (tid < K) {
                CompState<R, D> cs;
                if (warm) {
                    const size_t s0 = (size_t)c * kmax;
                    double wsum = 0.0;
                    for (int j = 0; j < K; ++j) wsum += A.init.omega[s0 + j];
                    const size_t sk = s0 + tid;
#pragma unroll
                    for (int d = 0; d < D; ++d) cs.mu[d] = (R)(A.init.mu[sk * D + d] - m[d]);
#pragma unroll
                    for (int q = 0; q < NT; ++q) cs.S[q] = (R)A.init.sigma[sk * NT + q];
                    cs.u = (R)(A.init.omega[sk] / wsum);
                } else {
                    const int ip = A.init_idx[(size_t)c * kInitSlots + tid];
#pragma unroll
                    for (int d = 0; d < D; ++d) cs.mu[d] = (R)(vc[(size_t)ip * D + d] - m[d]);
#pragma unroll
                    for (int q = 0; q < NT; ++q) cs.S[q] = (R)ci->C[q];
                    cs.u = (R)(1.0 / K);
                }
                if (factor_comp<R, D>(cs, trC, sdc)) s_flag = 1;
                comp[tid] = cs;
            }
            __syncthreads();
            if (s_flag) status |= GM_ST_COV_FLOOR;
            G = R(0);
            for (int j = 0; j < K; ++j) G += comp[j].u;

            const bool outer = A.outer != 0 && fixed <= 0;
            double L_best = -INFINITY;
            int K_best = 0, s_total = 0;
            R G_best = R(0);
            for (;;) {
                R inv_den = m_rcp((R)(N - halfT * K));
                const int cap_sweeps = fixed > 0 ? fixed : A.max_sweeps;
                int Kslots = K;
                uint32_t alive = (1u << K) - 1u;
                // base-2 log-sum-exp over the live slots at x: returns the
                // largest term in mx and sum_j 2^(t_j - mx)
                auto lse2 = [&](const R (&x)[D], R& mx) {
                    mx = R(-INFINITY);
                    for (int j = 0; j < Kslots; ++j)
                        if ((alive >> j) & 1u) mx = fmax(mx, log2_term<R, D>(comp[j], x));
                    R se = R(0);
                    for (int j = 0; j < Kslots; ++j)
                        if ((alive >> j) & 1u) se += fast_exp2(log2_term<R, D>(comp[j], x) - mx);
                    return se;
                };
                double L_prev = 0.0;
                for (s = 1; s <= cap_sweeps; ++s) {
                    bool annihilated = false;
                    for (int k = 0; k < Kslots; ++k) {
                        if (!((alive >> k) & 1u)) continue;
                        ++visits;
                        const CompState<R, D> ck = comp[k];
                        R sums[NS];
#pragma unroll
                        for (int t = 0; t < NS; ++t) sums[t] = R(0);
                        for (int i = tid; i < n; i += kBigThreads) {
                            R x[D], a;
                            load(i, x, a);
                            R mx;
                            const R se = lse2(x, mx);
                            const R g = a * fast_exp2(log2_term<R, D>(ck, x) - mx) / se;
                            R d[D];
#pragma unroll
                            for (int q = 0; q < D; ++q) d[q] = x[q] - ck.mu[q];
                            sums[0] += g;
#pragma unroll
                            for (int q = 0; q < D; ++q) {
                                const R gd = g * d[q];
                                sums[1 + q] += gd;
#pragma unroll
                                for (int r = q; r < D; ++r) sums[1 + D + tri_idx<D>(q, r)] += gd * d[r];
                            }
                        }
                        block_sum<16>(sums, red_r, par_r, NW);
                        const R Nk = sums[0];
                        const R NkT = Nk - (R)halfT;
                        if (fabs(NkT) < (R)(1e-5 * halfT)) status |= GM_ST_NEAR_TIE;
                        if (NkT <= R(0)) {
                            // annihilate k (eq. omegak); the weights renormalise through G
                            alive &= ~(1u << k);
                            G -= ck.u;
                            --K;
                            inv_den = m_rcp((R)(N - halfT * K));
                            annihilated = true;
                            continue;
                        }
                        // M-step (eqs. muk, sigmak about the new mean; eq. omegak)
                        CompState<R, D> cn;
                        const R invN = m_rcp(Nk);
                        R dl[D];
#pragma unroll
                        for (int q = 0; q < D; ++q) {
                            dl[q] = sums[1 + q] * invN;
                            cn.mu[q] = ck.mu[q] + dl[q];
                        }
#pragma unroll
                        for (int q = 0; q < D; ++q)
#pragma unroll
                            for (int r = q; r < D; ++r)
                                cn.S[tri_idx<D>(q, r)] = sums[1 + D + tri_idx<D>(q, r)] * invN - dl[q] * dl[r];
                        const R unew = NkT * inv_den * G;
                        G = G - ck.u + unew;
                        cn.u = unew;
                        if (factor_comp<R, D>(cn, trC, sdc)) status |= GM_ST_COV_FLOOR;
                        __syncthreads();  // every thread has read comp[k] for this update
                        if (tid == 0) comp[k] = cn;
                        __syncthreads();
                    }
                    // ---- end of sweep: eq. (lnL-GM) with the normalised weights ----
                    const R lg2G = fast_log2(G);
                    double lsum[1] = {0.0};
                    for (int i = tid; i < n; i += kBigThreads) {
                        R x[D], a;
                        load(i, x, a);
                        R mx;
                        const R se = lse2(x, mx);
                        lsum[0] += (double)a * (double)(mx + fast_log2(se) - lg2G);
                    }
                    block_sum<2>(lsum, red_d, par_d, NW);
                    __syncthreads();
                    if (tid < Kslots && ((alive >> tid) & 1u)) {
                        comp[tid].u = comp[tid].u * m_rcp(G);
                        comp[tid].c2 = comp[tid].c2 - lg2G;
                    }
                    __syncthreads();
                    R Gn = R(0);
                    double pen = 0.0;
                    for (int j = 0; j < Kslots; ++j)
                        if ((alive >> j) & 1u) Gn += comp[j].u;
                    for (int j = 0; j < Kslots; ++j)
                        if ((alive >> j) & 1u) pen += (double)fast_log2(comp[j].u * m_rcp(Gn));
                    G = Gn;
                    const double dpar = K * T + K - 1;
                    L_s = kLn2 * (lsum[0] - 0.5 * T * pen) + N * lnc0 - 0.5 * dpar * lnN;
                    // ---- compaction of dead slots, order kept ----
                    if (annihilated) {
                        __syncthreads();
                        if (tid == 0) {
                            int w = 0;
                            for (int j = 0; j < Kslots; ++j)
                                if ((alive >> j) & 1u) comp[w++] = comp[j];
                        }
                        __syncthreads();
                        Kslots = K;
                        alive = (1u << K) - 1u;
                    }
                    if (fixed > 0) {
                        if (s == fixed) break;
                        L_prev = L_s;
                        continue;
                    }
                    if (!isfinite(L_s)) break;
                    if (s >= 2 && !annihilated && fabs(L_s - L_prev) <= A.tol * fabs(L_s)) break;
                    if constexpr (std::is_same<R, float>::value)
                        if (s >= 2 && !annihilated && (L_s < L_prev || fabs(L_s - L_prev) <= A.tol * N)) break;  // as in k_em
                    if (s == A.max_sweeps) {
                        status |= GM_ST_MAXSWEEPS;
                        break;
                    }
                    L_prev = L_s;
                }
                if (s > cap_sweeps) s = cap_sweeps;
                s_total += s;
                if (!outer) break;
                if (K_best == 0 || L_s > L_best) {
                    __syncthreads();
                    if (tid < K) bestc[tid] = comp[tid];
                    L_best = L_s;
                    K_best = K;
                    G_best = G;
                }
                if (K <= 1 || !isfinite(L_s)) break;
                // remove the least probable component (smallest weight, lowest slot on ties)
                int kmin = 0;
                R umin = comp[0].u;
                for (int j = 1; j < K; ++j) {
                    const R uj = comp[j].u;
                    if (uj < umin) {
                        umin = uj;
                        kmin = j;
                    }
                }
                __syncthreads();
                if (tid == 0)
                    for (int j = kmin; j + 1 < K; ++j) comp[j] = comp[j + 1];
                __syncthreads();
                G -= umin;
                --K;
            }
            if (outer && K_best > 0) {
                __syncthreads();
                if (tid < K_best) comp[tid] = bestc[tid];
                __syncthreads();
                K = K_best;
                G = G_best;
                L_s = L_best;
            }
            s = s_total;
            if (!warm || fixed > 0 || L_s >= L_one - 1e-5 * fabs(L_one)) break;
            warm = false;
            status = GM_ST_WARM_FALLBACK;
            __syncthreads();
        }
        // penalised state into the output record (centred coordinates)
        if (tid < K) {
            const size_t sk = (size_t)c * kmax + tid;
            const CompState<R, D> cs = comp[tid];
            A.out.omega[sk] = (double)cs.u / (double)G;
            for (int d = 0; d < D; ++d) A.out.mu[sk * D + d] = (double)cs.mu[d];
            for (int q = 0; q < NT; ++q) A.out.sigma[sk * NT + q] = (double)cs.S[q];
        }
        if (tid == 0) {
            A.out.K[c] = K;
            A.out.L_pen[c] = L_s;
            A.out.sweeps[c] = s;
            A.out.visits[c] = visits;
            A.out.status[c] = status;
        }
        __syncthreads();
    }
}

// ===========================================================================
// k_finish
// ===========================================================================
template <int D>
struct CompF64 {
    double mu[D];
    double M[ntri(D)];  // inverse of the Cholesky factor, packed lower
    double lnw_c;       // ln w - D/2 ln(2 pi) - ln sqrt det
};

// ln(w N(x; mu, Sigma)) = lnw_c - |M (x - mu)|^2 / 2.  Every product-sum is
// an explicit fma and every other operation a single rounding, so each
// inlined copy evaluates a term bit for bit alike: the normaliser pass and
// the component passes see the same value.
template <int D>
__device__ __forceinline__ double ln_term(const CompF64<D>& c, const double (&x)[D])
{
    if constexpr (D == 1) {
        const double y0 = c.M[0] * (x[0] - c.mu[0]);
        return fma(-0.5, y0 * y0, c.lnw_c);
    } else {
        const double d0 = x[0] - c.mu[0], d1 = x[1] - c.mu[1], d2 = x[2] - c.mu[2];
        const double y0 = c.M[0] * d0;
        const double y1 = fma(c.M[1], d0, c.M[3] * d1);
        const double y2 = fma(c.M[2], d0, fma(c.M[4], d1, c.M[5] * d2));
        const double q = fma(y0, y0, fma(y1, y1, y2 * y2));
        return fma(-0.5, q, c.lnw_c);
    }
}

template <int D>
__device__ __forceinline__ bool make_f64(CompF64<D>& c, const double* mu, const double* S, double w)
{
    double Sd[ntri(D)], L[ntri(D)];
#pragma unroll
    for (int t = 0; t < ntri(D); ++t) Sd[t] = S[t];
    if (!chol<D, double>(Sd, L)) return false;
#pragma unroll
    for (int i = 0; i < D; ++i) c.mu[i] = mu[i];
    tri_inv<D, double>(L, c.M);
    double lndet = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) lndet += log(L[tri_idx<D>(i, i)]);
    c.lnw_c = log(w) - 0.5 * D * kLnTwoPi - lndet;
    return true;
}

constexpr int kFinishThreads = 256;
constexpr int kFinishCache = 2048;  // per-particle normalisers cached in LDS
// cells of at most this many particles are finished by one wave each (four
// per workgroup, no workgroup barrier); larger ones by a whole workgroup
constexpr int kFinishWaveMax = 512;
constexpr int kFinishCellsPerBlock = kFinishThreads / 64;

// orders one wave's LDS writes before its later LDS reads by other lanes
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int D, int KMAX, bool WAVE>
__global__ __launch_bounds__(kFinishThreads) void k_finish(CompressArgs A)
{
    constexpr int NT = ntri(D);
    constexpr int NS = 1 + D + NT;
    constexpr int SLOTS = WAVE ? kFinishCellsPerBlock : 1;
    constexpr int CACHE = WAVE ? kFinishWaveMax : kFinishCache;
    __shared__ CompF64<D> cf_s[SLOTS][KMAX];
    __shared__ double outw_s[SLOTS][KMAX], outmu_s[SLOTS][KMAX][D], outS_s[SLOTS][KMAX][NT];
    __shared__ double red[WAVE ? 1 : 2 * kMaxWaves * NS];
    __shared__ double mx_cache_s[SLOTS][CACHE], sum_cache_s[SLOTS][CACHE];
    __shared__ int s_ok_s[SLOTS];
    const int slot = WAVE ? (int)(threadIdx.x >> 6) : 0;
    const int64_t c = WAVE ? (int64_t)blockIdx.x * kFinishCellsPerBlock + slot : (int64_t)blockIdx.x;
    if (c >= A.n_cells) return;  // whole waves leave (wave mode only)
    const CellInfo<D>* ci = static_cast<const CellInfo<D>*>(A.cells) + c;
    // each cell is finished by exactly one of the two instantiations
    if (WAVE ? ci->n > kFinishWaveMax : ci->n <= kFinishWaveMax) return;
    CompF64<D>(&cf)[KMAX] = cf_s[slot];
    double(&outw)[KMAX] = outw_s[slot];
    double(&outmu)[KMAX][D] = outmu_s[slot];
    double(&outS)[KMAX][NT] = outS_s[slot];
    double* mx_cache = mx_cache_s[slot];
    double* sum_cache = sum_cache_s[slot];
    int& s_ok = s_ok_s[slot];
    const int tid = WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    const int nthreads = WAVE ? 64 : (int)blockDim.x, nwaves = nthreads >> 6;
    auto sync = [&]() {
        if constexpr (WAVE)
            wave_lds_sync();
        else
            __syncthreads();
    };
    int par = 0;
    const int kind = ci->kind;
    const int kmax = A.kmax;
    const double T = 0.5 * D * (D + 3);
    auto clear_slots = [&](int from) {
        for (int t = from + tid; t < kmax; t += nthreads) {
            const size_t sk = (size_t)c * kmax + t;
            A.out.omega[sk] = 0.0;
            for (int d = 0; d < D; ++d) A.out.mu[sk * D + d] = 0.0;
            for (int q = 0; q < NT; ++q) A.out.sigma[sk * NT + q] = 0.0;
        }
    };
    if (kind == CELL_INVALID || kind == CELL_EMPTY || kind == CELL_OVERSIZE) {
        clear_slots(0);
        if (tid == 0) {
            A.out.K[c] = 0;
            A.out.L_pen[c] = 0.0;
            A.out.L_final[c] = 0.0;
            A.out.sweeps[c] = 0;
            A.out.visits[c] = 0;
            A.out.status[c] = kind == CELL_INVALID ? GM_ST_NONFINITE_INPUT : GM_ST_DEGENERATE;
        }
        return;
    }
    const int n = ci->n;
    const int64_t o0 = A.off[c];
    const double* vc = A.v + o0 * D;
    const double* ac = A.alpha + o0;
    const double N = (double)n;
    const double wscale = N / ci->W;
    double m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = ci->m[d];

    auto load_x = [&](int i, double (&xv)[D]) {
#pragma unroll
        for (int d = 0; d < D; ++d) xv[d] = vc[(size_t)i * D + d] - m[d];
    };
    // largest log term and the sum of exp(term - largest) over cf[0..K-1]
    // (rolled loops: unrolled, the compiler would keep every component's
    // parameters in registers across the particle loop)
    auto norm_at = [&](const double (&xv)[D], int K, double& mx, double& se) {
        mx = -INFINITY;
#pragma unroll 1
        for (int j = 0; j < K; ++j) mx = fmax(mx, ln_term<D>(cf[j], xv));
        se = 0.0;
#pragma unroll 1
        for (int j = 0; j < K; ++j) se += exp(ln_term<D>(cf[j], xv) - mx);
    };
    auto lse_at = [&](const double (&xv)[D], int K) {
        double mx, se;
        norm_at(xv, K, mx, se);
        return mx + log(se);
    };
    auto loglik = [&](int K) {
        double s[1] = {0.0};
#pragma unroll 1
        for (int i = tid; i < n; i += nthreads) {
            double xv[D];
            load_x(i, xv);
            s[0] += ac[i] * wscale * lse_at(xv, K);
        }
        block_sum<NS>(s, red, par, nwaves);
        return s[0];
    };
    auto penalty = [&](int K) {
        double pen = 0.0;
        for (int j = 0; j < K; ++j) pen += log(outw[j]);
        const double dpar = K * T + K - 1;
        return -0.5 * dpar * log(N) - 0.5 * T * pen;
    };

    int K;
    int32_t status = 0;
    double L_pen = 0.0;
    int sweeps = 0;
    long long visits = 0;
    if (kind == CELL_CLOSED) {
        // a single Gaussian with the cell's own moments (n <= n_min or C singular)
        K = 1;
        status = GM_ST_SMALL_CELL_K1;
        if (tid == 0) {
            outw[0] = 1.0;
            for (int d = 0; d < D; ++d) outmu[0][d] = 0.0;
            for (int q = 0; q < NT; ++q) outS[0][q] = ci->C[q];
            s_ok = make_f64<D>(cf[0], outmu[0], outS[0], 1.0);
        }
        sync();
        if (!s_ok) status |= GM_ST_DEGENERATE;
        const double Lk = s_ok ? loglik(1) + penalty(1) : -INFINITY;
        L_pen = Lk;
        if (tid == 0) A.out.L_final[c] = Lk;
    } else {
        // unpenalised joint E-step with the penalised parameters, then
        // eqs. (muk), (sigmak), (omegak-mle)
        K = A.out.K[c];
        status = A.out.status[c];
        L_pen = A.out.L_pen[c];
        sweeps = A.out.sweeps[c];
        visits = A.out.visits[c];
        if (tid == 0) s_ok = 0;  // bit 0: a floor was needed, bit 1: a component did not factor
        sync();
        if (tid < K) {
            const size_t sk = (size_t)c * kmax + tid;
            double mu[D], S[NT];
            for (int d = 0; d < D; ++d) mu[d] = A.out.mu[sk * D + d];
            for (int q = 0; q < NT; ++q) S[q] = A.out.sigma[sk * NT + q];
            if (!make_f64<D>(cf[tid], mu, S, A.out.omega[sk])) {
                // a covariance that factored in FP32 iterations (floored or
                // not) can fail the FP64 factorisation when it is nearly
                // singular: the iteration's floor, eps I with eps = 1e-12
                // tr(C)/D growing tenfold; if even that fails the cell takes
                // the closed form below, so no component is left unset
                double eps = 1e-12 * ci->trC / D;
                bool ok = false;
                for (int it = 0; it < 40 && !ok; ++it) {
                    for (int i = 0; i < D; ++i) S[tri_idx<D>(i, i)] += eps;
                    ok = make_f64<D>(cf[tid], mu, S, A.out.omega[sk]);
                    eps *= 10.0;
                }
                atomicOr(&s_ok, ok ? 1 : 2);
            }
        }
        sync();
        const int fac = s_ok;
        if (fac & 2) {
            // no FP64 factor for some component: the closed form
            K = 1;
            status |= GM_ST_DEGENERATE;
            if (tid == 0) {
                outw[0] = 1.0;
                for (int d = 0; d < D; ++d) outmu[0][d] = 0.0;
                for (int q = 0; q < NT; ++q) outS[0][q] = ci->C[q];
                make_f64<D>(cf[0], outmu[0], outS[0], 1.0);
            }
            sync();
        } else if (fac & 1) {
            status |= GM_ST_COV_FLOOR;
        }
        // gamma_pk = a_p exp(l_k - mx_p) / sum_j exp(l_j - mx_p): a ratio of
        // the same exponentials, so sum_k gamma_pk = a_p to rounding (the
        // cache keeps 1 / sum)
        const bool cache = n <= CACHE;
        if (cache) {
            for (int i = tid; i < n; i += nthreads) {
                double xv[D], se;
                load_x(i, xv);
                norm_at(xv, K, mx_cache[i], se);
                sum_cache[i] = 1.0 / se;
            }
        }
        sync();
        for (int k = 0; k < K; ++k) {
            double sm[NS];
#pragma unroll
            for (int t = 0; t < NS; ++t) sm[t] = 0.0;
            const CompF64<D> ck = cf[k];
#pragma unroll 1
            for (int i = tid; i < n; i += nthreads) {
                double xv[D];
                load_x(i, xv);
                double mx, rse;
                if (cache) {
                    mx = mx_cache[i];
                    rse = sum_cache[i];
                } else {
                    double se;
                    norm_at(xv, K, mx, se);
                    rse = 1.0 / se;
                }
                const double g = ac[i] * wscale * exp(ln_term<D>(ck, xv) - mx) * rse;
                double d[D];
#pragma unroll
                for (int q = 0; q < D; ++q) d[q] = xv[q] - ck.mu[q];
                sm[0] += g;
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const double gd = g * d[q];
                    sm[1 + q] += gd;
#pragma unroll
                    for (int r = q; r < D; ++r) sm[1 + D + tri_idx<D>(q, r)] += gd * d[r];
                }
            }
            block_sum<NS>(sm, red, par, nwaves);
            if (tid == 0) {
                const double Nk = sm[0];
                double dl[D];
                for (int q = 0; q < D; ++q) {
                    dl[q] = sm[1 + q] / Nk;
                    outmu[k][q] = ck.mu[q] + dl[q];
                }
                for (int q = 0; q < D; ++q)
                    for (int r = q; r < D; ++r)
                        outS[k][tri_idx<D>(q, r)] = sm[1 + D + tri_idx<D>(q, r)] / Nk - dl[q] * dl[r];
                outw[k] = Nk / N;
            }
        }
        sync();
        // the output must factor; otherwise the closed form replaces it
        if (tid == 0) {
            bool ok = true;
            for (int k = 0; k < K; ++k) ok &= make_f64<D>(cf[k], outmu[k], outS[k], outw[k]);
            if (!ok) {
                outw[0] = 1.0;
                for (int d = 0; d < D; ++d) outmu[0][d] = 0.0;
                for (int q = 0; q < NT; ++q) outS[0][q] = ci->C[q];
                make_f64<D>(cf[0], outmu[0], outS[0], 1.0);
            }
            s_ok = ok;
        }
        sync();
        if (!s_ok) {
            status |= GM_ST_DEGENERATE;
            K = 1;
        }
        const double Lfin = loglik(K) + penalty(K);
        if (tid == 0) A.out.L_final[c] = Lfin;
    }
    // record: mixture in the input coordinates
    for (int t = tid; t < K; t += nthreads) {
        const size_t sk = (size_t)c * kmax + t;
        A.out.omega[sk] = outw[t];
        for (int d = 0; d < D; ++d) A.out.mu[sk * D + d] = outmu[t][d] + m[d];
        for (int q = 0; q < NT; ++q) A.out.sigma[sk * NT + q] = outS[t][q];
    }
    clear_slots(K);
    if (tid == 0) {
        A.out.K[c] = K;
        A.out.L_pen[c] = L_pen;
        A.out.sweeps[c] = sweeps;
        A.out.visits[c] = visits;
        A.out.status[c] = status;
    }
}

// ===========================================================================
// host-side launch helpers, instantiated per (D, precision) translation unit
// ===========================================================================
template <int D, int KMAX, typename R, typename F>
inline bool with_variant_kernel(int per_thread, int mode, F&& f)
{
    const bool store_e = (mode & kModeStoreE) != 0;
    if (mode & kModeLean) {
        // lean builds (at most 128 VGPRs): FP32 iterations only
        if constexpr (std::is_same<R, float>::value) {
            if (store_e && per_thread == 1) {
                f(k_em<D, KMAX, 1, true, R, true>);
                return true;
            }
            if (store_e && per_thread == 2) {
                f(k_em<D, KMAX, 2, true, R, true>);
                return true;
            }
            if (!store_e && per_thread == 4) {
                f(k_em<D, KMAX, 4, false, R, true>);
                return true;
            }
            if (!store_e && per_thread == 8) {
                f(k_em<D, KMAX, 8, false, R, true>);
                return true;
            }
        }
        return false;
    }
    if (!store_e) {
        if (per_thread == 8) {
            f(k_em<D, KMAX, 8, false, R, false>);
            return true;
        }
        if (per_thread == 16) {
            f(k_em<D, KMAX, 16, false, R, false>);
            return true;
        }
        return false;
    }
    switch (per_thread) {
        case 1: f(k_em<D, KMAX, 1, true, R, false>); return true;
        case 2: f(k_em<D, KMAX, 2, true, R, false>); return true;
        case 4: f(k_em<D, KMAX, 4, true, R, false>); return true;
        case 5:
        case 6:
        case 7:
            if constexpr (KMAX == 16 && std::is_same<R, float>::value) {
                if (per_thread == 5) f(k_em<D, KMAX, 5, true, R, false>);
                else if (per_thread == 6) f(k_em<D, KMAX, 6, true, R, false>);
                else f(k_em<D, KMAX, 7, true, R, false>);
                return true;
            }
            return false;
        case 8:
            if constexpr (KMAX == 8 || std::is_same<R, float>::value) {
                f(k_em<D, KMAX, 8, true, R, false>);
                return true;
            }
            return false;
        default: return false;
    }
}

template <int D, typename R>
int launch_bucket_dr(int kmax_tpl, int per_thread, int mode, int waves, const CompressArgs& a, int grid,
                     hipStream_t st)
{
    if (waves < 1 || waves > em_max_waves((mode & kModeLean) != 0) || a.nwaves != waves) return -1;
    const dim3 g(grid), b(64 * waves);
    bool ok = false;
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, b, 0, st, a); };
    if (kmax_tpl == 8)
        ok = with_variant_kernel<D, 8, R>(per_thread, mode, go);
    else if (kmax_tpl == 16)
        ok = with_variant_kernel<D, 16, R>(per_thread, mode, go);
    if (!ok) return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// persistent grid: resident workgroups per CU times the CU count (cached);
// 0 for a variant that is not built
template <int D, typename R>
int grid_dr(int kmax_tpl, int per_thread, int mode, int waves)
{
    static int cache[2][17][4][kEmMaxWaves + 1] = {};
    if (per_thread < 1 || per_thread > 16 || mode < 0 || mode > 3 || waves < 1 ||
        waves > em_max_waves((mode & kModeLean) != 0))
        return 0;
    const int ki = kmax_tpl == 8 ? 0 : 1;
    int& slot = cache[ki][per_thread][mode][waves];
    if (slot > 0) return slot;
    int dev = 0, ncu = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int block = 64 * waves;
    auto q = [&](auto kern) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kern), block, 0) !=
            hipSuccess)
            nb = 1;
    };
    bool ok = false;
    if (kmax_tpl == 8)
        ok = with_variant_kernel<D, 8, R>(per_thread, mode, q);
    else
        ok = with_variant_kernel<D, 16, R>(per_thread, mode, q);
    if (!ok) return 0;
    if (nb < 1) nb = 1;
    slot = nb * ncu;
    return slot;
}

// the big-cell sweeps: `grid` persistent workgroups (they leave at once when
// the batch has no big cell)
template <int D, typename R>
int launch_big_dr(int kmax_tpl, const CompressArgs& a, int grid, hipStream_t st)
{
    if (kmax_tpl == 8)
        hipLaunchKernelGGL((k_em_big<D, 8, R>), dim3(grid), dim3(kBigThreads), 0, st, a);
    else
        hipLaunchKernelGGL((k_em_big<D, 16, R>), dim3(grid), dim3(kBigThreads), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// pre- and post-EM kernels of one D
template <int D>
int launch_pre_dr(const CompressArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_plan_reset, dim3(1), dim3(64), 0, st, a.plan);
    hipLaunchKernelGGL(k_moments<D>, dim3((unsigned)((a.n_cells + kMomCellsPerBlock - 1) / kMomCellsPerBlock)),
                       dim3(64 * kMomCellsPerBlock), 0, st, a);
    hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(1), 0, st, a.plan);
    hipLaunchKernelGGL(k_plan_scatter<D>, dim3((unsigned)((a.n_cells + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int D>
int launch_finish_dr(int kmax_tpl, const CompressArgs& a, hipStream_t st)
{
    const unsigned nb_wave = (unsigned)((a.n_cells + kFinishCellsPerBlock - 1) / kFinishCellsPerBlock);
    if (kmax_tpl == 8) {
        hipLaunchKernelGGL((k_finish<D, 8, true>), dim3(nb_wave), dim3(kFinishThreads), 0, st, a);
        hipLaunchKernelGGL((k_finish<D, 8, false>), dim3((unsigned)a.n_cells), dim3(kFinishThreads), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_finish<D, 16, true>), dim3(nb_wave), dim3(kFinishThreads), 0, st, a);
        hipLaunchKernelGGL((k_finish<D, 16, false>), dim3((unsigned)a.n_cells), dim3(kFinishThreads), 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gm
