// gm_reconstruct.hip -- per-cell ancestral sampling of a Gaussian mixture
// (Sec. 2.4, eq. mix-dist-1) followed by a moment-matching projection, FP64
// throughout: Lemons' scalar form (Sec. 2.4.2, eqs. alpha/beta) or the one
// that matches the whole second-moment tensor; and the projection alone, of
// particles whose weights changed after sampling (the Gauss'-law correction
// of Sec. 2.4.1).
//
// A workgroup of four waves serves four consecutive cells: each cell of at
// most 512 particles is drawn by one wave on its own (no cross-wave
// reduction, no barrier), the larger ones afterwards by the whole
// workgroup, one after another.  Every particle is generated once from its
// own Philox counter and written unprojected; after the sample-moment
// reduction each thread reads back the velocities it wrote (from L2: a
// cell's output is a few ten KB) and overwrites them with their projected
// image, so HBM sees each output byte written once.
#include "gm_device.h"
#include "gm_launch.h"

namespace gm {

constexpr int kReconThreads = 256;

// Particle i of cell c: uniform j is word j % 4 of Philox block j / 4 with
// counter (i, c, j / 4, 0) and key (seed, "RECO").  Uniform 0 picks the
// component, the next ceil(D/2) pairs feed Box-Muller, the rest are positions.
template <int D>
__device__ __forceinline__ void draw_particle(uint64_t seed, int c, int64_t i, int K, const double* cum,
                                              const double (*mu)[D], const double (*L)[ntri(D)], int dx,
                                              double (&v)[D], double (&xpos)[3])
{
    constexpr int NPAIR = (D + 1) / 2;
    const u64x4 b0 = philox4x64_10((uint64_t)i, (uint64_t)c, 0, 0, seed, kTagRecon);
    double u[8];
    u[0] = unit53(b0.x);
    u[1] = unit53(b0.y);
    u[2] = unit53(b0.z);
    u[3] = unit53(b0.w);
    const int nu = 1 + 2 * NPAIR + dx;
    if (nu > 4) {
        const u64x4 b1 = philox4x64_10((uint64_t)i, (uint64_t)c, 1, 0, seed, kTagRecon);
        u[4] = unit53(b1.x);
        u[5] = unit53(b1.y);
        u[6] = unit53(b1.z);
        u[7] = unit53(b1.w);
    }
    // component by inverse CDF over the cumulative weights
    int k = 0;
    while (k < K - 1 && !(u[0] < cum[k])) ++k;
    // Box-Muller pairs
    double z[2 * NPAIR];
#pragma unroll
    for (int pr = 0; pr < NPAIR; ++pr) {
        const double r = sqrt(-2.0 * log(1.0 - u[1 + 2 * pr]));
        // angle 2 pi u: sincospi(2u) takes the exact argument 2u (no
        // reduction by a rounded pi)
        double sn, cs;
        sincospi(2.0 * u[2 + 2 * pr], &sn, &cs);
        z[2 * pr] = r * cs;
        z[2 * pr + 1] = r * sn;
    }
    // v = mu_k + L_k z   (L packed lower, row-major)
    if constexpr (D == 1) {
        v[0] = mu[k][0] + L[k][0] * z[0];
    } else {
        v[0] = mu[k][0] + L[k][0] * z[0];
        v[1] = mu[k][1] + (L[k][1] * z[0] + L[k][3] * z[1]);
        v[2] = mu[k][2] + (L[k][2] * z[0] + L[k][4] * z[1] + L[k][5] * z[2]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) xpos[d] = (d < dx) ? u[1 + 2 * NPAIR + d] : 0.0;
}

// Cholesky factor of a packed centred second moment whose pivots are not
// rounding noise: every pivot^2 above 1e-12 of ref (the mean diagonal of the
// uncentred moment it came from)
template <int D>
__device__ __forceinline__ bool chol_above(const double (&M)[ntri(D)], double ref, double (&L)[ntri(D)])
{
    if (!chol<D, double>(M, L)) return false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double l = L[tri_idx<D>(d, d)];
        if (!(l * l > 1e-12 * ref)) return false;
    }
    return true;
}

// product of packed lower-triangular matrices C = A B
template <int D>
__device__ __forceinline__ void tri_mul(const double (&A)[ntri(D)], const double (&B)[ntri(D)], double (&C)[ntri(D)])
{
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = j; k <= i; ++k) t += A[tri_idx<D>(k, i)] * B[tri_idx<D>(j, k)];
            C[tri_idx<D>(j, i)] = t;
        }
}

// Sums of a particle set that the projections need: N' = sum w, p' =
// sum w v and either S' = sum w v v^T (packed, TENSOR) or E' = sum w |v|^2 / 2.
template <int D, bool TENSOR>
struct SampleSums {
    static constexpr int NT = ntri(D);
    static constexpr int NA = TENSOR ? 1 + D + NT : 2 + D;
    double acc[NA];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int t = 0; t < NA; ++t) acc[t] = 0.0;
    }
    __device__ __forceinline__ void add(const double (&v)[D], double w)
    {
        acc[0] += w;
        if constexpr (TENSOR) {
#pragma unroll
            for (int d = 0; d < D; ++d) acc[1 + d] += w * v[d];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = i; j < D; ++j) acc[1 + D + tri_idx<D>(i, j)] += w * v[i] * v[j];
        } else {
            double e = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                acc[1 + d] += w * v[d];
                e += 0.5 * w * v[d] * v[d];
            }
            acc[1 + D] += e;
        }
    }
};

// The per-cell affine map of the projection, from the sample sums and the
// target moments record tg = (W, P, S packed).
//   TENSOR: v' = P / N' + A (v - p' / N'), A = L_t L_s^-1 with L_t L_t^T =
//     S - P P^T / N' and L_s L_s^T = S' - p' p'^T / N', so sum w v' = P and
//     sum w v' v'^T = S; skipped when a pivot^2 of either factor is not
//     above 1e-12 of the mean diagonal of its uncentred moment.
//   otherwise Lemons' scalar form (Sec. 2.4.2, eqs. alpha/beta) towards P and
//     E = tr(S) / 2: v' = a (v + beta), a = sqrt((2 E N' - |P|^2) / (2 E' N'
//     - |p'|^2)), beta = (P - a p') / (a N'); skipped when either bracket is
//     not above 1e-12 of its leading term 2 E N' or 2 E' N' (zero to
//     rounding: the denominator vanishes exactly when all velocities
//     coincide, as for n' = 1).
template <int D, bool TENSOR>
struct Projection {
    static constexpr int NT = ntri(D);
    bool ok;
    double shift[D];  // TENSOR: P / N'; scalar: beta
    double mean_s[D];
    double Am[NT];
    double sc;
    __device__ __forceinline__ void setup(const double (&acc)[SampleSums<D, TENSOR>::NA], const double* tg)
    {
        const double Np = acc[0];
        if constexpr (TENSOR) {
            double St[NT], Ss[NT], ref_t = 0.0, ref_s = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                ref_t += tg[1 + D + tri_idx<D>(d, d)] / D;
                ref_s += acc[1 + D + tri_idx<D>(d, d)] / D;
            }
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = i; j < D; ++j) {
                    const int q = tri_idx<D>(i, j);
                    St[q] = tg[1 + D + q] - tg[1 + i] * tg[1 + j] / Np;
                    Ss[q] = acc[1 + D + q] - acc[1 + i] * acc[1 + j] / Np;
                }
            double Lt[NT], Ls[NT], Li[NT];
            ok = chol_above<D>(St, ref_t, Lt) && chol_above<D>(Ss, ref_s, Ls);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                shift[d] = tg[1 + d] / Np;
                mean_s[d] = acc[1 + d] / Np;
            }
            if (ok) {
                tri_inv<D, double>(Ls, Li);
                tri_mul<D>(Lt, Li, Am);
            }
        } else {
            double E = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) E += tg[1 + D + tri_idx<D>(d, d)];
            E *= 0.5;
            const double Ep = acc[1 + D];
            double P2 = 0.0, pp2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                P2 += tg[1 + d] * tg[1 + d];
                pp2 += acc[1 + d] * acc[1 + d];
            }
            const double num = 2.0 * E * Np - P2;
            const double den = 2.0 * Ep * Np - pp2;
            ok = num > 1e-12 * (2.0 * E * Np) && den > 1e-12 * (2.0 * Ep * Np);
            sc = 1.0;
#pragma unroll
            for (int d = 0; d < D; ++d) shift[d] = 0.0;
            if (ok) {
                sc = sqrt(num / den);
#pragma unroll
                for (int d = 0; d < D; ++d) shift[d] = (tg[1 + d] - sc * acc[1 + d]) / (sc * Np);
            }
        }
    }
    // writes the image of v (v itself when the projection was skipped)
    __device__ __forceinline__ void write(const double (&v)[D], double* out) const
    {
        if constexpr (TENSOR) {
            double dv[D];
#pragma unroll
            for (int d = 0; d < D; ++d) dv[d] = v[d] - mean_s[d];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                double t = shift[a];
#pragma unroll
                for (int b = 0; b <= a; ++b) t += Am[tri_idx<D>(b, a)] * dv[b];
                out[a] = ok ? t : v[a];
            }
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) out[d] = ok ? sc * (v[d] + shift[d]) : v[d];
        }
    }
};

constexpr int kWaveCell = 512;  // largest cell drawn by one wave (8 particles per lane)

// Draw cell c's n' particles, reduce their sums, then write the projected
// velocities (TENSOR: full second moment; else Lemons' scalar form).  WAVE:
// the 64 lanes of one wave (t = lane) with the wave's own tables; else the
// whole workgroup (t = thread).  Statuses: LEMONS_SKIPPED when the
// projection has no solution, DEGENERATE when a covariance does not factor
// (its component is sampled at its mean) or K is out of range (zero output).
template <int D, bool TENSOR, bool WAVE>
__device__ __forceinline__ void recon_cell(const ReconArgs& A, int c, int64_t o0, int64_t n, int t,
                                           double (*s_mu)[D], double (*s_L)[ntri(D)], double* s_cum, int* s_bad,
                                           double* red, int& par)
{
    constexpr int NT = ntri(D);
    constexpr int G = WAVE ? 64 : kReconThreads;
    using Sums = SampleSums<D, TENSOR>;
    auto sync = [] {
        if constexpr (WAVE) {
            // LDS operations of one wave complete in order; the fence keeps
            // the compiler from moving them across
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };
    const int kmax = A.kmax;
    const int K = A.K[c];
    const int dx = A.dx;
    if (K < 1 || K > kmax) {
        for (int64_t i = t; i < n; i += G) {
            for (int d = 0; d < D; ++d) A.v_out[(o0 + i) * D + d] = 0.0;
            A.w_out[o0 + i] = 0.0;
            for (int d = 0; d < dx; ++d) A.x_out[(o0 + i) * dx + d] = 0.0;
        }
        if (t == 0) A.status[c] = GM_ST_DEGENERATE;
        return;
    }
    if (t == 0) *s_bad = 0;
    sync();
    if (t < K) {
        const size_t s = (size_t)c * kmax + t;
        double S[NT], L[NT];
        for (int q = 0; q < NT; ++q) S[q] = A.sigma[s * NT + q];
        if (!chol<D, double>(S, L)) {
            for (int q = 0; q < NT; ++q) L[q] = 0.0;  // sample the mean only
            *s_bad = 1;
        }
        for (int q = 0; q < NT; ++q) s_L[t][q] = L[q];
        for (int d = 0; d < D; ++d) s_mu[t][d] = A.mu[s * D + d];
    }
    if (t == 0) {
        double run = 0.0;
        for (int k = 0; k < K; ++k) {
            run += A.omega[(size_t)c * kmax + k];
            s_cum[k] = run;
        }
        s_cum[K - 1] = 1.0;
    }
    sync();
    // targets from the compress moments record: W, P = sum alpha v, S = sum
    // alpha v v^T (the scalar projection takes E = tr(S) / 2)
    const double* tg = A.target + (size_t)c * nmom(D);
    const double wp = tg[0] / (double)n;

    Sums sums;
    sums.zero();
    // pass 1: draw, write the particles (velocities unprojected), reduce the
    // sample's sums
    for (int64_t i = t; i < n; i += G) {
        double v[D], xp[3];
        draw_particle<D>(A.seed, c, i, K, s_cum, s_mu, s_L, dx, v, xp);
#pragma unroll
        for (int d = 0; d < D; ++d) A.v_out[(o0 + i) * D + d] = v[d];
        A.w_out[o0 + i] = wp;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (d < dx) A.x_out[(o0 + i) * dx + d] = xp[d];
        sums.add(v, wp);
    }
    if constexpr (WAVE) {
#pragma unroll
        for (int q = 0; q < Sums::NA; ++q) sums.acc[q] = wave_sum(sums.acc[q]);
    } else {
        block_sum<Sums::NA>(sums.acc, red, par, G >> 6);
    }
    Projection<D, TENSOR> pr;
    pr.setup(sums.acc, tg);
    // pass 2: every thread reads back the velocities it wrote (a cell's
    // particles are still in L2) and writes their projected image
    for (int64_t i = t; i < n; i += G) {
        double v[D];
#pragma unroll
        for (int d = 0; d < D; ++d) v[d] = A.v_out[(o0 + i) * D + d];
        pr.write(v, A.v_out + (o0 + i) * D);
    }
    if (t == 0) A.status[c] = (pr.ok ? 0 : GM_ST_LEMONS_SKIPPED) | (*s_bad ? GM_ST_DEGENERATE : 0);
}

// Workgroup b serves cells 4b .. 4b + 3: first each wave draws its own cell
// if that holds at most kWaveCell particles, then the whole workgroup draws
// the others in order (empty cells get status 0 and no output).
template <int D, bool TENSOR>
__global__ __launch_bounds__(kReconThreads) void k_reconstruct(ReconArgs A, int64_t n_cells)
{
    constexpr int NT = ntri(D);
    constexpr int KM = 16;
    constexpr int NW = kReconThreads / 64;
    using Sums = SampleSums<D, TENSOR>;
    __shared__ double s_mu[NW][KM][D], s_L[NW][KM][NT], s_cum[NW][KM];
    __shared__ double red[2 * kMaxWaves * Sums::NA];
    __shared__ int s_bad[NW];
    const int tid = threadIdx.x;
    const int wid = tid >> 6, lane = tid & 63;
    int par = 0;
    const int64_t cb = (int64_t)blockIdx.x * NW;
    {
        const int64_t c = cb + wid;
        if (c < n_cells) {
            const int64_t o0 = A.out_off[c];
            const int64_t n = A.out_off[c + 1] - o0;
            if (n <= 0) {
                if (lane == 0) A.status[c] = 0;
            } else if (n <= kWaveCell) {
                recon_cell<D, TENSOR, true>(A, (int)c, o0, n, lane, s_mu[wid], s_L[wid], s_cum[wid], &s_bad[wid],
                                            nullptr, par);
            }
        }
    }
#pragma unroll 1
    for (int j = 0; j < NW; ++j) {
        const int64_t c = cb + j;
        if (c >= n_cells) break;
        const int64_t o0 = A.out_off[c];
        const int64_t n = A.out_off[c + 1] - o0;
        if (n <= kWaveCell) continue;
        __syncthreads();  // the tables of wave 0 are free
        recon_cell<D, TENSOR, false>(A, (int)c, o0, n, tid, s_mu[0], s_L[0], s_cum[0], &s_bad[0], red, par);
    }
}

// Projection of given particles (v, w) of each cell towards the cell's
// moments record; v_out may alias v: every thread reads its own particles
// before the workgroup's reduction and writes the same particles after it.
template <int D, bool TENSOR>
__global__ __launch_bounds__(kReconThreads) void k_project(ProjArgs A)
{
    using Sums = SampleSums<D, TENSOR>;
    __shared__ double red[2 * kMaxWaves * Sums::NA];
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    int par = 0;
    const int64_t o0 = A.off[c];
    const int64_t n = A.off[c + 1] - o0;
    if (n <= 0) {
        if (tid == 0) A.status[c] = 0;
        return;
    }
    Sums sums;
    sums.zero();
    auto load = [&](int64_t i, double (&v)[D]) {
#pragma unroll
        for (int d = 0; d < D; ++d) v[d] = A.v[(o0 + i) * D + d];
    };
    for (int64_t i = tid; i < n; i += nthreads) {
        double v[D];
        load(i, v);
        sums.add(v, A.w[o0 + i]);
    }
    block_sum<Sums::NA>(sums.acc, red, par, nthreads >> 6);
    Projection<D, TENSOR> pr;
    pr.setup(sums.acc, A.moments + (size_t)c * nmom(D));
    // second read of the same particles (from L2 for cells of up to a few
    // ten thousand particles)
    for (int64_t i = tid; i < n; i += nthreads) {
        double v[D];
        load(i, v);
        pr.write(v, A.v_out + (o0 + i) * D);
    }
    if (tid == 0) A.status[c] = pr.ok ? 0 : GM_ST_LEMONS_SKIPPED;
}

int launch_reconstruct(const ReconArgs& a, int64_t n_cells, hipStream_t st)
{
    if (n_cells == 0) return 0;
    constexpr int NW = kReconThreads / 64;
    const dim3 grid((unsigned)((n_cells + NW - 1) / NW)), block(kReconThreads);
    if (a.D == 1) {
        if (a.tensor)
            hipLaunchKernelGGL((k_reconstruct<1, true>), grid, block, 0, st, a, n_cells);
        else
            hipLaunchKernelGGL((k_reconstruct<1, false>), grid, block, 0, st, a, n_cells);
    } else {
        if (a.tensor)
            hipLaunchKernelGGL((k_reconstruct<3, true>), grid, block, 0, st, a, n_cells);
        else
            hipLaunchKernelGGL((k_reconstruct<3, false>), grid, block, 0, st, a, n_cells);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_project(const ProjArgs& a, int64_t n_cells, hipStream_t st)
{
    if (n_cells == 0) return 0;
    const dim3 grid((unsigned)n_cells), block(kReconThreads);
    if (a.D == 1) {
        if (a.tensor)
            hipLaunchKernelGGL((k_project<1, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_project<1, false>), grid, block, 0, st, a);
    } else {
        if (a.tensor)
            hipLaunchKernelGGL((k_project<3, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_project<3, false>), grid, block, 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gm
