// gm_std.hip -- standard (non-adaptive) EM-GM with K-means start and Anderson
// acceleration (Sec. 3.4), FP32 E/M iterations, FP64 parameter mixing.
//
// One 256-thread workgroup (four waves) per cell, grid over the cells; only
// cells that k_moments marked for EM are fitted, k_finish then applies the
// unpenalised joint step (the standard EM step that follows the iteration)
// and handles every other cell.
//
//   start     K0 = min(K, n) components at the cold-start particles (the
//             same Philox draw as the adaptive path, without its cap), with
//             the cell covariance and equal weights; or K-means (Lloyd, FP64,
//             Euclidean, ties to the lowest slot, weighted centroids, an
//             emptied centre stays) from those particles, and the mixture of
//             its hard assignment (weights W_k / N, centroids, cluster
//             covariances with the covariance floor)
//   iterate   G(theta): joint E-step (log-sum-exp of base-2 terms per
//             particle, every component's terms in registers) and the M-step
//             sums of every component about its current mean, accumulated
//             per lane and reduced across the wave in one pass; weights
//             N_k / N, means, covariances with the new mean
//   mixing    theta = (w_k, mu_k, M2_k = Sigma_k + mu_k mu_k^T) per component
//             in FP64, lane k holding component k; Anderson mixing in the
//             difference form, theta_{i+1} = G(theta_i) - dG gamma with gamma
//             the least-squares coefficients of f_i on dF (modified
//             Gram-Schmidt, wave-wide dot products); a mixed iterate with a
//             negative weight, an indefinite Sigma or a dependent column
//             resets the history to the latest pair and takes G(theta_i); a
//             mixed iterate whose log-likelihood falls below the last
//             accepted one is rejected in favour of G of that iterate
//   stop      relative change of the log-likelihood at the accepted iterates
//             at most tol, or max_iter evaluations of G
#include "gm_compress_impl.h"

namespace gm {


// centred FP32 velocities and normalised weights of every EM particle; a
// cell whose particles lie beyond n_tot is not fitted (no access out of the
// staging buffers: it gets no mixture)
template <int D>
__global__ void k_std_stage(StdArgs P)
{
    const CompressArgs& A = P.a;
    const int c = blockIdx.x;
    CellInfo<D>* ci = static_cast<CellInfo<D>*>(A.cells) + c;
    if (ci->kind != CELL_EM && ci->kind != CELL_BIG) return;
    if (A.off[c + 1] > P.n_tot) {
        __syncthreads();
        if (threadIdx.x == 0) ci->kind = CELL_OVERSIZE;
        return;
    }
    const int64_t o0 = A.off[c];
    const int n = ci->n;
    const double wscale = (double)n / ci->W;
    float* xa = P.xa_w;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        float* o = xa + (o0 + i) * (D + 1);
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = (float)(A.v[(o0 + i) * D + d] - ci->m[d]);
        o[D] = (float)(A.alpha[o0 + i] * wscale);
    }
}

template <int D>
constexpr int std_len() { return 1 + D + ntri(D); }

// Cholesky of a packed FP64 covariance (validity of a mixed iterate)
template <int D>
__device__ __forceinline__ bool spd64(const double (&S)[ntri(D)])
{
    double L[ntri(D)];
    return chol<D, double>(S, L);
}

constexpr int kStdThreads = 256;
constexpr int kStdWaves = kStdThreads / 64;

template <int D, int KMAX>
__global__ __launch_bounds__(kStdThreads) void k_std(StdArgs P)
{
    constexpr int NT = ntri(D);
    constexpr int NS = 1 + D + NT;      // M-step sums per component
    constexpr int L = std_len<D>();     // mixed parameters per component
    constexpr int LEN = KMAX * L;
    constexpr int R = kStdAaMax + 1;    // history ring
    constexpr int NKM = KMAX * (1 + D); // K-means sums
    const CompressArgs& A = P.a;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int c = blockIdx.x;
    const CellInfo<D>* ci = static_cast<const CellInfo<D>*>(A.cells) + c;
    if (ci->kind != CELL_EM && ci->kind != CELL_BIG) return;

    __shared__ CompState<float, D> comp[KMAX];
    __shared__ double th[LEN];                  // theta_i, component k at k * L
    __shared__ double Fh[R][LEN], Gh[R][LEN];   // ring of (f, G); G of the last accepted iterate is the newest
    __shared__ double Q[kStdAaMax][LEN];        // orthonormalised differences of f
    __shared__ float red_f[kStdWaves][KMAX * NS];
    __shared__ float tot[KMAX * NS];
    __shared__ double red_d[2 * kMaxWaves * NKM];
    __shared__ double ctr[KMAX][D];
    __shared__ int s_ctl, s_status, s_resets;
    int par = 0;

    const int n = ci->n;
    const int64_t o0 = A.off[c];
    const double N = (double)n;
    const double trC = ci->trC;
    const double sdc64 = sqrt_det<D>(ci->C);
    const float sdc = (float)sdc64;
    const double lnc0 = -0.5 * D * kLnTwoPi - log(sdc64);
    const int K = min(P.K, n);
    const float* xa = P.xa_w + o0 * (D + 1);
    const double wscale = N / ci->W;
    if (tid == 0) {
        s_status = 0;
        s_resets = 0;
    }

    // component k's FP32 density parameters from its FP64 weight, mean and
    // covariance (floor where it does not factor); thread k only
    auto set_comp = [&](int k, double w, const double (&mu)[D], const double (&S)[NT]) {
        CompState<float, D> cs;
#pragma unroll
        for (int d = 0; d < D; ++d) cs.mu[d] = (float)mu[d];
#pragma unroll
        for (int q = 0; q < NT; ++q) cs.S[q] = (float)S[q];
        cs.u = (float)w;
        if (factor_comp<float, D>(cs, trC, sdc)) atomicOr(&s_status, GM_ST_COV_FLOOR);
        comp[k] = cs;
    };
    // theta of component k from a weight, mean and (float) covariance
    auto put_theta = [&](double* t, double w, const double (&mu)[D], const float (&S)[NT]) {
        t[0] = w;
#pragma unroll
        for (int d = 0; d < D; ++d) t[1 + d] = mu[d];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = i; j < D; ++j) t[1 + D + tri_idx<D>(i, j)] = (double)S[tri_idx<D>(i, j)] + mu[i] * mu[j];
    };
    // sums over the component lanes of wave 0 (lane k holds component k,
    // lanes from K on hold zeros): the tree of the first 8 or 16 lanes
    auto wsum = [&](double x) -> double {
        x += dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
        x += dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
        x += dpp_d<0x141>(x);  // row_half_mirror: 8-lane totals
        if constexpr (KMAX > 8) x += dpp_d<0x140>(x);  // row_mirror: 16-lane totals
        return lane_bcast(x, 0);
    };
    for (int t = tid; t < 2 * kMaxWaves * NKM; t += kStdThreads) red_d[t] = 0.0;
    __syncthreads();

    // ---------------- start ------------------------------------------------
    const int32_t* idx = A.init_idx + (size_t)c * kInitSlots;
    if (P.kmeans) {
        if (tid < K) {
            const int ip = idx[tid];
#pragma unroll
            for (int d = 0; d < D; ++d) ctr[tid][d] = A.v[(o0 + ip) * D + d] - ci->m[d];
        }
        for (int i = tid; i < n; i += kStdThreads) P.assign[o0 + i] = -1;
        __syncthreads();
        int pass = 0;
        for (pass = 1; pass <= 100; ++pass) {
            double acc[NKM];
#pragma unroll
            for (int t = 0; t < NKM; ++t) acc[t] = 0.0;
            int changed = 0;
            for (int i = tid; i < n; i += kStdThreads) {
                double x[D];
#pragma unroll
                for (int d = 0; d < D; ++d) x[d] = A.v[(o0 + i) * D + d] - ci->m[d];
                const double al = A.alpha[o0 + i] * wscale;
                int best = 0;
                double bd = INFINITY;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (k < K) {
                        double d2 = 0.0;
#pragma unroll
                        for (int d = 0; d < D; ++d) d2 += (x[d] - ctr[k][d]) * (x[d] - ctr[k][d]);
                        if (d2 < bd) {
                            bd = d2;
                            best = k;
                        }
                    }
                }
                if (P.assign[o0 + i] != best) {
                    changed = 1;
                    P.assign[o0 + i] = best;
                }
#pragma unroll
                for (int k = 0; k < KMAX; ++k)
                    if (k == best) {
                        acc[k * (1 + D)] += al;
#pragma unroll
                        for (int d = 0; d < D; ++d) acc[k * (1 + D) + 1 + d] += al * x[d];
                    }
            }
            if (!__syncthreads_or(changed)) break;
            block_sum<NKM, kStdWaves>(acc, red_d, par, kStdWaves);
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k == tid && k < K && acc[k * (1 + D)] > 0.0)
#pragma unroll
                    for (int d = 0; d < D; ++d) ctr[k][d] = acc[k * (1 + D) + 1 + d] / acc[k * (1 + D)];
            __syncthreads();
        }
        if (pass > 100) pass = 100;
        if (P.kmeans_passes && tid == 0) P.kmeans_passes[c] = pass;
        // the mixture of the hard assignment, one component per pass
        for (int k = 0; k < K; ++k) {
            double vals[1 + NT];
#pragma unroll
            for (int q = 0; q < 1 + NT; ++q) vals[q] = 0.0;
            for (int i = tid; i < n; i += kStdThreads) {
                if (P.assign[o0 + i] != k) continue;
                const double al = A.alpha[o0 + i] * wscale;
                double x[D];
#pragma unroll
                for (int d = 0; d < D; ++d) x[d] = A.v[(o0 + i) * D + d] - ci->m[d] - ctr[k][d];
                vals[0] += al;
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = a; b < D; ++b) vals[1 + tri_idx<D>(a, b)] += al * x[a] * x[b];
            }
            block_sum<NKM, kStdWaves>(vals, red_d, par, kStdWaves);
            if (tid == k) {
                const double W = vals[0];
                double S[NT], mu[D];
#pragma unroll
                for (int q = 0; q < NT; ++q) S[q] = W > 0.0 ? vals[1 + q] / W : 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) mu[d] = ctr[k][d];
                set_comp(k, W / N, mu, S);
                put_theta(th + k * L, W / N, mu, comp[k].S);
            }
        }
    } else if (tid < K) {
        const int ip = idx[tid];
        double mu[D], S[NT];
#pragma unroll
        for (int d = 0; d < D; ++d) mu[d] = A.v[(o0 + ip) * D + d] - ci->m[d];
#pragma unroll
        for (int q = 0; q < NT; ++q) S[q] = ci->C[q];
        set_comp(tid, 1.0 / K, mu, S);
        put_theta(th + tid * L, 1.0 / K, mu, comp[tid].S);
    }
    __syncthreads();

    // ---------------- iterations ---------------------------------------------
    // every wave runs the E-step; wave 0 alone runs the parameter update and
    // the mixing (lane k = component k) and publishes the control decision
    const int max_iter = A.max_sweeps;
    const double tol = A.tol;
    const int mm = P.aa_m;
    int nh = 0, head = 0, it = 0;
    bool mixed = false, have_prev = false, converged = false;
    double ll = 0.0, ll_prev = 0.0;
    while (it < max_iter) {
        ++it;
        // E-step and M-step sums about every component's current mean
        float sums[KMAX * NS];
#pragma unroll
        for (int t = 0; t < KMAX * NS; ++t) sums[t] = 0.0f;
        double lsum[1] = {0.0};
        for (int i = tid; i < n; i += kStdThreads) {
            float x[D];
#pragma unroll
            for (int d = 0; d < D; ++d) x[d] = xa[(size_t)i * (D + 1) + d];
            const float a = xa[(size_t)i * (D + 1) + D];
            float l[KMAX];
            float mx = -INFINITY;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                l[k] = k < K ? log2_term<float, D>(comp[k], x) : -INFINITY;
                mx = fmaxf(mx, l[k]);
            }
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                l[k] = k < K ? fast_exp2(l[k] - mx) : 0.0f;
                s += l[k];
            }
            lsum[0] += (double)a * (double)(mx + fast_log2(s));
            const float inv = a * fast_rcp(s);
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (k < K) {
                    const float g = l[k] * inv;
                    float d[D];
#pragma unroll
                    for (int q = 0; q < D; ++q) d[q] = x[q] - comp[k].mu[q];
                    float* sk = sums + k * NS;
                    sk[0] += g;
#pragma unroll
                    for (int q = 0; q < D; ++q) {
                        const float gd = g * d[q];
                        sk[1 + q] += gd;
#pragma unroll
                        for (int r = q; r < D; ++r) sk[1 + D + tri_idx<D>(q, r)] += gd * d[r];
                    }
                }
            }
        }
        // wave sums (the transposed reduction of the adaptive path: value v
        // ends in register v / 4, row tv_row(v); lane 15 of each row
        // publishes its row's values), then the waves' partials in wave order
        {
            constexpr int NV = KMAX * NS, NB = (NV + 3) / 4;
            float b[NB];
            wave_sums_transposed<NV>(sums, b);
            if ((lane & 15) == 15) {
                const int r = lane >> 4;
                const int off = 2 * (r & 1) + (r >> 1);
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    if (4 * q + off < NV) red_f[wid][4 * q + off] = b[q];
            }
        }
        block_sum<NKM, kStdWaves>(lsum, red_d, par, kStdWaves);
        for (int t = tid; t < KMAX * NS; t += kStdThreads) {
            float v = red_f[0][t];
#pragma unroll
            for (int w = 1; w < kStdWaves; ++w) v += red_f[w][t];
            tot[t] = v;
        }
        __syncthreads();
        ll = kLn2 * lsum[0] + N * lnc0;
        if (P.ll_trace && tid == 0) P.ll_trace[(size_t)c * max_iter + (it - 1)] = ll;

        if (wid == 0) {
            int ctl = 0;  // 0 go on, 1 converged, 2 stop (no finite likelihood), 3 rejected
            if (mixed && !(ll >= ll_prev)) {
                // the mixed iterate lowered the likelihood: back to G of the
                // last accepted iterate (the newest G of the ring), history cleared
                if (lane == 0) ++s_resets;
                if (lane < K) {
                    const double* gsrc = &Gh[(head + mm) % (mm + 1)][lane * L];
                    double mu[D], S[NT];
#pragma unroll
                    for (int d = 0; d < D; ++d) mu[d] = gsrc[1 + d];
#pragma unroll
                    for (int i = 0; i < D; ++i)
#pragma unroll
                        for (int j = i; j < D; ++j)
                            S[tri_idx<D>(i, j)] = gsrc[1 + D + tri_idx<D>(i, j)] - mu[i] * mu[j];
                    const double w = gsrc[0];
                    set_comp(lane, w, mu, S);
                    put_theta(th + lane * L, w, mu, comp[lane].S);
                }
                nh = 0;
                head = 0;
                mixed = false;
                ctl = 3;
            } else if (have_prev && fabs(ll - ll_prev) <= tol * fabs(ll)) {
                ctl = 1;
            } else if (!isfinite(ll)) {
                ctl = 2;
            } else {
                ll_prev = ll;
                have_prev = true;
                // G(theta): lane k forms component k's new weight, mean and
                // covariance (a component without responsibility keeps its mean
                // and covariance at weight 0)
                double gmu[D], gS[NT], gw = 0.0, greg[L];
#pragma unroll
                for (int t = 0; t < L; ++t) greg[t] = 0.0;
                if (lane < K) {
                    const float* sk = tot + lane * NS;
                    const CompState<float, D> ck = comp[lane];
                    const double Nk = sk[0];
                    if (Nk > 0.0) {
                        double dl[D];
#pragma unroll
                        for (int d = 0; d < D; ++d) {
                            dl[d] = (double)sk[1 + d] / Nk;
                            gmu[d] = (double)ck.mu[d] + dl[d];
                        }
#pragma unroll
                        for (int i = 0; i < D; ++i)
#pragma unroll
                            for (int j = i; j < D; ++j)
                                gS[tri_idx<D>(i, j)] = (double)sk[1 + D + tri_idx<D>(i, j)] / Nk - dl[i] * dl[j];
                        gw = Nk / N;
                    } else {
#pragma unroll
                        for (int d = 0; d < D; ++d) gmu[d] = ck.mu[d];
#pragma unroll
                        for (int q = 0; q < NT; ++q) gS[q] = ck.S[q];
                        gw = 0.0;
                    }
                    greg[0] = gw;
#pragma unroll
                    for (int d = 0; d < D; ++d) greg[1 + d] = gmu[d];
#pragma unroll
                    for (int i = 0; i < D; ++i)
#pragma unroll
                        for (int j = i; j < D; ++j)
                            greg[1 + D + tri_idx<D>(i, j)] = gS[tri_idx<D>(i, j)] + gmu[i] * gmu[j];
                }
                bool take_g = true;
                mixed = false;
                if (mm > 0) {
                    // push (f_i, G_i)
                    if (lane < K)
#pragma unroll
                        for (int t = 0; t < L; ++t) {
                            Fh[head][lane * L + t] = greg[t] - th[lane * L + t];
                            Gh[head][lane * L + t] = greg[t];
                        }
                    head = (head + 1) % (mm + 1);
                    if (nh < mm + 1) ++nh;
                    const int mk = nh - 1;
                    if (mk >= 1) {
                        const int cur = (head + mm) % (mm + 1);
                        // modified Gram-Schmidt on the differences of f, oldest first
                        double Rm[kStdAaMax][kStdAaMax], qf[kStdAaMax];
                        bool ok = true;
                        for (int j = 0; j < mk; ++j) {
                            const int i0 = (head - nh + j + 2 * (mm + 1)) % (mm + 1);
                            const int i1 = (i0 + 1) % (mm + 1);
                            double qj[L], n0 = 0.0;
#pragma unroll
                            for (int t = 0; t < L; ++t) qj[t] = 0.0;
                            if (lane < K)
#pragma unroll
                                for (int t = 0; t < L; ++t) {
                                    qj[t] = Fh[i1][lane * L + t] - Fh[i0][lane * L + t];
                                    n0 += qj[t] * qj[t];
                                }
                            n0 = wsum(n0);
                            for (int l = 0; l < j; ++l) {
                                double r = 0.0;
                                if (lane < K)
#pragma unroll
                                    for (int t = 0; t < L; ++t) r += Q[l][lane * L + t] * qj[t];
                                r = wsum(r);
                                Rm[l][j] = r;
                                if (lane < K)
#pragma unroll
                                    for (int t = 0; t < L; ++t) qj[t] -= r * Q[l][lane * L + t];
                            }
                            double nr = 0.0;
                            if (lane < K)
#pragma unroll
                                for (int t = 0; t < L; ++t) nr += qj[t] * qj[t];
                            nr = sqrt(wsum(nr));
                            if (!(nr > 1e-12 * sqrt(n0))) {
                                ok = false;
                                break;
                            }
                            Rm[j][j] = nr;
                            if (lane < K)
#pragma unroll
                                for (int t = 0; t < L; ++t) Q[j][lane * L + t] = qj[t] / nr;
                        }
                        if (ok) {
                            for (int j = 0; j < mk; ++j) {
                                double sq = 0.0;
                                if (lane < K)
#pragma unroll
                                    for (int t = 0; t < L; ++t) sq += Q[j][lane * L + t] * Fh[cur][lane * L + t];
                                qf[j] = wsum(sq);
                            }
                            double gam[kStdAaMax];
                            for (int j = mk - 1; j >= 0; --j) {
                                double sq = qf[j];
                                for (int l = j + 1; l < mk; ++l) sq -= Rm[j][l] * gam[l];
                                gam[j] = sq / Rm[j][j];
                            }
                            // candidate G_i - dG gamma, weights renormalised
                            double cand[L], w0 = 0.0;
#pragma unroll
                            for (int t = 0; t < L; ++t) cand[t] = 0.0;
                            if (lane < K) {
#pragma unroll
                                for (int t = 0; t < L; ++t) {
                                    double sq = greg[t];
                                    for (int j = 0; j < mk; ++j) {
                                        const int i0 = (head - nh + j + 2 * (mm + 1)) % (mm + 1);
                                        const int i1 = (i0 + 1) % (mm + 1);
                                        sq -= gam[j] * (Gh[i1][lane * L + t] - Gh[i0][lane * L + t]);
                                    }
                                    cand[t] = sq;
                                }
                                w0 = cand[0];
                            }
                            const double ws = wsum(w0);
                            // validity: weights >= 0, Sigma = M2 - mu mu^T positive definite
                            bool valid = ws > 0.0;
                            double cmu[D], cS[NT];
                            if (lane < K) {
                                cand[0] /= ws;
#pragma unroll
                                for (int d = 0; d < D; ++d) cmu[d] = cand[1 + d];
#pragma unroll
                                for (int i = 0; i < D; ++i)
#pragma unroll
                                    for (int j = i; j < D; ++j)
                                        cS[tri_idx<D>(i, j)] = cand[1 + D + tri_idx<D>(i, j)] - cmu[i] * cmu[j];
                                valid = valid && cand[0] >= 0.0 && spd64<D>(cS);
                            }
                            valid = __builtin_amdgcn_ballot_w64(!valid) == 0;
                            if (valid) {
                                if (lane < K) {
                                    set_comp(lane, cand[0], cmu, cS);
#pragma unroll
                                    for (int t = 0; t < L; ++t) th[lane * L + t] = cand[t];
                                }
                                take_g = false;
                                mixed = true;
                            }
                        }
                        if (take_g) {
                            // no usable mixed iterate: the history restarts from the latest pair
                            if (lane == 0) ++s_resets;
                            if (lane < K && cur != 0)
#pragma unroll
                                for (int t = 0; t < L; ++t) {
                                    Fh[0][lane * L + t] = Fh[cur][lane * L + t];
                                    Gh[0][lane * L + t] = Gh[cur][lane * L + t];
                                }
                            nh = 1;
                            head = 1 % (mm + 1);
                        }
                    }
                }
                if (take_g && lane < K) {
                    set_comp(lane, gw, gmu, gS);
                    put_theta(th + lane * L, gw, gmu, comp[lane].S);
                }
            }
            if (lane == 0) s_ctl = ctl;
        }
        __syncthreads();
        const int ctl = s_ctl;
        __syncthreads();  // s_ctl is rewritten in the next iteration
        if (ctl == 1) {
            converged = true;
            break;
        }
        if (ctl == 2) break;
    }

    // ---------------- state into the output record --------------------------
    // components left without weight are dropped, the others renormalised
    __shared__ int s_slot[KMAX];
    __shared__ double s_wsum;
    if (tid == 0) {
        int kk = 0;
        double ws = 0.0;
        for (int k = 0; k < K; ++k) {
            const double w = th[k * L];
            s_slot[k] = w > 0.0 ? kk++ : -1;
            if (w > 0.0) ws += w;
        }
        s_wsum = ws;
        A.out.K[c] = kk;
        A.out.L_pen[c] = ll;
        A.out.sweeps[c] = it;
        A.out.visits[c] = (int64_t)it * K;
        A.out.status[c] = s_status | (converged ? 0 : GM_ST_MAXSWEEPS);
        if (P.resets) P.resets[c] = s_resets;
    }
    __syncthreads();
    if (tid < K && s_slot[tid] >= 0) {
        const size_t sk = (size_t)c * A.kmax + s_slot[tid];
        const CompState<float, D> cs = comp[tid];
        A.out.omega[sk] = th[tid * L] / s_wsum;
        for (int d = 0; d < D; ++d) A.out.mu[sk * D + d] = (double)cs.mu[d];
        for (int q = 0; q < NT; ++q) A.out.sigma[sk * NT + q] = (double)cs.S[q];
    }
}

template <int D>
int launch_std_d(const StdArgs& p, int64_t n_cells, hipStream_t st)
{
    if (n_cells == 0) return 0;
    hipLaunchKernelGGL(k_std_stage<D>, dim3((unsigned)n_cells), dim3(256), 0, st, p);
    // the component count fixes the register arrays: K <= 8 runs the 8-slot
    // kernel whatever kmax the output record is padded to
    if (p.K <= 8)
        hipLaunchKernelGGL((k_std<D, 8>), dim3((unsigned)n_cells), dim3(kStdThreads), 0, st, p);
    else
        hipLaunchKernelGGL((k_std<D, 16>), dim3((unsigned)n_cells), dim3(kStdThreads), 0, st, p);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gm

namespace gm {
int launch_std_d1(const StdArgs& p, int64_t n_cells, hipStream_t st) { return launch_std_d<1>(p, n_cells, st); }
int launch_std_d3(const StdArgs& p, int64_t n_cells, hipStream_t st) { return launch_std_d<3>(p, n_cells, st); }
}  // namespace gm
