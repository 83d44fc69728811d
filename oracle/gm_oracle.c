/*
 * gm_oracle.c -- plain, slow FP64 CPU oracle for the Gaussian-mixture
 * checkpoint-restart method of Chen, Chacon & Nguyen, "Gaussian-mixture
 * checkpoint-restart for particle-in-cell" (arXiv:2007.12273).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library: every formula below is written again from
 * the paper.
 *
 * Every loop is written in the order the paper states it: no blocking, no
 * fusion, no incremental denominators.  The component-wise E-step recomputes
 * all log-densities of all particles for every component update, which makes
 * one sweep O(n K^2).  That is deliberate.
 *
 * Threads split the cell range into contiguous chunks; each cell is computed
 * by exactly one thread, so results do not depend on the thread count.
 *
 * Parity status of each function is listed at its definition.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 32
#define ORC_MAXD 3
#define ORC_AA_MAX 8 /* largest Anderson memory */

/* per-cell status bits (the library documents the same values) */
#define ORC_SMALL_CELL_K1 (1 << 0)
#define ORC_K0_CAPPED (1 << 1)
#define ORC_COV_FLOOR (1 << 2)
#define ORC_MAXSWEEPS (1 << 3)
#define ORC_NEAR_TIE (1 << 4)
#define ORC_WARM_FALLBACK (1 << 5)
#define ORC_NONFINITE_INPUT (1 << 6)
#define ORC_LEMONS_SKIPPED (1 << 7)
#define ORC_DEGENERATE (1 << 8)

/* oracle mode flags */
#define ORC_MODE_STANDARD_EM 1 /* joint E-step, MLE weights, no annihilation */
#define ORC_MODE_NO_FINISH 2   /* report the penalised state, skip the unpenalised step */
#define ORC_MODE_OUTER_K 4     /* outer search over K: after each converged run remove the
                                  least probable component and run again, keep the best */
#define ORC_MODE_ROUND32 8     /* perturbation of the component-wise sweeps: each update's
                                  responsibilities and the updated component's mean,
                                  covariance and weight rounded to FP32 (binary32) before
                                  use; sizes how far FP32 rounding alone moves a fit, for
                                  the parity bars of FP32 iterations (test use only) */

static const double LN_2PI = 1.8378770664093454835606594728112;
static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror & Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).             */
/* Pinned against numpy.random.Philox in the tests.                   */
/* ------------------------------------------------------------------ */
static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    __uint128_t p = (__uint128_t)a * (__uint128_t)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c[0], &hi0, &lo0);
        mul128(M1, c[2], &hi1, &lo1);
        uint64_t n0 = hi1 ^ c[1] ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c[3] ^ k1;
        uint64_t n3 = lo0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* 53 random bits -> double in [0, 1) */
static double u53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

#define ORC_TAG_INIT 0x494E4954ULL  /* "INIT" */
#define ORC_TAG_RECON 0x5245434FULL /* "RECO" */

/* ------------------------------------------------------------------ */
/* small dense linear algebra (D <= 3), row-major D x D                */
/* ------------------------------------------------------------------ */

/* Cholesky S = L L^T; returns 0 on success, -1 if S is not positive definite. */
static int chol(int D, const double S[ORC_MAXD][ORC_MAXD], double L[ORC_MAXD][ORC_MAXD])
{
    for (int i = 0; i < ORC_MAXD; ++i)
        for (int j = 0; j < ORC_MAXD; ++j) L[i][j] = 0.0;
    for (int j = 0; j < D; ++j) {
        double s = S[j][j];
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0.0) || !isfinite(s)) return -1;
        L[j][j] = sqrt(s);
        for (int i = j + 1; i < D; ++i) {
            double t = S[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    return 0;
}

/* ln N(x; mu, Sigma) with Sigma = L L^T:
 *   -D/2 ln 2pi - 1/2 ln|Sigma| - 1/2 (x-mu)^T Sigma^-1 (x-mu)   (Sec. 2, Gaussian density)
 * The quadratic form is |y|^2 with L y = x - mu (forward substitution). */
static double log_normal(int D, const double* x, const double* mu, const double L[ORC_MAXD][ORC_MAXD])
{
    double y[ORC_MAXD];
    double logdet = 0.0, q = 0.0;
    for (int i = 0; i < D; ++i) {
        double t = x[i] - mu[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
        q += y[i] * y[i];
        logdet += 2.0 * log(L[i][i]);
    }
    return -0.5 * D * LN_2PI - 0.5 * logdet - 0.5 * q;
}

/* ------------------------------------------------------------------ */
/* mixture state of one cell                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    int K;
    double w[ORC_MAXK];
    double mu[ORC_MAXK][ORC_MAXD];
    double S[ORC_MAXK][ORC_MAXD][ORC_MAXD];
    double L[ORC_MAXK][ORC_MAXD][ORC_MAXD];
} mixture;

static void remove_component(mixture* m, int k)
{
    for (int j = k; j + 1 < m->K; ++j) {
        m->w[j] = m->w[j + 1];
        memcpy(m->mu[j], m->mu[j + 1], sizeof(m->mu[j]));
        memcpy(m->S[j], m->S[j + 1], sizeof(m->S[j]));
        memcpy(m->L[j], m->L[j + 1], sizeof(m->L[j]));
    }
    m->K -= 1;
}

/* renormalise the mixing weights to sum 1 (Sec. 2.3, step 3) */
static void renormalise(mixture* m)
{
    double s = 0.0;
    for (int j = 0; j < m->K; ++j) s += m->w[j];
    for (int j = 0; j < m->K; ++j) m->w[j] /= s;
}

/* ln sum_j w_j f_j(x) by log-sum-exp; also returns ell_j = ln w_j + ln f_j(x) */
static double mixture_lse(int D, const mixture* m, const double* x, double* ell)
{
    double mx = -INFINITY;
    for (int j = 0; j < m->K; ++j) {
        ell[j] = log(m->w[j]) + log_normal(D, x, m->mu[j], m->L[j]);
        if (ell[j] > mx) mx = ell[j];
    }
    double s = 0.0;
    for (int j = 0; j < m->K; ++j) s += exp(ell[j] - mx);
    return mx + log(s);
}

/* Penalised log-likelihood, eq. (lnL-GM):
 *   L = sum_p a_p ln sum_k w_k f_k(v_p) - d/2 ln N - T/2 sum_k ln w_k,
 * with T = D(D+3)/2 parameters per component and d = K T + K - 1 in total
 * (Appendix A).  N = sum_p a_p. */
static double penalised_L(int D, double T, const mixture* m, int n, const double* x, const double* a, double N)
{
    double ell[ORC_MAXK];
    double ll = 0.0;
    for (int p = 0; p < n; ++p) ll += a[p] * mixture_lse(D, m, x + (size_t)p * D, ell);
    double d = m->K * T + m->K - 1;
    double pen = 0.0;
    for (int k = 0; k < m->K; ++k) pen += log(m->w[k]);
    return ll - 0.5 * d * log(N) - 0.5 * T * pen;
}

/* Cholesky of component k with the covariance floor used when it fails
 * (the paper is silent on singular covariances): add eps*I, eps = 1e-12 tr(C)/D,
 * growing tenfold until it factors.  Returns 1 if a floor was added. */
static int factor_component(int D, mixture* m, int k, double trC)
{
    if (chol(D, (const double(*)[ORC_MAXD])m->S[k], m->L[k]) == 0) return 0;
    double eps = 1e-12 * trC / D;
    for (int it = 0; it < 40; ++it) {
        for (int i = 0; i < D; ++i) m->S[k][i][i] += eps;
        if (chol(D, (const double(*)[ORC_MAXD])m->S[k], m->L[k]) == 0) return 1;
        eps *= 10.0;
    }
    return 1;
}

/* Cold-start particle choice: partial Fisher-Yates over 0..n-1.  Draw j uses
 * Philox with key (seed, "INIT") and counter (j, cell, 0, 0); the swap target
 * is j + floor(x (n - j) / 2^64) for the first 64-bit output x.  On return
 * perm[0..K0-1] are the chosen indices (perm must hold n ints). */
void orc_init_indices(int n, int K0, uint64_t seed, uint64_t cell, int* perm)
{
    for (int p = 0; p < n; ++p) perm[p] = p;
    uint64_t key[2] = {seed, ORC_TAG_INIT};
    for (int j = 0; j < K0; ++j) {
        uint64_t ctr[4] = {(uint64_t)j, cell, 0, 0}, r4[4];
        orc_philox4x64_10(ctr, key, r4);
        uint64_t hi, lo;
        mul128(r4[0], (uint64_t)(n - j), &hi, &lo);
        int r = j + (int)hi;
        int t = perm[j];
        perm[j] = perm[r];
        perm[r] = t;
    }
}

/* ------------------------------------------------------------------ */
/* compress                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    /* inputs */
    const double* v;
    const double* alpha;
    const int64_t* off;
    int64_t n_cells;
    int D, kmax, n_min, max_sweeps;
    const int32_t* fixed_sweeps; /* nullable; >0 = run exactly that many */
    double tol;
    uint64_t seed;
    int mode;
    double T_override; /* < 0: use D(D+3)/2 */
    /* optional initial mixtures (warm start / test init), nullable */
    const int32_t* init_K;
    const double* init_w;
    const double* init_mu;
    const double* init_S; /* packed upper triangle */
    /* outputs, padded to kmax */
    int32_t* K;
    double* w;
    double* mu;
    double* S;      /* packed upper triangle, D(D+1)/2 per component */
    double* mom;    /* W, P[D], S[D(D+1)/2] */
    double* L_pen;
    double* L_final;
    int32_t* sweeps;
    int32_t* status;
    int64_t* visits;   /* component E/M updates performed */
    double* L_trace;   /* nullable: [n_cells * max_sweeps] penalised L after each sweep */
    int32_t* K_trace;  /* nullable: [n_cells * max_sweeps] live K after each sweep */
    double* margin;    /* nullable: [n_cells] smallest |N_k - T/2| / (T/2) over the annihilation
                          decisions of the sweeps (+inf when none was taken) */
} compress_job;

static int ntri(int D) { return D * (D + 1) / 2; }

static void pack_sym(int D, const double S[ORC_MAXD][ORC_MAXD], double* out)
{
    int t = 0;
    for (int i = 0; i < D; ++i)
        for (int j = i; j < D; ++j) out[t++] = S[i][j];
}

static void unpack_sym(int D, const double* in, double S[ORC_MAXD][ORC_MAXD])
{
    int t = 0;
    for (int i = 0; i < D; ++i)
        for (int j = i; j < D; ++j) {
            S[i][j] = in[t];
            S[j][i] = in[t];
            ++t;
        }
}

/* gamma_pj = a_p w_j f_j(v_p) / sum_i w_i f_i(v_p) for all j (eq.
 * responsibility), formed as a ratio of the same exponentials (scaled by the
 * largest term) so that sum_j gamma_pj = a_p (eq. Sum_responsibility) holds to
 * rounding whatever the size of the log-densities. */
static void particle_responsibilities(int D, const mixture* m, const double* x, double a, double* g)
{
    double ell[ORC_MAXK];
    double mx = -INFINITY;
    for (int j = 0; j < m->K; ++j) {
        ell[j] = log(m->w[j]) + log_normal(D, x, m->mu[j], m->L[j]);
        if (ell[j] > mx) mx = ell[j];
    }
    double s = 0.0;
    for (int j = 0; j < m->K; ++j) {
        g[j] = exp(ell[j] - mx);
        s += g[j];
    }
    for (int j = 0; j < m->K; ++j) g[j] = a * g[j] / s;
}

/* One E-step for component k with the current parameters of all live
 * components. */
static void responsibilities(int D, const mixture* m, int k, int n, const double* x, const double* a, double* g)
{
    double gp[ORC_MAXK];
    for (int p = 0; p < n; ++p) {
        particle_responsibilities(D, m, x + (size_t)p * D, a[p], gp);
        g[p] = gp[k];
    }
}

/* M-step for one component from its responsibilities, eqs. (muk), (sigmak):
 *   mu_k = sum_p g_p v_p / N_k;  Sigma_k = sum_p g_p (v_p - mu_k)(v_p - mu_k)^T / N_k
 * (the covariance uses the new mean). */
static void mean_cov(int D, int n, const double* x, const double* g, double Nk, double* mu, double S[ORC_MAXD][ORC_MAXD])
{
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
        for (int p = 0; p < n; ++p) s += g[p] * x[(size_t)p * D + i];
        mu[i] = s / Nk;
    }
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
            for (int p = 0; p < n; ++p) s += g[p] * (x[(size_t)p * D + i] - mu[i]) * (x[(size_t)p * D + j] - mu[j]);
            S[i][j] = s / Nk;
        }
}

/* Unpenalised ("MLE") finish, Sec. 2.3.1: one joint E-step with the final
 * parameters, then eqs. (muk), (sigmak) and w_k = N_k / N (eq. omegak-mle).
 * Returns 0, or -1 if a resulting covariance is not positive definite. */
static int mle_finish(int D, mixture* m, int n, const double* x, const double* a, double N, double* g_all)
{
    double gp[ORC_MAXK];
    int K = m->K;
    /* joint E-step: every gamma_p. comes from the same parameters */
    for (int p = 0; p < n; ++p) {
        particle_responsibilities(D, m, x + (size_t)p * D, a[p], gp);
        for (int k = 0; k < K; ++k) g_all[(size_t)k * n + p] = gp[k];
    }
    mixture out = *m;
    for (int k = 0; k < K; ++k) {
        const double* g = g_all + (size_t)k * n;
        double Nk = 0.0;
        for (int p = 0; p < n; ++p) Nk += g[p];
        mean_cov(D, n, x, g, Nk, out.mu[k], out.S[k]);
        out.w[k] = Nk / N;
        if (chol(D, (const double(*)[ORC_MAXD])out.S[k], out.L[k]) != 0) return -1;
    }
    *m = out;
    return 0;
}

static void write_mixture(const compress_job* J, int64_t c, const mixture* m, const double* mean)
{
    int D = J->D, kmax = J->kmax, nt = ntri(D);
    J->K[c] = m->K;
    for (int k = 0; k < kmax; ++k) {
        double* wo = J->w + (size_t)c * kmax + k;
        double* mo = J->mu + ((size_t)c * kmax + k) * D;
        double* so = J->S + ((size_t)c * kmax + k) * nt;
        if (k < m->K) {
            *wo = m->w[k];
            for (int i = 0; i < D; ++i) mo[i] = m->mu[k][i] + mean[i];
            pack_sym(D, (const double(*)[ORC_MAXD])m->S[k], so);
        } else {
            *wo = 0.0;
            for (int i = 0; i < D; ++i) mo[i] = 0.0;
            for (int i = 0; i < nt; ++i) so[i] = 0.0;
        }
    }
}

static void compress_cell(const compress_job* J, int64_t c, double* x, double* a, double* g)
{
    const int D = J->D, nt = ntri(D);
    const int64_t o0 = J->off[c], o1 = J->off[c + 1];
    const int n = (int)(o1 - o0);
    const double T = J->T_override >= 0.0 ? J->T_override : 0.5 * D * (D + 3);
    const double* v = J->v + (size_t)o0 * D;
    const double* al = J->alpha + o0;
    int32_t status = 0;
    mixture m;
    memset(&m, 0, sizeof(m));
    double* mom = J->mom + (size_t)c * (1 + D + nt);
    for (int i = 0; i < 1 + D + nt; ++i) mom[i] = 0.0;
    J->L_pen[c] = 0.0;
    J->L_final[c] = 0.0;
    J->sweeps[c] = 0;
    J->visits[c] = 0;

    /* invalid input: non-finite values or non-positive weights */
    for (int p = 0; p < n; ++p) {
        int bad = !isfinite(al[p]) || !(al[p] > 0.0);
        for (int i = 0; i < D; ++i) bad |= !isfinite(v[(size_t)p * D + i]);
        if (bad) {
            double zero[ORC_MAXD] = {0, 0, 0};
            m.K = 0;
            write_mixture(J, c, &m, zero);
            J->status[c] = ORC_NONFINITE_INPUT;
            return;
        }
    }
    if (n == 0) {
        double zero[ORC_MAXD] = {0, 0, 0};
        m.K = 0;
        write_mixture(J, c, &m, zero);
        J->status[c] = ORC_DEGENERATE;
        return;
    }

    /* O1: preserved moments W = sum a, P = sum a v, S = sum a v v^T (Sec. 2.4.2),
     * mean m = P / W and the weighted covariance about it (two passes). */
    double W = 0.0, P[ORC_MAXD] = {0, 0, 0}, S2[ORC_MAXD][ORC_MAXD];
    memset(S2, 0, sizeof(S2));
    for (int p = 0; p < n; ++p) {
        W += al[p];
        for (int i = 0; i < D; ++i) {
            P[i] += al[p] * v[(size_t)p * D + i];
            for (int j = 0; j < D; ++j) S2[i][j] += al[p] * v[(size_t)p * D + i] * v[(size_t)p * D + j];
        }
    }
    mom[0] = W;
    for (int i = 0; i < D; ++i) mom[1 + i] = P[i];
    pack_sym(D, (const double(*)[ORC_MAXD])S2, mom + 1 + D);
    double mean[ORC_MAXD] = {0, 0, 0};
    for (int i = 0; i < D; ++i) mean[i] = P[i] / W;
    double C[ORC_MAXD][ORC_MAXD];
    memset(C, 0, sizeof(C));
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
            for (int p = 0; p < n; ++p) s += al[p] * (v[(size_t)p * D + i] - mean[i]) * (v[(size_t)p * D + j] - mean[j]);
            C[i][j] = s / W;
        }
    double trC = 0.0;
    for (int i = 0; i < D; ++i) trC += C[i][i];
    /* centred velocities and weights normalised so that sum a = N = n
     * (the paper takes sum alpha_p = N, eq. lnL-GM) */
    const double N = (double)n;
    for (int p = 0; p < n; ++p) {
        a[p] = al[p] * (double)n / W;
        for (int i = 0; i < D; ++i) x[(size_t)p * D + i] = v[(size_t)p * D + i] - mean[i];
    }

    /* O2: too few particles (the paper asks for more than ~10 per cell) or a
     * singular covariance: a single Gaussian with the cell's own moments. */
    double LC[ORC_MAXD][ORC_MAXD];
    int c_spd = chol(D, (const double(*)[ORC_MAXD])C, LC) == 0;
    int have_init = J->init_K != NULL && J->init_K[c] > 0;
    if (n <= J->n_min || !c_spd) {
        m.K = 1;
        m.w[0] = 1.0;
        memcpy(m.S[0], C, sizeof(C));
        memcpy(m.L[0], LC, sizeof(LC));
        status |= c_spd ? ORC_SMALL_CELL_K1 : (ORC_SMALL_CELL_K1 | ORC_DEGENERATE);
        if (c_spd) {
            double Lk = penalised_L(D, T, &m, n, x, a, N);
            J->L_pen[c] = Lk;
            J->L_final[c] = Lk;
        } else {
            J->L_pen[c] = -INFINITY;
            J->L_final[c] = -INFINITY;
        }
        write_mixture(J, c, &m, mean);
        J->status[c] = status;
        return;
    }

    /* A warm start (the paper starts cold, Sec. 2.3; a better start only
     * speeds the iteration up, Sec. 3.4) is accepted when its converged
     * penalised likelihood is at least that of the single Gaussian with the
     * cell's own moments, less 1e-5 of its magnitude (so that a warm start
     * that converges to that single Gaussian is kept whatever the rounding);
     * otherwise the cell is fitted again from the cold start and flagged.  Replay mode (fixed sweep counts) never restarts. */
    const int fixed = J->fixed_sweeps ? J->fixed_sweeps[c] : 0;
    double L_one = 0.0;
    if (have_init) {
        mixture one;
        memset(&one, 0, sizeof(one));
        one.K = 1;
        one.w[0] = 1.0;
        memcpy(one.S[0], C, sizeof(C));
        memcpy(one.L[0], LC, sizeof(LC));
        L_one = penalised_L(D, T, &one, n, x, a, N);
    }
    /* A supplied start is used only where eq. (omegak) is defined for it:
     * N - T K / 2 > 0 and N w_k > T/2 for every supplied component (weights
     * renormalised over the K used); otherwise the cell starts cold and is
     * flagged as a rejected warm start. */
    if (have_init) {
        int K0 = J->init_K[c] < J->kmax ? J->init_K[c] : J->kmax;
        double ws = 0.0;
        for (int k = 0; k < K0; ++k) ws += J->init_w[(size_t)c * J->kmax + k];
        int usable = N - 0.5 * T * K0 > 0.0 && ws > 0.0 && isfinite(ws);
        for (int k = 0; k < K0; ++k) usable &= N * (J->init_w[(size_t)c * J->kmax + k] / ws) > 0.5 * T;
        if (!usable) {
            have_init = 0;
            status = ORC_WARM_FALLBACK;
        }
    }
    int64_t visits = 0;
    double L_s = 0.0;
    double margin = INFINITY;
    int s = 0;
    for (int attempt = 0;; ++attempt) {
        if (have_init) {
            /* supplied initial mixture (learned warm start or a test's fixed init) */
            int K0 = J->init_K[c];
            if (K0 > J->kmax) K0 = J->kmax;
            m.K = K0;
            for (int k = 0; k < K0; ++k) {
                size_t s = (size_t)c * J->kmax + k;
                m.w[k] = J->init_w[s];
                for (int i = 0; i < D; ++i) m.mu[k][i] = J->init_mu[s * D + i] - mean[i];
                unpack_sym(D, J->init_S + s * nt, m.S[k]);
                if (factor_component(D, &m, k, trC)) status |= ORC_COV_FLOOR;
            }
            renormalise(&m);
        } else {
            /* O3: cold start (Sec. 2.3): K0 components, each mean at a distinct
             * randomly chosen particle, each covariance the whole cell's covariance,
             * equal weights.  K0 is capped so that N - T K0 / 2 > 0 in eq. (omegak). */
            int K0 = J->kmax < n ? J->kmax : n;
            if (T > 0.0) {
                double cap = floor(N / T);
                if (cap < 1.0) cap = 1.0;
                if ((double)K0 > cap) {
                    K0 = (int)cap;
                    status |= ORC_K0_CAPPED;
                }
            }
            /* partial Fisher-Yates over particle indices; draw j uses Philox with
             * key (seed, "INIT") and counter (j, cell, 0, 0); the index offset is
             * floor(x * (n - j) / 2^64) of the first 64-bit output x. */
            int* perm = (int*)malloc(sizeof(int) * (size_t)n);
            orc_init_indices(n, K0, J->seed, (uint64_t)c, perm);
            m.K = K0;
            for (int k = 0; k < K0; ++k) {
                m.w[k] = 1.0 / K0;
                for (int i = 0; i < D; ++i) m.mu[k][i] = x[(size_t)perm[k] * D + i];
                memcpy(m.S[k], C, sizeof(C));
                memcpy(m.L[k], LC, sizeof(LC));
            }
            free(perm);
        }

        /* O4-O6: component-wise adaptive EM sweeps (Sec. 2.3 steps 1-4).
         * With the outer search over K (the component-wise algorithm the
         * paper cites for its penalised likelihood, Sec. 1): after every
         * converged run the state is kept if its penalised L is the best so
         * far, the least probable component (smallest weight, lowest slot
         * on ties) is removed, the weights renormalised, and the sweeps run
         * again, down to K = 1; the best state is the result.  Each run
         * counts its own sweeps for the stop test and the cap. */
        const int standard = (J->mode & ORC_MODE_STANDARD_EM) != 0;
        const int outer = (J->mode & ORC_MODE_OUTER_K) != 0 && fixed <= 0 && !standard;
        const int round32 = (J->mode & ORC_MODE_ROUND32) != 0;
        const int cap_sweeps = fixed > 0 ? fixed : J->max_sweeps;
        const double half_T = 0.5 * T;
        mixture best;
        double L_best = -INFINITY;
        int have_best = 0, s_total = 0;
        for (;;) {
            double L_prev = 0.0;
            for (s = 1; s <= cap_sweeps; ++s) {
                int annihilated = 0;
                if (standard) {
                    /* plain EM: joint E-step, then every component's M-step with
                     * w_k = N_k / N (eq. omegak-mle); used only as a test mode */
                    double* gk = g;
                    mixture next = m;
                    double gp[ORC_MAXK];
                    for (int p = 0; p < n; ++p) {
                        particle_responsibilities(D, &m, x + (size_t)p * D, a[p], gp);
                        for (int k = 0; k < m.K; ++k) gk[(size_t)k * n + p] = gp[k];
                    }
                    for (int k = 0; k < m.K; ++k) {
                        double Nk = 0.0;
                        for (int p = 0; p < n; ++p) Nk += gk[(size_t)k * n + p];
                        mean_cov(D, n, x, gk + (size_t)k * n, Nk, next.mu[k], next.S[k]);
                        next.w[k] = Nk / N;
                        if (factor_component(D, &next, k, trC)) status |= ORC_COV_FLOOR;
                    }
                    visits += m.K;
                    m = next;
                } else {
                    int k = 0;
                    while (k < m.K) {
                        /* step 1: E-step for component k with the current parameters */
                        responsibilities(D, &m, k, n, x, a, g);
                        if (round32)
                            for (int p = 0; p < n; ++p) g[p] = (double)(float)g[p];
                        double Nk = 0.0;
                        for (int p = 0; p < n; ++p) Nk += g[p];
                        ++visits;
                        if (fabs(Nk - half_T) < 1e-5 * half_T) status |= ORC_NEAR_TIE;
                        if (half_T > 0.0 && fabs(Nk - half_T) / half_T < margin) margin = fabs(Nk - half_T) / half_T;
                        /* step 2: annihilate when N_k - T/2 <= 0 (eq. omegak) */
                        if (Nk - half_T <= 0.0) {
                            remove_component(&m, k);
                            renormalise(&m);
                            annihilated = 1;
                            continue;
                        }
                        mean_cov(D, n, x, g, Nk, m.mu[k], m.S[k]);
                        /* eq. (omegak) with K the current number of live components */
                        m.w[k] = (Nk - half_T) / (N - half_T * m.K);
                        if (round32) {
                            m.w[k] = (double)(float)m.w[k];
                            for (int i = 0; i < D; ++i) {
                                m.mu[k][i] = (double)(float)m.mu[k][i];
                                for (int j = 0; j < D; ++j) m.S[k][i][j] = (double)(float)m.S[k][i][j];
                            }
                        }
                        /* step 3: renormalise */
                        renormalise(&m);
                        if (factor_component(D, &m, k, trC)) status |= ORC_COV_FLOOR;
                        ++k;
                    }
                }
                /* step 4: monitor the penalised log-likelihood */
                L_s = penalised_L(D, T, &m, n, x, a, N);
                if (s_total + s <= J->max_sweeps) {
                    if (J->L_trace) J->L_trace[(size_t)c * J->max_sweeps + (s_total + s - 1)] = L_s;
                    if (J->K_trace) J->K_trace[(size_t)c * J->max_sweeps + (s_total + s - 1)] = m.K;
                }
                if (fixed > 0) {
                    if (s == fixed) break;
                    L_prev = L_s;
                    continue;
                }
                if (!isfinite(L_s)) break; /* eq. (lnL-GM) undefined: no further sweep can help */
                if (s >= 2 && !annihilated && fabs(L_s - L_prev) <= J->tol * fabs(L_s)) break;
                if (s == J->max_sweeps) {
                    status |= ORC_MAXSWEEPS;
                    break;
                }
                L_prev = L_s;
            }
            if (s > cap_sweeps) s = cap_sweeps;
            s_total += s;
            if (!outer) break;
            if (!have_best || L_s > L_best) {
                best = m;
                L_best = L_s;
                have_best = 1;
            }
            if (m.K <= 1 || !isfinite(L_s)) break;
            int kmin = 0;
            for (int k = 1; k < m.K; ++k)
                if (m.w[k] < m.w[kmin]) kmin = k;
            remove_component(&m, kmin);
            renormalise(&m);
        }
        if (outer && have_best) {
            m = best;
            L_s = L_best;
        }
        s = s_total;
        if (!have_init || fixed > 0 || L_s >= L_one - 1e-5 * fabs(L_one)) break;
        /* rejected warm start: cold start, flags of the cold fit only */
        have_init = 0;
        status = ORC_WARM_FALLBACK;
    }
    J->sweeps[c] = s;
    J->visits[c] = visits;
    J->L_pen[c] = L_s;
    if (J->margin) J->margin[c] = margin;

    /* O7: one unpenalised joint step restores exact moments (Sec. 2.3.1) */
    if ((J->mode & ORC_MODE_NO_FINISH) == 0 && mle_finish(D, &m, n, x, a, N, g) != 0) {
        /* degenerate output: fall back to the single-Gaussian closed form */
        m.K = 1;
        m.w[0] = 1.0;
        memcpy(m.S[0], C, sizeof(C));
        memcpy(m.L[0], LC, sizeof(LC));
        memset(m.mu[0], 0, sizeof(m.mu[0]));
        status |= ORC_DEGENERATE;
    }
    /* O8: penalised L at the output parameters */
    J->L_final[c] = penalised_L(D, T, &m, n, x, a, N);
    write_mixture(J, c, &m, mean);
    J->status[c] = status;
}

typedef struct {
    const compress_job* J;
    int64_t c0, c1;
} compress_chunk;

static int64_t max_cell_len(const int64_t* off, int64_t c0, int64_t c1)
{
    int64_t mx = 0;
    for (int64_t c = c0; c < c1; ++c)
        if (off[c + 1] - off[c] > mx) mx = off[c + 1] - off[c];
    return mx;
}

static void* compress_worker(void* arg)
{
    compress_chunk* ch = (compress_chunk*)arg;
    const compress_job* J = ch->J;
    int64_t nmax = max_cell_len(J->off, ch->c0, ch->c1);
    if (nmax < 1) nmax = 1;
    double* x = (double*)malloc(sizeof(double) * (size_t)nmax * J->D);
    double* a = (double*)malloc(sizeof(double) * (size_t)nmax);
    double* g = (double*)malloc(sizeof(double) * (size_t)nmax * ORC_MAXK);
    for (int64_t c = ch->c0; c < ch->c1; ++c) compress_cell(J, c, x, a, g);
    free(x);
    free(a);
    free(g);
    return NULL;
}

static void run_chunks(int64_t n_cells, int nthreads, void* (*fn)(void*), void* job, size_t chunk_size,
                       void (*fill)(void* chunk, void* job, int64_t c0, int64_t c1))
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n_cells) nthreads = n_cells > 0 ? (int)n_cells : 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    char* chunks = (char*)malloc(chunk_size * nthreads);
    for (int t = 0; t < nthreads; ++t) {
        int64_t c0 = n_cells * t / nthreads, c1 = n_cells * (t + 1) / nthreads;
        fill(chunks + chunk_size * t, job, c0, c1);
    }
    if (nthreads == 1) {
        fn(chunks);
    } else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, fn, chunks + chunk_size * t);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    free(th);
    free(chunks);
}

static void fill_compress(void* chunk, void* job, int64_t c0, int64_t c1)
{
    compress_chunk* ch = (compress_chunk*)chunk;
    ch->J = (const compress_job*)job;
    ch->c0 = c0;
    ch->c1 = c1;
}

int orc_compress(const double* v, const double* alpha, const int64_t* off, int64_t n_cells, int D, int kmax,
                 int n_min, int max_sweeps, const int32_t* fixed_sweeps, double tol, uint64_t seed, int mode,
                 double T_override, const int32_t* init_K, const double* init_w, const double* init_mu,
                 const double* init_S, int32_t* K, double* w, double* mu, double* S, double* mom, double* L_pen,
                 double* L_final, int32_t* sweeps, int32_t* status, int64_t* visits, double* L_trace,
                 int32_t* K_trace, double* margin, int nthreads)
{
    if (D < 1 || D > ORC_MAXD || kmax < 1 || kmax > ORC_MAXK || max_sweeps < 1) return -1;
    compress_job J = {v, alpha, off, n_cells, D, kmax, n_min, max_sweeps, fixed_sweeps, tol, seed, mode, T_override,
                      init_K, init_w, init_mu, init_S, K, w, mu, S, mom, L_pen, L_final, sweeps, status, visits,
                      L_trace, K_trace, margin};
    run_chunks(n_cells, nthreads, compress_worker, &J, sizeof(compress_chunk), fill_compress);
    return 0;
}

/* Unpenalised joint finish applied to an arbitrary mixture (test entry for
 * the conservation property of Sec. 2.3.1). Mixture arrays are in and out;
 * mu in original coordinates. Returns 0 or -1 if a covariance is not SPD. */
int orc_mle_finish(const double* v, const double* alpha, int n, int D, int K, double* w, double* mu, double* S)
{
    if (n < 1 || D < 1 || D > ORC_MAXD || K < 1 || K > ORC_MAXK) return -1;
    double W = 0.0;
    for (int p = 0; p < n; ++p) W += alpha[p];
    double* a = (double*)malloc(sizeof(double) * n);
    double* g = (double*)malloc(sizeof(double) * (size_t)n * K);
    for (int p = 0; p < n; ++p) a[p] = alpha[p] * n / W;
    mixture m;
    memset(&m, 0, sizeof(m));
    m.K = K;
    int nt = ntri(D);
    for (int k = 0; k < K; ++k) {
        m.w[k] = w[k];
        for (int i = 0; i < D; ++i) m.mu[k][i] = mu[k * D + i];
        unpack_sym(D, S + k * nt, m.S[k]);
        if (chol(D, (const double(*)[ORC_MAXD])m.S[k], m.L[k]) != 0) {
            free(a);
            free(g);
            return -1;
        }
    }
    int rc = mle_finish(D, &m, n, v, a, (double)n, g);
    if (rc == 0)
        for (int k = 0; k < K; ++k) {
            w[k] = m.w[k];
            for (int i = 0; i < D; ++i) mu[k * D + i] = m.mu[k][i];
            pack_sym(D, (const double(*)[ORC_MAXD])m.S[k], S + k * nt);
        }
    free(a);
    free(g);
    return rc;
}

/* Penalised log-likelihood of a given mixture on given particles (weights
 * normalised to sum n), eq. (lnL-GM).  T < 0 selects D(D+3)/2. */
double orc_penalised_L(const double* v, const double* alpha, int n, int D, int K, const double* w, const double* mu,
                       const double* S, double T)
{
    if (T < 0.0) T = 0.5 * D * (D + 3);
    double W = 0.0;
    for (int p = 0; p < n; ++p) W += alpha[p];
    double* a = (double*)malloc(sizeof(double) * n);
    for (int p = 0; p < n; ++p) a[p] = alpha[p] * n / W;
    mixture m;
    memset(&m, 0, sizeof(m));
    m.K = K;
    int nt = ntri(D);
    for (int k = 0; k < K; ++k) {
        m.w[k] = w[k];
        for (int i = 0; i < D; ++i) m.mu[k][i] = mu[k * D + i];
        unpack_sym(D, S + k * nt, m.S[k]);
        if (chol(D, (const double(*)[ORC_MAXD])m.S[k], m.L[k]) != 0) {
            free(a);
            return NAN;
        }
    }
    double L = penalised_L(D, T, &m, n, v, a, (double)n);
    free(a);
    return L;
}

/* ------------------------------------------------------------------ */
/* reconstruct: ancestral sampling (Sec. 2.4) + Lemons projection      */
/* (Sec. 2.4.2, eqs. alpha/beta)                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    const int32_t* K;
    const double* w;
    const double* mu;
    const double* S;
    int kmax;
    const int64_t* out_off;
    const double* target; /* W, P[D], E per cell */
    int64_t n_cells;
    int D, dx;
    uint64_t seed;
    double* v_out;
    double* w_out;
    double* x_out;
    int32_t* status;
    double* stats; /* nullable: [n_cells * 4] = a (scale), N', |p'|, E' */
    int tensor;    /* 0: scalar projection (target W, P, E); 1: full second moment (target W, P, S packed) */
} recon_job;

/* uniform number j (0-based) of particle i in cell c:
 * block b = j / 4 of Philox with key (seed, "RECO") and counter (i, c, b, 0) */
static void particle_uniforms(uint64_t seed, int64_t c, int64_t i, int count, double* u)
{
    uint64_t key[2] = {seed, ORC_TAG_RECON};
    for (int b = 0; b * 4 < count; ++b) {
        uint64_t ctr[4] = {(uint64_t)i, (uint64_t)c, (uint64_t)b, 0}, r[4];
        orc_philox4x64_10(ctr, key, r);
        for (int t = 0; t < 4 && 4 * b + t < count; ++t) u[4 * b + t] = u53(r[t]);
    }
}

/* Cholesky factor of a centred second moment whose pivots are not rounding
 * noise: every pivot^2 above 1e-12 of ref, the mean diagonal of the
 * uncentred moment it came from. */
static int chol_above(int D, const double M[ORC_MAXD][ORC_MAXD], double ref, double L[ORC_MAXD][ORC_MAXD])
{
    if (chol(D, M, L) != 0) return -1;
    for (int d = 0; d < D; ++d)
        if (!(L[d][d] * L[d][d] > 1e-12 * ref)) return -1;
    return 0;
}

/* Projection that matches the full second moment as well: with the sample's
 * mass N', momentum p', second moment S' and the target's P, S,
 *   v' = P / N' + A (v - p' / N'),   A = L_t L_s^-1,
 * where L_t L_t^T = S - P P^T / N' and L_s L_s^T = S' - p' p'^T / N'.  Then
 * sum w v' = P and sum w v' v'^T = S exactly (N' = W for the equal weights
 * W / n' of the sampling; N' differs after the Gauss'-law correction).
 * The scalar projection of Sec. 2.4.2 (eqs. alpha, beta) matches tr(S) only;
 * this one also restores the pressure tensor that the exact-moment step of
 * Sec. 2.3.1 conserves in the mixture.  Returns the status bits. */
static int32_t project_tensor(const recon_job* J, int64_t c, const double* tg, int64_t o0, int64_t n)
{
    const int D = J->D;
    double Np = 0.0, pp[ORC_MAXD] = {0, 0, 0}, Sp[ORC_MAXD][ORC_MAXD];
    memset(Sp, 0, sizeof(Sp));
    for (int64_t i = 0; i < n; ++i) {
        const double* vi = J->v_out + (size_t)(o0 + i) * D;
        const double wi = J->w_out[o0 + i];
        Np += wi;
        for (int a = 0; a < D; ++a) {
            pp[a] += wi * vi[a];
            for (int b = 0; b < D; ++b) Sp[a][b] += wi * vi[a] * vi[b];
        }
    }
    const double* P = tg + 1;
    double St[ORC_MAXD][ORC_MAXD], Ss[ORC_MAXD][ORC_MAXD];
    unpack_sym(D, tg + 1 + D, St);
    double ref_t = 0.0, ref_s = 0.0;
    for (int d = 0; d < D; ++d) {
        ref_t += St[d][d] / D;
        ref_s += Sp[d][d] / D;
    }
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            St[a][b] -= P[a] * P[b] / Np;
            Ss[a][b] = Sp[a][b] - pp[a] * pp[b] / Np;
        }
    double Lt[ORC_MAXD][ORC_MAXD], Ls[ORC_MAXD][ORC_MAXD];
    if (chol_above(D, (const double(*)[ORC_MAXD])St, ref_t, Lt) != 0 ||
        chol_above(D, (const double(*)[ORC_MAXD])Ss, ref_s, Ls) != 0)
        return ORC_LEMONS_SKIPPED; /* no projection; the sample stays as drawn */
    /* A = L_t L_s^-1: solve X L_s = L_t row by row (back substitution) */
    double Am[ORC_MAXD][ORC_MAXD];
    for (int r = 0; r < D; ++r)
        for (int col = D - 1; col >= 0; --col) {
            double t = Lt[r][col];
            for (int k = col + 1; k < D; ++k) t -= Am[r][k] * Ls[k][col];
            Am[r][col] = t / Ls[col][col];
        }
    double mean_s[ORC_MAXD];
    for (int d = 0; d < D; ++d) mean_s[d] = pp[d] / Np;
    for (int64_t i = 0; i < n; ++i) {
        double* vi = J->v_out + (size_t)(o0 + i) * D;
        double dv[ORC_MAXD];
        for (int d = 0; d < D; ++d) dv[d] = vi[d] - mean_s[d];
        for (int a = 0; a < D; ++a) {
            double t = P[a] / Np;
            for (int b = 0; b < D; ++b) t += Am[a][b] * dv[b];
            vi[a] = t;
        }
    }
    if (J->stats) {
        J->stats[(size_t)c * 4 + 0] = 1.0;
        J->stats[(size_t)c * 4 + 1] = Np;
    }
    return 0;
}

static int32_t project_scalar(const recon_job* J, int64_t c, double W, const double* Pt, double E, int64_t o0,
                              int64_t n);

static void reconstruct_cell(const recon_job* J, int64_t c)
{
    const int D = J->D, nt = ntri(D), dx = J->dx;
    const int64_t o0 = J->out_off[c], o1 = J->out_off[c + 1];
    const int64_t n = o1 - o0;
    int32_t st = 0;
    const double* tg = J->target + (size_t)c * (J->tensor ? 1 + D + nt : 2 + D);
    if (J->stats)
        for (int i = 0; i < 4; ++i) J->stats[(size_t)c * 4 + i] = 0.0;
    int K = J->K[c];
    if (n == 0) {
        J->status[c] = 0;
        return;
    }
    if (K < 1 || K > J->kmax) {
        J->status[c] = ORC_DEGENERATE;
        for (int64_t i = 0; i < n; ++i) {
            for (int d = 0; d < D; ++d) J->v_out[(size_t)(o0 + i) * D + d] = 0.0;
            J->w_out[o0 + i] = 0.0;
            for (int d = 0; d < dx; ++d) J->x_out[(size_t)(o0 + i) * dx + d] = 0.0;
        }
        return;
    }
    /* R1: Cholesky factors and cumulative weights (c_{K-1} := 1) */
    double L[ORC_MAXK][ORC_MAXD][ORC_MAXD], cum[ORC_MAXK];
    double run = 0.0;
    for (int k = 0; k < K; ++k) {
        double Sk[ORC_MAXD][ORC_MAXD];
        unpack_sym(D, J->S + ((size_t)c * J->kmax + k) * nt, Sk);
        if (chol(D, (const double(*)[ORC_MAXD])Sk, L[k]) != 0) {
            /* singular component: sample its mean only */
            memset(L[k], 0, sizeof(L[k]));
            st |= ORC_DEGENERATE;
        }
        run += J->w[(size_t)c * J->kmax + k];
        cum[k] = run;
    }
    cum[K - 1] = 1.0;
    const double W = tg[0];
    const double wp = W / (double)n; /* equal weights (Sec. 2.4) */
    const int nu = 1 + 2 * ((D + 1) / 2) + dx;
    /* R2: ancestral sampling: component by inverse CDF, then v = mu_k + L_k z
     * with Box-Muller normals; positions uniform in the cell. */
    for (int64_t i = 0; i < n; ++i) {
        double u[8];
        particle_uniforms(J->seed, c, i, nu, u);
        int k = 0;
        while (k < K - 1 && !(u[0] < cum[k])) ++k;
        double z[4];
        for (int pr = 0; pr < (D + 1) / 2; ++pr) {
            double r = sqrt(-2.0 * log(1.0 - u[1 + 2 * pr]));
            double th = TWO_PI * u[2 + 2 * pr];
            z[2 * pr] = r * cos(th);
            z[2 * pr + 1] = r * sin(th);
        }
        const double* mk = J->mu + ((size_t)c * J->kmax + k) * D;
        for (int d = 0; d < D; ++d) {
            double s = mk[d];
            for (int e = 0; e <= d; ++e) s += L[k][d][e] * z[e];
            J->v_out[(size_t)(o0 + i) * D + d] = s;
        }
        J->w_out[o0 + i] = wp;
        for (int d = 0; d < dx; ++d) J->x_out[(size_t)(o0 + i) * dx + d] = u[1 + 2 * ((D + 1) / 2) + d];
    }
    if (J->tensor) {
        J->status[c] = st | project_tensor(J, c, tg, o0, n);
        return;
    }
    J->status[c] = st | project_scalar(J, c, tg[0], tg + 1, tg[1 + D], o0, n);
}

/* R3-R5 on the particles of cell c already in v_out, w_out: Lemons'
 * projection towards momentum P and energy E (eqs. alpha, beta). */
static int32_t project_scalar(const recon_job* J, int64_t c, double W, const double* Pt, double E, int64_t o0,
                              int64_t n)
{
    (void)W;
    const int D = J->D;
    int32_t st = 0;
    /* R3: moments of the sample */
    double Np = 0.0, pp[ORC_MAXD] = {0, 0, 0}, Ep = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double* vi = J->v_out + (size_t)(o0 + i) * D;
        double wi = J->w_out[o0 + i];
        Np += wi;
        for (int d = 0; d < D; ++d) {
            pp[d] += wi * vi[d];
            Ep += 0.5 * wi * vi[d] * vi[d];
        }
    }
    /* R4: scale a and shift beta, eq. (alpha):
     *   a = sqrt((2 E N' - |P|^2) / (2 E' N' - |p'|^2)),  beta = (P - a p') / (a N') */
    double P2 = 0.0, pp2 = 0.0;
    for (int d = 0; d < D; ++d) {
        P2 += Pt[d] * Pt[d];
        pp2 += pp[d] * pp[d];
    }
    double num = 2.0 * E * Np - P2;
    double den = 2.0 * Ep * Np - pp2;
    double scale = 0.0;
    /* Each bracket is a difference of two terms of size 2 E N'; it vanishes
     * exactly when all velocities coincide (the denominator for n' = 1), so a
     * value within rounding of zero (1e-12 of either term) counts as zero. */
    if (num > 1e-12 * (2.0 * E * Np) && den > 1e-12 * (2.0 * Ep * Np)) {
        scale = sqrt(num / den);
        double beta[ORC_MAXD];
        for (int d = 0; d < D; ++d) beta[d] = (Pt[d] - scale * pp[d]) / (scale * Np);
        for (int64_t i = 0; i < n; ++i) {
            double* vi = J->v_out + (size_t)(o0 + i) * D;
            for (int d = 0; d < D; ++d) vi[d] = scale * (vi[d] + beta[d]);
        }
    } else {
        /* R5: the projection has no real solution; leave the sample as drawn */
        st |= ORC_LEMONS_SKIPPED;
    }
    if (J->stats) {
        J->stats[(size_t)c * 4 + 0] = scale;
        J->stats[(size_t)c * 4 + 1] = Np;
        J->stats[(size_t)c * 4 + 2] = sqrt(pp2);
        J->stats[(size_t)c * 4 + 3] = Ep;
    }
    return st;
}

typedef struct {
    const recon_job* J;
    int64_t c0, c1;
} recon_chunk;

static void* recon_worker(void* arg)
{
    recon_chunk* ch = (recon_chunk*)arg;
    for (int64_t c = ch->c0; c < ch->c1; ++c) reconstruct_cell(ch->J, c);
    return NULL;
}

static void fill_recon(void* chunk, void* job, int64_t c0, int64_t c1)
{
    recon_chunk* ch = (recon_chunk*)chunk;
    ch->J = (const recon_job*)job;
    ch->c0 = c0;
    ch->c1 = c1;
}

int orc_reconstruct(const int32_t* K, const double* w, const double* mu, const double* S, int kmax,
                    const int64_t* out_off, const double* target, int64_t n_cells, int D, int dx, uint64_t seed,
                    double* v_out, double* w_out, double* x_out, int32_t* status, double* stats, int nthreads)
{
    if (D < 1 || D > ORC_MAXD || dx < 0 || dx > 3 || kmax < 1 || kmax > ORC_MAXK) return -1;
    recon_job J = {K, w, mu, S, kmax, out_off, target, n_cells, D, dx, seed, v_out, w_out, x_out, status, stats, 0};
    run_chunks(n_cells, nthreads, recon_worker, &J, sizeof(recon_chunk), fill_recon);
    return 0;
}

/* Projection alone, on particles already in v, w (e.g. after the Gauss'-law
 * weight correction): target = the moments record (W, P, S packed) per cell;
 * tensor = 0: Lemons' scalar projection towards P and E = tr(S) / 2;
 * tensor = 1: the full second moment. */
int orc_project(double* v, double* w, const int64_t* off, const double* moments, int64_t n_cells, int D,
                int tensor, int32_t* status)
{
    if (D < 1 || D > ORC_MAXD) return -1;
    const int nt = ntri(D);
    recon_job J;
    memset(&J, 0, sizeof(J));
    J.D = D;
    J.v_out = v;
    J.w_out = w;
    J.tensor = tensor;
    for (int64_t c = 0; c < n_cells; ++c) {
        const int64_t o0 = off[c], n = off[c + 1] - off[c];
        const double* tg = moments + (size_t)c * (1 + D + nt);
        if (n <= 0) {
            status[c] = 0;
            continue;
        }
        if (tensor) {
            status[c] = project_tensor(&J, c, tg, o0, n);
        } else {
            double E = 0.0;
            for (int d = 0; d < D; ++d) E += 0.5 * tg[1 + D + d * D - d * (d - 1) / 2];
            status[c] = project_scalar(&J, c, tg[0], tg + 1, E, o0, n);
        }
    }
    return 0;
}

/* Same sampling; the full-second-moment projection with target = the
 * moments record (W, P, S packed) per cell. */
int orc_reconstruct_tensor(const int32_t* K, const double* w, const double* mu, const double* S, int kmax,
                           const int64_t* out_off, const double* moments, int64_t n_cells, int D, int dx,
                           uint64_t seed, double* v_out, double* w_out, double* x_out, int32_t* status, int nthreads)
{
    if (D < 1 || D > ORC_MAXD || dx < 0 || dx > 3 || kmax < 1 || kmax > ORC_MAXK) return -1;
    recon_job J = {K, w, mu, S, kmax, out_off, moments, n_cells, D, dx, seed, v_out, w_out, x_out, status, NULL, 1};
    run_chunks(n_cells, nthreads, recon_worker, &J, sizeof(recon_chunk), fill_recon);
    return 0;
}

/* ------------------------------------------------------------------ */
/* standard (non-adaptive) EM with K-means initialisation and Anderson */
/* acceleration (Sec. 3.4)                                             */
/* ------------------------------------------------------------------ */
/* The parameter vector accelerated by Anderson mixing holds, per component
 * in slot order, the weight w_k, the mean mu_k and the second moment
 * M2_k = Sigma_k + mu_k mu_k^T (packed upper triangle): the paper mixes M2
 * rather than Sigma because M2 is linear in the mixture. */
static int std_len(int D) { return 1 + D + ntri(D); }

static void theta_from_mixture(int D, const mixture* m, double* th)
{
    const int L = std_len(D);
    for (int k = 0; k < m->K; ++k) {
        double* t = th + (size_t)k * L;
        t[0] = m->w[k];
        for (int i = 0; i < D; ++i) t[1 + i] = m->mu[k][i];
        int q = 0;
        for (int i = 0; i < D; ++i)
            for (int j = i; j < D; ++j) t[1 + D + q++] = m->S[k][i][j] + m->mu[k][i] * m->mu[k][j];
    }
}

/* Decode a parameter vector; returns 0 if every weight is >= 0 and every
 * Sigma_k = M2_k - mu_k mu_k^T has a Cholesky factor, else -1. */
static int mixture_from_theta(int D, int K, const double* th, mixture* m)
{
    const int L = std_len(D);
    m->K = K;
    for (int k = 0; k < K; ++k) {
        const double* t = th + (size_t)k * L;
        if (!(t[0] >= 0.0)) return -1;
        m->w[k] = t[0];
        for (int i = 0; i < D; ++i) m->mu[k][i] = t[1 + i];
        int q = 0;
        for (int i = 0; i < D; ++i)
            for (int j = i; j < D; ++j) {
                const double s = t[1 + D + q++] - t[1 + i] * t[1 + j];
                m->S[k][i][j] = s;
                m->S[k][j][i] = s;
            }
        if (chol(D, (const double(*)[ORC_MAXD])m->S[k], m->L[k]) != 0) return -1;
    }
    return 0;
}

/* One standard EM step G(theta) (joint E-step, eqs. muk, sigmak, omegak-mle).
 * A component without responsibility (N_k = 0, only possible with w_k = 0)
 * keeps its mean and covariance and stays at weight 0.  Returns the
 * log-likelihood sum_p a_p ln sum_k w_k f_k(v_p) at the input parameters. */
static double std_em_step(int D, const mixture* m, int n, const double* x, const double* a, double N, double* g_all,
                          mixture* out)
{
    const int K = m->K;
    double gp[ORC_MAXK], ell[ORC_MAXK];
    double ll = 0.0;
    for (int p = 0; p < n; ++p) {
        const double* xp = x + (size_t)p * D;
        double mx = -INFINITY;
        for (int j = 0; j < K; ++j) {
            ell[j] = (m->w[j] > 0.0 ? log(m->w[j]) : -INFINITY) + log_normal(D, xp, m->mu[j], m->L[j]);
            if (ell[j] > mx) mx = ell[j];
        }
        double s = 0.0;
        for (int j = 0; j < K; ++j) {
            gp[j] = exp(ell[j] - mx);
            s += gp[j];
        }
        ll += a[p] * (mx + log(s));
        for (int j = 0; j < K; ++j) g_all[(size_t)j * n + p] = a[p] * gp[j] / s;
    }
    *out = *m;
    for (int k = 0; k < K; ++k) {
        const double* g = g_all + (size_t)k * n;
        double Nk = 0.0;
        for (int p = 0; p < n; ++p) Nk += g[p];
        if (!(Nk > 0.0)) {
            out->w[k] = 0.0;
            continue;
        }
        mean_cov(D, n, x, g, Nk, out->mu[k], out->S[k]);
        out->w[k] = Nk / N;
    }
    return ll;
}

/* K-means (Lloyd) from the given centres on the weighted centred particles,
 * Euclidean distance, ties to the lowest slot, weighted centroids; a centre
 * that loses all its particles stays where it is.  Stops when no assignment
 * changes (or after 100 passes).  On return m holds the initial mixture of
 * the hard assignment: w_k = W_k / N, mu_k the centroid, Sigma_k the
 * cluster's weighted covariance (the covariance floor where it does not
 * factor).  Returns the number of assignment passes. */
static int kmeans_init(int D, int K, int n, const double* x, const double* a, double N, const int* idx, double trC,
                       mixture* m, int* assign, int32_t* status)
{
    double c[ORC_MAXK][ORC_MAXD];
    for (int k = 0; k < K; ++k)
        for (int i = 0; i < D; ++i) c[k][i] = x[(size_t)idx[k] * D + i];
    for (int p = 0; p < n; ++p) assign[p] = -1;
    int pass = 0;
    for (pass = 1; pass <= 100; ++pass) {
        int changed = 0;
        for (int p = 0; p < n; ++p) {
            const double* xp = x + (size_t)p * D;
            int best = 0;
            double bd = INFINITY;
            for (int k = 0; k < K; ++k) {
                double d2 = 0.0;
                for (int i = 0; i < D; ++i) d2 += (xp[i] - c[k][i]) * (xp[i] - c[k][i]);
                if (d2 < bd) {
                    bd = d2;
                    best = k;
                }
            }
            if (best != assign[p]) {
                changed = 1;
                assign[p] = best;
            }
        }
        if (!changed) break;
        for (int k = 0; k < K; ++k) {
            double W = 0.0, s[ORC_MAXD] = {0, 0, 0};
            for (int p = 0; p < n; ++p)
                if (assign[p] == k) {
                    W += a[p];
                    for (int i = 0; i < D; ++i) s[i] += a[p] * x[(size_t)p * D + i];
                }
            if (W > 0.0)
                for (int i = 0; i < D; ++i) c[k][i] = s[i] / W;
        }
    }
    if (pass > 100) pass = 100;
    m->K = K;
    for (int k = 0; k < K; ++k) {
        double W = 0.0;
        for (int p = 0; p < n; ++p)
            if (assign[p] == k) W += a[p];
        for (int i = 0; i < D; ++i) m->mu[k][i] = c[k][i];
        m->w[k] = W / N;
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                double s = 0.0;
                for (int p = 0; p < n; ++p)
                    if (assign[p] == k) s += a[p] * (x[(size_t)p * D + i] - c[k][i]) * (x[(size_t)p * D + j] - c[k][j]);
                m->S[k][i][j] = W > 0.0 ? s / W : 0.0;
            }
        if (factor_component(D, m, k, trC)) *status |= ORC_COV_FLOOR;
    }
    return pass;
}

/* Least squares min |f - dF gamma| over the columns of dF (len x mk, column
 * j at dF + j * len) by modified Gram-Schmidt; returns -1 when a column is
 * numerically dependent on the earlier ones (|R_jj| <= 1e-12 |dF_j|). */
static int aa_solve(int len, int mk, const double* dF, const double* f, double* gamma)
{
    double Q[ORC_AA_MAX][ORC_MAXK * 10], R[ORC_AA_MAX][ORC_AA_MAX], qf[ORC_AA_MAX];
    for (int j = 0; j < mk; ++j) {
        double nrm0 = 0.0;
        for (int t = 0; t < len; ++t) {
            Q[j][t] = dF[(size_t)j * len + t];
            nrm0 += Q[j][t] * Q[j][t];
        }
        for (int l = 0; l < j; ++l) {
            double r = 0.0;
            for (int t = 0; t < len; ++t) r += Q[l][t] * Q[j][t];
            R[l][j] = r;
            for (int t = 0; t < len; ++t) Q[j][t] -= r * Q[l][t];
        }
        double nrm = 0.0;
        for (int t = 0; t < len; ++t) nrm += Q[j][t] * Q[j][t];
        nrm = sqrt(nrm);
        if (!(nrm > 1e-12 * sqrt(nrm0))) return -1;
        R[j][j] = nrm;
        for (int t = 0; t < len; ++t) Q[j][t] /= nrm;
    }
    for (int j = 0; j < mk; ++j) {
        double s = 0.0;
        for (int t = 0; t < len; ++t) s += Q[j][t] * f[t];
        qf[j] = s;
    }
    for (int j = mk - 1; j >= 0; --j) {
        double s = qf[j];
        for (int l = j + 1; l < mk; ++l) s -= R[j][l] * gamma[l];
        gamma[j] = s / R[j][j];
    }
    return 0;
}

typedef struct {
    const double* v;
    const double* alpha;
    const int64_t* off;
    int D, kmax, K, n_min, max_iter;
    double tol;
    uint64_t seed;
    int kmeans, aa_m;
    int32_t* Kout;
    double* w;
    double* mu;
    double* S;
    double* mom;
    double* ll_out;
    double* L_final;
    int32_t* iters;
    int32_t* status;
    int32_t* resets;
    int32_t* kmeans_passes;
    double* ll_trace; /* nullable [n_cells * max_iter] */
} std_job;

/* Standard (non-adaptive) EM of one cell, Sec. 3.4: K0 = min(K, n)
 * components started at the cold-start particles (or K-means from them),
 * then G(theta) iterations, Anderson-mixed when aa_m > 0 (Walker & Ni, the
 * unconstrained difference form: theta_{i+1} = G(theta_i) - dG gamma with
 * gamma = argmin |f_i - dF gamma|, f = G(theta) - theta, dF/dG the last
 * min(aa_m, i) differences).  A mixed state with a negative weight or an
 * indefinite Sigma, or a dependent least-squares column, resets the
 * mixing: the step becomes G(theta_i) and the history restarts from it.
 * Mixed weights are renormalised to sum 1.  Stop when the log-likelihood
 * at theta_i changes by at most tol relative, or after max_iter
 * iterations; the state theta_i is the result, and the unpenalised joint
 * step of the finish (Sec. 2.3.1) is the standard EM step that follows it. */
static void std_cell(const std_job* J, int64_t c, double* x, double* a, double* g, int* assign, double* hist)
{
    const int D = J->D, nt = ntri(D), L = std_len(D);
    const int64_t o0 = J->off[c], o1 = J->off[c + 1];
    const int n = (int)(o1 - o0);
    const double T = 0.5 * D * (D + 3);
    const double* v = J->v + (size_t)o0 * D;
    const double* al = J->alpha + o0;
    int32_t status = 0;
    mixture m;
    memset(&m, 0, sizeof(m));
    double* mom = J->mom + (size_t)c * (1 + D + nt);
    for (int i = 0; i < 1 + D + nt; ++i) mom[i] = 0.0;
    J->ll_out[c] = 0.0;
    J->L_final[c] = 0.0;
    J->iters[c] = 0;
    J->resets[c] = 0;
    J->kmeans_passes[c] = 0;
    compress_job W0;
    memset(&W0, 0, sizeof(W0));
    W0.D = D;
    W0.kmax = J->kmax;
    W0.K = J->Kout;
    W0.w = J->w;
    W0.mu = J->mu;
    W0.S = J->S;
    double zero[ORC_MAXD] = {0, 0, 0};
    for (int p = 0; p < n; ++p) {
        int bad = !isfinite(al[p]) || !(al[p] > 0.0);
        for (int i = 0; i < D; ++i) bad |= !isfinite(v[(size_t)p * D + i]);
        if (bad) {
            m.K = 0;
            write_mixture(&W0, c, &m, zero);
            J->status[c] = ORC_NONFINITE_INPUT;
            return;
        }
    }
    if (n == 0) {
        m.K = 0;
        write_mixture(&W0, c, &m, zero);
        J->status[c] = ORC_DEGENERATE;
        return;
    }
    /* moments, centring and weights summing to N = n, as for compress */
    double W = 0.0, P[ORC_MAXD] = {0, 0, 0}, S2[ORC_MAXD][ORC_MAXD];
    memset(S2, 0, sizeof(S2));
    for (int p = 0; p < n; ++p) {
        W += al[p];
        for (int i = 0; i < D; ++i) {
            P[i] += al[p] * v[(size_t)p * D + i];
            for (int j = 0; j < D; ++j) S2[i][j] += al[p] * v[(size_t)p * D + i] * v[(size_t)p * D + j];
        }
    }
    mom[0] = W;
    for (int i = 0; i < D; ++i) mom[1 + i] = P[i];
    pack_sym(D, (const double(*)[ORC_MAXD])S2, mom + 1 + D);
    double mean[ORC_MAXD] = {0, 0, 0};
    for (int i = 0; i < D; ++i) mean[i] = P[i] / W;
    double C[ORC_MAXD][ORC_MAXD];
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
            for (int p = 0; p < n; ++p) s += al[p] * (v[(size_t)p * D + i] - mean[i]) * (v[(size_t)p * D + j] - mean[j]);
            C[i][j] = s / W;
        }
    double trC = 0.0;
    for (int i = 0; i < D; ++i) trC += C[i][i];
    const double N = (double)n;
    for (int p = 0; p < n; ++p) {
        a[p] = al[p] * (double)n / W;
        for (int i = 0; i < D; ++i) x[(size_t)p * D + i] = v[(size_t)p * D + i] - mean[i];
    }
    double LC[ORC_MAXD][ORC_MAXD];
    const int c_spd = chol(D, (const double(*)[ORC_MAXD])C, LC) == 0;
    if (n <= J->n_min || !c_spd) {
        m.K = 1;
        m.w[0] = 1.0;
        memcpy(m.S[0], C, sizeof(C));
        memcpy(m.L[0], LC, sizeof(LC));
        status |= c_spd ? ORC_SMALL_CELL_K1 : (ORC_SMALL_CELL_K1 | ORC_DEGENERATE);
        J->L_final[c] = c_spd ? penalised_L(D, T, &m, n, x, a, N) : -INFINITY;
        J->ll_out[c] = J->L_final[c];
        write_mixture(&W0, c, &m, mean);
        J->status[c] = status;
        return;
    }
    /* start: the cold-start particles, K0 = min(K, n) (no penalty, no cap) */
    const int K0 = J->K < n ? J->K : n;
    int* perm = (int*)malloc(sizeof(int) * (size_t)n);
    orc_init_indices(n, K0, J->seed, (uint64_t)c, perm);
    if (J->kmeans) {
        J->kmeans_passes[c] = kmeans_init(D, K0, n, x, a, N, perm, trC, &m, assign, &status);
    } else {
        m.K = K0;
        for (int k = 0; k < K0; ++k) {
            m.w[k] = 1.0 / K0;
            for (int i = 0; i < D; ++i) m.mu[k][i] = x[(size_t)perm[k] * D + i];
            memcpy(m.S[k], C, sizeof(C));
            memcpy(m.L[k], LC, sizeof(LC));
        }
    }
    free(perm);
    /* iterations: hist holds up to aa_m + 1 pairs (f, G) of length len */
    const int len = K0 * L, mmax = J->aa_m;
    double* th = hist;                        /* theta_i */
    double* fg = th + (size_t)len;            /* G(theta_i) */
    double* Fh = fg + (size_t)len;            /* ring of f, (mmax + 1) x len */
    double* Gh = Fh + (size_t)(mmax + 1) * len; /* ring of G, (mmax + 1) x len */
    double* dF = Gh + (size_t)(mmax + 1) * len; /* mmax x len */
    double* dG = dF + (size_t)mmax * len;
    double gamma[ORC_AA_MAX];
    theta_from_mixture(D, &m, th);
    int nh = 0, head = 0, resets = 0, it = 0, mixed = 0, have_prev = 0, converged = 0;
    double ll = 0.0, ll_prev = 0.0;
    mixture gm, g_acc;
    memset(&g_acc, 0, sizeof(g_acc));
    while (it < J->max_iter) {
        ++it;
        ll = std_em_step(D, &m, n, x, a, N, g, &gm);
        if (J->ll_trace) J->ll_trace[(size_t)c * J->max_iter + (it - 1)] = ll;
        if (mixed && !(ll >= ll_prev)) {
            /* the mixed iterate lowered the likelihood: back to the plain
             * step of the last accepted iterate, history cleared */
            ++resets;
            m = g_acc;
            m.K = K0;
            for (int k = 0; k < K0; ++k)
                if (factor_component(D, &m, k, trC)) status |= ORC_COV_FLOOR;
            theta_from_mixture(D, &m, th);
            nh = 0;
            head = 0;
            mixed = 0;
            continue;
        }
        if (have_prev && fabs(ll - ll_prev) <= J->tol * fabs(ll)) {
            converged = 1;
            break;
        }
        if (!isfinite(ll)) break;
        ll_prev = ll;
        have_prev = 1;
        g_acc = gm;
        theta_from_mixture(D, &gm, fg);
        int take_g = 1;
        mixed = 0;
        if (mmax > 0) {
            /* push (f_i, G_i) */
            double* fslot = Fh + (size_t)head * len;
            double* gslot = Gh + (size_t)head * len;
            for (int t = 0; t < len; ++t) {
                fslot[t] = fg[t] - th[t];
                gslot[t] = fg[t];
            }
            head = (head + 1) % (mmax + 1);
            if (nh < mmax + 1) ++nh;
            const int mk = nh - 1;
            if (mk >= 1) {
                /* columns j = 0..mk-1: oldest difference first */
                for (int j = 0; j < mk; ++j) {
                    const int i0 = (head - nh + j + 2 * (mmax + 1)) % (mmax + 1);
                    const int i1 = (i0 + 1) % (mmax + 1);
                    for (int t = 0; t < len; ++t) {
                        dF[(size_t)j * len + t] = Fh[(size_t)i1 * len + t] - Fh[(size_t)i0 * len + t];
                        dG[(size_t)j * len + t] = Gh[(size_t)i1 * len + t] - Gh[(size_t)i0 * len + t];
                    }
                }
                const double* fcur = Fh + (size_t)((head + mmax) % (mmax + 1)) * len;
                if (aa_solve(len, mk, dF, fcur, gamma) == 0) {
                    double cand[ORC_MAXK * 10];
                    for (int t = 0; t < len; ++t) {
                        double s = fg[t];
                        for (int j = 0; j < mk; ++j) s -= gamma[j] * dG[(size_t)j * len + t];
                        cand[t] = s;
                    }
                    double ws = 0.0;
                    for (int k = 0; k < K0; ++k) ws += cand[(size_t)k * L];
                    for (int k = 0; k < K0; ++k) cand[(size_t)k * L] /= ws;
                    mixture cm;
                    if (ws > 0.0 && mixture_from_theta(D, K0, cand, &cm) == 0) {
                        memcpy(th, cand, sizeof(double) * (size_t)len);
                        m = cm;
                        take_g = 0;
                        mixed = 1;
                    }
                }
                if (take_g) {
                    /* no usable mixed iterate: the plain step, and the
                     * history restarts from the latest pair */
                    ++resets;
                    const int last = (head + mmax) % (mmax + 1);
                    if (last != 0) {
                        memcpy(Fh, Fh + (size_t)last * len, sizeof(double) * (size_t)len);
                        memcpy(Gh, Gh + (size_t)last * len, sizeof(double) * (size_t)len);
                    }
                    nh = 1;
                    head = 1 % (mmax + 1);
                }
            }
        }
        if (take_g) {
            /* G keeps Sigma positive definite unless a component collapsed */
            m = gm;
            m.K = K0;
            for (int k = 0; k < K0; ++k)
                if (factor_component(D, &m, k, trC)) status |= ORC_COV_FLOOR;
            theta_from_mixture(D, &m, th);
        }
    }
    if (!converged) status |= ORC_MAXSWEEPS;
    J->iters[c] = it;
    J->resets[c] = resets;
    J->ll_out[c] = ll;
    /* components left without weight are dropped */
    for (int k = m.K - 1; k >= 0; --k)
        if (!(m.w[k] > 0.0)) remove_component(&m, k);
    renormalise(&m);
    if (mle_finish(D, &m, n, x, a, N, g) != 0) {
        m.K = 1;
        m.w[0] = 1.0;
        memcpy(m.S[0], C, sizeof(C));
        memcpy(m.L[0], LC, sizeof(LC));
        memset(m.mu[0], 0, sizeof(m.mu[0]));
        status |= ORC_DEGENERATE;
    }
    J->L_final[c] = penalised_L(D, T, &m, n, x, a, N);
    write_mixture(&W0, c, &m, mean);
    J->status[c] = status;
}

typedef struct {
    const std_job* J;
    int64_t c0, c1;
} std_chunk;

static void* std_worker(void* arg)
{
    std_chunk* ch = (std_chunk*)arg;
    const std_job* J = ch->J;
    int64_t nmax = max_cell_len(J->off, ch->c0, ch->c1);
    if (nmax < 1) nmax = 1;
    const size_t len = (size_t)J->K * std_len(J->D);
    double* x = (double*)malloc(sizeof(double) * (size_t)nmax * J->D);
    double* a = (double*)malloc(sizeof(double) * (size_t)nmax);
    double* g = (double*)malloc(sizeof(double) * (size_t)nmax * ORC_MAXK);
    int* assign = (int*)malloc(sizeof(int) * (size_t)nmax);
    double* hist = (double*)malloc(sizeof(double) * len * (2 + 4 * (size_t)J->aa_m + 2));
    for (int64_t c = ch->c0; c < ch->c1; ++c) std_cell(J, c, x, a, g, assign, hist);
    free(x);
    free(a);
    free(g);
    free(assign);
    free(hist);
    return NULL;
}

static void fill_std(void* chunk, void* job, int64_t c0, int64_t c1)
{
    std_chunk* ch = (std_chunk*)chunk;
    ch->J = (const std_job*)job;
    ch->c0 = c0;
    ch->c1 = c1;
}

/* Standard EM of every cell (Sec. 3.4): K components (K <= kmax), random
 * or K-means start, Anderson memory aa_m (0 = plain EM, at most 8). */
int orc_compress_std(const double* v, const double* alpha, const int64_t* off, int64_t n_cells, int D, int kmax,
                     int K, int n_min, int max_iter, double tol, uint64_t seed, int kmeans, int aa_m, int32_t* Kout,
                     double* w, double* mu, double* S, double* mom, double* ll_out, double* L_final, int32_t* iters,
                     int32_t* status, int32_t* resets, int32_t* kmeans_passes, double* ll_trace, int nthreads)
{
    if (D < 1 || D > ORC_MAXD || kmax < 1 || kmax > ORC_MAXK || K < 1 || K > kmax || max_iter < 1 || aa_m < 0 ||
        aa_m > ORC_AA_MAX)
        return -1;
    std_job J = {v, alpha, off, D, kmax, K, n_min, max_iter, tol, seed, kmeans, aa_m, Kout, w, mu, S, mom, ll_out,
                 L_final, iters, status, resets, kmeans_passes, ll_trace};
    run_chunks(n_cells, nthreads, std_worker, &J, sizeof(std_chunk), fill_std);
    return 0;
}

/* Test entry: the Anderson least-squares step on given columns. */
int orc_aa_solve(int len, int mk, const double* dF, const double* f, double* gamma)
{
    if (len < 1 || len > ORC_MAXK * 10 || mk < 1 || mk > ORC_AA_MAX) return -2;
    return aa_solve(len, mk, dF, f, gamma);
}

/* Test entry: K-means from the given start indices on centred particles x
 * (n x D) with weights a; writes the hard-assignment mixture (w, mu, S
 * packed) and the assignment; returns the number of passes. */
int orc_kmeans(const double* x, const double* a, int n, int D, int K, const int* idx, double* w, double* mu,
               double* S, int* assign)
{
    if (D < 1 || D > ORC_MAXD || K < 1 || K > ORC_MAXK || n < 1) return -1;
    double N = 0.0, trC = 0.0;
    for (int p = 0; p < n; ++p) N += a[p];
    for (int i = 0; i < D; ++i) {
        double m = 0.0, s = 0.0;
        for (int p = 0; p < n; ++p) m += a[p] * x[(size_t)p * D + i];
        m /= N;
        for (int p = 0; p < n; ++p) s += a[p] * (x[(size_t)p * D + i] - m) * (x[(size_t)p * D + i] - m);
        trC += s / N;
    }
    mixture m;
    memset(&m, 0, sizeof(m));
    int32_t st = 0;
    const int passes = kmeans_init(D, K, n, x, a, N, idx, trC, &m, assign, &st);
    for (int k = 0; k < K; ++k) {
        w[k] = m.w[k];
        for (int i = 0; i < D; ++i) mu[(size_t)k * D + i] = m.mu[k][i];
        pack_sym(D, (const double(*)[ORC_MAXD])m.S[k], S + (size_t)k * ntri(D));
    }
    return passes;
}
