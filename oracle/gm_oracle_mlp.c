/*
 * gm_oracle_mlp.c -- FP64 oracle of the learned warm start (test
 * infrastructure only, like gm_oracle.c; shares nothing with the library).
 *
 * The paper does not learn its initial mixtures: it starts every cell from
 * random particles (Sec. 2.3) and notes that better starting points speed up
 * the EM iteration (Sec. 3.4).  The warm start built here maps per-cell
 * features to an initial mixture with a small multilayer perceptron:
 *
 *   features (105): whitened velocities u = L_C^-1 (v - m) of the cell (m, C
 *     its weighted mean and covariance, C = L_C L_C^T); three 32-bin
 *     histograms of u_x, u_y, u_z over [-4, 4) (bin width 1/4, values outside
 *     clamped to the end bins) weighted by alpha_p / W; then E[u_d^3] (3),
 *     E[u_d^4] - 3 (3) and E[u_d^2 u_e^2] - 1 for (d,e) = (x,y), (x,z), (y,z)
 *     (3), expectations weighted by alpha_p / W.
 *   network: 105 -> 256 -> 256 -> 160, ReLU on the hidden layers; weights
 *     row-major [in][out].
 *   output: 16 slots x (logit, mu_hat[3], l00, l10, l11, l20, l21, l22) with
 *     the diagonal entries of the lower factor L_hat as logarithms.
 *   decode: w = softmax(logit); keep slots with N w > T/2 (slot order; if
 *     none, the largest), renormalise; mu = m + L_C mu_hat; Sigma = L L^T with
 *     L = L_C L_hat.  A cell without a frame (empty, or a singular
 *     covariance) decodes to K = 0: it keeps the cold start.
 *   loss: soft cross-entropy of the target weights against softmax(logit)
 *     plus lambda sum_j w_t,j (|mu_hat_j - mu_t,j|^2 + |l_j - l_t,j|^2),
 *     averaged over the batch; targets are the plain-EM mixtures expressed in
 *     the same whitened frame, sorted by weight (descending, ties by mu_x).
 *
 * With `bf16` set, values are rounded to bfloat16 at the points where the
 * GPU kernels round them (inputs and weights of every product, hidden
 * activations, the output gradient and the hidden gradients), first to
 * FP32 and then to BF16 with round-to-nearest-even.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NF 105
#define NH 256
#define NO 160
#define NSLOT 16
#define SLOT 10

static double bf16r(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan */
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7fffu + lsb;
    b &= 0xffff0000u;
    memcpy(&f, &b, 4);
    return (double)f;
}

static double rnd(double x, int bf16) { return bf16 ? bf16r(x) : x; }

/* Cholesky of a packed upper 3x3 (00 01 02 11 12 22); L row-major 3x3 */
static int chol3(const double* S, double L[3][3])
{
    memset(L, 0, sizeof(double) * 9);
    double a00 = S[0];
    if (!(a00 > 0)) return -1;
    L[0][0] = sqrt(a00);
    L[1][0] = S[1] / L[0][0];
    L[2][0] = S[2] / L[0][0];
    double a11 = S[3] - L[1][0] * L[1][0];
    if (!(a11 > 0)) return -1;
    L[1][1] = sqrt(a11);
    L[2][1] = (S[4] - L[2][0] * L[1][0]) / L[1][1];
    double a22 = S[5] - L[2][0] * L[2][0] - L[2][1] * L[2][1];
    if (!(a22 > 0)) return -1;
    L[2][2] = sqrt(a22);
    return 0;
}

/* solve L y = b (lower) */
static void lsolve(double L[3][3], const double* b, double* y)
{
    y[0] = b[0] / L[0][0];
    y[1] = (b[1] - L[1][0] * y[0]) / L[1][1];
    y[2] = (b[2] - L[2][0] * y[0] - L[2][1] * y[1]) / L[2][2];
}

/* features of every 3V cell; frame = (m[3], L_C packed lower 00 10 11 20 21 22) */
int orc_features(const double* v, const double* alpha, const int64_t* off, int64_t n_cells, double* feats,
                 double* frame)
{
    for (int64_t c = 0; c < n_cells; ++c) {
        const int64_t o0 = off[c], n = off[c + 1] - off[c];
        double* f = feats + (size_t)c * NF;
        double* fr = frame + (size_t)c * 9;
        memset(f, 0, sizeof(double) * NF);
        memset(fr, 0, sizeof(double) * 9);
        if (n < 1) continue;
        double W = 0, m[3] = {0, 0, 0};
        for (int64_t p = 0; p < n; ++p) {
            W += alpha[o0 + p];
            for (int d = 0; d < 3; ++d) m[d] += alpha[o0 + p] * v[(o0 + p) * 3 + d];
        }
        for (int d = 0; d < 3; ++d) m[d] /= W;
        double C[6] = {0, 0, 0, 0, 0, 0};
        int t = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j, ++t) {
                double s = 0;
                for (int64_t p = 0; p < n; ++p)
                    s += alpha[o0 + p] * (v[(o0 + p) * 3 + i] - m[i]) * (v[(o0 + p) * 3 + j] - m[j]);
                C[t] = s / W;
            }
        double L[3][3];
        for (int d = 0; d < 3; ++d) fr[d] = m[d];
        if (chol3(C, L) != 0) continue; /* singular cell: zero features, frame has the mean only */
        fr[3] = L[0][0];
        fr[4] = L[1][0];
        fr[5] = L[1][1];
        fr[6] = L[2][0];
        fr[7] = L[2][1];
        fr[8] = L[2][2];
        for (int64_t p = 0; p < n; ++p) {
            double q = alpha[o0 + p] / W, b[3], u[3];
            for (int d = 0; d < 3; ++d) b[d] = v[(o0 + p) * 3 + d] - m[d];
            lsolve(L, b, u);
            for (int d = 0; d < 3; ++d) {
                int bin = (int)floor((u[d] + 4.0) * 4.0);
                if (bin < 0) bin = 0;
                if (bin > 31) bin = 31;
                f[32 * d + bin] += q;
                f[96 + d] += q * u[d] * u[d] * u[d];
                f[99 + d] += q * u[d] * u[d] * u[d] * u[d];
            }
            f[102] += q * u[0] * u[0] * u[1] * u[1];
            f[103] += q * u[0] * u[0] * u[2] * u[2];
            f[104] += q * u[1] * u[1] * u[2] * u[2];
        }
        for (int d = 0; d < 3; ++d) f[99 + d] -= 3.0;
        for (int d = 102; d < 105; ++d) f[d] -= 1.0;
    }
    return 0;
}

/* Y = act(X W + b) for X [B x nin], W [nin x nout] */
static void dense(const double* X, int B, int nin, const double* W, const double* b, int nout, int relu, int bf16,
                  double* Y)
{
    for (int r = 0; r < B; ++r)
        for (int j = 0; j < nout; ++j) {
            double s = 0;
            for (int i = 0; i < nin; ++i) s += rnd(X[(size_t)r * nin + i], bf16) * rnd(W[(size_t)i * nout + j], bf16);
            s += b[j];
            Y[(size_t)r * nout + j] = relu ? (s > 0 ? s : 0) : s;
        }
}

int orc_mlp_forward(const double* X, int B, const double* W1, const double* b1, const double* W2, const double* b2,
                    const double* W3, const double* b3, int bf16, double* H1, double* H2, double* Y)
{
    dense(X, B, NF, W1, b1, NH, 1, bf16, H1);
    dense(H1, B, NH, W2, b2, NH, 1, bf16, H2);
    dense(H2, B, NH, W3, b3, NO, 0, bf16, Y);
    return 0;
}

/* loss and dLoss/dY for one batch (mean over rows) */
static double loss_grad(const double* Y, const double* Tg, int B, double lambda, double* dY)
{
    double total = 0;
    for (int r = 0; r < B; ++r) {
        const double* y = Y + (size_t)r * NO;
        const double* t = Tg + (size_t)r * NO;
        double* g = dY + (size_t)r * NO;
        double mx = -INFINITY;
        for (int j = 0; j < NSLOT; ++j)
            if (y[j * SLOT] > mx) mx = y[j * SLOT];
        double se = 0;
        for (int j = 0; j < NSLOT; ++j) se += exp(y[j * SLOT] - mx);
        double lse = mx + log(se);
        double wsum = 0;
        for (int j = 0; j < NSLOT; ++j) wsum += t[j * SLOT];
        for (int j = 0; j < NSLOT; ++j) {
            double wt = t[j * SLOT];
            double pj = exp(y[j * SLOT] - lse);
            total += -wt * (y[j * SLOT] - lse);
            g[j * SLOT] = (pj * wsum - wt) / B;
            for (int q = 1; q < SLOT; ++q) {
                double d = y[j * SLOT + q] - t[j * SLOT + q];
                total += lambda * wt * d * d;
                g[j * SLOT + q] = 2.0 * lambda * wt * d / B;
            }
        }
    }
    return total / B;
}

/* backward of the three dense layers; returns the loss */
double orc_mlp_loss_backward(const double* X, int B, const double* W1, const double* b1, const double* W2,
                             const double* b2, const double* W3, const double* b3, const double* Tg, double lambda,
                             int bf16, double* gW1, double* gb1, double* gW2, double* gb2, double* gW3, double* gb3,
                             double* dY_out)
{
    double* H1 = (double*)malloc(sizeof(double) * (size_t)B * NH);
    double* H2 = (double*)malloc(sizeof(double) * (size_t)B * NH);
    double* Y = (double*)malloc(sizeof(double) * (size_t)B * NO);
    double* dY = (double*)malloc(sizeof(double) * (size_t)B * NO);
    double* dH2 = (double*)malloc(sizeof(double) * (size_t)B * NH);
    double* dH1 = (double*)malloc(sizeof(double) * (size_t)B * NH);
    orc_mlp_forward(X, B, W1, b1, W2, b2, W3, b3, bf16, H1, H2, Y);
    double L = loss_grad(Y, Tg, B, lambda, dY);
    if (dY_out) memcpy(dY_out, dY, sizeof(double) * (size_t)B * NO);
    /* layer 3: Y = H2 W3 + b3 */
    for (int i = 0; i < NH; ++i)
        for (int j = 0; j < NO; ++j) {
            double s = 0;
            for (int r = 0; r < B; ++r) s += rnd(H2[(size_t)r * NH + i], bf16) * rnd(dY[(size_t)r * NO + j], bf16);
            gW3[(size_t)i * NO + j] = s;
        }
    for (int j = 0; j < NO; ++j) {
        double s = 0;
        for (int r = 0; r < B; ++r) s += dY[(size_t)r * NO + j];
        gb3[j] = s;
    }
    for (int r = 0; r < B; ++r)
        for (int i = 0; i < NH; ++i) {
            double s = 0;
            for (int j = 0; j < NO; ++j) s += rnd(dY[(size_t)r * NO + j], bf16) * rnd(W3[(size_t)i * NO + j], bf16);
            dH2[(size_t)r * NH + i] = H2[(size_t)r * NH + i] > 0 ? s : 0;
        }
    /* layer 2: H2 = relu(H1 W2 + b2) */
    for (int i = 0; i < NH; ++i)
        for (int j = 0; j < NH; ++j) {
            double s = 0;
            for (int r = 0; r < B; ++r) s += rnd(H1[(size_t)r * NH + i], bf16) * rnd(dH2[(size_t)r * NH + j], bf16);
            gW2[(size_t)i * NH + j] = s;
        }
    for (int j = 0; j < NH; ++j) {
        double s = 0;
        for (int r = 0; r < B; ++r) s += dH2[(size_t)r * NH + j];
        gb2[j] = s;
    }
    for (int r = 0; r < B; ++r)
        for (int i = 0; i < NH; ++i) {
            double s = 0;
            for (int j = 0; j < NH; ++j) s += rnd(dH2[(size_t)r * NH + j], bf16) * rnd(W2[(size_t)i * NH + j], bf16);
            dH1[(size_t)r * NH + i] = H1[(size_t)r * NH + i] > 0 ? s : 0;
        }
    /* layer 1: H1 = relu(X W1 + b1) */
    for (int i = 0; i < NF; ++i)
        for (int j = 0; j < NH; ++j) {
            double s = 0;
            for (int r = 0; r < B; ++r) s += rnd(X[(size_t)r * NF + i], bf16) * rnd(dH1[(size_t)r * NH + j], bf16);
            gW1[(size_t)i * NH + j] = s;
        }
    for (int j = 0; j < NH; ++j) {
        double s = 0;
        for (int r = 0; r < B; ++r) s += dH1[(size_t)r * NH + j];
        gb1[j] = s;
    }
    free(H1);
    free(H2);
    free(Y);
    free(dY);
    free(dH2);
    free(dH1);
    return L;
}

/* initial mixtures from network outputs (D = 3) */
int orc_warm_decode(const double* Y, const double* frame, const int64_t* off, int64_t n_cells, int kmax, int32_t* K,
                    double* w, double* mu, double* S)
{
    const double halfT = 4.5;
    for (int64_t c = 0; c < n_cells; ++c) {
        const double* y = Y + (size_t)c * NO;
        const double* fr = frame + (size_t)c * 9;
        const double N = (double)(off[c + 1] - off[c]);
        for (int q = 0; q < kmax; ++q) {
            size_t s = (size_t)c * kmax + q;
            w[s] = 0;
            for (int d = 0; d < 3; ++d) mu[s * 3 + d] = 0;
            for (int d = 0; d < 6; ++d) S[s * 6 + d] = 0;
        }
        /* no whitening frame (empty cell or singular covariance): no warm
         * start, the cell keeps the cold start */
        if (!(fr[3] > 0)) {
            K[c] = 0;
            continue;
        }
        double mx = -INFINITY;
        for (int j = 0; j < NSLOT; ++j)
            if (y[j * SLOT] > mx) mx = y[j * SLOT];
        double p[NSLOT], se = 0;
        for (int j = 0; j < NSLOT; ++j) {
            p[j] = exp(y[j * SLOT] - mx);
            se += p[j];
        }
        int keep[NSLOT], nk = 0, best = 0;
        for (int j = 0; j < NSLOT; ++j) {
            p[j] /= se;
            if (p[j] > p[best]) best = j;
        }
        for (int j = 0; j < NSLOT && nk < kmax; ++j)
            if (N * p[j] > halfT) keep[nk++] = j;
        if (nk == 0) keep[nk++] = best;
        double ws = 0;
        for (int q = 0; q < nk; ++q) ws += p[keep[q]];
        double LC[3][3] = {{fr[3], 0, 0}, {fr[4], fr[5], 0}, {fr[6], fr[7], fr[8]}};
        K[c] = nk;
        for (int q = 0; q < nk; ++q) {
            size_t s = (size_t)c * kmax + q;
            const double* o = y + keep[q] * SLOT;
            w[s] = p[keep[q]] / ws;
            for (int d = 0; d < 3; ++d) {
                double t = fr[d];
                for (int e = 0; e <= d; ++e) t += LC[d][e] * o[1 + e];
                mu[s * 3 + d] = t;
            }
            double Lh[3][3] = {{exp(o[4]), 0, 0}, {o[5], exp(o[6]), 0}, {o[7], o[8], exp(o[9])}};
            double L[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double t = 0;
                    for (int e = 0; e < 3; ++e) t += LC[i][e] * Lh[e][j];
                    L[i][j] = t;
                }
            int t = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = i; j < 3; ++j, ++t) {
                    double a = 0;
                    for (int e = 0; e < 3; ++e) a += L[i][e] * L[j][e];
                    S[s * 6 + t] = a;
                }
        }
    }
    return 0;
}

/* training targets from plain-EM mixtures, in the whitened frame */
int orc_warm_targets(const int32_t* K, const double* w, const double* mu, const double* S, const double* frame,
                     int64_t n_cells, int kmax, double* Tg)
{
    for (int64_t c = 0; c < n_cells; ++c) {
        double* t = Tg + (size_t)c * NO;
        memset(t, 0, sizeof(double) * NO);
        const double* fr = frame + (size_t)c * 9;
        if (!(fr[3] > 0)) continue;
        double LC[3][3] = {{fr[3], 0, 0}, {fr[4], fr[5], 0}, {fr[6], fr[7], fr[8]}};
        int k = K[c] < NSLOT ? K[c] : NSLOT;
        double rec[NSLOT][SLOT];
        int order[NSLOT];
        for (int q = 0; q < k; ++q) {
            size_t s = (size_t)c * kmax + q;
            rec[q][0] = w[s];
            double b[3], mh[3];
            for (int d = 0; d < 3; ++d) b[d] = mu[s * 3 + d] - fr[d];
            lsolve(LC, b, mh);
            for (int d = 0; d < 3; ++d) rec[q][1 + d] = mh[d];
            /* Sigma_hat = L_C^-1 Sigma L_C^-T: columns by two triangular solves */
            double Sg[3][3];
            int tt = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = i; j < 3; ++j, ++tt) Sg[i][j] = Sg[j][i] = S[s * 6 + tt];
            double Z[3][3], Sh[3][3];
            for (int j = 0; j < 3; ++j) {
                double col[3] = {Sg[0][j], Sg[1][j], Sg[2][j]}, y[3];
                lsolve(LC, col, y);
                for (int i = 0; i < 3; ++i) Z[i][j] = y[i];
            }
            for (int i = 0; i < 3; ++i) {
                double row[3] = {Z[i][0], Z[i][1], Z[i][2]}, y[3];
                lsolve(LC, row, y);
                for (int j = 0; j < 3; ++j) Sh[i][j] = y[j];
            }
            double sp[6] = {Sh[0][0], 0.5 * (Sh[0][1] + Sh[1][0]), 0.5 * (Sh[0][2] + Sh[2][0]), Sh[1][1],
                            0.5 * (Sh[1][2] + Sh[2][1]), Sh[2][2]};
            double Lh[3][3];
            if (chol3(sp, Lh) != 0) {
                memset(Lh, 0, sizeof(Lh));
                Lh[0][0] = Lh[1][1] = Lh[2][2] = 1e-3;
            }
            rec[q][4] = log(Lh[0][0]);
            rec[q][5] = Lh[1][0];
            rec[q][6] = log(Lh[1][1]);
            rec[q][7] = Lh[2][0];
            rec[q][8] = Lh[2][1];
            rec[q][9] = log(Lh[2][2]);
            order[q] = q;
        }
        /* weight descending, ties by mu_hat_x ascending (insertion sort) */
        for (int a = 1; a < k; ++a) {
            int x = order[a], b = a - 1;
            while (b >= 0 && (rec[order[b]][0] < rec[x][0] ||
                              (rec[order[b]][0] == rec[x][0] && rec[order[b]][1] > rec[x][1]))) {
                order[b + 1] = order[b];
                --b;
            }
            order[b + 1] = x;
        }
        for (int q = 0; q < k; ++q)
            for (int e = 0; e < SLOT; ++e) t[q * SLOT + e] = rec[order[q]][e];
    }
    return 0;
}
