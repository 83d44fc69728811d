// gm_warm.hip -- learned warm start for gm_compress on gfx950.
//
// A small multilayer perceptron maps per-cell features of the velocity
// distribution to an initial mixture, so the adaptive EM starts near its
// answer instead of from random particles (the paper starts from random
// particles, Sec. 2.3, and notes that better starting points speed the EM
// iteration up, Sec. 3.4).  Everything runs in kernels here:
//
//   k_features  FP64 whitening u = L_C^-1 (v - m) per cell, three 32-bin
//               histograms of u over [-4, 4) weighted by alpha / W
//               (deterministic fixed-point LDS atomics), and 9 moments
//               E[u_d^3], E[u_d^4] - 3, E[u_d^2 u_e^2] - 1 -> 105 BF16 values
//               (padded to 128) and the frame (m, L_C)
//   k_gemm      C = A B with BF16 operands on v_mfma_f32_16x16x32_bf16, FP32
//               accumulation, fused bias / ReLU / mask epilogue, FP32 and/or
//               BF16 outputs; arbitrary element strides cover the transposed
//               products of the backward pass
//   k_loss      soft cross-entropy of the target weights + weighted squared
//               error of the whitened means and log-Cholesky factors, and its
//               gradient
//   k_colsum    bias gradients (fixed-order column sums)
//   k_adam      Adam on FP32 master weights, refreshing the BF16 copies
//   k_decode    network outputs -> initial mixtures (gm_init layout)
//   k_targets   plain-EM mixtures -> training targets in the whitened frame
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "gm_device.h"

namespace gm {

constexpr int NF = 105, NFP = 128, NH = 256, NO = 160, NSLOT = 16, SLOT = 10;

// parameter layout (FP32 master, also the host layout of get/set_params)
constexpr size_t OFF_W1 = 0;
constexpr size_t OFF_B1 = OFF_W1 + (size_t)NFP * NH;
constexpr size_t OFF_W2 = OFF_B1 + NH;
constexpr size_t OFF_B2 = OFF_W2 + (size_t)NH * NH;
constexpr size_t OFF_W3 = OFF_B2 + NH;
constexpr size_t OFF_B3 = OFF_W3 + (size_t)NH * NO;
constexpr size_t NPARAM = OFF_B3 + NO;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return (uint16_t)((b >> 16) | ((b & 0xffffu) ? 0x40u : 0u));
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
constexpr int kFeatThreads = 256;
constexpr double kHistScale = 1099511627776.0;  // 2^40 fixed point for the histogram weights

__global__ __launch_bounds__(kFeatThreads) void k_features3(const double* v, const double* alpha, const int64_t* off,
                                                             uint16_t* feats, double* frame)
{
    __shared__ double red[2 * kMaxWaves * 10];
    __shared__ unsigned long long hist[96];
    __shared__ double sL[6];
    __shared__ int s_ok;
    const int c = blockIdx.x, tid = threadIdx.x, nthreads = blockDim.x, nwaves = nthreads >> 6;
    int par = 0;
    const int64_t o0 = off[c];
    const int64_t n = off[c + 1] - o0;
    uint16_t* f = feats + (size_t)c * NFP;
    double* fr = frame + (size_t)c * 9;
    for (int t = tid; t < 96; t += nthreads) hist[t] = 0ull;
    if (n <= 0) {
        for (int t = tid; t < NFP; t += nthreads) f[t] = 0;
        if (tid < 9) fr[tid] = 0.0;
        return;
    }
    const double* vc = v + o0 * 3;
    const double* ac = alpha + o0;
    double s[4] = {0, 0, 0, 0};
    for (int64_t i = tid; i < n; i += nthreads) {
        const double a = ac[i];
        s[0] += a;
        for (int d = 0; d < 3; ++d) s[1 + d] += a * vc[i * 3 + d];
    }
    block_sum<10>(s, red, par, nwaves);
    const double W = s[0];
    const double m[3] = {s[1] / W, s[2] / W, s[3] / W};
    double cv[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = tid; i < n; i += nthreads) {
        const double a = ac[i];
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = vc[i * 3 + d] - m[d];
        cv[0] += a * x[0] * x[0];
        cv[1] += a * x[0] * x[1];
        cv[2] += a * x[0] * x[2];
        cv[3] += a * x[1] * x[1];
        cv[4] += a * x[1] * x[2];
        cv[5] += a * x[2] * x[2];
    }
    block_sum<10>(cv, red, par, nwaves);
    if (tid == 0) {
        double C[6], L[6];
        for (int t = 0; t < 6; ++t) C[t] = cv[t] / W;
        s_ok = chol<3, double>(C, L);
        for (int t = 0; t < 6; ++t) sL[t] = s_ok ? L[t] : 0.0;
        for (int d = 0; d < 3; ++d) fr[d] = m[d];
        // frame factor, packed lower row-major: 00, 10, 11, 20, 21, 22
        fr[3] = sL[0];
        fr[4] = sL[1];
        fr[5] = sL[3];
        fr[6] = sL[2];
        fr[7] = sL[4];
        fr[8] = sL[5];
    }
    __syncthreads();
    if (!s_ok) {
        for (int t = tid; t < NFP; t += nthreads) f[t] = 0;
        return;
    }
    const double l00 = sL[0], l10 = sL[1], l20 = sL[2], l11 = sL[3], l21 = sL[4], l22 = sL[5];
    double mo[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = tid; i < n; i += nthreads) {
        const double q = ac[i] / W;
        const double b0 = vc[i * 3 + 0] - m[0], b1 = vc[i * 3 + 1] - m[1], b2 = vc[i * 3 + 2] - m[2];
        double u[3];
        u[0] = b0 / l00;
        u[1] = (b1 - l10 * u[0]) / l11;
        u[2] = (b2 - l20 * u[0] - l21 * u[1]) / l22;
        const unsigned long long qi = (unsigned long long)llrint(q * kHistScale);
        for (int d = 0; d < 3; ++d) {
            int bin = (int)floor((u[d] + 4.0) * 4.0);
            bin = bin < 0 ? 0 : (bin > 31 ? 31 : bin);
            atomicAdd(&hist[32 * d + bin], qi);
            const double u2 = u[d] * u[d];
            mo[d] += q * u2 * u[d];
            mo[3 + d] += q * u2 * u2;
        }
        mo[6] += q * u[0] * u[0] * u[1] * u[1];
        mo[7] += q * u[0] * u[0] * u[2] * u[2];
        mo[8] += q * u[1] * u[1] * u[2] * u[2];
    }
    block_sum<10>(mo, red, par, nwaves);
    __syncthreads();
    for (int t = tid; t < NFP; t += nthreads) {
        double val = 0.0;
        if (t < 96)
            val = (double)hist[t] / kHistScale;
        else if (t < 99)
            val = mo[t - 96];
        else if (t < 102)
            val = mo[t - 96] - 3.0;
        else if (t < 105)
            val = mo[t - 96] - 1.0;
        f[t] = f2bf((float)val);
    }
}

// ---------------------------------------------------------------------------
// BF16 GEMM on MFMA 16x16x32: one wave per 16x16 output tile, four waves per
// workgroup (a 32x32 block tile).  A(i,k) = A[i*sa_i + k*sa_k],
// B(k,j) = B[k*sb_k + j*sb_j].  Each 32-wide step of k stages the block's
// A and B slices through LDS, loaded along whichever index is contiguous in
// memory (the transposed operands of the backward products included) and
// stored k-contiguous, so every MFMA operand is one 16-byte LDS read.
// Epilogue: + bias[j], ReLU, mask (keep where mask(i,j) > 0), then FP32
// and/or BF16 stores.
// ---------------------------------------------------------------------------
struct GemmArgs {
    const uint16_t* A;
    int64_t sa_i, sa_k;
    const uint16_t* B;
    int64_t sb_k, sb_j;
    int M, N, K;
    const float* bias;
    const float* mask;
    int64_t ldm;
    int relu;
    float* C32;
    int64_t ldc;
    uint16_t* C16;
    int64_t ldc16;
};

constexpr int kGemmPad = 40;  // LDS row length of a staged slice (32 values + 8 of padding)

// 32 x 32 slice of a strided matrix into s[r][k] (row r, k contiguous):
// M(r, k) = P[r * s_r + k * s_k], rows r0.., columns k0.., zero outside
// [0, nr) x [0, nk).  Where one stride is 1 and the eight values a thread
// takes are inside the matrix and 16-byte aligned, they come in one vector
// load (128 threads); otherwise element by element.
__device__ __forceinline__ void stage_slice(const uint16_t* P, int64_t s_r, int64_t s_k, int r0, int k0, int nr,
                                            int nk, uint16_t (*s)[kGemmPad])
{
    const int t = threadIdx.x & 127;
    const bool kfast = s_k == 1;
    // this thread's run of eight along the contiguous index
    const int run = t & 3, other = t >> 2;        // 4 runs of 8 along the fast index, 32 along the other
    const int r = kfast ? other : run * 8;        // first row of the run
    const int k = kfast ? run * 8 : other;        // first column of the run
    const int gr = r0 + r, gk = k0 + k;
    const int64_t base = (int64_t)gr * s_r + (int64_t)gk * s_k;
    const bool inside = kfast ? (gr < nr && gk + 8 <= nk) : (gk < nk && gr + 8 <= nr);
    const bool vec = (kfast || s_r == 1) && inside && ((reinterpret_cast<uintptr_t>(P + base) & 15) == 0);
    u16x8 val;
    if (vec) {
        val = *reinterpret_cast<const u16x8*>(P + base);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int rr = kfast ? gr : gr + e, kk = kfast ? gk + e : gk;
            val[e] = (rr < nr && kk < nk) ? P[(int64_t)rr * s_r + (int64_t)kk * s_k] : (uint16_t)0;
        }
    }
    if (kfast) {
        *reinterpret_cast<u16x8*>(&s[r][k]) = val;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) s[r + e][k] = val[e];
    }
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    __shared__ __align__(16) uint16_t sA[32][kGemmPad];
    __shared__ __align__(16) uint16_t sB[32][kGemmPad];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bi = blockIdx.x * 32, bj = blockIdx.y * 32;
    const int ti = (wave >> 1) * 16, tj = (wave & 1) * 16;
    const int kq = (lane >> 4) * 8;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        __syncthreads();  // the previous step's operand reads are done
        if (threadIdx.x < 128)
            stage_slice(g.A, g.sa_i, g.sa_k, bi, k0, g.M, g.K, sA);
        else
            stage_slice(g.B, g.sb_j, g.sb_k, bj, k0, g.N, g.K, sB);
        __syncthreads();
        const u16x8 a = *reinterpret_cast<const u16x8*>(&sA[ti + (lane & 15)][kq]);
        const u16x8 b = *reinterpret_cast<const u16x8*>(&sB[tj + (lane & 15)][kq]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      acc, 0, 0, 0);
    }
    const int i0 = bi + ti, j = bj + tj + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + (lane >> 4) * 4 + r;
        if (i >= g.M || j >= g.N) continue;
        float x = acc[r];
        if (g.bias) x += g.bias[j];
        if (g.relu) x = x > 0.f ? x : 0.f;
        if (g.mask) x = g.mask[(int64_t)i * g.ldm + j] > 0.f ? x : 0.f;
        if (g.C32) g.C32[(int64_t)i * g.ldc + j] = x;
        if (g.C16) g.C16[(int64_t)i * g.ldc16 + j] = f2bf(x);
    }
}

static int gemm(const GemmArgs& a, hipStream_t st)
{
    if (a.M <= 0 || a.N <= 0) return 0;
    dim3 grid((a.M + 31) / 32, (a.N + 31) / 32);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// loss and its gradient, one thread per row
// ---------------------------------------------------------------------------
__global__ void k_loss(const float* Y, const float* T, int B, float lambda, float* dY, uint16_t* dYb, float* loss)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    const float* y = Y + (size_t)r * NO;
    const float* t = T + (size_t)r * NO;
    float* g = dY + (size_t)r * NO;
    uint16_t* gb = dYb + (size_t)r * NO;
    float mx = -INFINITY;
    for (int j = 0; j < NSLOT; ++j) mx = fmaxf(mx, y[j * SLOT]);
    float se = 0.f, wsum = 0.f;
    for (int j = 0; j < NSLOT; ++j) {
        se += expf(y[j * SLOT] - mx);
        wsum += t[j * SLOT];
    }
    const float lse = mx + logf(se);
    const float invB = 1.0f / (float)B;
    float l = 0.f;
    for (int j = 0; j < NSLOT; ++j) {
        const float wt = t[j * SLOT];
        const float pj = expf(y[j * SLOT] - lse);
        l += -wt * (y[j * SLOT] - lse);
        const float gl = (pj * wsum - wt) * invB;
        g[j * SLOT] = gl;
        gb[j * SLOT] = f2bf(gl);
        for (int q = 1; q < SLOT; ++q) {
            const float d = y[j * SLOT + q] - t[j * SLOT + q];
            l += lambda * wt * d * d;
            const float gq = 2.f * lambda * wt * d * invB;
            g[j * SLOT + q] = gq;
            gb[j * SLOT + q] = f2bf(gq);
        }
    }
    if (loss) loss[r] = l;
}

// column sums: a 32 x 32 block per 32 columns; thread (ty, tx) adds rows
// ty, ty + 32, ... of column tx, then row 0 adds the 32 partials in order
constexpr int kColTile = 32;
__global__ __launch_bounds__(kColTile * kColTile) void k_colsum(const float* X, int rows, int cols, int64_t ld,
                                                                 float* out)
{
    __shared__ float part[kColTile][kColTile + 1];
    const int tx = threadIdx.x % kColTile, ty = threadIdx.x / kColTile;
    const int j = blockIdx.x * kColTile + tx;
    float s = 0.f;
    if (j < cols)
        for (int r = ty; r < rows; r += kColTile) s += X[(size_t)r * ld + j];
    part[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && j < cols) {
        float t = part[0][tx];
        for (int q = 1; q < kColTile; ++q) t += part[q][tx];
        out[j] = t;
    }
}

__global__ void k_adam(float* w, float* m, float* v, const float* g, uint16_t* wb, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float* w, uint16_t* wb, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}

// batch rows; an index outside [0, n_rows) gives a zero row (zero features
// and zero target weights, so it adds nothing to the loss or the gradient)
__global__ void k_gather(const uint16_t* feats, const float* T, const int32_t* idx, int64_t n_rows, uint16_t* Xb,
                         float* Tb)
{
    const int r = blockIdx.x;
    const int64_t src = idx[r];
    const bool ok = src >= 0 && src < n_rows;
    for (int t = threadIdx.x; t < NFP; t += blockDim.x) Xb[(size_t)r * NFP + t] = ok ? feats[src * NFP + t] : 0;
    for (int t = threadIdx.x; t < NO; t += blockDim.x) Tb[(size_t)r * NO + t] = ok ? T[src * NO + t] : 0.f;
}

// Glorot-uniform weights from Philox (key (seed, "WARM"), counter (index, tensor, 0, 0)), zero biases
__global__ void k_init_params(float* w, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)NPARAM) return;
    int tensor = 0, fin = 0, fout = 0;
    int64_t local = 0;
    bool bias = false, pad = false;
    if (i < (int64_t)OFF_B1) {
        tensor = 1, fin = NF, fout = NH, local = i;
        pad = (local / NH) >= NF;
    } else if (i < (int64_t)OFF_W2) {
        bias = true;
    } else if (i < (int64_t)OFF_B2) {
        tensor = 2, fin = NH, fout = NH, local = i - OFF_W2;
    } else if (i < (int64_t)OFF_W3) {
        bias = true;
    } else if (i < (int64_t)OFF_B3) {
        tensor = 3, fin = NH, fout = NO, local = i - OFF_W3;
    } else {
        bias = true;
    }
    if (bias || pad) {
        w[i] = 0.f;
        return;
    }
    const u64x4 r = philox4x64_10((uint64_t)local, (uint64_t)tensor, 0, 0, seed, 0x5741524Dull);
    const double u = unit53(r.x) * 2.0 - 1.0;
    w[i] = (float)(u * sqrt(6.0 / (fin + fout)));
}

// ---------------------------------------------------------------------------
// decode: network outputs -> initial mixtures, one thread per cell
// ---------------------------------------------------------------------------
// decode of one cell's network outputs y [NO] with its frame fr [9] (mean,
// then the packed lower Cholesky factor of the cell covariance) into kmax
// gm_init slots: softmax weights, slots whose expected count N p_j is not
// above T/2 dropped (the most probable one kept if none is), the remaining
// weights renormalised; means m + L_C mu_hat, covariances L_C L_hat L_hat^T
// L_C^T with L_hat's diagonal exponentiated
__device__ void decode_row(const float* y, const double* fr, double N, int kmax, int32_t& Kc, double* w, double* mu,
                           double* S)
{
    const double halfT = 4.5;
    for (int q = 0; q < kmax; ++q) {
        w[q] = 0.0;
        for (int d = 0; d < 3; ++d) mu[q * 3 + d] = 0.0;
        for (int d = 0; d < 6; ++d) S[q * 6 + d] = 0.0;
    }
    if (!(fr[3] > 0.0)) {
        Kc = 0;  // no frame (singular or empty cell): cold start
        return;
    }
    double mx = -INFINITY;
    for (int j = 0; j < NSLOT; ++j) mx = fmax(mx, (double)y[j * SLOT]);
    double p[NSLOT], se = 0.0;
    for (int j = 0; j < NSLOT; ++j) {
        p[j] = exp((double)y[j * SLOT] - mx);
        se += p[j];
    }
    int best = 0;
    for (int j = 0; j < NSLOT; ++j) {
        p[j] /= se;
        if (p[j] > p[best]) best = j;
    }
    int keep[NSLOT], nk = 0;
    for (int j = 0; j < NSLOT && nk < kmax; ++j)
        if (N * p[j] > halfT) keep[nk++] = j;
    if (nk == 0) keep[nk++] = best;
    double ws = 0.0;
    for (int q = 0; q < nk; ++q) ws += p[keep[q]];
    const double LC[3][3] = {{fr[3], 0, 0}, {fr[4], fr[5], 0}, {fr[6], fr[7], fr[8]}};
    Kc = nk;
    for (int q = 0; q < nk; ++q) {
        const float* o = y + keep[q] * SLOT;
        w[q] = p[keep[q]] / ws;
        for (int d = 0; d < 3; ++d) {
            double t = fr[d];
            for (int e = 0; e <= d; ++e) t += LC[d][e] * (double)o[1 + e];
            mu[q * 3 + d] = t;
        }
        const double Lh[3][3] = {{exp((double)o[4]), 0, 0}, {(double)o[5], exp((double)o[6]), 0},
                                 {(double)o[7], (double)o[8], exp((double)o[9])}};
        double L[3][3];
        for (int i = 0; i < 3; ++i)
            for (int jj = 0; jj < 3; ++jj) {
                double t = 0.0;
                for (int e = 0; e < 3; ++e) t += LC[i][e] * Lh[e][jj];
                L[i][jj] = t;
            }
        int t = 0;
        for (int i = 0; i < 3; ++i)
            for (int jj = i; jj < 3; ++jj, ++t) {
                double a = 0.0;
                for (int e = 0; e < 3; ++e) a += L[i][e] * L[jj][e];
                S[q * 6 + t] = a;
            }
    }
}

__global__ void k_decode3(const float* Y, const double* frame, const int64_t* off, int64_t n_cells, int kmax,
                          int32_t* K, double* w, double* mu, double* S)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const size_t s0 = (size_t)c * kmax;
    decode_row(Y + (size_t)c * NO, frame + (size_t)c * 9, (double)(off[c + 1] - off[c]), kmax, K[c], w + s0,
               mu + s0 * 3, S + s0 * 6);
}

// ---------------------------------------------------------------------------
// Fused inference: the three layers and the decode for a tile of kInferRows
// cells per 256-thread workgroup.  Activations stay in LDS (BF16 between
// layers, FP32 network outputs); each layer's weights pass through LDS in
// blocks of 32 input rows, stored transposed so every MFMA operand is one
// 16-byte read.  Each 16x16 output tile accumulates over the inputs in the
// order of k_gemm with the same MFMA, then the same bias, ReLU and BF16
// rounding, so the outputs equal the separate launches' bit for bit.
// ---------------------------------------------------------------------------
constexpr int kInferRows = 32;
constexpr int kInferThreads = 256;

__global__ __launch_bounds__(kInferThreads) void k_mlp_infer(const uint16_t* X, int rows, const uint16_t* wb,
                                                              const float* w, const double* frame, const int64_t* off,
                                                              int kmax, int32_t* K, double* om, double* mu, double* S)
{
    __shared__ __align__(16) uint16_t s_a[kInferRows * NH];         // X (NFP wide), later H2 (NH wide)
    __shared__ __align__(16) unsigned char s_hy[kInferRows * NO * 4]; // H1 (BF16), later the FP32 outputs
    __shared__ __align__(16) uint16_t s_wt[NH * 32];                // one weight block, transposed [col][32]
    uint16_t* s_h1 = reinterpret_cast<uint16_t*>(s_hy);
    float* s_y = reinterpret_cast<float*>(s_hy);
    static_assert(kInferRows * NO * 4 >= kInferRows * NH * 2, "H1 must fit the output buffer");
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r0 = blockIdx.x * kInferRows;
    for (int t = tid; t < kInferRows * NFP / 8; t += kInferThreads) {
        const int r = t / (NFP / 8), q = t % (NFP / 8);
        u16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
        if (r0 + r < rows) val = reinterpret_cast<const u16x8*>(X + (size_t)(r0 + r) * NFP)[q];
        reinterpret_cast<u16x8*>(s_a + r * NFP)[q] = val;
    }
    // OUT[32 x N] = IN[32 x KD] W[KD x N] + bias (ReLU): a wave owns output
    // tiles t = wave, wave + 4, ... (two row tiles by N / 16 column tiles),
    // at most NH / 16 * 2 / 4 = 8 per wave
    auto layer = [&](const uint16_t* in, int KD, const uint16_t* W, int N, const float* bias, bool relu,
                     uint16_t* out16, float* out32) {
        const int ntile = 2 * (N / 16);
        f32x4 acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int kq = (lane >> 4) * 8;
        for (int k0 = 0; k0 < KD; k0 += 32) {
            __syncthreads();  // the previous block's reads (and the input writes) are done
            for (int t = tid; t < 32 * N; t += kInferThreads) {
                const int kk = t / N, j = t % N;
                s_wt[j * 32 + kk] = W[(size_t)(k0 + kk) * N + j];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = wave + 4 * u;
                if (t >= ntile) break;
                const int i0 = (t & 1) * 16, j0 = (t >> 1) * 16;
                const u16x8 a = *reinterpret_cast<const u16x8*>(in + (i0 + (lane & 15)) * KD + k0 + kq);
                const u16x8 b = *reinterpret_cast<const u16x8*>(s_wt + (j0 + (lane & 15)) * 32 + kq);
                acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                                 __builtin_bit_cast(bf16x8, b), acc[u], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read `in` before it is overwritten
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = wave + 4 * u;
            if (t >= ntile) break;
            const int i0 = (t & 1) * 16, j = (t >> 1) * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + (lane >> 4) * 4 + r;
                float x = acc[u][r] + bias[j];
                if (relu) x = x > 0.f ? x : 0.f;
                if (out16) out16[i * N + j] = f2bf(x);
                if (out32) out32[i * N + j] = x;
            }
        }
    };
    layer(s_a, NFP, wb + OFF_W1, NH, w + OFF_B1, true, s_h1, nullptr);
    layer(s_h1, NH, wb + OFF_W2, NH, w + OFF_B2, true, s_a, nullptr);
    layer(s_a, NH, wb + OFF_W3, NO, w + OFF_B3, false, nullptr, s_y);
    __syncthreads();
    if (tid < kInferRows && r0 + tid < rows) {
        const int64_t c = r0 + tid;
        const size_t s0 = (size_t)c * kmax;
        decode_row(s_y + tid * NO, frame + (size_t)c * 9, (double)(off[c + 1] - off[c]), kmax, K[c], om + s0,
                   mu + s0 * 3, S + s0 * 6);
    }
}

// ---------------------------------------------------------------------------
// training targets from compress outputs, one thread per cell
// ---------------------------------------------------------------------------
__device__ inline void lsolve3(const double L[3][3], const double* b, double* y)
{
    y[0] = b[0] / L[0][0];
    y[1] = (b[1] - L[1][0] * y[0]) / L[1][1];
    y[2] = (b[2] - L[2][0] * y[0] - L[2][1] * y[1]) / L[2][2];
}

__global__ void k_targets3(const int32_t* Kin, const double* w, const double* mu, const double* S, int kmax,
                           const double* frame, int64_t n_cells, float* T)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    float* t = T + (size_t)c * NO;
    for (int q = 0; q < NO; ++q) t[q] = 0.f;
    const double* fr = frame + (size_t)c * 9;
    if (!(fr[3] > 0.0)) return;
    const double LC[3][3] = {{fr[3], 0, 0}, {fr[4], fr[5], 0}, {fr[6], fr[7], fr[8]}};
    const int k = min(Kin[c], min(kmax, NSLOT));
    double rec[NSLOT][SLOT];
    int order[NSLOT];
    for (int q = 0; q < k; ++q) {
        const size_t s = (size_t)c * kmax + q;
        rec[q][0] = w[s];
        double b[3], mh[3];
        for (int d = 0; d < 3; ++d) b[d] = mu[s * 3 + d] - fr[d];
        lsolve3(LC, b, mh);
        for (int d = 0; d < 3; ++d) rec[q][1 + d] = mh[d];
        double Sg[3][3];
        int tt = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j, ++tt) Sg[i][j] = Sg[j][i] = S[s * 6 + tt];
        double Z[3][3], Sh[3][3];
        for (int j = 0; j < 3; ++j) {
            const double col[3] = {Sg[0][j], Sg[1][j], Sg[2][j]};
            double y[3];
            lsolve3(LC, col, y);
            for (int i = 0; i < 3; ++i) Z[i][j] = y[i];
        }
        for (int i = 0; i < 3; ++i) {
            const double row[3] = {Z[i][0], Z[i][1], Z[i][2]};
            double y[3];
            lsolve3(LC, row, y);
            for (int j = 0; j < 3; ++j) Sh[i][j] = y[j];
        }
        double sp[6] = {Sh[0][0], 0.5 * (Sh[0][1] + Sh[1][0]), 0.5 * (Sh[0][2] + Sh[2][0]), Sh[1][1],
                        0.5 * (Sh[1][2] + Sh[2][1]), Sh[2][2]};
        double Lp[6];
        double l00 = 1e-3, l10 = 0, l11 = 1e-3, l20 = 0, l21 = 0, l22 = 1e-3;
        if (chol<3, double>(sp, Lp)) {
            l00 = Lp[0], l10 = Lp[1], l20 = Lp[2], l11 = Lp[3], l21 = Lp[4], l22 = Lp[5];
        }
        rec[q][4] = log(l00);
        rec[q][5] = l10;
        rec[q][6] = log(l11);
        rec[q][7] = l20;
        rec[q][8] = l21;
        rec[q][9] = log(l22);
        order[q] = q;
    }
    for (int a = 1; a < k; ++a) {
        const int x = order[a];
        int b = a - 1;
        while (b >= 0 && (rec[order[b]][0] < rec[x][0] || (rec[order[b]][0] == rec[x][0] && rec[order[b]][1] > rec[x][1]))) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = x;
    }
    for (int q = 0; q < k; ++q)
        for (int e = 0; e < SLOT; ++e) t[q * SLOT + e] = (float)rec[order[q]][e];
}

}  // namespace gm

// ===========================================================================
// C ABI
// ===========================================================================
struct gm_warm {
    int D, kmax, batch;
    int64_t step;
    float* w;        // FP32 master parameters (NPARAM)
    float* m;        // Adam first moment
    float* v;        // Adam second moment
    float* grad;     // gradients (NPARAM)
    uint16_t* wb;    // BF16 copy of the parameters (weights used by the products)
    // batch scratch
    uint16_t *Xb, *H1b, *H2b, *dYb, *dH2b, *dH1b;
    float *Tb, *H1, *H2, *Y, *dY, *dH2, *dH1, *loss;
    void* block;     // one allocation holding everything
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

bool ok(hipError_t e) { return e == hipSuccess; }

int launch_ok() { return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP; }

gm::GemmArgs ga(const uint16_t* A, int64_t sa_i, int64_t sa_k, const uint16_t* B, int64_t sb_k, int64_t sb_j, int M,
                int N, int K)
{
    gm::GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.A = A;
    g.sa_i = sa_i;
    g.sa_k = sa_k;
    g.B = B;
    g.sb_k = sb_k;
    g.sb_j = sb_j;
    g.M = M;
    g.N = N;
    g.K = K;
    return g;
}

// forward of rows [0, rows) of X (BF16, NFP wide) into H1b/H2b (BF16) and Y (FP32);
// FP32 hidden copies when given (training)
int forward(const gm_warm* mdl, const uint16_t* X, int rows, uint16_t* H1b, float* H1, uint16_t* H2b, float* H2,
            float* Y, hipStream_t st)
{
    using namespace gm;
    GemmArgs g = ga(X, NFP, 1, mdl->wb + OFF_W1, NH, 1, rows, NH, NFP);
    g.bias = mdl->w + OFF_B1;
    g.relu = 1;
    g.C32 = H1;
    g.ldc = NH;
    g.C16 = H1b;
    g.ldc16 = NH;
    if (gemm(g, st)) return GM_EHIP;
    g = ga(H1b, NH, 1, mdl->wb + OFF_W2, NH, 1, rows, NH, NH);
    g.bias = mdl->w + OFF_B2;
    g.relu = 1;
    g.C32 = H2;
    g.ldc = NH;
    g.C16 = H2b;
    g.ldc16 = NH;
    if (gemm(g, st)) return GM_EHIP;
    g = ga(H2b, NH, 1, mdl->wb + OFF_W3, NO, 1, rows, NO, NH);
    g.bias = mdl->w + OFF_B3;
    g.C32 = Y;
    g.ldc = NO;
    if (gemm(g, st)) return GM_EHIP;
    return GM_OK;
}

}  // namespace

extern "C" {

size_t gm_warm_param_count(void) { return gm::NPARAM; }

int gm_warm_create(gm_warm** out, int32_t D, int32_t kmax, int32_t batch, uint64_t seed, void* stream)
{
    using namespace gm;
    if (!out || D != 3 || kmax < 1 || kmax > 16 || batch < 1 || batch > (1 << 20)) return GM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    gm_warm* m = new gm_warm;
    memset(m, 0, sizeof(*m));
    m->D = D;
    m->kmax = kmax;
    m->batch = batch;
    const size_t B = (size_t)batch;
    size_t sz[20], tot = 0;
    int i = 0;
    sz[i++] = al256(NPARAM * 4);        // w
    sz[i++] = al256(NPARAM * 4);        // m
    sz[i++] = al256(NPARAM * 4);        // v
    sz[i++] = al256(NPARAM * 4);        // grad
    sz[i++] = al256(NPARAM * 2);        // wb
    sz[i++] = al256(B * NFP * 2);       // Xb
    sz[i++] = al256(B * NH * 2);        // H1b
    sz[i++] = al256(B * NH * 2);        // H2b
    sz[i++] = al256(B * NO * 2);        // dYb
    sz[i++] = al256(B * NH * 2);        // dH2b
    sz[i++] = al256(B * NH * 2);        // dH1b
    sz[i++] = al256(B * NO * 4);        // Tb
    sz[i++] = al256(B * NH * 4);        // H1
    sz[i++] = al256(B * NH * 4);        // H2
    sz[i++] = al256(B * NO * 4);        // Y
    sz[i++] = al256(B * NO * 4);        // dY
    sz[i++] = al256(B * NH * 4);        // dH2
    sz[i++] = al256(B * NH * 4);        // dH1
    sz[i++] = al256(B * 4);             // loss
    const int nb = i;
    for (int k = 0; k < nb; ++k) tot += sz[k];
    if (!ok(hipMalloc(&m->block, tot))) {
        delete m;
        return GM_ENOMEM;
    }
    char* p = (char*)m->block;
    void** ptrs[20] = {(void**)&m->w,   (void**)&m->m,   (void**)&m->v,   (void**)&m->grad, (void**)&m->wb,
                       (void**)&m->Xb,  (void**)&m->H1b, (void**)&m->H2b, (void**)&m->dYb,  (void**)&m->dH2b,
                       (void**)&m->dH1b, (void**)&m->Tb, (void**)&m->H1,  (void**)&m->H2,   (void**)&m->Y,
                       (void**)&m->dY,  (void**)&m->dH2, (void**)&m->dH1, (void**)&m->loss};
    for (int k = 0; k < nb; ++k) {
        *ptrs[k] = p;
        p += sz[k];
    }
    const int nblk = (int)((NPARAM + 255) / 256);
    hipLaunchKernelGGL(k_init_params, dim3(nblk), dim3(256), 0, st, m->w, seed);
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk), dim3(256), 0, st, m->w, m->wb, (int64_t)NPARAM);
    if (!ok(hipMemsetAsync(m->m, 0, NPARAM * 4, st)) || !ok(hipMemsetAsync(m->v, 0, NPARAM * 4, st)) ||
        launch_ok() != GM_OK) {
        (void)hipFree(m->block);
        delete m;
        return GM_EHIP;
    }
    *out = m;
    return GM_OK;
}

void gm_warm_destroy(gm_warm* m)
{
    if (!m) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(m->block);
    delete m;
}

int gm_warm_get_params(const gm_warm* m, float* host)
{
    if (!m || !host) return GM_EINVAL;
    if (!ok(hipDeviceSynchronize())) return GM_EHIP;
    return ok(hipMemcpy(host, m->w, gm::NPARAM * 4, hipMemcpyDeviceToHost)) ? GM_OK : GM_EHIP;
}

int gm_warm_set_params(gm_warm* m, const float* host)
{
    using namespace gm;
    if (!m || !host) return GM_EINVAL;
    if (!ok(hipDeviceSynchronize())) return GM_EHIP;
    if (!ok(hipMemcpy(m->w, host, NPARAM * 4, hipMemcpyHostToDevice))) return GM_EHIP;
    if (!ok(hipMemset(m->m, 0, NPARAM * 4)) || !ok(hipMemset(m->v, 0, NPARAM * 4))) return GM_EHIP;
    m->step = 0;
    const int nblk = (int)((NPARAM + 255) / 256);
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk), dim3(256), 0, 0, m->w, m->wb, (int64_t)NPARAM);
    if (launch_ok() != GM_OK) return GM_EHIP;
    return ok(hipDeviceSynchronize()) ? GM_OK : GM_EHIP;
}

// Model file: the 8 bytes "GMCRWRM1", int32 D, int32 kmax, uint64 parameter
// count, then the FP32 parameters in the get/set layout (host byte order).
static const char kWarmMagic[8] = {'G', 'M', 'C', 'R', 'W', 'R', 'M', '1'};

int gm_warm_save(const gm_warm* m, const char* path)
{
    if (!m || !path) return GM_EINVAL;
    std::vector<float> h(gm::NPARAM);
    const int rc = gm_warm_get_params(m, h.data());
    if (rc != GM_OK) return rc;
    FILE* f = fopen(path, "wb");
    if (!f) return GM_EIO;
    const int32_t dk[2] = {m->D, m->kmax};
    const uint64_t np = gm::NPARAM;
    bool good = fwrite(kWarmMagic, 1, 8, f) == 8 && fwrite(dk, 4, 2, f) == 2 && fwrite(&np, 8, 1, f) == 1 &&
                fwrite(h.data(), 4, h.size(), f) == h.size();
    good = (fclose(f) == 0) && good;
    return good ? GM_OK : GM_EIO;
}

int gm_warm_load(gm_warm** out, const char* path, int32_t batch, void* stream)
{
    if (!out || !path || batch < 1 || batch > (1 << 20)) return GM_EINVAL;
    FILE* f = fopen(path, "rb");
    if (!f) return GM_EIO;
    char magic[8];
    int32_t dk[2] = {0, 0};
    uint64_t np = 0;
    std::vector<float> h(gm::NPARAM);
    int rc = GM_OK;
    if (fread(magic, 1, 8, f) != 8 || fread(dk, 4, 2, f) != 2 || fread(&np, 8, 1, f) != 1)
        rc = GM_EIO;
    else if (memcmp(magic, kWarmMagic, 8) != 0 || dk[0] != 3 || dk[1] < 1 || dk[1] > 16 || np != gm::NPARAM)
        rc = GM_EINVAL;  // not a model file of this library, or of another layout
    else if (fread(h.data(), 4, h.size(), f) != h.size() || fgetc(f) != EOF)
        rc = GM_EIO;     // truncated, or trailing bytes
    fclose(f);
    if (rc != GM_OK) return rc;
    gm_warm* m = nullptr;
    rc = gm_warm_create(&m, dk[0], dk[1], batch, 0, stream);
    if (rc != GM_OK) return rc;
    rc = gm_warm_set_params(m, h.data());
    if (rc != GM_OK) {
        gm_warm_destroy(m);
        return rc;
    }
    *out = m;
    return GM_OK;
}

int gm_warm_features(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells, int32_t D,
                     uint16_t* feats, double* frame, void* stream)
{
    if (D != 3 || n_cells < 0 || n_cells > 0x7fffffff) return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!v || !alpha || !cell_off || !feats || !frame) return GM_EINVAL;
    hipLaunchKernelGGL(gm::k_features3, dim3((unsigned)n_cells), dim3(gm::kFeatThreads), 0, (hipStream_t)stream, v,
                       alpha, cell_off, feats, frame);
    return launch_ok();
}

int gm_warm_forward(const gm_warm* m, const uint16_t* feats, int64_t n_rows, float* Y, void* ws, size_t ws_bytes,
                    void* stream)
{
    using namespace gm;
    if (!m || n_rows < 0 || n_rows > 0x7fffffff) return GM_EINVAL;
    if (n_rows == 0) return GM_OK;
    if (!feats || !Y) return GM_EINVAL;
    const size_t need = al256((size_t)n_rows * NH * 2) * 2;
    if (!ws || ws_bytes < need) return GM_ENOMEM;
    uint16_t* H1b = (uint16_t*)ws;
    uint16_t* H2b = (uint16_t*)((char*)ws + al256((size_t)n_rows * NH * 2));
    return forward(m, feats, (int)n_rows, H1b, nullptr, H2b, nullptr, Y, (hipStream_t)stream);
}

int gm_warm_model_kmax(const gm_warm* m) { return m ? m->kmax : 0; }

size_t gm_warm_forward_workspace(int64_t n_rows)
{
    if (n_rows < 0) return 0;
    return al256((size_t)n_rows * gm::NH * 2) * 2;
}

int gm_warm_infer(const gm_warm* m, const uint16_t* feats, const double* frame, const int64_t* cell_off,
                  int64_t n_cells, int32_t kmax, int32_t* K, double* omega, double* mu, double* sigma, void* stream)
{
    if (!m || n_cells < 0 || n_cells > 0x7fffffff || kmax < 1 || kmax > 16) return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!feats || !frame || !cell_off || !K || !omega || !mu || !sigma) return GM_EINVAL;
    const unsigned nb = (unsigned)((n_cells + gm::kInferRows - 1) / gm::kInferRows);
    hipLaunchKernelGGL(gm::k_mlp_infer, dim3(nb), dim3(gm::kInferThreads), 0, (hipStream_t)stream, feats,
                       (int)n_cells, m->wb, m->w, frame, cell_off, kmax, K, omega, mu, sigma);
    return launch_ok();
}

int gm_warm_decode(const float* Y, const double* frame, const int64_t* cell_off, int64_t n_cells, int32_t kmax,
                   int32_t* K, double* omega, double* mu, double* sigma, void* stream)
{
    if (n_cells < 0 || kmax < 1 || kmax > 16) return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!Y || !frame || !cell_off || !K || !omega || !mu || !sigma) return GM_EINVAL;
    const unsigned nb = (unsigned)((n_cells + 127) / 128);
    hipLaunchKernelGGL(gm::k_decode3, dim3(nb), dim3(128), 0, (hipStream_t)stream, Y, frame, cell_off, n_cells, kmax,
                       K, omega, mu, sigma);
    return launch_ok();
}

int gm_warm_targets(const int32_t* K, const double* omega, const double* mu, const double* sigma, int32_t kmax,
                    const double* frame, int64_t n_cells, float* targets, void* stream)
{
    if (n_cells < 0 || kmax < 1 || kmax > 16) return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!K || !omega || !mu || !sigma || !frame || !targets) return GM_EINVAL;
    const unsigned nb = (unsigned)((n_cells + 127) / 128);
    hipLaunchKernelGGL(gm::k_targets3, dim3(nb), dim3(128), 0, (hipStream_t)stream, K, omega, mu, sigma, kmax, frame,
                       n_cells, targets);
    return launch_ok();
}

int gm_warm_train_step(gm_warm* m, const uint16_t* feats, const float* targets, int64_t n_rows, const int32_t* idx,
                       float lr, float lambda, float* loss_rows, void* stream)
{
    using namespace gm;
    if (!m || !feats || !targets || !idx || n_rows < 1 || !(lr > 0.f) || !(lambda >= 0.f)) return GM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int B = m->batch;
    hipLaunchKernelGGL(k_gather, dim3(B), dim3(128), 0, st, feats, targets, idx, n_rows, m->Xb, m->Tb);
    if (launch_ok() != GM_OK) return GM_EHIP;
    int rc = forward(m, m->Xb, B, m->H1b, m->H1, m->H2b, m->H2, m->Y, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_loss, dim3((B + 127) / 128), dim3(128), 0, st, m->Y, m->Tb, B, lambda, m->dY, m->dYb,
                       loss_rows ? loss_rows : m->loss);
    if (launch_ok() != GM_OK) return GM_EHIP;
    // layer 3: dW3 = H2^T dY, db3 = colsum dY, dH2 = (dY W3^T) * [H2 > 0]
    GemmArgs g = ga(m->H2b, 1, NH, m->dYb, NO, 1, NH, NO, B);
    g.C32 = m->grad + OFF_W3;
    g.ldc = NO;
    if (gemm(g, st)) return GM_EHIP;
    hipLaunchKernelGGL(k_colsum, dim3((NO + kColTile - 1) / kColTile), dim3(kColTile * kColTile), 0, st, m->dY, B, NO, (int64_t)NO, m->grad + OFF_B3);
    g = ga(m->dYb, NO, 1, m->wb + OFF_W3, 1, NO, B, NH, NO);
    g.mask = m->H2;
    g.ldm = NH;
    g.C32 = m->dH2;
    g.ldc = NH;
    g.C16 = m->dH2b;
    g.ldc16 = NH;
    if (gemm(g, st)) return GM_EHIP;
    // layer 2
    g = ga(m->H1b, 1, NH, m->dH2b, NH, 1, NH, NH, B);
    g.C32 = m->grad + OFF_W2;
    g.ldc = NH;
    if (gemm(g, st)) return GM_EHIP;
    hipLaunchKernelGGL(k_colsum, dim3((NH + kColTile - 1) / kColTile), dim3(kColTile * kColTile), 0, st, m->dH2, B, NH, (int64_t)NH, m->grad + OFF_B2);
    g = ga(m->dH2b, NH, 1, m->wb + OFF_W2, 1, NH, B, NH, NH);
    g.mask = m->H1;
    g.ldm = NH;
    g.C32 = m->dH1;
    g.ldc = NH;
    g.C16 = m->dH1b;
    g.ldc16 = NH;
    if (gemm(g, st)) return GM_EHIP;
    // layer 1 (rows of W1 beyond the 105 features get zero gradient: X is zero there)
    g = ga(m->Xb, 1, NFP, m->dH1b, NH, 1, NFP, NH, B);
    g.C32 = m->grad + OFF_W1;
    g.ldc = NH;
    if (gemm(g, st)) return GM_EHIP;
    hipLaunchKernelGGL(k_colsum, dim3((NH + kColTile - 1) / kColTile), dim3(kColTile * kColTile), 0, st, m->dH1, B, NH, (int64_t)NH, m->grad + OFF_B1);
    if (launch_ok() != GM_OK) return GM_EHIP;
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - powf(b1, (float)m->step), bc2 = 1.f - powf(b2, (float)m->step);
    const int nblk = (int)((NPARAM + 255) / 256);
    hipLaunchKernelGGL(k_adam, dim3(nblk), dim3(256), 0, st, m->w, m->m, m->v, m->grad, m->wb, (int64_t)NPARAM, lr, b1,
                       b2, 1e-8f, bc1, bc2);
    return launch_ok();
}

int gm_warm_gradients(const gm_warm* m, float* host)
{
    if (!m || !host) return GM_EINVAL;
    if (!ok(hipDeviceSynchronize())) return GM_EHIP;
    return ok(hipMemcpy(host, m->grad, gm::NPARAM * 4, hipMemcpyDeviceToHost)) ? GM_OK : GM_EHIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Training loop: epochs of shuffled mini-batches.  The permutation of an
// epoch is a Fisher-Yates shuffle (from the top index down, j uniform in
// [0, i] as the high 64 bits of draw * (i + 1)) driven by splitmix64
// (Steele, Lea and Flood 2014) started at seed ^ (0xD1B54A32D192ED03 *
// (epoch + 1)).
// ---------------------------------------------------------------------------
namespace {

uint64_t splitmix64_next(uint64_t& x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void epoch_permutation(int32_t* perm, int64_t n, uint64_t seed, int32_t epoch)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    uint64_t x = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(epoch + 1));
    for (int64_t i = n - 1; i >= 1; --i) {
        const uint64_t r = splitmix64_next(x);
        const int64_t j = (int64_t)(((unsigned __int128)r * (uint64_t)(i + 1)) >> 64);
        const int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
}

size_t al256h(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

size_t gm_warm_train_workspace(int64_t n_rows, int32_t batch)
{
    if (n_rows < 1 || n_rows > 0x7fffffff || batch < 1 || n_rows < batch) return 0;
    const int64_t steps = n_rows / batch;
    return al256h((size_t)n_rows * 4) + al256h((size_t)(steps * batch) * 4);
}

int gm_warm_train(gm_warm* m, const uint16_t* feats, const float* targets, int64_t n_rows, int32_t epochs,
                  float lr, float lambda, uint64_t seed, void* ws, size_t ws_bytes, float* epoch_loss, void* stream)
{
    if (!m || !feats || !targets || epochs < 1 || !(lr > 0.f) || !(lambda >= 0.f)) return GM_EINVAL;
    const size_t need = gm_warm_train_workspace(n_rows, m->batch);
    if (need == 0) return GM_EINVAL;  // fewer rows than one batch, or too many rows
    if (!ws || ws_bytes < need) return GM_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    const int B = m->batch;
    const int64_t steps = n_rows / B;
    int32_t* dperm = (int32_t*)ws;
    float* dloss = (float*)((char*)ws + al256h((size_t)n_rows * 4));
    std::vector<int32_t> perm((size_t)n_rows);
    std::vector<float> hl((size_t)(steps * B));
    for (int32_t e = 0; e < epochs; ++e) {
        epoch_permutation(perm.data(), n_rows, seed, e);
        if (hipMemcpyAsync(dperm, perm.data(), (size_t)n_rows * 4, hipMemcpyHostToDevice, st) != hipSuccess)
            return GM_EHIP;
        for (int64_t s = 0; s < steps; ++s) {
            const int rc = gm_warm_train_step(m, feats, targets, n_rows, dperm + s * B, lr, lambda, dloss + s * B,
                                              stream);
            if (rc != GM_OK) return rc;
        }
        // the host permutation is rewritten next epoch: wait for this one
        if (epoch_loss) {
            if (hipMemcpyAsync(hl.data(), dloss, hl.size() * 4, hipMemcpyDeviceToHost, st) != hipSuccess)
                return GM_EHIP;
        }
        if (hipStreamSynchronize(st) != hipSuccess) return GM_EHIP;
        if (epoch_loss) {
            double t = 0.0;
            for (float x : hl) t += x;
            epoch_loss[e] = (float)(t / (double)hl.size());
        }
    }
    return GM_OK;
}

}  // extern "C"
