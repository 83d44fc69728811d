// gm_gauss.hip -- Gauss'-law weight correction after resampling (Sec. 2.4.1).
//
// Mesh: periodic, nx cells (dx = 1) or nx * ny cells (dx = 2, cell c at
// (c % nx, c / nx)), unit cells; cell i has centre X_i = i + 1/2 and a
// particle of cell c with cell-local position x sits at X = (cell) + x.
//
//   k_stencil   one wave per cell: the quadratic B-spline weights
//               S2(X_i - X_p) of its particles on the 3 (1D) or 9 (2D) mesh
//               cells around it, summed plain (the cell's column of the mass
//               matrix M_ij = sum_{p in j} S2(X_i - X_p), eq.
//               p-weight-correction with the top-hat S0) and weighted by w_p
//               (the cell's share of the deposit D_i = sum_p w_p S2(X_i -
//               X_p)); FP64, fixed-order sums
//   k_deposit   D_i or (M a)_i from the neighbouring cells' columns in a
//               fixed order (a gather: no atomics, deterministic)
//   solver      M dA = D_target - D(w) by BiCGSTAB with the Jacobi
//               preconditioner diag(M) applied on the right.  Every scalar
//               of the iteration stays in device memory: one-thread
//               epilogues fold the fixed-order block partials of the dot
//               products into rho, alpha, omega and a done flag, and every
//               vector kernel returns at once when the flag is set, so the
//               host enqueues iterations in chunks and reads the state once
//               per chunk.  A restart recomputes the true residual b - M dA,
//               which alone decides convergence (below tol |b|).
//   k_apply_dA  w_p += dA_{cell(p)} (eq. new-p-weight)
#include <cmath>

#include "gm_device.h"

namespace gm {

constexpr int kStencilThreads = 256;
constexpr int kVecThreads = 256;

__device__ __forceinline__ double bspline2(double s)
{
    const double a = fabs(s);
    if (a <= 0.5) return 0.75 - a * a;
    if (a <= 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

// slot o of a cell's stencil: 1D o = ox + 1 (ox = -1, 0, 1); 2D o = 3 (oy +
// 1) + (ox + 1); the cell's own slot is 1 (1D) or 4 (2D)
template <int DX>
constexpr int kSlots = DX == 1 ? 3 : 9;
template <int DX>
constexpr int kCentre = DX == 1 ? 1 : 4;

// one wave per cell (kStencilThreads / 64 cells per workgroup): lanes stride
// over the cell's particles, then a wave-wide DPP sum per slot (fixed order)
template <int DX>
__global__ __launch_bounds__(kStencilThreads) void k_stencil(const double* x, const double* w, const int64_t* off,
                                                             int64_t n_cells, double* colM, double* colW)
{
    constexpr int NS = kSlots<DX>;
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * (kStencilThreads / 64) + (threadIdx.x >> 6);
    if (c >= n_cells) return;  // whole waves leave; no workgroup barrier follows
    const int64_t o0 = off[c], n = off[c + 1] - o0;
    double acc[2 * NS];
#pragma unroll
    for (int t = 0; t < 2 * NS; ++t) acc[t] = 0.0;
    for (int64_t i = lane; i < n; i += 64) {
        const double wp = w[o0 + i];
        double sx[3], sy[3] = {1.0, 0.0, 0.0};
        const double px = x[(o0 + i) * DX];
#pragma unroll
        for (int o = 0; o < 3; ++o) sx[o] = bspline2((o - 1) + 0.5 - px);
        if constexpr (DX == 2) {
            const double py = x[(o0 + i) * DX + 1];
#pragma unroll
            for (int o = 0; o < 3; ++o) sy[o] = bspline2((o - 1) + 0.5 - py);
        }
#pragma unroll
        for (int oy = 0; oy < (DX == 2 ? 3 : 1); ++oy)
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const double s = DX == 2 ? sx[ox] * sy[oy] : sx[ox];
                acc[oy * 3 + ox] += s;
                acc[NS + oy * 3 + ox] += wp * s;
            }
    }
#pragma unroll
    for (int t = 0; t < 2 * NS; ++t) acc[t] = wave_sum(acc[t]);
    // every lane holds the totals; lane t stores slot t (static indices keep
    // acc in registers)
#pragma unroll
    for (int t = 0; t < NS; ++t)
        if (lane == t) {
            if (colM) colM[c * NS + t] = acc[t];
            colW[c * NS + t] = acc[NS + t];
        }
}

// sum over the stencil slots o of col[j(i, o)][o] * f(j), j = the cell whose
// slot o lands on mesh cell i
template <int DX, typename F>
__device__ __forceinline__ double gather(const double* col, int64_t i, int64_t n_cells, int nx, int ny, F f)
{
    constexpr int NS = kSlots<DX>;
    double t = 0.0;
    if constexpr (DX == 1) {
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            int64_t j = i - (o - 1);
            j = j < 0 ? j + n_cells : (j >= n_cells ? j - n_cells : j);
            t += col[j * NS + o] * f(j);
        }
    } else {
        const int ix = (int)(i % nx), iy = (int)(i / nx);
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            int jy = iy - (oy - 1);
            jy = jy < 0 ? jy + ny : (jy >= ny ? jy - ny : jy);
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                int jx = ix - (ox - 1);
                jx = jx < 0 ? jx + nx : (jx >= nx ? jx - nx : jx);
                const int64_t j = (int64_t)jy * nx + jx;
                t += col[j * NS + oy * 3 + ox] * f(j);
            }
        }
    }
    return t;
}

// the deposit D_i from the weighted columns
template <int DX>
__global__ __launch_bounds__(kVecThreads) void k_deposit(const double* colW, int64_t n_cells, int nx, int ny,
                                                        double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_cells) return;
    out[i] = gather<DX>(colW, i, n_cells, nx, ny, [](int64_t) { return 1.0; });
}

// ---------------------------------------------------------------------------
// solver state (device): the scalars of the iteration and its flags
// ---------------------------------------------------------------------------
enum : int { S_RHO, S_ALPHA, S_OMEGA, S_BETA, S_TOL2B2, S_R2, S_DONE, S_ITERS, S_EMPTY, S_COUNT };
// S_DONE: 0 running, 1 converged, 2 stopped (a breakdown or a vanishing
// omega; the host restarts from the true residual)

// Block partials of two dot products: every thread adds its own terms, the
// workgroup reduces them in a fixed order, thread 0 stores them.
__device__ __forceinline__ void store_partials(double a0, double a1, double* partial)
{
    __shared__ double red[2 * kMaxWaves * 2];
    int par = 0;
    double acc[2] = {a0, a1};
    block_sum<2>(acc, red, par, blockDim.x >> 6);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = acc[0];
        partial[2 * blockIdx.x + 1] = acc[1];
    }
}

__device__ __forceinline__ bool halted(const double* st) { return st[S_DONE] != 0.0; }

enum : int { E_INIT, E_RESTART, E_ALPHA, E_OMEGA, E_RES_RHO };

// Folds the block partials (fixed order) and updates the state:
//   E_INIT     s0 = b.b, s1 = number of empty cells
//   E_RESTART  s0 = r.r of the true residual (rh = r, p = v = 0): converged
//              when s0 <= tol^2 b.b, else a fresh start with rho = rh.r = s0
//   E_ALPHA    s0 = rh.v: alpha = rho / s0
//   E_OMEGA    s0 = t.s, s1 = t.t: omega = s0 / s1
//   E_RES_RHO  s0 = r.r, s1 = rh.r of the new residual: one more iteration;
//              done, or beta = (s1 / rho) (alpha / omega) and rho = s1
__global__ __launch_bounds__(kVecThreads) void k_fold(const double* partial, int nblocks, double* st, int mode,
                                                      double tol)
{
    __shared__ double red[2 * kMaxWaves * 2];
    int par = 0;
    double acc[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        acc[0] += partial[2 * b];
        acc[1] += partial[2 * b + 1];
    }
    block_sum<2>(acc, red, par, blockDim.x >> 6);
    if (threadIdx.x != 0) return;
    const double s0 = acc[0], s1 = acc[1];
    switch (mode) {
        case E_INIT:
            st[S_TOL2B2] = tol * tol * s0;
            st[S_EMPTY] = s1;
            st[S_R2] = s0;
            st[S_ITERS] = 0.0;
            st[S_DONE] = s0 == 0.0 ? 1.0 : 0.0;
            break;
        case E_RESTART:
            st[S_R2] = s0;
            st[S_ALPHA] = 1.0;
            st[S_OMEGA] = 1.0;
            st[S_RHO] = s0;
            st[S_BETA] = 0.0;
            st[S_DONE] = s0 <= st[S_TOL2B2] ? 1.0 : (isfinite(s0) ? 0.0 : 2.0);
            break;
        case E_ALPHA:
            if (st[S_DONE] != 0.0) break;
            if (s0 == 0.0 || !isfinite(s0))
                st[S_DONE] = 2.0;
            else
                st[S_ALPHA] = st[S_RHO] / s0;
            break;
        case E_OMEGA:
            if (st[S_DONE] != 0.0) break;
            st[S_OMEGA] = s1 > 0.0 ? s0 / s1 : 0.0;
            break;
        case E_RES_RHO:
            if (st[S_DONE] != 0.0) break;
            st[S_ITERS] += 1.0;
            st[S_R2] = s0;
            if (s0 <= st[S_TOL2B2]) {
                st[S_DONE] = 1.0;
            } else if (st[S_OMEGA] == 0.0 || s1 == 0.0 || !isfinite(s0) || !isfinite(s1)) {
                st[S_DONE] = 2.0;
            } else {
                st[S_BETA] = (s1 / st[S_RHO]) * (st[S_ALPHA] / st[S_OMEGA]);
                st[S_RHO] = s1;
            }
            break;
    }
}

// dinv_j = 1 / M_jj (a cell with particles has M_jj >= n_j / 4 > 0), b =
// target - D(w), dA = 0; partials of (b.b, number of empty cells)
template <int DX>
__global__ __launch_bounds__(kVecThreads) void k_setup(const double* colM, const double* colW,
                                                       const double* target, const int64_t* off, int64_t n_cells,
                                                       int nx, int ny, double* dinv, double* b, double* x,
                                                       double* partial)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double bb = 0.0, e = 0.0;
    if (i < n_cells) {
        const bool empty = off[i + 1] <= off[i];
        dinv[i] = empty ? 0.0 : 1.0 / colM[i * kSlots<DX> + kCentre<DX>];
        const double bi = target[i] - gather<DX>(colW, i, n_cells, nx, ny, [](int64_t) { return 1.0; });
        b[i] = bi;
        x[i] = 0.0;
        bb = bi * bi;
        e = empty ? 1.0 : 0.0;
    }
    store_partials(bb, e, partial);
}

// restart: r = rh = b - M dA, p = v = 0; partials of (r.r, r.r)
template <int DX>
__global__ __launch_bounds__(kVecThreads) void k_restart(const double* colM, const double* b, const double* x,
                                                         int64_t n_cells, int nx, int ny, double* r, double* rh,
                                                         double* p, double* v, double* partial)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (i < n_cells) {
        const double ri = b[i] - gather<DX>(colM, i, n_cells, nx, ny, [&](int64_t j) { return x[j]; });
        r[i] = ri;
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
        rr = ri * ri;
    }
    store_partials(rr, rr, partial);
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kVecThreads) void k_update_p(const double* st, const double* r, const double* v,
                                                          double* p, int64_t n)
{
    if (halted(st)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = r[i] + st[S_BETA] * (p[i] - st[S_OMEGA] * v[i]);
}

// y = M diag(dinv) a; partials of (rh.y, 0), or (y.a, y.y) when TS
template <int DX, bool TS>
__global__ __launch_bounds__(kVecThreads) void k_spmv(const double* st, const double* colM, const double* dinv,
                                                      const double* a, const double* rh, int64_t n_cells, int nx,
                                                      int ny, double* y, double* partial)
{
    if (halted(st)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double q0 = 0.0, q1 = 0.0;
    if (i < n_cells) {
        const double yi = gather<DX>(colM, i, n_cells, nx, ny, [&](int64_t j) { return dinv[j] * a[j]; });
        y[i] = yi;
        if constexpr (TS) {
            q0 = yi * a[i];
            q1 = yi * yi;
        } else {
            q0 = rh[i] * yi;
        }
    }
    store_partials(q0, q1, partial);
}

// s = r - alpha v
__global__ __launch_bounds__(kVecThreads) void k_update_s(const double* st, const double* r, const double* v,
                                                          double* s, int64_t n)
{
    if (halted(st)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = r[i] - st[S_ALPHA] * v[i];
}

// dA += dinv (alpha p + omega s), r = s - omega t; partials of (r.r, rh.r)
__global__ __launch_bounds__(kVecThreads) void k_update_xr(const double* st, const double* dinv, const double* p,
                                                           const double* s, const double* t, const double* rh,
                                                           double* x, double* r, int64_t n, double* partial)
{
    if (halted(st)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double q0 = 0.0, q1 = 0.0;
    if (i < n) {
        const double al = st[S_ALPHA], om = st[S_OMEGA];
        x[i] += dinv[i] * (al * p[i] + om * s[i]);
        const double ri = s[i] - om * t[i];
        r[i] = ri;
        q0 = ri * ri;
        q1 = rh[i] * ri;
    }
    store_partials(q0, q1, partial);
}

__global__ void k_apply_dA(double* w, const int64_t* off, const double* dA)
{
    const int c = blockIdx.x;
    const int64_t o0 = off[c], n = off[c + 1] - o0;
    const double d = dA[c];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) w[o0 + i] += d;
}

}  // namespace gm

namespace {

constexpr size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct GaussWs {
    double *colM, *colW, *dinv, *b, *x, *r, *rh, *p, *v, *s, *t, *partial, *st;
    size_t total;
};

int64_t vec_blocks(int64_t n_cells) { return (n_cells + gm::kVecThreads - 1) / gm::kVecThreads; }

unsigned stencil_blocks(int64_t n_cells)
{
    const int64_t per = gm::kStencilThreads / 64;
    return (unsigned)((n_cells + per - 1) / per);
}

GaussWs gauss_layout(int64_t n_cells, int dx, char* base)
{
    GaussWs g;
    const size_t n = (size_t)n_cells, ns = dx == 1 ? 3 : 9;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        double* ptr = base ? (double*)(base + o) : nullptr;
        o += al256(bytes);
        return ptr;
    };
    g.colM = take(n * ns * 8);
    g.colW = take(n * ns * 8);
    g.dinv = take(n * 8);
    g.b = take(n * 8);
    g.x = take(n * 8);
    g.r = take(n * 8);
    g.rh = take(n * 8);
    g.p = take(n * 8);
    g.v = take(n * 8);
    g.s = take(n * 8);
    g.t = take(n * 8);
    g.partial = take((size_t)vec_blocks(n_cells) * 2 * 8);
    g.st = take(gm::S_COUNT * 8);
    g.total = o;
    return g;
}

bool mesh_ok(int64_t n_cells, int dx, int nx)
{
    if (n_cells < 1 || n_cells > 0x7fffffff) return false;
    if (dx == 1) return nx == n_cells || nx <= 0;
    if (dx == 2) return nx >= 1 && n_cells % nx == 0;
    return false;
}

// iterations enqueued between two reads of the solver state
constexpr int kChunk = 8;
// restarts from the true residual before the solve gives up
constexpr int kMaxRestarts = 8;

template <int DX>
int gauss_correct_impl(const double* x, double* w, const int64_t* off, int64_t n, int nx, int ny,
                       const double* target, double tol, int max_iter, const GaussWs& g, hipStream_t st,
                       int32_t* iters_out, double* resid_out)
{
    using namespace gm;
    const unsigned nb = (unsigned)vec_blocks(n);
    const dim3 vb(kVecThreads);
    double hs[S_COUNT];
    auto read_state = [&]() -> bool {
        if (hipGetLastError() != hipSuccess) return false;
        if (hipMemcpyAsync(hs, g.st, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
        return hipStreamSynchronize(st) == hipSuccess;
    };
    auto fold = [&](int mode) {
        hipLaunchKernelGGL(k_fold, dim3(1), vb, 0, st, g.partial, (int)nb, g.st, mode, tol);
    };
    hipLaunchKernelGGL(k_stencil<DX>, dim3(stencil_blocks(n)), dim3(kStencilThreads), 0, st, x, w, off, n, g.colM,
                       g.colW);
    hipLaunchKernelGGL(k_setup<DX>, dim3(nb), vb, 0, st, g.colM, g.colW, target, off, n, nx, ny, g.dinv, g.b, g.x,
                       g.partial);
    fold(E_INIT);
    if (!read_state()) return GM_EHIP;
    if (hs[S_EMPTY] != 0.0) return GM_EINVAL;  // a cell without particles: M is singular
    const double b2 = hs[S_R2];
    bool converged = hs[S_DONE] == 1.0;
    int iters = 0;
    double r2 = b2;
    for (int rs = 0; !converged && rs <= kMaxRestarts; ++rs) {
        // the true residual of the current dA decides convergence
        hipLaunchKernelGGL(k_restart<DX>, dim3(nb), vb, 0, st, g.colM, g.b, g.x, n, nx, ny, g.r, g.rh, g.p, g.v,
                           g.partial);
        fold(E_RESTART);
        if (!read_state()) return GM_EHIP;
        r2 = hs[S_R2];
        if (hs[S_DONE] == 1.0) {
            converged = true;
            break;
        }
        if (hs[S_DONE] != 0.0 || iters >= max_iter) break;
        while (iters < max_iter) {
            const int k = max_iter - iters < kChunk ? max_iter - iters : kChunk;
            for (int it = 0; it < k; ++it) {
                hipLaunchKernelGGL(k_update_p, dim3(nb), vb, 0, st, g.st, g.r, g.v, g.p, n);
                hipLaunchKernelGGL((k_spmv<DX, false>), dim3(nb), vb, 0, st, g.st, g.colM, g.dinv, g.p, g.rh, n, nx,
                                   ny, g.v, g.partial);
                fold(E_ALPHA);
                hipLaunchKernelGGL(k_update_s, dim3(nb), vb, 0, st, g.st, g.r, g.v, g.s, n);
                hipLaunchKernelGGL((k_spmv<DX, true>), dim3(nb), vb, 0, st, g.st, g.colM, g.dinv, g.s, g.rh, n, nx,
                                   ny, g.t, g.partial);
                fold(E_OMEGA);
                hipLaunchKernelGGL(k_update_xr, dim3(nb), vb, 0, st, g.st, g.dinv, g.p, g.s, g.t, g.rh, g.x, g.r, n,
                                   g.partial);
                fold(E_RES_RHO);
            }
            if (!read_state()) return GM_EHIP;
            iters = (int)hs[S_ITERS];  // iterations since the start, over every restart
            if (hs[S_DONE] != 0.0) break;
        }
    }
    hipLaunchKernelGGL(k_apply_dA, dim3((unsigned)n), dim3(256), 0, st, w, off, g.x);
    if (hipGetLastError() != hipSuccess) return GM_EHIP;
    const double rel = b2 > 0.0 ? std::sqrt(r2 / b2) : 0.0;
    if (iters_out) *iters_out = iters;
    if (resid_out) *resid_out = rel;
    return converged && std::isfinite(rel) ? GM_OK : GM_ENOCONV;
}

}  // namespace

extern "C" {

size_t gm_gauss_workspace(int64_t n_cells, int32_t dx)
{
    if (!mesh_ok(n_cells, dx, dx == 1 ? (int)n_cells : 1)) return 0;
    return gauss_layout(n_cells, dx, nullptr).total;
}

int gm_deposit(const double* x, const double* w, const int64_t* cell_off, int64_t n_cells, int32_t dx, int32_t nx,
               double* dep, void* ws, size_t ws_bytes, void* stream)
{
    using namespace gm;
    if (!mesh_ok(n_cells, dx, nx)) return GM_EINVAL;
    if (!x || !w || !cell_off || !dep) return GM_EINVAL;
    GaussWs g = gauss_layout(n_cells, dx, (char*)ws);
    if (!ws || ws_bytes < g.total) return GM_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    const int NX = dx == 1 ? (int)n_cells : nx, NY = dx == 1 ? 1 : (int)(n_cells / nx);
    const unsigned nb = (unsigned)vec_blocks(n_cells);
    if (dx == 1) {
        hipLaunchKernelGGL(k_stencil<1>, dim3(stencil_blocks(n_cells)), dim3(kStencilThreads), 0, st, x, w,
                           cell_off, n_cells, nullptr, g.colW);
        hipLaunchKernelGGL(k_deposit<1>, dim3(nb), dim3(kVecThreads), 0, st, g.colW, n_cells, NX, NY, dep);
    } else {
        hipLaunchKernelGGL(k_stencil<2>, dim3(stencil_blocks(n_cells)), dim3(kStencilThreads), 0, st, x, w,
                           cell_off, n_cells, nullptr, g.colW);
        hipLaunchKernelGGL(k_deposit<2>, dim3(nb), dim3(kVecThreads), 0, st, g.colW, n_cells, NX, NY, dep);
    }
    return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP;
}

int gm_gauss_correct(const double* x, double* w, const int64_t* cell_off, int64_t n_cells, int32_t dx, int32_t nx,
                     const double* dep_target, double tol, int32_t max_iter, void* ws, size_t ws_bytes, void* stream,
                     int32_t* iters_out, double* resid_out)
{
    if (!mesh_ok(n_cells, dx, nx) || !(tol > 0.0) || !(tol < 1.0) || max_iter < 1) return GM_EINVAL;
    if (!x || !w || !cell_off || !dep_target) return GM_EINVAL;
    GaussWs g = gauss_layout(n_cells, dx, (char*)ws);
    if (!ws || ws_bytes < g.total) return GM_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    const int NX = dx == 1 ? (int)n_cells : nx, NY = dx == 1 ? 1 : (int)(n_cells / nx);
    if (dx == 1)
        return gauss_correct_impl<1>(x, w, cell_off, n_cells, NX, NY, dep_target, tol, max_iter, g, st, iters_out,
                                     resid_out);
    return gauss_correct_impl<2>(x, w, cell_off, n_cells, NX, NY, dep_target, tol, max_iter, g, st, iters_out,
                                 resid_out);
}

}  // extern "C"
