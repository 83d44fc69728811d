// gm_device.h -- device helpers shared by the gfx950 kernels of libgmcr.
//
// Counter-based Philox4x64-10, 64-lane DPP reductions, workgroup
// reductions through LDS, and 1x1 / 3x3 Cholesky factorisations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/gmcr.h"

namespace gm {

constexpr int ntri(int D) { return D * (D + 1) / 2; }
constexpr int nmom(int D) { return 1 + D + ntri(D); }  // W, P[D], S[ntri]

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;  // 1024 threads per workgroup

constexpr uint64_t kTagInit = 0x494E4954ull;   // "INIT"
constexpr uint64_t kTagRecon = 0x5245434Full;  // "RECO"

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with the Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
struct u64x4 {
    uint64_t x, y, z, w;
};

// Full 128-bit product of two 64-bit words from four 32 x 32 + 64 -> 64
// multiply-adds (v_mad_u64_u32), each partial product's carry folded into
// the next one's addend: hi:lo = m * x exactly.
__device__ __forceinline__ void mul_64x64_128(uint64_t m, uint64_t x, uint64_t& hi, uint64_t& lo)
{
    const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32), x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
    const uint64_t t = (uint64_t)m0 * x0;
    const uint64_t u = (uint64_t)m1 * x0 + (t >> 32);       // < 2^64: (2^32 - 1)^2 + 2^32 - 1
    const uint64_t w = (uint64_t)m0 * x1 + (uint32_t)u;
    const uint64_t y = (uint64_t)m1 * x1 + (u >> 32);
    hi = y + (w >> 32);
    lo = (w << 32) | (uint32_t)t;
}

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mul_64x64_128(M0, c0, hi0, lo0);
        mul_64x64_128(M1, c2, hi1, lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return {c0, c1, c2, c3};
}

// top 53 bits -> [0, 1)
__device__ __forceinline__ double unit53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

// ---------------------------------------------------------------------------
// 64-lane sums with DPP: quad swaps, half-row and row mirrors give every lane
// its 16-lane row total; two row broadcasts (lane 15 of each row into the
// next row, lane 31 into rows 2 and 3) fold the rows into lane 63, which
// ends with (R3 + R2) + (R1 + R0).  Only lane 63's value is used, so the
// broadcasts write every row (a lane without a source row adds zero): with
// full row masks the move fuses into the add, one instruction per level.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xf, true);
}

__device__ __forceinline__ float wave_sum(float x)
{
    x += __int_as_float(dpp_i<0xB1>(__float_as_int(x)));       // quad_perm [1,0,3,2]
    x += __int_as_float(dpp_i<0x4E>(__float_as_int(x)));       // quad_perm [2,3,0,1]
    x += __int_as_float(dpp_i<0x141>(__float_as_int(x)));      // row_half_mirror
    x += __int_as_float(dpp_i<0x140>(__float_as_int(x)));      // row_mirror
    x += __int_as_float(dpp_i<0x142>(__float_as_int(x))); // row_bcast:15
    x += __int_as_float(dpp_i<0x143>(__float_as_int(x))); // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_d(double x)
{
    const int64_t b = __double_as_longlong(x);
    const int lo = dpp_i<CTRL, ROW_MASK>((int)(uint32_t)b);
    const int hi = dpp_i<CTRL, ROW_MASK>((int)(uint32_t)(b >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_d<0xB1>(x);
    x += dpp_d<0x4E>(x);
    x += dpp_d<0x141>(x);
    x += dpp_d<0x140>(x);
    x += dpp_d<0x142>(x);
    x += dpp_d<0x143>(x);
    const int64_t b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Workgroup-wide sum of NV values; every thread receives the totals.  Lane
// 0 of every wave publishes its wave's sums; after one barrier lane v < NV
// adds the per-wave partials of value v in wave order (MAXW bounds the wave
// count so the loads can all be issued together) and the totals are
// broadcast back with readlane.  The order of additions is fixed, so all
// threads and all runs see identical totals.  `buf` holds two halves of
// kMaxWaves * NVMAX values (NVMAX >= every NV used with the buffer);
// `parity` alternates halves so one barrier per call suffices: a wave can
// only overwrite a half after every wave has passed the barrier of the call
// that last used it.
__device__ __forceinline__ float lane_bcast(float x, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

__device__ __forceinline__ double lane_bcast(double x, int lane)
{
    const int64_t b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

template <int NVMAX, int MAXW = kMaxWaves, typename T, int NV>
__device__ __forceinline__ void block_sum(T (&x)[NV], T* buf, int& parity, int nwaves)
{
    static_assert(NV <= NVMAX && NVMAX <= 64, "reduction buffer too small");
    static_assert(MAXW <= kMaxWaves, "more waves than the buffer holds");
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = wave_sum(x[v]);
    if (nwaves == 1) return;
    T* b = buf + parity * (kMaxWaves * NVMAX);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) b[wid * NVMAX + v] = x[v];
    }
    __syncthreads();
    T t = T(0);
    if (lane < NV) {
        // all MAXW partials are loaded at once (slots of absent waves are in
        // the buffer and discarded), then added in wave order
        T part[MAXW];
#pragma unroll
        for (int w = 0; w < MAXW; ++w) part[w] = b[w * NVMAX + lane];
        t = part[0];
#pragma unroll
        for (int w = 1; w < MAXW; ++w)
            if (w < nwaves) t += part[w];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = lane_bcast(t, v);
    parity ^= 1;
}

// ---------------------------------------------------------------------------
// Small symmetric matrices, packed upper triangle row-major (= packed lower
// triangle row-major for the factor): D = 3 -> (00, 01, 02, 11, 12, 22).
// ---------------------------------------------------------------------------
template <int D>
__host__ __device__ constexpr int tri_idx(int i, int j)
{
    // i <= j, row-major upper
    return i * D - i * (i - 1) / 2 + (j - i);
}

// Cholesky of packed S into packed lower factor L (L[tri_idx(j,i)] = L_ij for
// i >= j); returns false if S is not numerically positive definite.
template <int D, typename R>
__device__ __forceinline__ bool chol(const R (&S)[ntri(D)], R (&L)[ntri(D)])
{
    if constexpr (D == 1) {
        if (!(S[0] > R(0)) || !isfinite(S[0])) return false;
        L[0] = sqrt(S[0]);
        return true;
    } else {
        // S packed: 0=00 1=01 2=02 3=11 4=12 5=22 ; L packed same slots as (row>=col): 0=L00 1=L10 2=L20 3=L11 4=L21 5=L22
        const R s00 = S[0];
        if (!(s00 > R(0)) || !isfinite(s00)) return false;
        const R l00 = sqrt(s00);
        const R l10 = S[1] / l00;
        const R l20 = S[2] / l00;
        const R t11 = S[3] - l10 * l10;
        if (!(t11 > R(0)) || !isfinite(t11)) return false;
        const R l11 = sqrt(t11);
        const R l21 = (S[4] - l20 * l10) / l11;
        const R t22 = S[5] - l20 * l20 - l21 * l21;
        if (!(t22 > R(0)) || !isfinite(t22)) return false;
        const R l22 = sqrt(t22);
        L[0] = l00;
        L[1] = l10;
        L[2] = l20;
        L[3] = l11;
        L[4] = l21;
        L[5] = l22;
        return true;
    }
}

// Inverse of the packed lower factor (same packing).
template <int D, typename R>
__device__ __forceinline__ void tri_inv(const R (&L)[ntri(D)], R (&M)[ntri(D)])
{
    if constexpr (D == 1) {
        M[0] = R(1) / L[0];
    } else {
        const R m00 = R(1) / L[0], m11 = R(1) / L[3], m22 = R(1) / L[5];
        const R m10 = -L[1] * m00 * m11;
        const R m21 = -L[4] * m11 * m22;
        const R m20 = -(L[2] * m00 + L[4] * m10) * m22;
        M[0] = m00;
        M[1] = m10;
        M[2] = m20;
        M[3] = m11;
        M[4] = m21;
        M[5] = m22;
    }
}

// |M d|^2 for packed lower-triangular M
template <int D, typename R>
__device__ __forceinline__ R tri_quad(const R* M, const R (&d)[D])
{
    if constexpr (D == 1) {
        const R z = M[0] * d[0];
        return z * z;
    } else {
        const R z0 = M[0] * d[0];
        const R z1 = M[1] * d[0] + M[3] * d[1];
        const R z2 = M[2] * d[0] + M[4] * d[1] + M[5] * d[2];
        return z0 * z0 + z1 * z1 + z2 * z2;
    }
}

// sum of log2 of the factor's diagonal = log2 sqrt(det S)
template <int D, typename R>
__device__ __forceinline__ R tri_log2diag(const R (&L)[ntri(D)])
{
    if constexpr (D == 1) {
        return log2(L[0]);
    } else {
        return log2(L[0] * L[3] * L[5]);
    }
}

template <typename R>
__device__ __forceinline__ R fast_exp2(R x)
{
    if constexpr (std::is_same<R, float>::value) {
        return __builtin_amdgcn_exp2f(x);
    } else {
        return exp2(x);
    }
}

template <typename R>
__device__ __forceinline__ R fast_log2(R x)
{
    if constexpr (std::is_same<R, float>::value) {
        return __builtin_amdgcn_logf(x);
    } else {
        return log2(x);
    }
}

template <typename R>
__device__ __forceinline__ R fast_rcp(R x)
{
    if constexpr (std::is_same<R, float>::value) {
        return __builtin_amdgcn_rcpf(x);
    } else {
        return R(1) / x;
    }
}

}  // namespace gm
