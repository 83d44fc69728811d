// gm_launch.h -- internal launch interface between the C ABI layer and the
// kernel translation units of libgmcr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gmcr.h"

namespace gm {

// ---- compress ------------------------------------------------------------
struct CompressArgs;

// Length buckets: cell n -> first bucket with n <= max_n (64 * 2^b).  Each
// bucket is run by one persistent launch of 64 * waves threads per
// workgroup, each thread holding `per_thread` particles.  `store_e` buckets
// keep every density term in registers, so the particles per thread depend
// on the number of component slots (KMAX): the register file holds
// (KMAX + D + 2) values per particle.
struct Bucket {
    int max_n;
    int per_thread;
    int waves;
    bool store_e;
};
constexpr int kNumBuckets = 12;
// KMAX = 8: 8 register-resident particles per thread up to 8 waves (4096
// particles), then the recompute mode.
constexpr Bucket kBuckets8[kNumBuckets] = {
    {64, 1, 1, true},    {128, 2, 1, true},   {256, 4, 1, true},    {512, 8, 1, true},
    {1024, 8, 2, true},  {1536, 8, 3, true},  {2048, 8, 4, true},   {2560, 8, 5, true},
    {3072, 8, 6, true},  {3584, 8, 7, true},  {4096, 8, 8, true},   {8192, 16, 8, false},
};
// KMAX = 16: 4 register-resident particles per thread, one bucket per wave
// count up to 8 waves (2048 particles), then the recompute mode; cells of
// 2049-4096 particles in two buckets (their FP32 launch plans keep 5 and 8
// particles per thread in registers).  Cells of up to 128 particles share
// one bucket (two particles per thread; such cells are rare in the
// workloads that use 16 slots).
constexpr Bucket kBuckets16[kNumBuckets] = {
    {128, 2, 1, true},   {256, 4, 1, true},   {512, 4, 2, true},    {768, 4, 3, true},
    {1024, 4, 4, true},  {1280, 4, 5, true},  {1536, 4, 6, true},   {1792, 4, 7, true},
    {2048, 4, 8, true},  {2560, 8, 5, false}, {4096, 8, 8, false},  {8192, 16, 8, false},
};
__host__ __device__ constexpr const Bucket& bucket_cfg(int kmax_tpl, int b)
{
    return kmax_tpl == 8 ? kBuckets8[b] : kBuckets16[b];
}
// largest cell of the register-resident launches; larger cells go to k_em_big
constexpr int kMaxCellParticles = 8192;

// Launch variants a bucket can run with (the autotuner picks among them):
// particles per thread, whether the density terms stay in registers, and
// the build: standard (workgroups of up to 512 threads, up to 256 VGPRs per
// lane, two waves per SIMD; three for FP32 with one register-resident
// particle per thread) or lean (up to 1024 threads, at most 128 VGPRs, four
// waves per SIMD: more cells in flight per CU, and 16-wave workgroups for
// the largest cells).  Lean builds exist for FP32 iterations
// only.  A variant fits a bucket when 64 * waves * per_thread >= max_n with
// waves = ceil(max_n / (64 * per_thread)) <= the build's waves.
// Register-resident densities with 8 particles per thread are built for
// kmax 8 only (16 slots x 8 particles do not fit the register file); with
// 5, 6 and 7 for FP32 iterations at kmax 16 only, so that the cells of
// 1025-1792 particles run as four waves, one per SIMD: with five to seven
// waves some SIMD carries two of the cell's waves and every component
// update waits for it.
// Launch mode bits: kModeStoreE (densities in registers), kModeLean.
constexpr int kModeStoreE = 1;
constexpr int kModeLean = 2;
struct EmVariant {
    int per_thread;
    bool store_e;
    bool lean;
};
constexpr int kNumVariants = 13;
constexpr EmVariant kVariants[kNumVariants] = {{1, true, false}, {2, true, false}, {4, true, false},
                                              {8, true, false}, {8, false, false}, {16, false, false},
                                              {1, true, true},  {2, true, true},  {4, false, true},
                                              {8, false, true}, {5, true, false}, {6, true, false},
                                              {7, true, false}};
// the 5-, 6- and 7-particle register-resident builds exist for FP32 at
// kmax 16 only; the 8-particle one for kmax 8, and for FP32 at kmax 16
__host__ __device__ constexpr bool em_variant_built(int D, int kt, bool fp64, int per_thread, bool store_e)
{
    return (void)D, !store_e || (per_thread >= 5 && per_thread <= 7 ? (kt == 16 && !fp64)
                                 : per_thread == 8              ? (kt == 8 || !fp64)
                                                                : true);
}
constexpr int kEmMaxThreads = 512;
constexpr int kEmLeanThreads = 1024;
__host__ __device__ constexpr int em_max_waves(bool lean) { return (lean ? kEmLeanThreads : kEmMaxThreads) / 64; }
constexpr int kEmMaxWaves = kEmLeanThreads / 64;
// launch-plan code of a variant: per_thread * 1000 + waves * 10 + mode
__host__ __device__ constexpr int em_variant_code(int per_thread, int waves, int mode)
{
    return per_thread * 1000 + waves * 10 + mode;
}

// ---- reconstruct ---------------------------------------------------------
struct ReconArgs {
    const int32_t* K;
    const double* omega;
    const double* mu;
    const double* sigma;
    int32_t kmax;
    const int64_t* out_off;
    const double* target;
    int32_t D, dx;
    uint64_t seed;
    double* v_out;
    double* w_out;
    double* x_out;
    int32_t* status;
    int32_t tensor;  // 0: scalar projection (W, P, tr S); 1: full second moment (W, P, S)
};

int launch_reconstruct(const ReconArgs& a, int64_t n_cells, hipStream_t st);

// arguments of the projection of given particles
struct ProjArgs {
    const double* v;
    const double* w;
    const int64_t* off;
    const double* moments;
    int32_t D;
    int32_t tensor;
    double* v_out;
    int32_t* status;
};

int launch_project(const ProjArgs& a, int64_t n_cells, hipStream_t st);

}  // namespace gm
