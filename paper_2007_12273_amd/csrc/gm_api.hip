// gm_api.hip -- the C ABI of libgmcr: argument checks, workspace layout and
// launch sequencing.  All arithmetic happens in the kernels.
#include <stdio.h>
#include <string.h>

#include "gm_compress_impl.h"

#include <algorithm>
#include <string>
#include <vector>
#include <mutex>

namespace gm {
int launch_compress_d1_float(int, int, int, int, const CompressArgs&, int, hipStream_t);
int launch_compress_d3_float(int, int, int, int, const CompressArgs&, int, hipStream_t);
int launch_compress_d1_double(int, int, int, int, const CompressArgs&, int, hipStream_t);
int launch_compress_d3_double(int, int, int, int, const CompressArgs&, int, hipStream_t);
int grid_compress_d1_float(int, int, int, int);
int grid_compress_d3_float(int, int, int, int);
int grid_compress_d1_double(int, int, int, int);
int grid_compress_d3_double(int, int, int, int);
int launch_compress_big_d1_float(int, const CompressArgs&, int, hipStream_t);
int launch_compress_big_d3_float(int, const CompressArgs&, int, hipStream_t);
int launch_compress_big_d1_double(int, const CompressArgs&, int, hipStream_t);
int launch_compress_big_d3_double(int, const CompressArgs&, int, hipStream_t);
int launch_compress_pre_d1(const CompressArgs&, hipStream_t);
int launch_compress_pre_d3(const CompressArgs&, hipStream_t);
int launch_compress_requeue_d1(const CompressArgs&, hipStream_t);
int launch_compress_requeue_d3(const CompressArgs&, hipStream_t);
int launch_compress_finish_d1(int, const CompressArgs&, hipStream_t);
int launch_compress_finish_d3(int, const CompressArgs&, hipStream_t);
int launch_std_d1(const StdArgs&, int64_t, hipStream_t);
int launch_std_d3(const StdArgs&, int64_t, hipStream_t);
}  // namespace gm

namespace {

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// phase timing: events recorded on the caller's stream around the compress
// phases (plan, EM, finish) and the reconstruct launch
enum { EV_PRE = 0, EV_EM, EV_FIN, EV_END, EV_REC0, EV_REC1, EV_COUNT };
bool g_prof = false;
bool g_prof_ready = false;
hipEvent_t g_ev[EV_COUNT];
bool g_ev_used[EV_COUNT];

void prof_mark(int which, hipStream_t st)
{
    if (!g_prof) return;
    if (!g_prof_ready) {
        for (int i = 0; i < EV_COUNT; ++i)
            if (hipEventCreate(&g_ev[i]) != hipSuccess) return;
        g_prof_ready = true;
    }
    if (hipEventRecord(g_ev[which], st) == hipSuccess) g_ev_used[which] = true;
}

size_t cellinfo_bytes(int D) { return D == 1 ? sizeof(gm::CellInfo<1>) : sizeof(gm::CellInfo<3>); }

struct WsLayout {
    size_t plan, cells, list, init, total;
};

// Streams of the EM phase, one set per device: every length bucket runs on
// a library stream of its own and the big-cell launch on the caller's
// stream, so the thirteen launches can run concurrently.  HIP maps streams
// onto GPU_MAX_HW_QUEUES hardware queues (default 4); they only all run at
// once with at least thirteen.  With fewer, streams share queues
// round-robin and the launches sharing a queue run one after another.
constexpr int kLanes = gm::kNumBuckets + 1;
struct Fork {
    hipStream_t aux[kLanes - 1];
    hipEvent_t fork;
    hipEvent_t fork2;  // releases the launches that do not fill a CU
    hipEvent_t join[kLanes - 1];
    long long hold_ticks;  // kHoldUs in ticks of the device's wall clock
};
constexpr int kMaxDevices = 64;
Fork* g_fork[kMaxDevices] = {};

// The EM phase releases its launches in two steps.  A bucket whose
// workgroups fill a CU's register file (eight or more waves of a standard
// build, sixteen of a lean one) can only start on an empty CU; launched
// together with the smaller buckets, whose persistent workgroups spread
// over every CU first, such a bucket's cells (in 3V the slowest fits)
// started up to several milliseconds late.  Its launches are therefore
// released first, and the others kHoldUs later, after a one-wave wait on
// the caller's stream that ends at once when those buckets hold no cell.
constexpr int kHoldUs = 40;
__global__ void k_hold(long long ticks, const int32_t* plan, unsigned heavy)
{
    int cells = 0;
    for (int b = 0; b < gm::kNumBuckets; ++b)
        if ((heavy >> b) & 1u) cells += plan[gm::PLAN_COUNT + b];
    if (cells == 0) return;
    const long long t0 = wall_clock64();
    for (int i = 0; i < (1 << 16); ++i) {  // bounded: about 13 ms of sleeps at most
        if (wall_clock64() - t0 >= ticks) break;
        __builtin_amdgcn_s_sleep(8);
    }
}

Fork* fork_for_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    if (g_fork[dev]) return g_fork[dev];
    Fork* f = new Fork;
    for (int i = 0; i < kLanes - 1; ++i) {
        if (hipStreamCreateWithFlags(&f->aux[i], hipStreamNonBlocking) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&f->join[i], hipEventDisableTiming) != hipSuccess) return nullptr;
    }
    if (hipEventCreateWithFlags(&f->fork, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&f->fork2, hipEventDisableTiming) != hipSuccess) return nullptr;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) return nullptr;
    f->hold_ticks = (long long)khz * kHoldUs / 1000;
    g_fork[dev] = f;
    return f;
}

// ---- EM launch plans ------------------------------------------------------
// Per bucket: launch variant (particles per thread, register-resident
// densities, waves), stream lane and launch order.  The default plan comes
// from the bucket tables; gm_autotune replaces it per (device, D, kmax
// template, precision, warm or cold start) with measured choices.
struct EmPlan {
    int8_t per_thread[gm::kNumBuckets];
    int8_t mode[gm::kNumBuckets];  // gm::kModeStoreE | gm::kModeLean
    int8_t waves[gm::kNumBuckets];
    int8_t lane[gm::kNumBuckets];
    int8_t order[gm::kNumBuckets];  // launch order, first launched first
    bool tuned;
};

// bucket b on library stream b
constexpr int kNumLaneOf(int b) { return b; }
// persistent workgroups of the big-cell launch
constexpr int kBigGrid = 64;

// Buckets of cells above 2048 particles (kmax 16) hold few cells, and one
// long fit among them can set the length of the whole EM phase: there the
// per-update latency of a single cell matters more than the bucket's
// throughput.  FP32 iterations run them with a lean build of more than 8
// waves (four waves per SIMD, the cell's CU to itself; in 3V the cells of
// 2049-4096 particles take the register-resident builds of the next rule
// instead).  On the Weibel-like batch one
// 2049-particle cell running 1000 sweeps made the warm phase 9.6-10.4 ms
// with it against 13.9-14.8 ms with the 8-wave builds, while a batch without
// such a fit cannot tell the builds apart, so the tuner keeps this choice.
constexpr int kChainMinN = 2048;
inline bool chain_bucket(int kt, bool fp64, int b)
{
    return !fp64 && kt == 16 && gm::bucket_cfg(kt, b).max_n > kChainMinN;
}

// The cells of 1025-1792 particles (FP32, kmax 16) run as four waves,
// one per SIMD, with 5, 6 or 7 register-resident particles per thread
// instead of five to seven waves of 4: every update then waits for a SIMD
// with one of the cell's waves, not two.  On the Weibel-like batch the warm
// EM phase took 8.1 ms with them against 10.0-10.2 ms.
inline bool four_wave_bucket(int D, int kt, bool fp64, int b)
{
    const int n = gm::bucket_cfg(kt, b).max_n;
    return (void)D, kt == 16 && !fp64 && n > 1024 && n <= 1792;
}

// In 3V the cells of 2049-2560 and 2561-4096 particles (FP32, kmax 16) run
// as eight waves with 5 and 8 register-resident particles per thread (two
// waves per SIMD, the CU to the cell as with the 16-wave lean build): each
// update then evaluates one density per particle instead of recomputing the
// old one beside the new one, and a cell near 2049 particles computes 5
// particle slots per lane, not 8.  The 8-particle build spills a few
// per-cell values, which it reloads inside the update.  On the Weibel-like
// batch, where these cells hold the longest cold fits, with built-in plans:
// judged-fallback refit 20.7-20.9 ms against 26.7-29.3 ms with the lean
// build, headline step 30.6-31.0 ms against 35.5-38.9 ms; the warm phase
// (8.8 ms against 8.3-8.4 ms) ends on a 2049-particle cell that runs 4005
// component updates (the sweep cap) here and 957 with the lean build's
// rounding.  The tuner may still pick a lean build there.
inline bool resident8_bucket(int D, int kt, bool fp64, int b)
{
    const int n = gm::bucket_cfg(kt, b).max_n;
    return D == 3 && kt == 16 && !fp64 && n > 2048 && n <= 4096;
}

EmPlan default_plan(int D, int kt, bool fp64)
{
    EmPlan p;
    for (int b = 0; b < gm::kNumBuckets; ++b) {
        const gm::Bucket& c = gm::bucket_cfg(kt, b);
        p.per_thread[b] = (int8_t)c.per_thread;
        p.mode[b] = (int8_t)(c.store_e ? gm::kModeStoreE : 0);
        p.waves[b] = (int8_t)c.waves;
        if (four_wave_bucket(D, kt, fp64, b)) {
            p.per_thread[b] = (int8_t)(c.max_n / 256);
            p.mode[b] = (int8_t)gm::kModeStoreE;
            p.waves[b] = 4;
        }
        if (chain_bucket(kt, fp64, b)) {
            // the lean builds recompute 4 or 8 particles per thread
            const int P = c.max_n <= 64 * gm::em_max_waves(true) * 4 ? 4 : 8;
            p.per_thread[b] = (int8_t)P;
            p.mode[b] = (int8_t)gm::kModeLean;
            p.waves[b] = (int8_t)((c.max_n + 64 * P - 1) / (64 * P));
        }
        if (resident8_bucket(D, kt, fp64, b)) {
            p.per_thread[b] = (int8_t)(c.max_n / (64 * 8));
            p.mode[b] = (int8_t)gm::kModeStoreE;
            p.waves[b] = 8;
        }
        p.lane[b] = (int8_t)(kNumLaneOf(b));
        p.order[b] = (int8_t)(gm::kNumBuckets - 1 - b);  // largest cells first
    }
    p.tuned = false;
    return p;
}

EmPlan* g_plans[kMaxDevices][2][2][2][2] = {};  // [dev][D == 3][kt == 16][fp64][warm]

EmPlan* plan_slot(int D, int kt, bool fp64, bool warm, bool create)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    EmPlan*& p = g_plans[dev][D == 3][kt == 16][fp64 ? 1 : 0][warm ? 1 : 0];
    if (!p && create) {
        p = new EmPlan(default_plan(D, kt, fp64));
    }
    return p;
}

int launch_em_bucket(int D, bool fp64, int kt, int b, const EmPlan& p, gm::CompressArgs& a, int64_t n_cells,
                     hipStream_t st)
{
    const int P = p.per_thread[b], W = p.waves[b];
    const int mode = p.mode[b];
    int grid = 0;
    if (D == 1)
        grid = fp64 ? gm::grid_compress_d1_double(kt, P, mode, W) : gm::grid_compress_d1_float(kt, P, mode, W);
    else
        grid = fp64 ? gm::grid_compress_d3_double(kt, P, mode, W) : gm::grid_compress_d3_float(kt, P, mode, W);
    if (grid < 1) return -1;
    if ((int64_t)grid > n_cells) grid = (int)n_cells;
    a.bucket = b;
    a.nwaves = W;
    if (D == 1)
        return fp64 ? gm::launch_compress_d1_double(kt, P, mode, W, a, grid, st)
                    : gm::launch_compress_d1_float(kt, P, mode, W, a, grid, st);
    return fp64 ? gm::launch_compress_d3_double(kt, P, mode, W, a, grid, st)
                : gm::launch_compress_d3_float(kt, P, mode, W, a, grid, st);
}

// the EM phase: fork onto the lanes, launch every bucket in plan order, join
int launch_em_phase(int D, bool fp64, int kt, const EmPlan& p, gm::CompressArgs& a, int64_t n_cells, hipStream_t st)
{
    Fork* fk = fork_for_device();
    if (!fk) return -1;
    hipStream_t lanes[kLanes];
    for (int i = 0; i < kLanes - 1; ++i) lanes[i] = fk->aux[i];
    lanes[kLanes - 1] = st;
    if (hipEventRecord(fk->fork, st) != hipSuccess) return -1;
    for (int i = 0; i < kLanes - 1; ++i)
        if (hipStreamWaitEvent(fk->aux[i], fk->fork, 0) != hipSuccess) return -1;
    // buckets whose workgroups fill a CU first, then, after the hold, the rest
    bool heavy[gm::kNumBuckets];
    bool any_heavy = false, any_light = false;
    unsigned heavy_mask = 0;
    for (int b = 0; b < gm::kNumBuckets; ++b) {
        const int fill = (p.mode[b] & gm::kModeLean) ? 16 : 8;
        heavy[b] = p.waves[b] >= fill && p.lane[b] != kLanes - 1;  // none waits behind the hold
        any_heavy |= heavy[b];
        any_light |= !heavy[b];
        if (heavy[b]) heavy_mask |= 1u << b;
    }
    for (int i = 0; i < gm::kNumBuckets; ++i) {
        const int b = p.order[i];
        if (heavy[b] && launch_em_bucket(D, fp64, kt, b, p, a, n_cells, lanes[p.lane[b]])) return -1;
    }
    if (any_heavy && any_light) {
        k_hold<<<1, 64, 0, st>>>(fk->hold_ticks, a.plan, heavy_mask);
        if (hipGetLastError() != hipSuccess) return -1;
        if (hipEventRecord(fk->fork2, st) != hipSuccess) return -1;
        bool waited[kLanes] = {};
        for (int b = 0; b < gm::kNumBuckets; ++b) {
            const int l = p.lane[b];
            if (heavy[b] || l == kLanes - 1 || waited[l]) continue;
            if (hipStreamWaitEvent(lanes[l], fk->fork2, 0) != hipSuccess) return -1;
            waited[l] = true;
        }
    }
    for (int i = 0; i < gm::kNumBuckets; ++i) {
        const int b = p.order[i];
        if (!heavy[b] && launch_em_bucket(D, fp64, kt, b, p, a, n_cells, lanes[p.lane[b]])) return -1;
    }
    // cells larger than the buckets hold, on the caller's stream
    {
        const int g = (int)std::min<int64_t>(kBigGrid, n_cells);
        int rc = 0;
        if (D == 1)
            rc = fp64 ? gm::launch_compress_big_d1_double(kt, a, g, st) : gm::launch_compress_big_d1_float(kt, a, g, st);
        else
            rc = fp64 ? gm::launch_compress_big_d3_double(kt, a, g, st) : gm::launch_compress_big_d3_float(kt, a, g, st);
        if (rc) return -1;
    }
    for (int i = 0; i < kLanes - 1; ++i) {
        if (hipEventRecord(fk->join[i], fk->aux[i]) != hipSuccess) return -1;
        if (hipStreamWaitEvent(st, fk->join[i], 0) != hipSuccess) return -1;
    }
    return 0;
}

WsLayout ws_layout(int64_t n_cells, int D)
{
    WsLayout w;
    w.plan = 0;
    w.cells = align256(gm::PLAN_SIZE * sizeof(int32_t));
    w.list = w.cells + align256((size_t)n_cells * cellinfo_bytes(D));
    w.init = w.list + align256((size_t)n_cells * sizeof(int32_t));
    w.total = w.init + align256((size_t)n_cells * gm::kInitSlots * sizeof(int32_t));
    return w;
}

bool valid_opts(const gm_opts* o)
{
    if (!o) return false;
    if (o->D != 1 && o->D != 3) return false;
    if (o->kmax < 1 || o->kmax > 16) return false;
    const int half_T_floor = o->D * (o->D + 3) / 4;  // floor(T / 2)
    if (o->n_min < half_T_floor) return false;
    if (o->max_sweeps < 1) return false;
    if (!(o->tol_rel >= 0.0)) return false;
    if (o->estep_fp64 != 0 && o->estep_fp64 != 1) return false;
    if (o->outer_k != 0 && o->outer_k != 1) return false;
    return true;
}

// ---- compress: argument checks and the launch sequence shared by
// gm_compress (caller workspace) and gm_compress_noalloc (fixed scratch) ----
int compress_check(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells, const gm_opts* o,
                   const gm_init* init, const gm_mix* out)
{
    if (!valid_opts(o) || n_cells < 0 || n_cells > 0x7fffffff || !out) return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!v || !alpha || !cell_off) return GM_EINVAL;
    if (!out->K || !out->omega || !out->mu || !out->sigma || !out->moments || !out->L_pen || !out->L_final ||
        !out->sweeps || !out->status || !out->visits)
        return GM_EINVAL;
    if (init && init->K && (!init->omega || !init->mu || !init->sigma)) return GM_EINVAL;
    return GM_OK;
}

int compress_run(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells, const gm_opts* o,
                 const int32_t* fixed_sweeps, const gm_init* init, const gm_mix* out, char* w, hipStream_t st)
{
    const WsLayout L = ws_layout(n_cells, o->D);
    gm::CompressArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.alpha = alpha;
    a.off = cell_off;
    a.n_cells = n_cells;
    a.cells = w + L.cells;
    a.list = (int32_t*)(w + L.list);
    a.init_idx = (int32_t*)(w + L.init);
    a.plan = (int32_t*)(w + L.plan);
    a.kmax = o->kmax;
    a.n_min = o->n_min;
    a.max_sweeps = o->max_sweeps;
    a.tol = o->tol_rel;
    a.seed = o->seed;
    a.outer = o->outer_k;
    a.fixed = fixed_sweeps;
    if (init && init->K) a.init = *init;
    a.out = *out;
    const int kt = o->kmax <= 8 ? 8 : 16;
    const bool fp64 = o->estep_fp64 != 0;
    const int D = o->D;

    prof_mark(EV_PRE, st);
    int rc = D == 1 ? gm::launch_compress_pre_d1(a, st) : gm::launch_compress_pre_d3(a, st);
    if (rc) return GM_EHIP;
    prof_mark(EV_EM, st);
    // Length buckets run concurrently on the caller's stream and three
    // auxiliary streams (fork/join through events, so the sequence can be
    // captured into a graph), in the order and lanes of the launch plan.
    {
        const EmPlan* tuned = plan_slot(D, kt, fp64, init && init->K, false);
        const EmPlan p = tuned ? *tuned : default_plan(D, kt, fp64);
        if (launch_em_phase(D, fp64, kt, p, a, n_cells, st)) return GM_EHIP;
    }
    prof_mark(EV_FIN, st);
    rc = D == 1 ? gm::launch_compress_finish_d1(kt, a, st) : gm::launch_compress_finish_d3(kt, a, st);
    prof_mark(EV_END, st);
    return rc ? GM_EHIP : GM_OK;
}

// ---- fixed scratch of gm_compress_noalloc ----
// The workspace of up to GM_NOALLOC_MAX_CELLS cells (the larger of the 1V
// and 3V layouts), one copy per device for the life of the process.  Host
// code never uses the array's name as an address: the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes =
    align256(gm::PLAN_SIZE * sizeof(int32_t)) + align256((size_t)GM_NOALLOC_MAX_CELLS * sizeof(gm::CellInfo<3>)) +
    align256((size_t)GM_NOALLOC_MAX_CELLS * sizeof(int32_t)) +
    align256((size_t)GM_NOALLOC_MAX_CELLS * gm::kInitSlots * sizeof(int32_t));
__device__ __align__(256) unsigned char scratch[kScratchBytes];

char* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// device address of this device's scratch (and its library streams), set
// up on the first call on the device; nullptr on a HIP error
char* scratch_for_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        if (!fork_for_device()) return nullptr;
        g_scratch[dev] = static_cast<char*>(p);
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" {

void gm_opts_default(gm_opts* o, int32_t D, int32_t kmax)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->D = D;
    o->kmax = kmax;
    o->n_min = 10;
    o->max_sweeps = 1000;
    o->tol_rel = 1e-7;
    o->seed = 0;
    o->estep_fp64 = 0;
    o->outer_k = 0;
}

size_t gm_compress_workspace(int64_t n_cells, const gm_opts* o)
{
    if (!o || n_cells < 0) return 0;
    return ws_layout(n_cells, o->D).total;
}

int gm_compress(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells, const gm_opts* o,
                const int32_t* fixed_sweeps, const gm_init* init, const gm_mix* out, void* ws, size_t ws_bytes,
                void* stream)
{
    const int rc = compress_check(v, alpha, cell_off, n_cells, o, init, out);
    if (rc != GM_OK || n_cells == 0) return rc;
    if (!ws || ws_bytes < ws_layout(n_cells, o->D).total) return GM_ENOMEM;
    return compress_run(v, alpha, cell_off, n_cells, o, fixed_sweeps, init, out, (char*)ws, (hipStream_t)stream);
}

int gm_compress_noalloc(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                        const gm_opts* o, const int32_t* fixed_sweeps, const gm_init* init, const gm_mix* out,
                        void* stream)
{
    const int rc = compress_check(v, alpha, cell_off, n_cells, o, init, out);
    if (rc != GM_OK || n_cells == 0) return rc;
    if (n_cells > GM_NOALLOC_MAX_CELLS) return GM_ETOOBIG;
    char* w = scratch_for_device();
    if (!w) return GM_EHIP;
    return compress_run(v, alpha, cell_off, n_cells, o, fixed_sweeps, init, out, w, (hipStream_t)stream);
}

// ---- warm start + compress in one call ----
namespace {
struct WarmWs {
    size_t feats, frame, K, omega, mu, sigma, total;
};
WarmWs warm_layout(int64_t n_cells, const gm_opts* o)
{
    WarmWs w;
    const size_t n = (size_t)n_cells, km = (size_t)o->kmax;
    w.feats = ws_layout(n_cells, o->D).total;
    w.frame = w.feats + align256(n * 128 * sizeof(uint16_t));
    w.K = w.frame + align256(n * 9 * sizeof(double));
    w.omega = w.K + align256(n * sizeof(int32_t));
    w.mu = w.omega + align256(n * km * sizeof(double));
    w.sigma = w.mu + align256(n * km * 3 * sizeof(double));
    w.total = w.sigma + align256(n * km * 6 * sizeof(double));
    return w;
}
}  // namespace

size_t gm_compress_warm_workspace(int64_t n_cells, const gm_opts* o)
{
    if (!valid_opts(o) || o->D != 3 || n_cells < 0) return 0;
    return warm_layout(n_cells, o).total;
}

int gm_compress_warm(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                     const gm_opts* o, const gm_warm* model, const gm_mix* out, void* ws, size_t ws_bytes,
                     void* stream)
{
    int rc = compress_check(v, alpha, cell_off, n_cells, o, nullptr, out);
    if (rc != GM_OK) return rc;
    if (!model || o->D != 3 || gm_warm_model_kmax(model) != o->kmax) return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    const WarmWs L = warm_layout(n_cells, o);
    if (!ws || ws_bytes < L.total) return GM_ENOMEM;
    char* w = (char*)ws;
    uint16_t* feats = (uint16_t*)(w + L.feats);
    double* frame = (double*)(w + L.frame);
    gm_init init;
    init.K = (const int32_t*)(w + L.K);
    init.omega = (const double*)(w + L.omega);
    init.mu = (const double*)(w + L.mu);
    init.sigma = (const double*)(w + L.sigma);
    if ((rc = gm_warm_features(v, alpha, cell_off, n_cells, 3, feats, frame, stream)) != GM_OK) return rc;
    if ((rc = gm_warm_infer(model, feats, frame, cell_off, n_cells, o->kmax, (int32_t*)(w + L.K),
                            (double*)(w + L.omega), (double*)(w + L.mu), (double*)(w + L.sigma), stream)) != GM_OK)
        return rc;
    return compress_run(v, alpha, cell_off, n_cells, o, nullptr, &init, out, w, (hipStream_t)stream);
}

size_t gm_compress_standard_workspace(int64_t n_cells, int64_t n_tot, const gm_opts* o)
{
    if (!valid_opts(o) || n_cells < 0 || n_tot < 0) return 0;
    return ws_layout(n_cells, o->D).total + align256((size_t)n_tot * (o->D + 1) * sizeof(float)) +
           align256((size_t)n_tot * sizeof(int32_t));
}

int gm_compress_standard(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells,
                         int64_t n_tot, const gm_opts* o, int32_t K, int32_t kmeans, int32_t aa_memory,
                         const gm_mix* out, int32_t* resets, int32_t* kmeans_passes, double* ll_trace, void* ws,
                         size_t ws_bytes, void* stream)
{
    if (!valid_opts(o) || o->outer_k != 0 || n_cells < 0 || n_cells > 0x7fffffff || n_tot < 0 || !out)
        return GM_EINVAL;
    if (K < 1 || K > o->kmax || (kmeans != 0 && kmeans != 1) || aa_memory < 0 || aa_memory > gm::kStdAaMax)
        return GM_EINVAL;
    if (o->estep_fp64 != 0) return GM_ENOTIMPL;
    if (n_cells == 0) return GM_OK;
    if (!v || !alpha || !cell_off) return GM_EINVAL;
    if (!out->K || !out->omega || !out->mu || !out->sigma || !out->moments || !out->L_pen || !out->L_final ||
        !out->sweeps || !out->status || !out->visits)
        return GM_EINVAL;
    const WsLayout L = ws_layout(n_cells, o->D);
    const size_t need = gm_compress_standard_workspace(n_cells, n_tot, o);
    if (!ws || ws_bytes < need) return GM_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    gm::StdArgs p;
    memset(&p, 0, sizeof(p));
    gm::CompressArgs& a = p.a;
    a.v = v;
    a.alpha = alpha;
    a.off = cell_off;
    a.n_cells = n_cells;
    a.cells = w + L.cells;
    a.list = (int32_t*)(w + L.list);
    a.init_idx = (int32_t*)(w + L.init);
    a.plan = (int32_t*)(w + L.plan);
    a.kmax = o->kmax;
    a.n_min = o->n_min;
    a.max_sweeps = o->max_sweeps;
    a.tol = o->tol_rel;
    a.seed = o->seed;
    a.std_K = K;
    a.out = *out;
    p.n_tot = n_tot;
    p.xa_w = (float*)(w + L.total);
    p.assign = (int32_t*)(w + L.total + align256((size_t)n_tot * (o->D + 1) * sizeof(float)));
    p.K = K;
    p.kmeans = kmeans;
    p.aa_m = aa_memory;
    p.resets = resets;
    p.kmeans_passes = kmeans_passes;
    p.ll_trace = ll_trace;
    const int kt = o->kmax <= 8 ? 8 : 16;
    const int D = o->D;
    if (D == 1 ? gm::launch_compress_pre_d1(a, st) : gm::launch_compress_pre_d3(a, st)) return GM_EHIP;
    if (D == 1 ? gm::launch_std_d1(p, n_cells, st) : gm::launch_std_d3(p, n_cells, st)) return GM_EHIP;
    if (D == 1 ? gm::launch_compress_finish_d1(kt, a, st) : gm::launch_compress_finish_d3(kt, a, st)) return GM_EHIP;
    return GM_OK;
}

int gm_autotune(const double* v, const double* alpha, const int64_t* cell_off, int64_t n_cells, const gm_opts* o,
                const gm_init* init, const gm_mix* out, void* ws, size_t ws_bytes, void* stream, double* report,
                int32_t report_len)
{
    if (!valid_opts(o) || n_cells < 1 || n_cells > 0x7fffffff || !out) return GM_EINVAL;
    if (!v || !alpha || !cell_off) return GM_EINVAL;
    if (!out->K || !out->omega || !out->mu || !out->sigma || !out->moments || !out->L_pen || !out->L_final ||
        !out->sweeps || !out->status || !out->visits)
        return GM_EINVAL;
    if (init && init->K && (!init->omega || !init->mu || !init->sigma)) return GM_EINVAL;
    if (report && report_len < GM_TUNE_REPORT_LEN) return GM_EINVAL;
    if (g_prof) return GM_EINVAL;  // the tuner records its own events
    const WsLayout L = ws_layout(n_cells, o->D);
    if (!ws || ws_bytes < L.total) return GM_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    gm::CompressArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.alpha = alpha;
    a.off = cell_off;
    a.n_cells = n_cells;
    a.cells = w + L.cells;
    a.list = (int32_t*)(w + L.list);
    a.init_idx = (int32_t*)(w + L.init);
    a.plan = (int32_t*)(w + L.plan);
    a.kmax = o->kmax;
    a.n_min = o->n_min;
    a.max_sweeps = o->max_sweeps;
    a.tol = o->tol_rel;
    a.seed = o->seed;
    a.outer = o->outer_k;
    a.fixed = nullptr;
    const bool warm = init && init->K;
    if (warm) a.init = *init;
    a.out = *out;
    const int kt = o->kmax <= 8 ? 8 : 16;
    const bool fp64 = o->estep_fp64 != 0;
    const int D = o->D;
    auto requeue = [&]() { return D == 1 ? gm::launch_compress_requeue_d1(a, st) : gm::launch_compress_requeue_d3(a, st); };

    if (D == 1 ? gm::launch_compress_pre_d1(a, st) : gm::launch_compress_pre_d3(a, st)) return GM_EHIP;
    int32_t counts[gm::kNumBuckets];
    if (hipMemcpyAsync(counts, a.plan + gm::PLAN_COUNT, sizeof(counts), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return GM_EHIP;

    // candidate variants of every bucket
    int cand[gm::kNumBuckets][gm::kNumVariants][2];  // (variant index, waves)
    int ncand[gm::kNumBuckets];
    int maxc = 0;
    for (int b = 0; b < gm::kNumBuckets; ++b) {
        ncand[b] = 0;
        const int max_n = gm::bucket_cfg(kt, b).max_n;
        for (int vi = 0; vi < gm::kNumVariants; ++vi) {
            const gm::EmVariant& var = gm::kVariants[vi];
            if (var.lean && fp64) continue;
            if (!gm::em_variant_built(D, kt, fp64, var.per_thread, var.store_e)) continue;
            const int waves = (max_n + 64 * var.per_thread - 1) / (64 * var.per_thread);
            if (waves < 1 || waves > gm::em_max_waves(var.lean)) continue;
            if (chain_bucket(kt, fp64, b) && !(var.lean && waves > gm::em_max_waves(false)) &&
                !(resident8_bucket(D, kt, fp64, b) && var.store_e && waves == 8))
                continue;
            cand[b][ncand[b]][0] = vi;
            cand[b][ncand[b]][1] = waves;
            ++ncand[b];
        }
        maxc = std::max(maxc, ncand[b]);
    }

    hipEvent_t ev[2 * gm::kNumBuckets];
    for (int i = 0; i < 2 * gm::kNumBuckets; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) return GM_EHIP;
    int rc = GM_OK;
    double best_ms[gm::kNumBuckets];
    int best_c[gm::kNumBuckets];
    double lean_ms[gm::kNumBuckets];  // fastest lean-build candidate
    int lean_c[gm::kNumBuckets];
    EmPlan trial = default_plan(D, kt, fp64);
    for (int b = 0; b < gm::kNumBuckets; ++b) {
        best_ms[b] = lean_ms[b] = 0.0;
        best_c[b] = lean_c[b] = -1;
    }
    // every bucket alone on the device, once per candidate
    for (int r = 0; r < maxc && rc == GM_OK; ++r) {
        if (requeue()) rc = GM_EHIP;
        bool used[gm::kNumBuckets] = {};
        for (int b = gm::kNumBuckets - 1; b >= 0 && rc == GM_OK; --b) {
            if (counts[b] <= 0 || r >= ncand[b]) continue;
            const gm::EmVariant& var = gm::kVariants[cand[b][r][0]];
            trial.per_thread[b] = (int8_t)var.per_thread;
            trial.mode[b] = (int8_t)((var.store_e ? gm::kModeStoreE : 0) | (var.lean ? gm::kModeLean : 0));
            trial.waves[b] = (int8_t)cand[b][r][1];
            if (hipEventRecord(ev[2 * b], st) != hipSuccess ||
                launch_em_bucket(D, fp64, kt, b, trial, a, n_cells, st) ||
                hipEventRecord(ev[2 * b + 1], st) != hipSuccess)
                rc = GM_EHIP;
            used[b] = true;
        }
        if (rc == GM_OK && hipStreamSynchronize(st) != hipSuccess) rc = GM_EHIP;
        for (int b = 0; b < gm::kNumBuckets && rc == GM_OK; ++b) {
            if (!used[b]) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[2 * b], ev[2 * b + 1]) != hipSuccess) {
                rc = GM_EHIP;
                break;
            }
            if (best_c[b] < 0 || t < best_ms[b]) {
                best_ms[b] = t;
                best_c[b] = r;
            }
            if (gm::kVariants[cand[b][r][0]].lean && (lean_c[b] < 0 || t < lean_ms[b])) {
                lean_ms[b] = t;
                lean_c[b] = r;
            }
        }
    }
    // A tuned plan from a choice of candidate per bucket: buckets spread
    // over the streams longest first onto the least-loaded one (with a
    // stream per bucket, each bucket gets its own), and launched in that
    // order.  Two choices: the fastest variant alone, and the
    // fastest lean-build variant where the bucket has one.  Alone, a bucket
    // has the device to itself; in the concurrent phase the lean builds
    // leave room on a CU for the other buckets' workgroups, which can beat
    // a variant that is faster alone.
    auto make_plan = [&](const int* choice, const double* ms) {
        EmPlan t = default_plan(D, kt, fp64);
        int idx[gm::kNumBuckets];
        for (int b = 0; b < gm::kNumBuckets; ++b) {
            idx[b] = b;
            if (choice[b] >= 0) {
                const gm::EmVariant& var = gm::kVariants[cand[b][choice[b]][0]];
                t.per_thread[b] = (int8_t)var.per_thread;
                t.mode[b] = (int8_t)((var.store_e ? gm::kModeStoreE : 0) | (var.lean ? gm::kModeLean : 0));
                t.waves[b] = (int8_t)cand[b][choice[b]][1];
            }
        }
        std::stable_sort(idx, idx + gm::kNumBuckets, [&](int x, int y) { return ms[x] > ms[y]; });
        double load[kLanes] = {};
        for (int i = 0; i < gm::kNumBuckets; ++i) {
            const int b = idx[i];
            int l = 0;
            for (int q = 1; q < kLanes; ++q)
                if (load[q] < load[l]) l = q;
            t.lane[b] = (int8_t)l;
            load[l] += ms[b];
            t.order[i] = (int8_t)b;
        }
        t.tuned = true;
        return t;
    };
    int pref_c[gm::kNumBuckets];
    double pref_ms[gm::kNumBuckets];
    for (int b = 0; b < gm::kNumBuckets; ++b) {
        const bool lean = lean_c[b] >= 0;
        pref_c[b] = lean ? lean_c[b] : best_c[b];
        pref_ms[b] = lean ? lean_ms[b] : best_ms[b];
    }
    // keep whichever plan runs the concurrent phase fastest
    constexpr int kPlans = 3;
    double phase_ms[kPlans] = {0.0, 0.0, 0.0};
    const EmPlan cands[kPlans] = {default_plan(D, kt, fp64), make_plan(best_c, best_ms), make_plan(pref_c, pref_ms)};
    // each plan's phase time is the median of three runs, the plans run in
    // turn (a drift of the device's clocks affects all of them alike): the
    // concurrent phase varies from run to run with the order in which the
    // buckets' workgroups reach the CUs, and a lucky minimum predicts the
    // next batch worse than the median does
    constexpr int kReps = 3;
    double runs[kPlans][kReps] = {};
    for (int rep = 0; rep < kReps && rc == GM_OK; ++rep)
        for (int pi = 0; pi < kPlans && rc == GM_OK; ++pi) {
            float t = 0.f;
            if (requeue() || hipEventRecord(ev[0], st) != hipSuccess ||
                launch_em_phase(D, fp64, kt, cands[pi], a, n_cells, st) || hipEventRecord(ev[1], st) != hipSuccess ||
                hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess)
                rc = GM_EHIP;
            runs[pi][rep] = t;
        }
    for (int pi = 0; pi < kPlans; ++pi) {
        std::sort(runs[pi], runs[pi] + kReps);
        phase_ms[pi] = runs[pi][kReps / 2];
    }
    int pick = 0;
    for (int pi = 1; pi < kPlans; ++pi)
        if (phase_ms[pi] < phase_ms[pick]) pick = pi;
    const EmPlan& chosen = cands[rc == GM_OK ? pick : 0];
    if (rc == GM_OK) {
        EmPlan* slot = plan_slot(D, kt, fp64, warm, true);
        if (!slot) {
            rc = GM_EHIP;
        } else {
            // installed as a measured choice also where it is the built-in
            // plan, so that a plan file keeps the decision
            *slot = chosen;
            slot->tuned = true;
        }
    }
    // leave a complete compress result in `out`
    if (rc == GM_OK && (requeue() || launch_em_phase(D, fp64, kt, chosen, a, n_cells, st) ||
                        (D == 1 ? gm::launch_compress_finish_d1(kt, a, st) : gm::launch_compress_finish_d3(kt, a, st))))
        rc = GM_EHIP;
    if (rc == GM_OK && hipStreamSynchronize(st) != hipSuccess) rc = GM_EHIP;
    for (int i = 0; i < 2 * gm::kNumBuckets; ++i) (void)hipEventDestroy(ev[i]);
    if (rc == GM_OK && report) {
        report[0] = phase_ms[0];
        report[1] = std::min(phase_ms[1], phase_ms[2]);
        for (int b = 0; b < gm::kNumBuckets; ++b) {
            report[2 + b] = best_ms[b];
            report[2 + gm::kNumBuckets + b] =
                gm::em_variant_code(chosen.per_thread[b], chosen.waves[b], chosen.mode[b]);
            report[2 + 2 * gm::kNumBuckets + b] = chosen.lane[b];
        }
    }
    return rc;
}

namespace {

// A plan from launch-plan codes (as in the autotune report), checked: every
// variant built and covering its bucket, lanes in range, the launch order
// (nullable: the built-in order) a permutation of the buckets.
int plan_from_codes(int D, int kt, bool fp64, const int32_t* variant, const int32_t* lane, const int32_t* order,
                    EmPlan& p)
{
    p = default_plan(D, kt, fp64);
    for (int b = 0; b < gm::kNumBuckets; ++b) {
        const int code = variant[b];
        const int P = code / 1000, W = (code / 10) % 100, mode = code % 10;
        if (code < 0 || mode > (gm::kModeStoreE | gm::kModeLean)) return GM_EINVAL;
        const bool se = (mode & gm::kModeStoreE) != 0, lean = (mode & gm::kModeLean) != 0;
        bool known = false;
        for (int vi = 0; vi < gm::kNumVariants; ++vi)
            known |= gm::kVariants[vi].per_thread == P && gm::kVariants[vi].store_e == se &&
                     gm::kVariants[vi].lean == lean;
        if (!known || (lean && fp64) || !gm::em_variant_built(D, kt, fp64 != 0, P, se))
            return GM_EINVAL;
        if (W < 1 || W > gm::em_max_waves(lean) || 64 * P * W < gm::bucket_cfg(kt, b).max_n) return GM_EINVAL;
        p.per_thread[b] = (int8_t)P;
        p.waves[b] = (int8_t)W;
        p.mode[b] = (int8_t)mode;
        if (lane) {
            if (lane[b] < 0 || lane[b] >= kLanes) return GM_EINVAL;
            p.lane[b] = (int8_t)lane[b];
        }
    }
    if (order) {
        bool seen[gm::kNumBuckets] = {};
        for (int b = 0; b < gm::kNumBuckets; ++b) {
            if (order[b] < 0 || order[b] >= gm::kNumBuckets || seen[order[b]]) return GM_EINVAL;
            seen[order[b]] = true;
            p.order[b] = (int8_t)order[b];
        }
    }
    p.tuned = true;
    return GM_OK;
}

// ---- launch-plan file ----
// One line per tuned plan:
//   gmcr-plan 1 <arch> <CUs> <D> <kmax class> <fp64> <warm> v[12] lane[12] order[12]
// The device key is the architecture name and CU count of the device the
// plan was tuned on; a file may hold the plans of several devices.
constexpr const char* kPlanTag = "gmcr-plan";
constexpr int kPlanFileVersion = 1;

bool device_key(char* arch, size_t n, int& cus)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    size_t i = 0;
    for (; i + 1 < n && prop.gcnArchName[i] && prop.gcnArchName[i] != ' '; ++i) arch[i] = prop.gcnArchName[i];
    arch[i] = 0;
    cus = prop.multiProcessorCount;
    return i > 0;
}

struct PlanLine {
    char arch[64];
    int cus, D, kt, fp64, warm;
    int32_t v[gm::kNumBuckets], lane[gm::kNumBuckets], order[gm::kNumBuckets];
};

// parse one line; false if it is not a well-formed plan line
bool parse_plan_line(const char* line, PlanLine& pl)
{
    char tag[16];
    int ver = 0, used = 0;
    if (sscanf(line, "%15s %d %63s %d %d %d %d %d%n", tag, &ver, pl.arch, &pl.cus, &pl.D, &pl.kt, &pl.fp64, &pl.warm,
               &used) != 8)
        return false;
    if (strcmp(tag, kPlanTag) != 0 || ver != kPlanFileVersion) return false;
    const char* q = line + used;
    int32_t* dst[3] = {pl.v, pl.lane, pl.order};
    for (int f = 0; f < 3; ++f)
        for (int b = 0; b < gm::kNumBuckets; ++b) {
            int x = 0, k = 0;
            if (sscanf(q, "%d%n", &x, &k) != 1) return false;
            dst[f][b] = x;
            q += k;
        }
    while (*q == ' ' || *q == '\t' || *q == '\r' || *q == '\n') ++q;
    return *q == 0 && (pl.D == 1 || pl.D == 3) && (pl.kt == 8 || pl.kt == 16) && (pl.fp64 == 0 || pl.fp64 == 1) &&
           (pl.warm == 0 || pl.warm == 1);
}

}  // namespace

int gm_autotune_set(int32_t D, int32_t kmax, int32_t fp64, int32_t warm, const int32_t* variant, const int32_t* lane)
{
    if ((D != 1 && D != 3) || kmax < 1 || kmax > 16 || !variant) return GM_EINVAL;
    const int kt = kmax <= 8 ? 8 : 16;
    EmPlan p;
    const int rc = plan_from_codes(D, kt, fp64 != 0, variant, lane, nullptr, p);
    if (rc != GM_OK) return rc;
    EmPlan* slot = plan_slot(D, kt, fp64 != 0, warm != 0, true);
    if (!slot) return GM_EHIP;
    *slot = p;
    return GM_OK;
}

int gm_autotune_get(int32_t D, int32_t kmax, int32_t fp64, int32_t warm, int32_t* variant, int32_t* lane,
                    int32_t* order)
{
    if ((D != 1 && D != 3) || kmax < 1 || kmax > 16 || !variant) return GM_EINVAL;
    const int kt = kmax <= 8 ? 8 : 16;
    const EmPlan* slot = plan_slot(D, kt, fp64 != 0, warm != 0, false);
    const EmPlan p = slot ? *slot : default_plan(D, kt, fp64 != 0);
    for (int b = 0; b < gm::kNumBuckets; ++b) {
        variant[b] = gm::em_variant_code(p.per_thread[b], p.waves[b], p.mode[b]);
        if (lane) lane[b] = p.lane[b];
        if (order) order[b] = p.order[b];
    }
    return p.tuned ? 1 : 0;
}

int gm_autotune_save(const char* path)
{
    if (!path || !path[0]) return GM_EINVAL;
    char arch[64];
    int cus = 0, dev = 0;
    if (!device_key(arch, sizeof(arch), cus) || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return GM_EHIP;
    // keep the lines of other devices from an existing file
    std::vector<std::string> keep;
    if (FILE* f = fopen(path, "r")) {
        char buf[1024];
        while (fgets(buf, sizeof(buf), f)) {
            PlanLine pl;
            if (parse_plan_line(buf, pl) && !(strcmp(pl.arch, arch) == 0 && pl.cus == cus)) keep.emplace_back(buf);
        }
        fclose(f);
    }
    FILE* f = fopen(path, "w");
    if (!f) return GM_EIO;
    bool ok = true;
    for (const std::string& l : keep) ok &= fputs(l.c_str(), f) >= 0;
    for (int d3 = 0; d3 < 2; ++d3)
        for (int k16 = 0; k16 < 2; ++k16)
            for (int f64 = 0; f64 < 2; ++f64)
                for (int w = 0; w < 2; ++w) {
                    const EmPlan* p = g_plans[dev][d3][k16][f64][w];
                    if (!p || !p->tuned) continue;
                    ok &= fprintf(f, "%s %d %s %d %d %d %d %d", kPlanTag, kPlanFileVersion, arch, cus, d3 ? 3 : 1,
                                  k16 ? 16 : 8, f64, w) > 0;
                    for (int b = 0; b < gm::kNumBuckets; ++b)
                        ok &= fprintf(f, " %d", gm::em_variant_code(p->per_thread[b], p->waves[b], p->mode[b])) > 0;
                    for (int b = 0; b < gm::kNumBuckets; ++b) ok &= fprintf(f, " %d", p->lane[b]) > 0;
                    for (int b = 0; b < gm::kNumBuckets; ++b) ok &= fprintf(f, " %d", p->order[b]) > 0;
                    ok &= fputc('\n', f) != EOF;
                }
    ok &= fclose(f) == 0;
    return ok ? GM_OK : GM_EIO;
}

int gm_autotune_load(const char* path)
{
    if (!path || !path[0]) return GM_EINVAL;
    char arch[64];
    int cus = 0;
    if (!device_key(arch, sizeof(arch), cus)) return GM_EHIP;
    FILE* f = fopen(path, "r");
    if (!f) return GM_EIO;
    // check every line first, install only a wholly valid file
    std::vector<std::pair<PlanLine, EmPlan>> plans;
    char buf[1024];
    int rc = GM_OK;
    while (rc == GM_OK && fgets(buf, sizeof(buf), f)) {
        const char* q = buf;
        while (*q == ' ' || *q == '\t') ++q;
        if (*q == '\n' || *q == '\r' || *q == 0 || *q == '#') continue;
        PlanLine pl;
        if (!parse_plan_line(buf, pl)) {
            rc = GM_EINVAL;
            break;
        }
        if (strcmp(pl.arch, arch) != 0 || pl.cus != cus) continue;  // another device's plan
        EmPlan p;
        rc = plan_from_codes(pl.D, pl.kt, pl.fp64 != 0, pl.v, pl.lane, pl.order, p);
        if (rc == GM_OK) plans.emplace_back(pl, p);
    }
    const bool read_err = ferror(f) != 0;
    fclose(f);
    if (read_err) return GM_EIO;
    if (rc != GM_OK) return rc;
    for (const auto& e : plans) {
        EmPlan* slot = plan_slot(e.first.D, e.first.kt, e.first.fp64 != 0, e.first.warm != 0, true);
        if (!slot) return GM_EHIP;
        *slot = e.second;
    }
    return (int)plans.size();
}

int gm_autotune_reset(void)
{
    for (auto& a : g_plans)
        for (auto& b : a)
            for (auto& c : b)
                for (auto& d : c)
                    for (auto& p : d) {
                        delete p;
                        p = nullptr;
                    }
    return GM_OK;
}

size_t gm_reconstruct_workspace(int64_t n_cells, int32_t D)
{
    (void)n_cells;
    (void)D;
    return 0;
}

namespace {
int reconstruct_impl(const int32_t* K, const double* omega, const double* mu, const double* sigma, int32_t kmax,
                     const int64_t* out_off, const double* target, int64_t n_cells, int32_t D, int32_t dx,
                     uint64_t seed, double* v_out, double* w_out, double* x_out, int32_t* status, void* stream,
                     int tensor)
{
    if ((D != 1 && D != 3) || kmax < 1 || kmax > 16 || dx < 0 || dx > 3 || n_cells < 0 || n_cells > 0x7fffffff)
        return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!K || !omega || !mu || !sigma || !out_off || !target || !v_out || !w_out || !status) return GM_EINVAL;
    if (dx > 0 && !x_out) return GM_EINVAL;
    gm::ReconArgs a;
    memset(&a, 0, sizeof(a));
    a.K = K;
    a.omega = omega;
    a.mu = mu;
    a.sigma = sigma;
    a.kmax = kmax;
    a.out_off = out_off;
    a.target = target;
    a.D = D;
    a.dx = dx;
    a.seed = seed;
    a.v_out = v_out;
    a.w_out = w_out;
    a.x_out = x_out;
    a.status = status;
    a.tensor = tensor;
    prof_mark(EV_REC0, (hipStream_t)stream);
    const int rc = gm::launch_reconstruct(a, n_cells, (hipStream_t)stream);
    prof_mark(EV_REC1, (hipStream_t)stream);
    return rc ? GM_EHIP : GM_OK;
}
}  // namespace

int gm_reconstruct(const int32_t* K, const double* omega, const double* mu, const double* sigma, int32_t kmax,
                   const int64_t* out_off, const double* target, int64_t n_cells, int32_t D, int32_t dx,
                   uint64_t seed, double* v_out, double* w_out, double* x_out, int32_t* status, void* ws,
                   size_t ws_bytes, void* stream)
{
    (void)ws;
    (void)ws_bytes;
    return reconstruct_impl(K, omega, mu, sigma, kmax, out_off, target, n_cells, D, dx, seed, v_out, w_out, x_out,
                            status, stream, 0);
}

int gm_reconstruct_tensor(const int32_t* K, const double* omega, const double* mu, const double* sigma,
                          int32_t kmax, const int64_t* out_off, const double* target, int64_t n_cells, int32_t D,
                          int32_t dx, uint64_t seed, double* v_out, double* w_out, double* x_out, int32_t* status,
                          void* ws, size_t ws_bytes, void* stream)
{
    (void)ws;
    (void)ws_bytes;
    return reconstruct_impl(K, omega, mu, sigma, kmax, out_off, target, n_cells, D, dx, seed, v_out, w_out, x_out,
                            status, stream, 1);
}

int gm_project(const double* v, const double* w, const int64_t* cell_off, const double* moments, int64_t n_cells,
               int32_t D, int32_t tensor, double* v_out, int32_t* status, void* stream)
{
    if ((D != 1 && D != 3) || (tensor != 0 && tensor != 1) || n_cells < 0 || n_cells > 0x7fffffff)
        return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!v || !w || !cell_off || !moments || !v_out || !status) return GM_EINVAL;
    gm::ProjArgs a;
    a.v = v;
    a.w = w;
    a.off = cell_off;
    a.moments = moments;
    a.D = D;
    a.tensor = tensor;
    a.v_out = v_out;
    a.status = status;
    return gm::launch_project(a, n_cells, (hipStream_t)stream) ? GM_EHIP : GM_OK;
}

void gm_profile_enable(int on) { g_prof = on != 0; }

int gm_profile_read(double* ms, int n)
{
    if (!ms || n < 4) return GM_EINVAL;
    const int pairs[4][2] = {{EV_PRE, EV_EM}, {EV_EM, EV_FIN}, {EV_FIN, EV_END}, {EV_REC0, EV_REC1}};
    for (int i = 0; i < 4; ++i) {
        ms[i] = -1.0;
        const int a0 = pairs[i][0], a1 = pairs[i][1];
        if (!g_prof_ready || !g_ev_used[a0] || !g_ev_used[a1]) continue;
        if (hipEventSynchronize(g_ev[a1]) != hipSuccess) return GM_EHIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, g_ev[a0], g_ev[a1]) != hipSuccess) return GM_EHIP;
        ms[i] = t;
    }
    return GM_OK;
}

const char* gm_strerror(int code)
{
    switch (code) {
        case GM_OK: return "success";
        case GM_EINVAL: return "invalid argument";
        case GM_EHIP: return "HIP runtime error";
        case GM_ENOMEM: return "workspace missing or too small";
        case GM_ENOTIMPL: return "not implemented in this build";
        case GM_ENOCONV: return "iterative solve did not reach its tolerance";
        case GM_EIO: return "file could not be opened, read or written";
        case GM_ETOOBIG: return "input larger than the fixed scratch of the allocation-free entry point";
        default: return "unknown error";
    }
}

int gm_version(void) { return 100; }

}  // extern "C"
