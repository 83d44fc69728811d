// gm_api.hip -- the C ABI of libgmcr: argument checks, workspace layout and
// launch sequencing.  All arithmetic happens in the kernels.
#include <string.h>

#include "gm_compress_impl.h"

namespace gm {
int launch_compress_d1_float(int, int, const CompressArgs&, int, hipStream_t);
int launch_compress_d3_float(int, int, const CompressArgs&, int, hipStream_t);
int launch_compress_d1_double(int, int, const CompressArgs&, int, hipStream_t);
int launch_compress_d3_double(int, int, const CompressArgs&, int, hipStream_t);
int grid_compress_d1_float(int, int);
int grid_compress_d3_float(int, int);
int grid_compress_d1_double(int, int);
int grid_compress_d3_double(int, int);
int launch_compress_pre_d1(const CompressArgs&, hipStream_t);
int launch_compress_pre_d3(const CompressArgs&, hipStream_t);
int launch_compress_finish_d1(int, const CompressArgs&, hipStream_t);
int launch_compress_finish_d3(int, const CompressArgs&, hipStream_t);
}  // namespace gm

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

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

// auxiliary streams for concurrent length buckets, one set per device
constexpr int kLanes = 4;
// bucket -> lane (0..2 auxiliary, 3 the caller's stream).  Each bucket's
// makespan is set by its slowest cell, so the mapping spreads the buckets
// that measured longest on the 1D3V Weibel-like workload over different
// lanes (the 257-512 bucket holds small cells that keep 16 components for
// the whole sweep cap; the two recompute-mode buckets hold the largest
// cells); buckets are launched largest first on every lane.
constexpr int kBucketLane16[gm::kNumBuckets] = {0, 0, 0, 0, 3, 3, 1, 2, 3, 3, 1, 2};
constexpr int kBucketLane8[gm::kNumBuckets] = {0, 1, 2, 3, 0, 1, 2, 3, 0, 1, 2, 3};
struct Fork {
    hipStream_t aux[kLanes - 1];
    hipEvent_t fork;
    hipEvent_t join[kLanes - 1];
};
constexpr int kMaxDevices = 64;
Fork* g_fork[kMaxDevices] = {};

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
    g_fork[dev] = f;
    return f;
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
    if (o->reserved != 0) return false;
    return true;
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
    o->reserved = 0;
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
    if (!valid_opts(o) || n_cells < 0 || n_cells > 0x7fffffff || !out) return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!v || !alpha || !cell_off) return GM_EINVAL;
    if (!out->K || !out->omega || !out->mu || !out->sigma || !out->moments || !out->L_pen || !out->L_final ||
        !out->sweeps || !out->status || !out->visits)
        return GM_EINVAL;
    if (init && init->K && (!init->omega || !init->mu || !init->sigma)) return GM_EINVAL;
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
    // captured into a graph).  The largest cells are launched first: their
    // workgroups are the longest-running.
    Fork* fk = fork_for_device();
    if (!fk) return GM_EHIP;
    hipStream_t lanes[kLanes] = {fk->aux[0], fk->aux[1], fk->aux[2], st};
    if (hipEventRecord(fk->fork, st) != hipSuccess) return GM_EHIP;
    for (int i = 0; i < kLanes - 1; ++i)
        if (hipStreamWaitEvent(fk->aux[i], fk->fork, 0) != hipSuccess) return GM_EHIP;
    for (int b = gm::kNumBuckets - 1; b >= 0; --b) {
        hipStream_t bs = lanes[kt == 8 ? kBucketLane8[b] : kBucketLane16[b]];
        int grid = 0;
        if (D == 1)
            grid = fp64 ? gm::grid_compress_d1_double(kt, b) : gm::grid_compress_d1_float(kt, b);
        else
            grid = fp64 ? gm::grid_compress_d3_double(kt, b) : gm::grid_compress_d3_float(kt, b);
        if (grid < 1) return GM_EHIP;
        if ((int64_t)grid > n_cells) grid = (int)n_cells;
        a.bucket = b;
        a.nwaves = gm::bucket_cfg(kt, b).waves;
        if (D == 1)
            rc = fp64 ? gm::launch_compress_d1_double(kt, b, a, grid, bs) : gm::launch_compress_d1_float(kt, b, a, grid, bs);
        else
            rc = fp64 ? gm::launch_compress_d3_double(kt, b, a, grid, bs) : gm::launch_compress_d3_float(kt, b, a, grid, bs);
        if (rc) return GM_EHIP;
    }
    for (int i = 0; i < kLanes - 1; ++i) {
        if (hipEventRecord(fk->join[i], fk->aux[i]) != hipSuccess) return GM_EHIP;
        if (hipStreamWaitEvent(st, fk->join[i], 0) != hipSuccess) return GM_EHIP;
    }
    prof_mark(EV_FIN, st);
    rc = D == 1 ? gm::launch_compress_finish_d1(kt, a, st) : gm::launch_compress_finish_d3(kt, a, st);
    prof_mark(EV_END, st);
    return rc ? GM_EHIP : GM_OK;
}

size_t gm_reconstruct_workspace(int64_t n_cells, int32_t D)
{
    (void)n_cells;
    (void)D;
    return 0;
}

int gm_reconstruct(const int32_t* K, const double* omega, const double* mu, const double* sigma, int32_t kmax,
                   const int64_t* out_off, const double* target, int64_t n_cells, int32_t D, int32_t dx,
                   uint64_t seed, double* v_out, double* w_out, double* x_out, int32_t* status, void* ws,
                   size_t ws_bytes, void* stream)
{
    (void)ws;
    (void)ws_bytes;
    if ((D != 1 && D != 3) || kmax < 1 || kmax > 16 || dx < 0 || dx > 3 || n_cells < 0 || n_cells > 0x7fffffff)
        return GM_EINVAL;
    if (n_cells == 0) return GM_OK;
    if (!K || !omega || !mu || !sigma || !out_off || !target || !v_out || !w_out || !status) return GM_EINVAL;
    if (dx > 0 && !x_out) return GM_EINVAL;
    gm::ReconArgs a;
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
    prof_mark(EV_REC0, (hipStream_t)stream);
    const int rc = gm::launch_reconstruct(a, n_cells, (hipStream_t)stream);
    prof_mark(EV_REC1, (hipStream_t)stream);
    return rc ? GM_EHIP : GM_OK;
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
        default: return "unknown error";
    }
}

int gm_version(void) { return 100; }

}  // extern "C"
