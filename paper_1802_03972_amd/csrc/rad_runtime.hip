// Host runtime of the C ABI declared in include/rad.h: grid lifetime, validation, launch
// shapes, and the stream-ordered push / fold / read-out sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rad.h"
#include "rad_internal.h"

using rad::AccArgs;
using rad::LaunchShape;

namespace {

thread_local std::string t_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(RAD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define RAD_HIP(call)                                         \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

constexpr double kC = 299792458.0;
constexpr double kQe = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

// Normalised Table 1 shape factor |F~(omega)|^2 (F~(0) = 1), evaluated on the host once
// per grid and uploaded as (g, 1 - g) in FP32.
double shape_factor(int shape, double L, double omega)
{
    switch (shape) {
    case RAD_SHAPE_POINT: return 1.0;
    case RAD_SHAPE_GAUSS: {
        const double a = omega * L / kC;
        return std::exp(-a * a);
    }
    default: {
        const double x = 0.5 * omega * L / kC;
        const double s = x == 0.0 ? 1.0 : std::sin(x) / x;
        const double s2 = s * s;
        if (shape == RAD_SHAPE_CIC) return s2;
        if (shape == RAD_SHAPE_TSC) return s2 * s2;
        return s2 * s2 * s2;
    }
    }
}

bool is_shape3(int shape) { return shape >= RAD_SHAPE_CIC3D && shape <= RAD_SHAPE_QSC3D; }

// Cubic cell of side L: product over the axes of the 1-D shape factor at omega * n_c.
double shape_factor3(int shape, double L, const double n[3], double omega)
{
    const int s1 = shape - RAD_SHAPE_CIC3D + RAD_SHAPE_CIC;
    double g = 1.0;
    for (int c = 0; c < 3; ++c) g *= shape_factor(s1, L, omega * std::fabs(n[c]));
    return g;
}

// Orthonormal basis (e1, e2) of the plane normal to unit n.
void normal_basis(const double n[3], double e1[3], double e2[3])
{
    int a = 0;
    if (std::fabs(n[1]) < std::fabs(n[a])) a = 1;
    if (std::fabs(n[2]) < std::fabs(n[a])) a = 2;
    double u[3] = {0, 0, 0};
    u[a] = 1.0;
    const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    for (int c = 0; c < 3; ++c) e1[c] = u[c] - un * n[c];
    const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int c = 0; c < 3; ++c) e1[c] /= l1;
    e2[0] = n[1] * e1[2] - n[2] * e1[1];
    e2[1] = n[2] * e1[0] - n[0] * e1[2];
    e2[2] = n[0] * e1[1] - n[1] * e1[0];
    const double l2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    for (int c = 0; c < 3; ++c) e2[c] /= l2;
}

// ---- fixed scratch of the no-allocation push (rad_push_step_noalloc) ----------------
// That entry point keeps its FP32 partial sums in this file-scope device array instead of
// a grid's own buffers.  In host code the name `scratch` is only a host-side handle of the
// symbol, not a device address: the array's address on each GPU is looked up once per
// device (hipGetSymbolAddress, with that device current, when the first grid is created
// on it) and only that address is ever passed to kernels.
constexpr int kScratchDevices = 64;
static __device__ __align__(256) float scratch[RAD_NOALLOC_SCRATCH_BYTES / sizeof(float)];
std::mutex g_scratch_mu;
std::atomic<float*> g_scratch_addr[kScratchDevices];

// Looks up the scratch address on the current device `dev` (once per device).
int scratch_setup(int dev)
{
    if (dev < 0 || dev >= kScratchDevices)
        return fail(RAD_ERR_INVALID_ARG, "device %d beyond the %d devices the library supports", dev, kScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_addr[dev].load(std::memory_order_acquire)) return RAD_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(RAD_ERR_DEVICE, "no device address for the no-allocation scratch");
    g_scratch_addr[dev].store(static_cast<float*>(p), std::memory_order_release);
    return RAD_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct rad_grid {
    int device = 0;
    int n_dir = 0, n_omega = 0;
    double omega0 = 0, domega = 0, dt = 0, shape_len = 0;
    int shape = 0, precision = 0;
    double C = 0;
    int cus = 0;
    rad_tile tile{};
    double* d_dirs9 = nullptr;
    double* d_omega = nullptr;
    float2* d_gtab = nullptr;
    double* d_S = nullptr;
    // Two partial-sum buffers, used in turn: a push on one stream may start its
    // accumulate while the fold of the previous push (issued on another stream) still
    // reads the other buffer.
    float* d_part[2] = {nullptr, nullptr};
    int64_t part_splits = 0;
    int part_next = 0;
    // Ordering hub of the writes of S: every single-push fold (run on the pushing stream),
    // batched fold, reset and device read-out is chained into it; a call on another stream
    // than the last write's waits for its last event.
    hipStream_t fold_stream = nullptr;
    hipEvent_t ev_fold_done[2] = {nullptr, nullptr};
    hipStream_t fold_done_on[2] = {nullptr, nullptr};   // stream that orders the write each event marks
    hipEvent_t ev_write = nullptr;   // end of a write of S on a caller's stream (reset)
    bool fold_recorded[2] = {false, false};
    int last_fold = -1;
    int* d_err = nullptr;
    double* d_out = nullptr;
    float* d_g3 = nullptr;     // [n_dir][n_omega] for 3-D shapes
    double* d_bstep = nullptr; // per-block spacing of a piecewise-uniform frequency list
    int variant = 0;           // rad::kVarDirect | rad::kVarShape3
    // kernel timing (rad_profile_*)
    bool profiling = false;
    int64_t prof_period = 1;    // time every prof_period-th accumulate launch
    int64_t prof_count = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_acc, ev_fold;
    int64_t prof_updates = 0;
};

namespace {

// Particles handled per workgroup in one launch at most (bounds the FP32 partial sums;
// longer pushes are cut into several launches, each folded into the FP64 accumulator).
constexpr int64_t kMaxPerWorkgroup = 32768;

LaunchShape shape_of(const rad_tile& t, int variant = 0)
{
    return LaunchShape{t.w_per_lane, t.dir_per_wave, t.waves, variant};
}

int tiles_d(const rad_grid* g) { return (g->n_dir + g->tile.dir_per_wave - 1) / g->tile.dir_per_wave; }
int tiles_w(const rad_grid* g)
{
    const int to = rad::tile_omegas(shape_of(g->tile));
    return (g->n_omega + to - 1) / to;
}
int max_splits(const rad_grid* g)
{
    const int nt = tiles_d(g) * tiles_w(g);
    const int target = g->cus * g->tile.wg_per_cu;
    return std::max(1, (target + nt - 1) / nt);
}

rad_tile default_tile(int n_dir, int n_omega, int variant = 0)
{
    (void)variant;
    rad_tile t{};
    // 16 frequencies per lane (the four-waves-per-SIMD kernels); 32 directions per wave
    // where the grid has them and the frequencies are few, else 16.  Measured winners on
    // MI355X: 128 x 256 and 64 x 256 -> 32 x 8 waves, 128 x 512 and 64 x 1024 -> 16 x 8.
    t.w_per_lane = 16;
    t.dir_per_wave = (n_dir >= 32 && n_omega <= 256) ? 32 : 16;
    const int per_wave = (64 / t.dir_per_wave) * t.w_per_lane;
    t.waves = std::min(8, std::max(1, (n_omega + per_wave - 1) / per_wave));
    // 16 waves per CU fit (128 VGPRs); LDS also bounds the count.
    const size_t lds = rad::acc_lds_bytes(shape_of(t));
    const int by_waves = std::max(1, 16 / t.waves);
    const int by_lds = std::max(1, (int)((160 * 1024) / lds));
    t.wg_per_cu = std::max(2, std::min(by_waves, by_lds));
    return t;
}

int validate_tile(const rad_tile& t)
{
    if (t.w_per_lane != 16 && t.w_per_lane != 32)
        return fail(RAD_ERR_INVALID_ARG, "w_per_lane must be 16 or 32 (got %d)", t.w_per_lane);
    if (t.dir_per_wave != 16 && t.dir_per_wave != 32 && t.dir_per_wave != 64)
        return fail(RAD_ERR_INVALID_ARG, "dir_per_wave must be 16, 32 or 64 (got %d)", t.dir_per_wave);
    if (t.waves < 1 || t.waves > 8)
        return fail(RAD_ERR_INVALID_ARG, "waves must be in 1..8 (got %d)", t.waves);
    if (t.wg_per_cu < 1 || t.wg_per_cu > 16)
        return fail(RAD_ERR_INVALID_ARG, "wg_per_cu must be in 1..16 (got %d)", t.wg_per_cu);
    if (rad::acc_lds_bytes(shape_of(t)) > 160 * 1024)
        return fail(RAD_ERR_INVALID_ARG, "tile needs %zu B of LDS (> 160 KiB)",
                    rad::acc_lds_bytes(shape_of(t)));
    return RAD_OK;
}

int ensure_partials(rad_grid* g)
{
    const int64_t need = max_splits(g);
    if (need <= g->part_splits) return RAD_OK;
    if (g->d_part[0] || g->d_part[1]) {
        RAD_HIP(hipDeviceSynchronize());
        for (int b = 0; b < 2; ++b) {
            if (g->d_part[b]) RAD_HIP(hipFree(g->d_part[b]));
            g->d_part[b] = nullptr;
        }
        g->part_splits = 0;
    }
    const size_t bytes = (size_t)need * g->n_omega * g->n_dir * 4 * sizeof(float);
    for (int b = 0; b < 2; ++b) {
        if (hipMalloc(&g->d_part[b], bytes) != hipSuccess) {
            g->d_part[b] = nullptr;
            return fail(RAD_ERR_OOM, "cannot allocate 2 x %zu B of partial sums", bytes);
        }
    }
    g->part_splits = need;
    return RAD_OK;
}

void release_events(rad_grid* g)
{
    for (auto& e : g->ev_acc) { g->ev_pool.push_back(e.first); g->ev_pool.push_back(e.second); }
    for (auto& e : g->ev_fold) { g->ev_pool.push_back(e.first); g->ev_pool.push_back(e.second); }
    g->ev_acc.clear();
    g->ev_fold.clear();
}

hipError_t take_event(rad_grid* g, hipEvent_t* ev)
{
    if (!g->ev_pool.empty()) {
        *ev = g->ev_pool.back();
        g->ev_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

void free_grid(rad_grid* g)
{
    if (!g) return;
    DeviceGuard dg(g->device);
    release_events(g);
    for (hipEvent_t e : g->ev_pool) (void)hipEventDestroy(e);
    g->ev_pool.clear();
    if (g->d_dirs9) (void)hipFree(g->d_dirs9);
    if (g->d_omega) (void)hipFree(g->d_omega);
    if (g->d_gtab) (void)hipFree(g->d_gtab);
    if (g->d_S) (void)hipFree(g->d_S);
    for (int b = 0; b < 2; ++b) {
        if (g->d_part[b]) (void)hipFree(g->d_part[b]);
        if (g->ev_fold_done[b]) (void)hipEventDestroy(g->ev_fold_done[b]);
    }
    if (g->ev_write) (void)hipEventDestroy(g->ev_write);
    if (g->fold_stream) (void)hipStreamDestroy(g->fold_stream);
    if (g->d_err) (void)hipFree(g->d_err);
    if (g->d_out) (void)hipFree(g->d_out);
    if (g->d_g3) (void)hipFree(g->d_g3);
    if (g->d_bstep) (void)hipFree(g->d_bstep);
    delete g;
}

int check_particles(const rad_particles* p)
{
    if (!p) return fail(RAD_ERR_INVALID_ARG, "particles is NULL");
    if (p->dtype != RAD_F32 && p->dtype != RAD_F64)
        return fail(RAD_ERR_INVALID_ARG, "particle dtype must be RAD_F32 or RAD_F64 (got %d)", p->dtype);
    const void* f[10] = {p->x, p->y, p->z, p->bx, p->by, p->bz, p->dbx, p->dby, p->dbz, p->w};
    static const char* names[10] = {"x", "y", "z", "bx", "by", "bz", "dbx", "dby", "dbz", "w"};
    for (int i = 0; i < 10; ++i)
        if (!f[i]) return fail(RAD_ERR_INVALID_ARG, "particle field %s is NULL", names[i]);
    return RAD_OK;
}

void fill_job(rad::Job& j, const rad_grid* g, const rad_particles* p, double t0, int64_t n_per_step,
              const rad_tile& t)
{
    j.f[0] = p->x; j.f[1] = p->y; j.f[2] = p->z;
    j.f[3] = p->bx; j.f[4] = p->by; j.f[5] = p->bz;
    j.f[6] = p->dbx; j.f[7] = p->dby; j.f[8] = p->dbz; j.f[9] = p->w;
    j.n_per_step = n_per_step;
    j.t0 = t0;
    j.dt = g->dt;
    j.dirs9 = g->d_dirs9;
    j.omega = g->d_omega;
    j.gtab = g->d_gtab;
    j.g3 = g->d_g3;
    j.bstep = g->d_bstep;
    j.domega = g->domega;
    j.n_dir = g->n_dir;
    j.n_omega = g->n_omega;
    const int to = rad::tile_omegas(shape_of(t));
    j.tiles_d = (g->n_dir + t.dir_per_wave - 1) / t.dir_per_wave;
    j.tiles_w = (g->n_omega + to - 1) / to;
    j.err = g->d_err;
}

// Cuts particles [0, total) into launches of at most target_splits particle splits of at
// most kMaxPerWorkgroup particles each, and sets a's particle range, split count and
// chunks per split for each launch before calling fn() (which returns a status code).
template <typename Fn>
int for_each_launch(AccArgs& a, int64_t total, int64_t target_splits, Fn fn)
{
    const int64_t per_launch_cap = target_splits * kMaxPerWorkgroup;
    for (int64_t i0 = 0; i0 < total; i0 += per_launch_cap) {
        const int64_t i1 = std::min(total, i0 + per_launch_cap);
        const int64_t nchunks = (i1 - i0 + rad::kChunk - 1) / rad::kChunk;
        int64_t splits = std::min<int64_t>(target_splits, nchunks);
        const int64_t cps = (nchunks + splits - 1) / splits;
        splits = (nchunks + cps - 1) / cps;
        a.job.i_begin = i0;
        a.job.i_end = i1;
        a.splits = (int32_t)splits;
        a.chunks_per_split = cps;
        if (int rc = fn()) return rc;
    }
    return RAD_OK;
}

// Accumulate particles [0, total) (step of element i is i / n_per_step, t = t0 + step*dt).
int push_range(rad_grid* g, double t0, int64_t n_per_step, int64_t total, const rad_particles* p,
               hipStream_t st)
{
    int rc = ensure_partials(g);
    if (rc) return rc;
    const LaunchShape ls = shape_of(g->tile, g->variant);
    const int td = tiles_d(g), tw = tiles_w(g), nt = td * tw;
    const int64_t count = (int64_t)g->n_omega * g->n_dir * 4;
    const int64_t target_splits = max_splits(g);   // <= part_splits (capacity may be larger)
    AccArgs a{};
    fill_job(a.job, g, p, t0, n_per_step, g->tile);
    return for_each_launch(a, total, target_splits, [&]() -> int {
        const int64_t i0 = a.job.i_begin, i1 = a.job.i_end, splits = a.splits;
        const int b = g->part_next;
        g->part_next ^= 1;
        a.part = g->d_part[b];
        // the fold that last read this buffer must be done before it is overwritten (stream
        // order already guarantees it when that event was recorded on this stream)
        if (g->fold_recorded[b] && g->fold_done_on[b] != st) RAD_HIP(hipStreamWaitEvent(st, g->ev_fold_done[b], 0));
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
        if (g->profiling && g->prof_count++ % g->prof_period == 0) {
            RAD_HIP(take_event(g, &e0));
            RAD_HIP(take_event(g, &e1));
            RAD_HIP(take_event(g, &e2));
            RAD_HIP(take_event(g, &e3));
            g->ev_acc.emplace_back(e0, e1);
            g->ev_fold.emplace_back(e2, e3);
            g->prof_updates += (i1 - i0) * (int64_t)g->n_dir * g->n_omega;
        }
        hipError_t e = rad::launch_accumulate(a, p->dtype, g->precision, ls, (int)(splits * nt), st, e0, e1);
        if (e != hipSuccess) return hip_fail(e, "accumulate launch");
        // The fold runs right after the accumulate on the caller's stream, so it has the
        // whole GPU for its few microseconds (beside the next push's accumulate it would
        // trickle along in the few free wave slots).  It comes after every fold already
        // issued for this grid, on whatever stream, and the grid's fold stream -- the
        // ordering point of batched folds, resets and read-outs -- is chained behind it.
        // The fold's completion event is stamped by the fold launch itself (no separate
        // marker between this fold and the next push's accumulate: 0.4 % of the whole job
        // for per-step pushes); a timed fold stamps its timing event and records it after.
        if (g->last_fold >= 0 && g->fold_done_on[g->last_fold] != st)
            RAD_HIP(hipStreamWaitEvent(st, g->ev_fold_done[g->last_fold], 0));
        e = rad::launch_fold(g->d_part[b], g->d_S, (int)splits, count, st, e2, e3 ? e3 : g->ev_fold_done[b]);
        if (e != hipSuccess) return hip_fail(e, "fold launch");
        if (e3) RAD_HIP(hipEventRecord(g->ev_fold_done[b], st));
        RAD_HIP(hipStreamWaitEvent(g->fold_stream, g->ev_fold_done[b], 0));
        g->fold_done_on[b] = st;
        g->fold_recorded[b] = true;
        g->last_fold = b;
        return RAD_OK;
    });
}

// Make `st` wait for every fold already enqueued (the fold stream is in order, so the
// last one suffices).  Every call that touches the accumulator S on `st` does this first.
int after_folds(rad_grid* g, hipStream_t st)
{
    if (g->last_fold >= 0 && g->fold_done_on[g->last_fold] != st)
        RAD_HIP(hipStreamWaitEvent(st, g->ev_fold_done[g->last_fold], 0));
    return RAD_OK;
}

// S was just written (a batched fold, a reset) or read (a device read-out) on stream
// `origin` up to `ev`, after every earlier fold: later folds, resets and read-outs must come
// after it.  Chain the fold stream behind `ev` and move the last-fold mark there, owned by
// `origin`: later calls on `origin` are ordered by the stream itself and skip the wait (a
// wait on the fold stream's event costs a round trip through another hardware queue, about
// 0.1 ms), calls on any other stream wait for the fold stream's event.
int chain_fold_stream(rad_grid* g, hipEvent_t ev, hipStream_t origin)
{
    RAD_HIP(hipStreamWaitEvent(g->fold_stream, ev, 0));
    const int k = g->last_fold >= 0 ? g->last_fold : 0;
    RAD_HIP(hipEventRecord(g->ev_fold_done[k], g->fold_stream));
    g->fold_done_on[k] = origin;
    g->fold_recorded[k] = true;
    g->last_fold = k;
    return RAD_OK;
}

int read_err_flag(rad_grid* g, hipStream_t st, int* flag)
{
    RAD_HIP(hipMemcpyAsync(flag, g->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
}

}  // namespace

namespace {

// Validated host-side tables of a grid description: directions with their normal basis
// (n, e1, e2), the frequency list, the walk step, the Eq. 13 prefactor and the
// kernel variant.  check_shape = false skips the shape fields (chosen later).
struct GridTables {
    std::vector<double> dirs9, om;
    std::vector<double> bstep;   // per 16-frequency block spacing (piecewise-uniform lists)
    double domega = 0.0, C = 0.0;
    int variant = 0;
};

// How an explicit frequency list can be evaluated.  A list whose every aligned block of
// kBlockW frequencies is an arithmetic progression (to a few FP64 ulps) runs the frequency
// walk with a per-block step; if the steps also agree and the blocks continue one
// another, the list is one uniform grid.  Otherwise each term takes its own FP64 phase.
int classify_list(const std::vector<double>& om, std::vector<double>& bstep, double& domega)
{
    const int n = (int)om.size(), W = rad::kBlockW;
    const int nb = (n + W - 1) / W;
    bstep.assign((size_t)nb, 0.0);
    auto close = [](double a, double b) {
        const double tol = 16.0 * 2.220446049250313e-16 * std::max(std::fabs(a), std::fabs(b));
        return std::fabs(a - b) <= tol;
    };
    for (int b = 0; b < nb; ++b) {
        const int k0 = b * W, k1 = std::min(n, k0 + W);
        if (k1 - k0 < 2) continue;
        const double st = (om[k1 - 1] - om[k0]) / (double)(k1 - 1 - k0);
        for (int k = k0 + 2; k < k1; ++k)
            if (!close(om[k], om[k0] + (double)(k - k0) * st)) return rad::kVarDirect;
        bstep[b] = st;
    }
    if (n >= 2) {
        const double st = (om[n - 1] - om[0]) / (double)(n - 1);
        bool uniform = true;
        for (int k = 2; k < n && uniform; ++k) uniform = close(om[k], om[0] + (double)k * st);
        if (uniform) {
            domega = st;
            return 0;
        }
    } else {
        domega = 0.0;
        return 0;
    }
    return rad::kVarBlockStep;
}

int prepare_tables(const rad_grid_desc* d, bool check_shape, GridTables& tb)
{
    if (d->n_dir < 1 || !d->dirs) return fail(RAD_ERR_INVALID_ARG, "need n_dir >= 1 and dirs");
    if (d->n_omega < 1) return fail(RAD_ERR_INVALID_ARG, "need n_omega >= 1");
    if (d->omegas) {
        for (int k = 0; k < d->n_omega; ++k)
            if (!(d->omegas[k] >= 0.0) || !std::isfinite(d->omegas[k]))
                return fail(RAD_ERR_INVALID_ARG, "omegas[%d] must be finite and >= 0", k);
    } else if (!(d->omega0 >= 0.0) || !std::isfinite(d->omega0) || !(d->domega >= 0.0) || !std::isfinite(d->domega)) {
        return fail(RAD_ERR_INVALID_ARG, "omega0 and domega must be finite and >= 0");
    }
    if (check_shape) {
        if (d->shape < RAD_SHAPE_POINT || d->shape > RAD_SHAPE_QSC3D)
            return fail(RAD_ERR_INVALID_ARG, "unknown shape %d", d->shape);
        if (d->shape != RAD_SHAPE_POINT && !(d->shape_len > 0.0 && std::isfinite(d->shape_len)))
            return fail(RAD_ERR_INVALID_ARG, "shape_len must be finite and > 0");
    }
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(RAD_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (d->precision != RAD_PHASE_F64 && d->precision != RAD_ALL_F32)
        return fail(RAD_ERR_INVALID_ARG, "unknown precision mode %d", d->precision);
    const int64_t points = (int64_t)d->n_dir * d->n_omega;
    if (points > (int64_t)1 << 28) return fail(RAD_ERR_INVALID_ARG, "grid of %lld points too large", (long long)points);
    tb.dirs9.resize((size_t)d->n_dir * 9);
    for (int i = 0; i < d->n_dir; ++i) {
        const double* n = d->dirs + 3 * i;
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!std::isfinite(len) || std::fabs(len - 1.0) > 1e-6)
            return fail(RAD_ERR_INVALID_ARG, "direction %d is not a unit vector (|n| = %.17g)", i, len);
        double* o = tb.dirs9.data() + 9 * i;
        o[0] = n[0]; o[1] = n[1]; o[2] = n[2];
        normal_basis(n, o + 3, o + 6);
    }
    tb.om.resize((size_t)d->n_omega);
    for (int k = 0; k < d->n_omega; ++k) {
        if (d->omegas) {
            tb.om[k] = d->omegas[k];
        } else {
            volatile double kd = (double)k * d->domega;  // one rounding per operation, no fma
            tb.om[k] = d->omega0 + kd;
        }
    }
    tb.domega = d->domega;
    const int list_kind = d->omegas ? classify_list(tb.om, tb.bstep, tb.domega) : 0;
    if (list_kind != rad::kVarBlockStep) tb.bstep.clear();
    if (list_kind == rad::kVarDirect) tb.domega = 0.0;
    const double q = kQe * d->dt;
    tb.C = q * q / (16.0 * kPi * kPi * kPi * kEps0 * kC);
    tb.variant = list_kind | (check_shape && is_shape3(d->shape) ? rad::kVarShape3 : 0);
    return RAD_OK;
}

}  // namespace

void rad::set_last_error(const char* msg) { t_last_error = msg ? msg : ""; }

extern "C" {

const char* rad_last_error(void) { return t_last_error.c_str(); }

int rad_device_cus(int32_t device)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(RAD_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, n);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    return cus;
}

int rad_create_grid(rad_grid** out, const rad_grid_desc* d)
{
    if (!out || !d) return fail(RAD_ERR_INVALID_ARG, "out and desc must be non-NULL");
    GridTables tb;
    int vrc = prepare_tables(d, true, tb);
    if (vrc) return vrc;
    const int64_t points = (int64_t)d->n_dir * d->n_omega;
    std::vector<double>& dirs9 = tb.dirs9;
    const int cus = rad_device_cus(d->device);
    if (cus < 0) return cus;

    rad_grid* g = new rad_grid;
    g->device = d->device;
    g->n_dir = d->n_dir;
    g->n_omega = d->n_omega;
    g->omega0 = d->omega0;
    g->domega = d->domega;
    g->dt = d->dt;
    g->shape = d->shape;
    g->shape_len = d->shape_len;
    g->precision = d->precision;
    g->cus = cus;
    g->C = tb.C;
    g->variant = tb.variant;
    g->domega = tb.domega;
    g->tile = default_tile(d->n_dir, d->n_omega, g->variant);

    std::vector<double>& om = tb.om;
    std::vector<float2> gt((size_t)d->n_omega);
    for (int k = 0; k < d->n_omega; ++k) {
        const double gg = is_shape3(d->shape) ? 0.0 : shape_factor(d->shape, d->shape_len, om[k]);
        gt[k] = make_float2((float)gg, (float)(1.0 - gg));
    }
    std::vector<float> g3;
    if (is_shape3(d->shape)) {
        g3.resize((size_t)points);
        for (int i = 0; i < d->n_dir; ++i)
            for (int k = 0; k < d->n_omega; ++k)
                g3[(size_t)i * d->n_omega + k] = (float)shape_factor3(d->shape, d->shape_len, d->dirs + 3 * i, om[k]);
    }

    DeviceGuard dg(g->device);
    if (int rs = scratch_setup(g->device)) {
        free_grid(g);
        return rs;
    }
    const size_t sbytes = (size_t)points * 4 * sizeof(double);
    if (hipMalloc(&g->d_dirs9, dirs9.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&g->d_omega, om.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&g->d_gtab, gt.size() * sizeof(float2)) != hipSuccess ||
        hipMalloc(&g->d_S, sbytes) != hipSuccess ||
        hipMalloc(&g->d_err, sizeof(int)) != hipSuccess ||
        hipMalloc(&g->d_out, (size_t)points * 6 * sizeof(double)) != hipSuccess ||
        (!g3.empty() && hipMalloc(&g->d_g3, g3.size() * sizeof(float)) != hipSuccess) ||
        (!tb.bstep.empty() && hipMalloc(&g->d_bstep, tb.bstep.size() * sizeof(double)) != hipSuccess)) {
        free_grid(g);
        return fail(RAD_ERR_OOM, "device allocation failed for a %lld-point grid", (long long)points);
    }
    int rc = ensure_partials(g);
    if (rc) { free_grid(g); return rc; }
    if (hipStreamCreateWithFlags(&g->fold_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_fold_done[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_fold_done[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_write, hipEventDisableTiming) != hipSuccess) {
        free_grid(g);
        return fail(RAD_ERR_DEVICE, "cannot create the grid's fold stream and events");
    }
    hipError_t e;
    if ((e = hipMemcpy(g->d_dirs9, dirs9.data(), dirs9.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(g->d_omega, om.data(), om.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(g->d_gtab, gt.data(), gt.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
        (!g3.empty() && (e = hipMemcpy(g->d_g3, g3.data(), g3.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) ||
        (!tb.bstep.empty() &&
         (e = hipMemcpy(g->d_bstep, tb.bstep.data(), tb.bstep.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = rad::launch_fill(g->d_S, points * 4, 0.0, nullptr)) != hipSuccess ||
        (e = rad::launch_fill_int(g->d_err, 1, 0, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess) {
        free_grid(g);
        return hip_fail(e, "grid initialisation");
    }
    *out = g;
    return RAD_OK;
}

int rad_destroy_grid(rad_grid* g)
{
    if (!g) return RAD_OK;
    {
        DeviceGuard dg(g->device);
        (void)hipDeviceSynchronize();
    }
    free_grid(g);
    return RAD_OK;
}

int rad_reset(rad_grid* g, void* stream)
{
    if (!g) return fail(RAD_ERR_INVALID_ARG, "grid is NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc0 = after_folds(g, st)) return rc0;
    hipError_t e = rad::launch_fill(g->d_S, (int64_t)g->n_dir * g->n_omega * 4, 0.0, st);
    if (e == hipSuccess) e = rad::launch_fill_int(g->d_err, 1, 0, st);
    if (e == hipSuccess) e = hipEventRecord(g->ev_write, st);
    if (e != hipSuccess) return hip_fail(e, "reset");
    return chain_fold_stream(g, g->ev_write, st);
}

int rad_push_step(rad_grid* g, double t, int64_t n_particles, const rad_particles* p, void* stream)
{
    if (!g) return fail(RAD_ERR_INVALID_ARG, "grid is NULL");
    if (n_particles < 0) return fail(RAD_ERR_INVALID_ARG, "n_particles < 0");
    if (!std::isfinite(t)) return fail(RAD_ERR_INVALID_ARG, "t is not finite");
    if (n_particles == 0) return RAD_OK;
    int rc = check_particles(p);
    if (rc) return rc;
    DeviceGuard dg(g->device);
    return push_range(g, t, n_particles, n_particles, p, (hipStream_t)stream);
}

int rad_push_steps(rad_grid* g, double t0, int32_t n_steps, int64_t n_particles,
                   const rad_particles* p, void* stream)
{
    if (!g) return fail(RAD_ERR_INVALID_ARG, "grid is NULL");
    if (n_particles < 0 || n_steps < 0) return fail(RAD_ERR_INVALID_ARG, "negative size");
    if (!std::isfinite(t0)) return fail(RAD_ERR_INVALID_ARG, "t0 is not finite");
    if (n_particles == 0 || n_steps == 0) return RAD_OK;
    int rc = check_particles(p);
    if (rc) return rc;
    DeviceGuard dg(g->device);
    return push_range(g, t0, n_particles, (int64_t)n_steps * n_particles, p, (hipStream_t)stream);
}

int rad_push_step_noalloc(rad_grid* g, double t, int64_t n_particles, const rad_particles* p, void* stream)
{
    if (!g) return fail(RAD_ERR_INVALID_ARG, "grid is NULL");
    if (n_particles < 0) return fail(RAD_ERR_INVALID_ARG, "n_particles < 0");
    if (!std::isfinite(t)) return fail(RAD_ERR_INVALID_ARG, "t is not finite");
    if (n_particles == 0) return RAD_OK;
    int rc = check_particles(p);
    if (rc) return rc;
    const int64_t count = (int64_t)g->n_omega * g->n_dir * 4;        // FP32 values per split
    const int64_t split_bytes = count * (int64_t)sizeof(float);
    const int64_t cap_splits = (int64_t)(RAD_NOALLOC_SCRATCH_BYTES / (size_t)split_bytes);
    if (cap_splits < 1)
        return fail(RAD_ERR_INVALID_ARG,
                    "grid of %lld points needs %lld B of partial sums, more than the %zu B no-allocation "
                    "scratch (at most %zu points)", (long long)(count / 4), (long long)split_bytes,
                    (size_t)RAD_NOALLOC_SCRATCH_BYTES, (size_t)RAD_NOALLOC_SCRATCH_BYTES / 16);
    DeviceGuard dg(g->device);
    float* scr = g->device >= 0 && g->device < kScratchDevices
                     ? g_scratch_addr[g->device].load(std::memory_order_acquire) : nullptr;
    if (!scr) return fail(RAD_ERR_DEVICE, "no-allocation scratch not set up on device %d", g->device);
    hipStream_t st = (hipStream_t)stream;
    // Under stream capture the call records no event and waits on none (a wait on an event
    // recorded outside the capture, or another stream waiting on the capture, would break
    // it): the caller orders the captured push against the grid's other work.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    RAD_HIP(hipStreamIsCapturing(st, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    // every fold of this grid runs in issue order: the folds below come after every fold
    // already issued (on any stream), later folds, read-outs and resets after them
    if (!capturing) {
        if (int rc0 = after_folds(g, st)) return rc0;
    }
    const LaunchShape ls = shape_of(g->tile, g->variant);
    const int nt = tiles_d(g) * tiles_w(g);
    AccArgs a{};
    fill_job(a.job, g, p, t, n_particles, g->tile);
    a.part = scr;
    rc = for_each_launch(a, n_particles, std::min<int64_t>(max_splits(g), cap_splits), [&]() -> int {
        // same stream: a launch's accumulate rewrites the scratch only after the previous
        // launch's fold has read it
        hipError_t e = rad::launch_accumulate(a, p->dtype, g->precision, ls, (int)(a.splits * nt), st);
        if (e != hipSuccess) return hip_fail(e, "accumulate launch");
        e = rad::launch_fold(scr, g->d_S, a.splits, count, st);
        if (e != hipSuccess) return hip_fail(e, "fold launch");
        return RAD_OK;
    });
    if (rc) return rc;
    if (capturing) return RAD_OK;
    RAD_HIP(hipEventRecord(g->ev_write, st));
    return chain_fold_stream(g, g->ev_write, st);
}

int rad_spectrum_device(rad_grid* g, double* I_dev, void* stream)
{
    if (!g || !I_dev) return fail(RAD_ERR_INVALID_ARG, "grid and output must be non-NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc0 = after_folds(g, st)) return rc0;
    hipError_t e = rad::launch_finalize(g->d_S, I_dev, g->n_dir, g->n_omega, g->C, st);
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
    // The read-out does not synchronise: later folds and resets, on any stream, must not
    // write S before it has been read, so the read-out becomes the grid's last-write mark.
    RAD_HIP(hipEventRecord(g->ev_write, st));
    return chain_fold_stream(g, g->ev_write, st);
}

int rad_spectrum(rad_grid* g, double* I_host, void* stream)
{
    if (!g || !I_host) return fail(RAD_ERR_INVALID_ARG, "grid and output must be non-NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc0 = after_folds(g, st)) return rc0;
    hipError_t e = rad::launch_finalize(g->d_S, g->d_out, g->n_dir, g->n_omega, g->C, st);
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
    int flag = 0;
    int rc = read_err_flag(g, st, &flag);
    if (rc) return rc;
    if (flag) return fail(RAD_ERR_BAD_DATA, "device detected invalid particle data (non-finite, N < 0 or 1 - beta.n <= 0)");
    RAD_HIP(hipMemcpyAsync(I_host, g->d_out, (size_t)g->n_dir * g->n_omega * sizeof(double),
                           hipMemcpyDeviceToHost, st));
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
}

int rad_spectrum_complex(rad_grid* g, double* S_host, void* stream)
{
    if (!g || !S_host) return fail(RAD_ERR_INVALID_ARG, "grid and output must be non-NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc0 = after_folds(g, st)) return rc0;
    hipError_t e = rad::launch_cartesian(g->d_S, g->d_dirs9, g->d_out, g->n_dir, g->n_omega, st);
    if (e != hipSuccess) return hip_fail(e, "cartesian launch");
    int flag = 0;
    int rc = read_err_flag(g, st, &flag);
    if (rc) return rc;
    if (flag) return fail(RAD_ERR_BAD_DATA, "device detected invalid particle data");
    RAD_HIP(hipMemcpyAsync(S_host, g->d_out, (size_t)g->n_dir * g->n_omega * 6 * sizeof(double),
                           hipMemcpyDeviceToHost, st));
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
}

size_t rad_state_size(const rad_grid* g)
{
    return g ? (size_t)g->n_dir * g->n_omega * 4 : 0;
}

int rad_get_state(rad_grid* g, double* state_host, void* stream)
{
    if (!g || !state_host) return fail(RAD_ERR_INVALID_ARG, "grid and state must be non-NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc0 = after_folds(g, st)) return rc0;
    int flag = 0;
    int rc = read_err_flag(g, st, &flag);
    if (rc) return rc;
    if (flag) return fail(RAD_ERR_BAD_DATA, "device detected invalid particle data");
    RAD_HIP(hipMemcpyAsync(state_host, g->d_S, rad_state_size(g) * sizeof(double), hipMemcpyDeviceToHost, st));
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
}

int rad_set_state(rad_grid* g, const double* state_host, void* stream)
{
    if (!g || !state_host) return fail(RAD_ERR_INVALID_ARG, "grid and state must be non-NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc0 = after_folds(g, st)) return rc0;
    RAD_HIP(hipMemcpyAsync(g->d_S, state_host, rad_state_size(g) * sizeof(double), hipMemcpyHostToDevice, st));
    hipError_t e = rad::launch_fill_int(g->d_err, 1, 0, st);
    if (e != hipSuccess) return hip_fail(e, "set_state");
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
}

int rad_grid_variant(const rad_grid* g)
{
    if (!g) return fail(RAD_ERR_INVALID_ARG, "grid is NULL");
    return g->variant;
}

int rad_get_tile(const rad_grid* g, rad_tile* t)
{
    if (!g || !t) return fail(RAD_ERR_INVALID_ARG, "grid and tile must be non-NULL");
    *t = g->tile;
    return RAD_OK;
}

int rad_set_tile(rad_grid* g, const rad_tile* t)
{
    if (!g || !t) return fail(RAD_ERR_INVALID_ARG, "grid and tile must be non-NULL");
    int rc = validate_tile(*t);
    if (rc) return rc;
    if (g->variant != 0 && t->w_per_lane != 16)
        return fail(RAD_ERR_INVALID_ARG, "grids with a frequency list or a 3-D shape need w_per_lane = 16");
    DeviceGuard dg(g->device);
    const rad_tile old = g->tile;
    g->tile = *t;
    rc = ensure_partials(g);
    if (rc) g->tile = old;
    return rc;
}

}  // extern "C"

#include "rad_debug.h"

extern "C" int rad_debug_trig_probe(const float* in_dev, float* out_dev, int n, void* stream)
{
    if (n < 0 || (n > 0 && (!in_dev || !out_dev))) return fail(RAD_ERR_INVALID_ARG, "bad probe arguments");
    hipError_t e = rad::launch_trig_probe(in_dev, out_dev, n, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "trig probe launch");
    return RAD_OK;
}

extern "C" int rad_profile_enable(rad_grid* g, int enable)
{
    if (!g) return fail(RAD_ERR_INVALID_ARG, "grid is NULL");
    DeviceGuard dg(g->device);
    release_events(g);
    g->prof_updates = 0;
    g->profiling = enable > 0;
    g->prof_period = enable > 0 ? enable : 1;
    g->prof_count = 0;
    return RAD_OK;
}

extern "C" int rad_profile_read(rad_grid* g, rad_profile_stats* out)
{
    if (!g || !out) return fail(RAD_ERR_INVALID_ARG, "grid and stats must be non-NULL");
    DeviceGuard dg(g->device);
    rad_profile_stats s{};
    for (auto& e : g->ev_acc) {
        RAD_HIP(hipEventSynchronize(e.second));
        float ms = 0.f;
        RAD_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        s.accumulate_ms += ms;
        s.launches += 1;
    }
    for (auto& e : g->ev_fold) {
        RAD_HIP(hipEventSynchronize(e.second));
        float ms = 0.f;
        RAD_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        s.fold_ms += ms;
    }
    s.updates = g->prof_updates;
    g->prof_updates = 0;
    release_events(g);
    *out = s;
    return RAD_OK;
}

// ---------------------------------------------------------------------------------------
// Batched launches over several grids.
// ---------------------------------------------------------------------------------------
#include <map>
#include <utility>

struct BatchGraphKey {
    int dtype, precision, w, dpw, waves, R, slot;
    bool operator==(const BatchGraphKey& o) const
    {
        return dtype == o.dtype && precision == o.precision && w == o.w && dpw == o.dpw && waves == o.waves &&
               R == o.R && slot == o.slot;
    }
};

struct BatchGraph {
    BatchGraphKey key;
    int64_t gen;
    hipGraphExec_t exec;
};

struct rad_batcher {
    int device = 0;
    int max_items = 0;
    int cus = 0;
    // Two plan buffers (pinned host + device); a plan buffer is rewritten only after the
    // launch that read it two pushes earlier has finished (event `done`).
    struct Slot {
        unsigned char* host = nullptr;
        unsigned char* dev = nullptr;
        size_t cap = 0;
        hipEvent_t done = nullptr;
        bool used = false;
    } slot[2];
    int next = 0;
    float* seg_part = nullptr;
    size_t seg_part_floats = 0;
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_acc, ev_fold;
    std::vector<hipEvent_t> ev_pool;
    int64_t prof_updates = 0;
    // graph mode: captured [plan upload -> accumulate -> fold] per launch configuration
    bool tile_set = false;       // launch shape of the batched kernel (else the built-in
    rad_tile tile{};             // heuristic for the first item's grid shape)
    bool graph_mode = false;
    hipStream_t cap_stream = nullptr;
    std::vector<BatchGraph> graphs;
    int64_t graph_gen = 0;
    int64_t graph_launches = 0;
    int64_t graph_failures = 0;
};

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

hipError_t batch_event(rad_batcher* b, hipEvent_t* ev)
{
    if (!b->ev_pool.empty()) {
        *ev = b->ev_pool.back();
        b->ev_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

void batch_release_events(rad_batcher* b)
{
    for (auto& e : b->ev_acc) { b->ev_pool.push_back(e.first); b->ev_pool.push_back(e.second); }
    for (auto& e : b->ev_fold) { b->ev_pool.push_back(e.first); b->ev_pool.push_back(e.second); }
    b->ev_acc.clear();
    b->ev_fold.clear();
}

void free_batcher(rad_batcher* b)
{
    if (!b) return;
    DeviceGuard dg(b->device);
    for (auto& s : b->slot) {
        if (s.done) (void)hipEventSynchronize(s.done);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        if (s.done) (void)hipEventDestroy(s.done);
    }
    if (b->seg_part) (void)hipFree(b->seg_part);
    for (auto& ge : b->graphs) (void)hipGraphExecDestroy(ge.exec);
    b->graphs.clear();
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    batch_release_events(b);
    for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
    delete b;
}

struct ItemInfo {
    rad::Job job;
    int64_t chunks = 0;
    int64_t iters = 0;     // tiles * chunks
    int64_t iter_begin = 0;
    rad_grid* grid = nullptr;
};

// One launch's plan over the global iteration range [L0, L1).
struct LaunchPlan {
    std::vector<int32_t> wg_seg_begin;
    std::vector<rad::BatchSeg> segs;
    std::vector<rad::FoldJob> jobs;
    std::vector<int32_t> seg_list;
};

void build_plan(const std::vector<ItemInfo>& items, int64_t L0, int64_t L1, int R, LaunchPlan& pl)
{
    pl = LaunchPlan{};
    const int64_t I = L1 - L0;
    size_t it = 0;
    while (it < items.size() && items[it].iter_begin + items[it].iters <= L0) ++it;
    for (int r = 0; r < R; ++r) {
        pl.wg_seg_begin.push_back((int32_t)pl.segs.size());
        int64_t pos = L0 + I * r / R;
        const int64_t end = L0 + I * (r + 1) / R;
        while (pos < end) {
            while (items[it].iter_begin + items[it].iters <= pos) ++it;
            const ItemInfo& in = items[it];
            const int64_t local = pos - in.iter_begin;
            const int64_t tile = local / in.chunks;
            const int64_t c0 = local % in.chunks;
            const int64_t seg_end = std::min(end, in.iter_begin + (tile + 1) * in.chunks);
            pl.segs.push_back(rad::BatchSeg{(int32_t)it, (int32_t)tile, c0, c0 + (seg_end - pos)});
            pos = seg_end;
        }
    }
    pl.wg_seg_begin.push_back((int32_t)pl.segs.size());
    // fold jobs keyed by (grid, tile), segments listed in segment order.  The tile index is
    // in the batch's launch shape (the items' jobs), not the grid's own single-push shape.
    std::map<std::pair<const rad_grid*, int>, std::vector<int32_t>> groups;
    std::vector<std::pair<const rad_grid*, int>> order;
    std::vector<int> order_tiles_d;
    for (size_t sidx = 0; sidx < pl.segs.size(); ++sidx) {
        const auto& sg = pl.segs[sidx];
        auto key = std::make_pair((const rad_grid*)items[sg.item].grid, (int)sg.tile);
        auto f = groups.find(key);
        if (f == groups.end()) {
            order.push_back(key);
            order_tiles_d.push_back(items[sg.item].job.tiles_d);
            groups[key].push_back((int32_t)sidx);
        } else {
            f->second.push_back((int32_t)sidx);
        }
    }
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const auto& key = order[oi];
        const rad_grid* g = key.first;
        const int tdn = order_tiles_d[oi];
        rad::FoldJob fj{};
        fj.S = g->d_S;
        fj.n_dir = g->n_dir;
        fj.n_omega = g->n_omega;
        fj.td = key.second % tdn;
        fj.tw = key.second / tdn;
        fj.list_begin = (int32_t)pl.seg_list.size();
        for (int32_t sidx : groups[key]) pl.seg_list.push_back(sidx);
        fj.list_end = (int32_t)pl.seg_list.size();
        pl.jobs.push_back(fj);
    }
}

}  // namespace

extern "C" int rad_batcher_create(rad_batcher** out, int32_t device, int32_t max_items)
{
    if (!out) return fail(RAD_ERR_INVALID_ARG, "out is NULL");
    if (max_items < 1 || max_items > (1 << 20)) return fail(RAD_ERR_INVALID_ARG, "max_items must be in 1..2^20");
    const int cus = rad_device_cus(device);
    if (cus < 0) return cus;
    rad_batcher* b = new rad_batcher;
    b->device = device;
    b->max_items = max_items;
    b->cus = cus;
    DeviceGuard dg(device);
    for (auto& s : b->slot) {
        if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
            free_batcher(b);
            return fail(RAD_ERR_DEVICE, "cannot create batcher events");
        }
    }
    *out = b;
    return RAD_OK;
}

extern "C" int rad_batcher_destroy(rad_batcher* b)
{
    if (!b) return RAD_OK;
    {
        DeviceGuard dg(b->device);
        (void)hipDeviceSynchronize();
    }
    free_batcher(b);
    return RAD_OK;
}

extern "C" int rad_batcher_push(rad_batcher* b, const rad_batch_item* items, int32_t n_items, void* stream)
{
    if (!b) return fail(RAD_ERR_INVALID_ARG, "batcher is NULL");
    if (n_items < 0 || n_items > b->max_items)
        return fail(RAD_ERR_INVALID_ARG, "n_items %d outside 0..%d", n_items, b->max_items);
    if (n_items > 0 && !items) return fail(RAD_ERR_INVALID_ARG, "items is NULL");
    // validation
    std::vector<ItemInfo> info;
    std::vector<const rad_particles*> items_p;
    const rad_grid* g0 = nullptr;
    int dtype = -1;
    for (int32_t i = 0; i < n_items; ++i) {
        const rad_batch_item& itm = items[i];
        if (!itm.grid) return fail(RAD_ERR_INVALID_ARG, "item %d has no grid", i);
        if (itm.n_steps < 0 || itm.n_particles < 0) return fail(RAD_ERR_INVALID_ARG, "item %d has a negative size", i);
        if (!std::isfinite(itm.t0)) return fail(RAD_ERR_INVALID_ARG, "item %d: t0 is not finite", i);
        if (itm.grid->device != b->device)
            return fail(RAD_ERR_INVALID_ARG, "item %d: grid on device %d, batcher on %d", i, itm.grid->device, b->device);
        if (itm.n_steps == 0 || itm.n_particles == 0) continue;
        int rc = check_particles(&itm.p);
        if (rc) return rc;
        if (!g0) {
            g0 = itm.grid;
            dtype = itm.p.dtype;
        }
        if (itm.p.dtype != dtype) return fail(RAD_ERR_INVALID_ARG, "item %d: particle dtype differs within the batch", i);
        if (itm.grid->precision != g0->precision) return fail(RAD_ERR_INVALID_ARG, "item %d: precision mode differs", i);
        if (itm.grid->variant != g0->variant)
            return fail(RAD_ERR_INVALID_ARG, "item %d: frequency-list / 3-D-shape kind differs within the batch", i);
        ItemInfo in;
        in.grid = itm.grid;
        in.job.i_begin = 0;
        in.job.i_end = (int64_t)itm.n_steps * itm.n_particles;
        in.job.n_per_step = itm.n_particles;
        in.job.t0 = itm.t0;
        in.chunks = (in.job.i_end + rad::kChunk - 1) / rad::kChunk;
        info.push_back(in);
        items_p.push_back(&itm.p);
    }
    if (info.empty()) return RAD_OK;
    const rad_tile btile = b->tile_set ? b->tile : default_tile(g0->n_dir, g0->n_omega, g0->variant);
    if (g0->variant != 0 && btile.w_per_lane != 16)
        return fail(RAD_ERR_INVALID_ARG, "batches of grids with a frequency list or a 3-D shape need w_per_lane = 16");
    for (size_t i = 0; i < info.size(); ++i) {
        ItemInfo& in = info[i];
        const int64_t i_end = in.job.i_end, nps = in.job.n_per_step;
        const double t0 = in.job.t0;
        fill_job(in.job, in.grid, items_p[i], t0, nps, btile);
        in.job.i_begin = 0;
        in.job.i_end = i_end;
        in.iters = in.chunks * (int64_t)in.job.tiles_d * in.job.tiles_w;
    }
    DeviceGuard dg(b->device);
    hipStream_t st = (hipStream_t)stream;
    // earlier single-grid folds of these grids must land before the batch fold
    {
        std::vector<rad_grid*> seen;
        for (const auto& in : info) {
            if (std::find(seen.begin(), seen.end(), in.grid) != seen.end()) continue;
            seen.push_back(in.grid);
            if (int rc = after_folds(in.grid, st)) return rc;
        }
    }
    int64_t I = 0;
    for (auto& in : info) {
        in.iter_begin = I;
        I += in.iters;
    }
    const LaunchShape ls = shape_of(btile, g0->variant);
    const int TD = rad::tile_dirs(ls), TO = rad::tile_omegas(ls);
    const int R_target = std::max(1, b->cus * btile.wg_per_cu);
    const int64_t per_launch = (int64_t)R_target * (kMaxPerWorkgroup / rad::kChunk);
    hipEvent_t last_done = nullptr;
    for (int64_t L0 = 0; L0 < I; L0 += per_launch) {
        const int64_t L1 = std::min(I, L0 + per_launch);
        const int R = (int)std::min<int64_t>(R_target, L1 - L0);
        LaunchPlan pl;
        build_plan(info, L0, L1, R, pl);
        // Plan layout: header {n_items, n_segs, n_jobs, R} | items | wg_seg_begin | segs |
        // jobs | seg_list.  In graph mode the capacities (and the launched grid) are fixed
        // so one captured graph serves every plan that fits.
        const int R_fixed = R_target;
        const size_t segs_cap_g = (size_t)R_fixed + 16 * (size_t)b->max_items;
        bool use_graph = b->graph_mode && pl.segs.size() <= segs_cap_g && pl.jobs.size() <= segs_cap_g &&
                         pl.seg_list.size() <= segs_cap_g;
        const int R_launch = use_graph ? R_fixed : R;
        const size_t items_cap = use_graph ? (size_t)b->max_items : info.size();
        const size_t segs_cap = use_graph ? segs_cap_g : pl.segs.size();
        const size_t jobs_cap = use_graph ? segs_cap_g : pl.jobs.size();
        const size_t list_cap = use_graph ? segs_cap_g : pl.seg_list.size();
        const size_t o_hdr = 0;
        const size_t o_items = 16;
        const size_t o_wsb = align_up(o_items + items_cap * sizeof(rad::Job), 16);
        const size_t o_segs = align_up(o_wsb + ((size_t)R_launch + 1) * sizeof(int32_t), 16);
        const size_t o_jobs = align_up(o_segs + segs_cap * sizeof(rad::BatchSeg), 16);
        const size_t o_list = align_up(o_jobs + jobs_cap * sizeof(rad::FoldJob), 16);
        const size_t bytes = align_up(o_list + list_cap * sizeof(int32_t), 16);
        const int slot_index = b->next;
        auto& sl = b->slot[slot_index];
        b->next ^= 1;
        if (sl.used) RAD_HIP(hipEventSynchronize(sl.done));
        if (bytes > sl.cap) {
            if (sl.host) RAD_HIP(hipHostFree(sl.host));
            if (sl.dev) RAD_HIP(hipFree(sl.dev));
            sl.host = nullptr;
            sl.dev = nullptr;
            sl.cap = 0;
            const size_t cap = std::max<size_t>(bytes * 2, 64 * 1024);
            if (hipHostMalloc((void**)&sl.host, cap, hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void**)&sl.dev, cap) != hipSuccess)
                return fail(RAD_ERR_OOM, "cannot allocate a %zu B batch plan", cap);
            sl.cap = cap;
            b->graph_gen += 1;   // captured graphs refer to the old buffers
        }
        const int32_t hdr[4] = {(int32_t)info.size(), (int32_t)pl.segs.size(), (int32_t)pl.jobs.size(), (int32_t)R};
        std::memcpy(sl.host + o_hdr, hdr, sizeof(hdr));
        for (size_t i = 0; i < info.size(); ++i) std::memcpy(sl.host + o_items + i * sizeof(rad::Job), &info[i].job, sizeof(rad::Job));
        {
            int32_t* wsb = reinterpret_cast<int32_t*>(sl.host + o_wsb);
            std::memcpy(wsb, pl.wg_seg_begin.data(), pl.wg_seg_begin.size() * sizeof(int32_t));
            for (int r = R + 1; r <= R_launch; ++r) wsb[r] = (int32_t)pl.segs.size();   // idle workgroups
        }
        std::memcpy(sl.host + o_segs, pl.segs.data(), pl.segs.size() * sizeof(rad::BatchSeg));
        std::memcpy(sl.host + o_jobs, pl.jobs.data(), pl.jobs.size() * sizeof(rad::FoldJob));
        std::memcpy(sl.host + o_list, pl.seg_list.data(), pl.seg_list.size() * sizeof(int32_t));
        // segment scratch
        const size_t need = segs_cap * (size_t)TD * TO * 4;
        if (need > b->seg_part_floats) {
            if (b->seg_part) {
                RAD_HIP(hipDeviceSynchronize());
                RAD_HIP(hipFree(b->seg_part));
                b->seg_part = nullptr;
                b->seg_part_floats = 0;
            }
            const size_t alloc = need + need / 4;
            if (hipMalloc((void**)&b->seg_part, alloc * sizeof(float)) != hipSuccess)
                return fail(RAD_ERR_OOM, "cannot allocate %zu B of batch partial sums", alloc * sizeof(float));
            b->seg_part_floats = alloc;
            b->graph_gen += 1;
        }
        const rad::Job* d_items = reinterpret_cast<const rad::Job*>(sl.dev + o_items);
        const int32_t* d_wsb = reinterpret_cast<const int32_t*>(sl.dev + o_wsb);
        const rad::BatchSeg* d_segs = reinterpret_cast<const rad::BatchSeg*>(sl.dev + o_segs);
        const int32_t* d_njobs = reinterpret_cast<const int32_t*>(sl.dev + o_hdr) + 2;
        const rad::FoldJob* d_jobs = reinterpret_cast<const rad::FoldJob*>(sl.dev + o_jobs);
        const int32_t* d_list = reinterpret_cast<const int32_t*>(sl.dev + o_list);
        hipGraphExec_t exec = nullptr;
        if (use_graph) {
            const BatchGraphKey key{dtype, g0->precision * 16 + ls.variant, ls.w_per_lane, ls.dir_per_wave, ls.waves,
                                    R_launch, slot_index};
            for (auto& ge : b->graphs)
                if (ge.key == key && ge.gen == b->graph_gen) exec = ge.exec;
            if (!exec) {
                // capture [plan upload -> persistent accumulate -> fold] on the batcher's own stream
                hipGraph_t graph = nullptr;
                hipError_t e = rad::prepare_accumulate_batch(dtype, g0->precision, ls);
                if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    hipError_t e1 = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, b->cap_stream);
                    if (e1 == hipSuccess)
                        e1 = rad::launch_accumulate_batch(d_items, d_wsb, d_segs, b->seg_part, dtype, g0->precision,
                                                          ls, R_launch, b->cap_stream);
                    if (e1 == hipSuccess)
                        e1 = rad::launch_fold_batch(d_njobs, d_jobs, (int)jobs_cap, d_list, b->seg_part, TD, TO,
                                                    b->cap_stream);
                    hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
                    e = e1 != hipSuccess ? e1 : e2;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                if (graph) (void)hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    exec = nullptr;
                    b->graph_mode = false;   // fall back to direct launches from now on
                    b->graph_failures += 1;
                } else {
                    b->graphs.push_back(BatchGraph{key, b->graph_gen, exec});
                }
            }
            use_graph = exec != nullptr;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
        if (b->profiling) {
            RAD_HIP(batch_event(b, &e0));
            RAD_HIP(batch_event(b, &e1));
            RAD_HIP(batch_event(b, &e2));
            RAD_HIP(batch_event(b, &e3));
            b->ev_acc.emplace_back(e0, e1);
            b->ev_fold.emplace_back(e2, e3);
            for (const auto& sg : pl.segs) {
                const ItemInfo& in = info[sg.item];
                const int64_t lo = sg.c_begin * rad::kChunk;
                const int64_t hi = std::min(in.job.i_end, sg.c_end * rad::kChunk);
                const int td = sg.tile % in.job.tiles_d, tw = sg.tile / in.job.tiles_d;
                const int64_t nd = std::min(TD, in.job.n_dir - td * TD);
                const int64_t no = std::min(TO, in.job.n_omega - tw * TO);
                b->prof_updates += (hi - lo) * nd * no;   // in-grid terms only
            }
        }
        if (use_graph) {
            // timing of a replay covers the whole graph (upload, accumulate and fold)
            if (b->profiling) RAD_HIP(hipEventRecord(e0, st));
            RAD_HIP(hipGraphLaunch(exec, st));
            b->graph_launches += 1;
            if (b->profiling) {
                RAD_HIP(hipEventRecord(e1, st));
                RAD_HIP(hipEventRecord(e2, st));
                RAD_HIP(hipEventRecord(e3, st));
            }
        } else {
            RAD_HIP(hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, st));
            if (b->profiling) RAD_HIP(hipEventRecord(e0, st));
            hipError_t e = rad::launch_accumulate_batch(d_items, d_wsb, d_segs, b->seg_part, dtype, g0->precision,
                                                        ls, R_launch, st);
            if (e != hipSuccess) return hip_fail(e, "batch accumulate launch");
            if (b->profiling) {
                RAD_HIP(hipEventRecord(e1, st));
                RAD_HIP(hipEventRecord(e2, st));
            }
            e = rad::launch_fold_batch(d_njobs, d_jobs, (int)jobs_cap, d_list, b->seg_part, TD, TO, st);
            if (e != hipSuccess) return hip_fail(e, "batch fold launch");
            if (b->profiling) RAD_HIP(hipEventRecord(e3, st));
        }
        RAD_HIP(hipEventRecord(sl.done, st));
        sl.used = true;
        last_done = sl.done;
    }
    // Later single-grid folds (on whatever stream pushes them), resets and read-outs must
    // come after this batch's fold: chain each grid's fold stream behind it.
    if (last_done) {
        std::vector<rad_grid*> seen;
        for (const auto& in : info) {
            rad_grid* g = in.grid;
            if (std::find(seen.begin(), seen.end(), g) != seen.end()) continue;
            seen.push_back(g);
            if (int rc = chain_fold_stream(g, last_done, st)) return rc;
        }
    }
    return RAD_OK;
}

extern "C" int rad_batcher_profile_enable(rad_batcher* b, int enable)
{
    if (!b) return fail(RAD_ERR_INVALID_ARG, "batcher is NULL");
    batch_release_events(b);
    b->prof_updates = 0;
    b->profiling = enable != 0;
    return RAD_OK;
}

extern "C" int rad_batcher_profile_read(rad_batcher* b, rad_profile_stats* out)
{
    if (!b || !out) return fail(RAD_ERR_INVALID_ARG, "batcher and stats must be non-NULL");
    DeviceGuard dg(b->device);
    rad_profile_stats s{};
    for (auto& e : b->ev_acc) {
        RAD_HIP(hipEventSynchronize(e.second));
        float ms = 0.f;
        RAD_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        s.accumulate_ms += ms;
        s.launches += 1;
    }
    for (auto& e : b->ev_fold) {
        RAD_HIP(hipEventSynchronize(e.second));
        float ms = 0.f;
        RAD_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        s.fold_ms += ms;
    }
    s.updates = b->prof_updates;
    b->prof_updates = 0;
    batch_release_events(b);
    *out = s;
    return RAD_OK;
}

extern "C" int rad_batcher_set_graph(rad_batcher* b, int enable)
{
    if (!b) return fail(RAD_ERR_INVALID_ARG, "batcher is NULL");
    DeviceGuard dg(b->device);
    if (enable && !b->cap_stream) {
        if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(RAD_ERR_DEVICE, "cannot create the capture stream");
    }
    b->graph_mode = enable != 0;
    return RAD_OK;
}

extern "C" int rad_batcher_graph_stats(rad_batcher* b, int64_t* graphs, int64_t* launches, int64_t* failures)
{
    if (!b) return fail(RAD_ERR_INVALID_ARG, "batcher is NULL");
    if (graphs) *graphs = (int64_t)b->graphs.size();
    if (launches) *launches = b->graph_launches;
    if (failures) *failures = b->graph_failures;
    return RAD_OK;
}

extern "C" int rad_batcher_set_tile(rad_batcher* b, const rad_tile* t)
{
    if (!b) return fail(RAD_ERR_INVALID_ARG, "batcher is NULL");
    if (!t) {
        b->tile_set = false;
        return RAD_OK;
    }
    int rc = validate_tile(*t);
    if (rc) return rc;
    b->tile = *t;
    b->tile_set = true;
    return RAD_OK;
}

extern "C" int rad_batcher_get_tile(rad_batcher* b, rad_tile* t)
{
    if (!b || !t) return fail(RAD_ERR_INVALID_ARG, "batcher and tile must be non-NULL");
    if (!b->tile_set) return fail(RAD_ERR_INVALID_ARG, "no launch shape set (the heuristic for the first item's grid is used)");
    *t = b->tile;
    return RAD_OK;
}

// ---------------------------------------------------------------------------------------
// Post-processing variant: tracked particles with per-particle time integrals.
// ---------------------------------------------------------------------------------------
struct rad_tracked {
    int device = 0;
    int64_t n_particles = 0;
    int n_dir = 0, n_omega = 0;
    double domega = 0, dt = 0, C = 0;
    bool direct = false;
    std::vector<double> dirs, om;
    double* d_dirs9 = nullptr;
    double* d_omega = nullptr;
    double* d_T = nullptr;
    double* d_w = nullptr;
    double* d_g = nullptr;     // n_dir * n_omega shape factors of the last read-out
    double* d_I = nullptr;
    int* d_err = nullptr;
};

namespace {

void free_tracked(rad_tracked* tr)
{
    if (!tr) return;
    DeviceGuard dg(tr->device);
    for (double* p : {tr->d_dirs9, tr->d_omega, tr->d_T, tr->d_w, tr->d_g, tr->d_I})
        if (p) (void)hipFree(p);
    if (tr->d_err) (void)hipFree(tr->d_err);
    delete tr;
}

}  // namespace

extern "C" int rad_tracked_create(rad_tracked** out, const rad_grid_desc* d, int64_t n_particles)
{
    if (!out || !d) return fail(RAD_ERR_INVALID_ARG, "out and desc must be non-NULL");
    if (n_particles < 1) return fail(RAD_ERR_INVALID_ARG, "need n_particles >= 1");
    if (d->precision != RAD_PHASE_F64) return fail(RAD_ERR_INVALID_ARG, "tracked particles use the FP64-phase mode");
    GridTables tb;
    int rc = prepare_tables(d, false, tb);
    if (rc) return rc;
    const int64_t points = (int64_t)d->n_dir * d->n_omega;
    // 32 B per particle and grid point; refuse sizes whose byte count would not fit
    if (n_particles > ((int64_t)1 << 50) / (points * 32))
        return fail(RAD_ERR_INVALID_ARG, "%lld tracked particles x %lld points is too large",
                    (long long)n_particles, (long long)points);
    rad_tracked* tr = new rad_tracked;
    tr->device = d->device;
    tr->n_particles = n_particles;
    tr->n_dir = d->n_dir;
    tr->n_omega = d->n_omega;
    tr->domega = tb.domega;
    tr->dt = d->dt;
    tr->C = tb.C;
    // any non-uniform list takes the per-term phase here (tracked sets are small)
    tr->direct = (tb.variant & (rad::kVarDirect | rad::kVarBlockStep)) != 0;
    if (tr->direct) tr->domega = 0.0;
    tr->dirs.assign(d->dirs, d->dirs + 3 * (size_t)d->n_dir);
    tr->om = tb.om;
    DeviceGuard dg(d->device);
    const size_t tbytes = (size_t)n_particles * points * 4 * sizeof(double);
    if (hipMalloc(&tr->d_dirs9, tb.dirs9.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&tr->d_omega, tb.om.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&tr->d_T, tbytes) != hipSuccess ||
        hipMalloc(&tr->d_w, (size_t)n_particles * sizeof(double)) != hipSuccess ||
        hipMalloc(&tr->d_g, (size_t)points * sizeof(double)) != hipSuccess ||
        hipMalloc(&tr->d_I, (size_t)points * sizeof(double)) != hipSuccess ||
        hipMalloc(&tr->d_err, sizeof(int)) != hipSuccess) {
        free_tracked(tr);
        return fail(RAD_ERR_OOM, "cannot allocate %zu B of per-particle integrals", tbytes);
    }
    hipError_t e;
    if ((e = hipMemcpy(tr->d_dirs9, tb.dirs9.data(), tb.dirs9.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(tr->d_omega, tb.om.data(), tb.om.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = rad::launch_fill(tr->d_T, (int64_t)(tbytes / sizeof(double)), 0.0, nullptr)) != hipSuccess ||
        (e = rad::launch_fill_int(tr->d_err, 1, 0, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
        free_tracked(tr);
        return hip_fail(e, "tracked initialisation");
    }
    *out = tr;
    return RAD_OK;
}

extern "C" int rad_tracked_destroy(rad_tracked* tr)
{
    if (!tr) return RAD_OK;
    {
        DeviceGuard dg(tr->device);
        (void)hipDeviceSynchronize();
    }
    free_tracked(tr);
    return RAD_OK;
}

extern "C" int rad_tracked_reset(rad_tracked* tr, void* stream)
{
    if (!tr) return fail(RAD_ERR_INVALID_ARG, "tracked is NULL");
    DeviceGuard dg(tr->device);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = rad::launch_fill(tr->d_T, tr->n_particles * tr->n_dir * tr->n_omega * 4, 0.0, st);
    if (e == hipSuccess) e = rad::launch_fill_int(tr->d_err, 1, 0, st);
    if (e != hipSuccess) return hip_fail(e, "tracked reset");
    return RAD_OK;
}

namespace {

int tracked_push(rad_tracked* tr, double t0, int32_t n_steps, const rad_particles* p, void* stream)
{
    if (!tr) return fail(RAD_ERR_INVALID_ARG, "tracked is NULL");
    if (!std::isfinite(t0)) return fail(RAD_ERR_INVALID_ARG, "t is not finite");
    if (n_steps < 0) return fail(RAD_ERR_INVALID_ARG, "negative step count");
    if (!p) return fail(RAD_ERR_INVALID_ARG, "particles is NULL");
    if (n_steps == 0) return RAD_OK;
    rad_particles q = *p;
    if (!q.w) q.w = q.x;   // the weight field is not read here
    int rc = check_particles(&q);
    if (rc) return rc;
    DeviceGuard dg(tr->device);
    rad::TrackedArgs a{};
    a.f[0] = p->x; a.f[1] = p->y; a.f[2] = p->z;
    a.f[3] = p->bx; a.f[4] = p->by; a.f[5] = p->bz;
    a.f[6] = p->dbx; a.f[7] = p->dby; a.f[8] = p->dbz; a.f[9] = nullptr;
    a.n_particles = tr->n_particles;
    a.t = t0;
    a.dt = tr->dt;
    a.n_steps = n_steps;
    a.dirs9 = tr->d_dirs9;
    a.omega = tr->d_omega;
    a.domega = tr->domega;
    a.T = tr->d_T;
    a.err = tr->d_err;
    a.n_dir = tr->n_dir;
    a.n_omega = tr->n_omega;
    hipError_t e = rad::launch_tracked_accumulate(a, p->dtype, tr->direct, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "tracked accumulate launch");
    return RAD_OK;
}

}  // namespace

extern "C" int rad_tracked_push_step(rad_tracked* tr, double t, const rad_particles* p, void* stream)
{
    return tracked_push(tr, t, 1, p, stream);
}

namespace rad {
int tracked_step_group();   // rad_kernels.hip
}

extern "C" int rad_tracked_step_group(void) { return rad::tracked_step_group(); }

extern "C" int rad_tracked_push_steps(rad_tracked* tr, double t0, int32_t n_steps, const rad_particles* p,
                                      void* stream)
{
    return tracked_push(tr, t0, n_steps, p, stream);
}

extern "C" int rad_tracked_spectrum(rad_tracked* tr, const double* weights_host, int32_t shape, double shape_len,
                                    double* I_host, void* stream)
{
    if (!tr || !weights_host || !I_host) return fail(RAD_ERR_INVALID_ARG, "NULL argument");
    if (shape < RAD_SHAPE_POINT || shape > RAD_SHAPE_QSC3D) return fail(RAD_ERR_INVALID_ARG, "unknown shape %d", shape);
    if (shape != RAD_SHAPE_POINT && !(shape_len > 0.0 && std::isfinite(shape_len)))
        return fail(RAD_ERR_INVALID_ARG, "shape_len must be finite and > 0");
    for (int64_t m = 0; m < tr->n_particles; ++m)
        if (!(weights_host[m] >= 0.0) || !std::isfinite(weights_host[m]))
            return fail(RAD_ERR_INVALID_ARG, "weight %lld must be finite and >= 0", (long long)m);
    DeviceGuard dg(tr->device);
    hipStream_t st = (hipStream_t)stream;
    const bool s3 = is_shape3(shape);
    std::vector<double> g(s3 ? (size_t)tr->n_dir * tr->n_omega : (size_t)tr->n_omega);
    for (int d = 0; d < (s3 ? tr->n_dir : 1); ++d)
        for (int k = 0; k < tr->n_omega; ++k)
            g[(size_t)d * tr->n_omega + k] = s3 ? shape_factor3(shape, shape_len, tr->dirs.data() + 3 * d, tr->om[k])
                                                : shape_factor(shape, shape_len, tr->om[k]);
    RAD_HIP(hipMemcpyAsync(tr->d_g, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice, st));
    RAD_HIP(hipMemcpyAsync(tr->d_w, weights_host, (size_t)tr->n_particles * sizeof(double), hipMemcpyHostToDevice, st));
    hipError_t e = rad::launch_tracked_finalize(tr->d_T, tr->d_w, s3 ? nullptr : tr->d_g, s3 ? tr->d_g : nullptr,
                                                tr->n_particles, tr->n_dir, tr->n_omega, tr->C, tr->d_I, st);
    if (e != hipSuccess) return hip_fail(e, "tracked finalize launch");
    int flag = 0;
    RAD_HIP(hipMemcpyAsync(&flag, tr->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    RAD_HIP(hipStreamSynchronize(st));
    if (flag) return fail(RAD_ERR_BAD_DATA, "device detected invalid particle data");
    RAD_HIP(hipMemcpyAsync(I_host, tr->d_I, (size_t)tr->n_dir * tr->n_omega * sizeof(double), hipMemcpyDeviceToHost, st));
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
}
