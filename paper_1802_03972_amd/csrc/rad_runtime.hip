// Host runtime of the C ABI declared in include/rad.h: grid lifetime, validation, launch
// shapes, and the stream-ordered push / fold / read-out sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
    float* d_part = nullptr;
    int64_t part_splits = 0;
    int* d_err = nullptr;
    double* d_out = nullptr;
    // kernel timing (rad_profile_*)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_acc, ev_fold;
    int64_t prof_updates = 0;
};

namespace {

// Particles handled per workgroup in one launch at most (bounds the FP32 partial sums;
// longer pushes are cut into several launches, each folded into the FP64 accumulator).
constexpr int64_t kMaxPerWorkgroup = 32768;

LaunchShape shape_of(const rad_tile& t) { return LaunchShape{t.w_per_lane, t.dir_per_wave, t.waves}; }

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

rad_tile default_tile(int n_dir, int n_omega)
{
    rad_tile t{};
    t.dir_per_wave = n_dir <= 16 ? 16 : 32;
    const int subs = 64 / t.dir_per_wave;
    t.w_per_lane = n_omega >= 32 * subs ? 32 : 16;
    const int per_wave = subs * t.w_per_lane;
    t.waves = std::min(8, std::max(1, (n_omega + per_wave - 1) / per_wave));
    // Two waves per SIMD (8 per CU) at ~160-256 VGPRs; LDS also bounds the count.
    const size_t lds = rad::acc_lds_bytes(shape_of(t));
    int by_waves = std::max(1, 8 / t.waves);
    int by_lds = std::max(1, (int)((160 * 1024) / lds));
    t.wg_per_cu = std::min(by_waves, by_lds);
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
    if (g->d_part) {
        RAD_HIP(hipDeviceSynchronize());
        RAD_HIP(hipFree(g->d_part));
        g->d_part = nullptr;
        g->part_splits = 0;
    }
    const size_t bytes = (size_t)need * g->n_omega * g->n_dir * 4 * sizeof(float);
    if (hipMalloc(&g->d_part, bytes) != hipSuccess) {
        g->d_part = nullptr;
        return fail(RAD_ERR_OOM, "cannot allocate %zu B of partial sums", bytes);
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
    if (g->d_part) (void)hipFree(g->d_part);
    if (g->d_err) (void)hipFree(g->d_err);
    if (g->d_out) (void)hipFree(g->d_out);
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

// Accumulate particles [0, total) (step of element i is i / n_per_step, t = t0 + step*dt).
int push_range(rad_grid* g, double t0, int64_t n_per_step, int64_t total, const rad_particles* p,
               hipStream_t st)
{
    int rc = ensure_partials(g);
    if (rc) return rc;
    const LaunchShape ls = shape_of(g->tile);
    const int td = tiles_d(g), tw = tiles_w(g), nt = td * tw;
    const int64_t count = (int64_t)g->n_omega * g->n_dir * 4;
    const int64_t per_launch_cap = (int64_t)g->part_splits * kMaxPerWorkgroup;
    AccArgs a{};
    a.f[0] = p->x; a.f[1] = p->y; a.f[2] = p->z;
    a.f[3] = p->bx; a.f[4] = p->by; a.f[5] = p->bz;
    a.f[6] = p->dbx; a.f[7] = p->dby; a.f[8] = p->dbz; a.f[9] = p->w;
    a.n_per_step = n_per_step;
    a.t0 = t0;
    a.dt = g->dt;
    a.dirs9 = g->d_dirs9;
    a.omega = g->d_omega;
    a.gtab = g->d_gtab;
    a.domega = g->domega;
    a.part = g->d_part;
    a.err = g->d_err;
    a.n_dir = g->n_dir;
    a.n_omega = g->n_omega;
    a.tiles_d = td;
    a.tiles_w = tw;
    for (int64_t i0 = 0; i0 < total; i0 += per_launch_cap) {
        const int64_t i1 = std::min(total, i0 + per_launch_cap);
        const int64_t nchunks = (i1 - i0 + rad::kChunk - 1) / rad::kChunk;
        int64_t splits = std::min<int64_t>(g->part_splits, nchunks);
        const int64_t cps = (nchunks + splits - 1) / splits;
        splits = (nchunks + cps - 1) / cps;
        a.i_begin = i0;
        a.i_end = i1;
        a.splits = (int32_t)splits;
        a.chunks_per_split = cps;
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
        if (g->profiling) {
            RAD_HIP(take_event(g, &e0));
            RAD_HIP(take_event(g, &e1));
            RAD_HIP(take_event(g, &e2));
            RAD_HIP(take_event(g, &e3));
            g->ev_acc.emplace_back(e0, e1);
            g->ev_fold.emplace_back(e2, e3);
            g->prof_updates += (i1 - i0) * (int64_t)g->n_dir * g->n_omega;
            RAD_HIP(hipEventRecord(e0, st));
        }
        hipError_t e = rad::launch_accumulate(a, p->dtype, g->precision, ls, (int)(splits * nt), st);
        if (e != hipSuccess) return hip_fail(e, "accumulate launch");
        if (g->profiling) {
            RAD_HIP(hipEventRecord(e1, st));
            RAD_HIP(hipEventRecord(e2, st));
        }
        e = rad::launch_fold(g->d_part, g->d_S, (int)splits, count, st);
        if (e != hipSuccess) return hip_fail(e, "fold launch");
        if (g->profiling) RAD_HIP(hipEventRecord(e3, st));
    }
    return RAD_OK;
}

int read_err_flag(rad_grid* g, hipStream_t st, int* flag)
{
    RAD_HIP(hipMemcpyAsync(flag, g->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
}

}  // namespace

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
    if (d->n_dir < 1 || !d->dirs) return fail(RAD_ERR_INVALID_ARG, "need n_dir >= 1 and dirs");
    if (d->n_omega < 1) return fail(RAD_ERR_INVALID_ARG, "need n_omega >= 1");
    if (!(d->omega0 >= 0.0) || !std::isfinite(d->omega0) || !(d->domega >= 0.0) || !std::isfinite(d->domega))
        return fail(RAD_ERR_INVALID_ARG, "omega0 and domega must be finite and >= 0");
    if (d->shape < RAD_SHAPE_POINT || d->shape > RAD_SHAPE_GAUSS)
        return fail(RAD_ERR_INVALID_ARG, "unknown shape %d", d->shape);
    if (d->shape != RAD_SHAPE_POINT && !(d->shape_len > 0.0 && std::isfinite(d->shape_len)))
        return fail(RAD_ERR_INVALID_ARG, "shape_len must be finite and > 0");
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(RAD_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (d->precision != RAD_PHASE_F64 && d->precision != RAD_ALL_F32)
        return fail(RAD_ERR_INVALID_ARG, "unknown precision mode %d", d->precision);
    const int64_t points = (int64_t)d->n_dir * d->n_omega;
    if (points > (int64_t)1 << 28) return fail(RAD_ERR_INVALID_ARG, "grid of %lld points too large", (long long)points);
    std::vector<double> dirs9((size_t)d->n_dir * 9);
    for (int i = 0; i < d->n_dir; ++i) {
        const double* n = d->dirs + 3 * i;
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!std::isfinite(len) || std::fabs(len - 1.0) > 1e-6)
            return fail(RAD_ERR_INVALID_ARG, "direction %d is not a unit vector (|n| = %.17g)", i, len);
        double* o = dirs9.data() + 9 * i;
        o[0] = n[0]; o[1] = n[1]; o[2] = n[2];
        normal_basis(n, o + 3, o + 6);
    }
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
    const double q = kQe * d->dt;
    g->C = q * q / (16.0 * kPi * kPi * kPi * kEps0 * kC);
    g->tile = default_tile(d->n_dir, d->n_omega);

    std::vector<double> om((size_t)d->n_omega);
    std::vector<float2> gt((size_t)d->n_omega);
    for (int k = 0; k < d->n_omega; ++k) {
        volatile double kd = (double)k * d->domega;  // one rounding per operation, no fma
        om[k] = d->omega0 + kd;
        const double gg = shape_factor(d->shape, d->shape_len, om[k]);
        gt[k] = make_float2((float)gg, (float)(1.0 - gg));
    }

    DeviceGuard dg(g->device);
    const size_t sbytes = (size_t)points * 4 * sizeof(double);
    if (hipMalloc(&g->d_dirs9, dirs9.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&g->d_omega, om.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&g->d_gtab, gt.size() * sizeof(float2)) != hipSuccess ||
        hipMalloc(&g->d_S, sbytes) != hipSuccess ||
        hipMalloc(&g->d_err, sizeof(int)) != hipSuccess ||
        hipMalloc(&g->d_out, (size_t)points * 6 * sizeof(double)) != hipSuccess) {
        free_grid(g);
        return fail(RAD_ERR_OOM, "device allocation failed for a %lld-point grid", (long long)points);
    }
    int rc = ensure_partials(g);
    if (rc) { free_grid(g); return rc; }
    hipError_t e;
    if ((e = hipMemcpy(g->d_dirs9, dirs9.data(), dirs9.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(g->d_omega, om.data(), om.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(g->d_gtab, gt.data(), gt.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
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
    hipError_t e = rad::launch_fill(g->d_S, (int64_t)g->n_dir * g->n_omega * 4, 0.0, st);
    if (e == hipSuccess) e = rad::launch_fill_int(g->d_err, 1, 0, st);
    if (e != hipSuccess) return hip_fail(e, "reset");
    return RAD_OK;
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

int rad_spectrum_device(rad_grid* g, double* I_dev, void* stream)
{
    if (!g || !I_dev) return fail(RAD_ERR_INVALID_ARG, "grid and output must be non-NULL");
    DeviceGuard dg(g->device);
    hipError_t e = rad::launch_finalize(g->d_S, I_dev, g->n_dir, g->n_omega, g->C, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
    return RAD_OK;
}

int rad_spectrum(rad_grid* g, double* I_host, void* stream)
{
    if (!g || !I_host) return fail(RAD_ERR_INVALID_ARG, "grid and output must be non-NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
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
    RAD_HIP(hipMemcpyAsync(g->d_S, state_host, rad_state_size(g) * sizeof(double), hipMemcpyHostToDevice, st));
    hipError_t e = rad::launch_fill_int(g->d_err, 1, 0, st);
    if (e != hipSuccess) return hip_fail(e, "set_state");
    RAD_HIP(hipStreamSynchronize(st));
    return RAD_OK;
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
    g->profiling = enable != 0;
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
