// Auxiliary gfx950 kernels of the radiation library: the fixed-order FP64 folds of the
// accumulate kernels' FP32 partials, read-out (intensity and Cartesian spectrum), fills,
// the tracked-particle (post-processing) kernels and a transcendental probe.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "rad_device.h"
#include "rad_internal.h"

namespace rad {

namespace {

// ---------------------------------------------------------------------------------------
// Post-processing variant: tracked particles keep their own time integral
// T_m(n, omega) = sum_j A_{j,m}(n) exp(i omega tau_{j,m}) (no form factor) in FP64,
// layout [m][omega][dir][4]; the form factor is applied only when the spectrum is read.
//
// One workgroup of NT threads per (particle, tile of TD directions x OB blocks of
// W = kTrackW frequencies), OB = min(NT / W, smallest power of two >= the number of
// frequency blocks), TD = NT / OB.  The steps of a push are taken S = OB at a
// time: the S x TD (step, direction) geometries (FP64, as in the main path) are computed
// once, one per thread, into LDS, then every thread walks its W frequencies for each of the
// S steps with the main path's three-term walk from the block's middle frequency (or,
// for explicit frequency lists, the per-term FP64 phase).  The per-(step, direction) set-up is thus shared by OB * W
// frequencies.  Up to kStepGroup steps of one push are summed in FP32 registers before one
// read-modify-write of the FP64 integrals, so a multi-step push moves 64 B per particle and
// grid point per group instead of per step (the main path likewise sums hundreds of
// particles in FP32 per partial).  W = 8 (rather than 16) keeps the kernel at 162 VGPRs,
// three waves per SIMD.
// ---------------------------------------------------------------------------------------
constexpr int kStepGroup = 128;
constexpr int kTrackW = 8;
// Workgroup sizes: 256 threads for multi-step pushes, 512 for one-step pushes (measured:
// 512 is 7 % faster on one-step pushes, whose workgroups mostly wait for their integrals,
// and 42 % slower on a 100-step push).
constexpr int kTrackThreads = 256;
constexpr int kTrackThreadsOneStep = 512;

struct TrackedTiling {
    int ob;     // frequency blocks per workgroup (also the steps per sub-chunk)
    int td;     // directions per workgroup
    int n_dt;   // direction tiles
    int n_ot;   // frequency tiles
};

__host__ __device__ inline TrackedTiling tracked_tiling(int n_dir, int n_omega, int nt)
{
    const int max_ob = nt / kTrackW;
    const int n_blocks = (n_omega + kTrackW - 1) / kTrackW;
    int ob = 1;
    while (ob < n_blocks && ob < max_ob) ob *= 2;
    TrackedTiling t;
    t.ob = ob;
    t.td = nt / ob;
    t.n_dt = (n_dir + t.td - 1) / t.td;
    t.n_ot = (n_blocks + ob - 1) / ob;
    return t;
}

// Waves per SIMD the tracked kernel is compiled for: four (at most 128 VGPRs).  It fits
// without spills because the read-modify-write of the integrals keeps only two 32-byte
// loads in flight per thread (eight needed 166 VGPRs, i.e. three waves per SIMD; the
// four-wave build is 6 % faster on 100-step pushes and 8 % on one-step pushes).  More
// waves let one workgroup's read-modify-write overlap another's arithmetic.
#ifndef RAD_TRACK_WAVES
#define RAD_TRACK_WAVES 4
#endif

template <typename InT, bool DIRECT, int NT>
__global__ void __launch_bounds__(NT, RAD_TRACK_WAVES) k_tracked_accumulate(TrackedArgs a)
{
    constexpr int W = kTrackW;
    constexpr int SMAX = NT / kTrackW;
    __shared__ double raw[11 * SMAX];            // [field][step] of the sub-chunk
    __shared__ float4 geo[NT];                   // [step][direction]: A1, A2, w
    __shared__ double tau[NT];                   // [step][direction]: tau / (2 pi)
    const TrackedTiling tl = tracked_tiling(a.n_dir, a.n_omega, NT);
    const int S = tl.ob, TD = tl.td;
    const int tid = threadIdx.x;
    int64_t b = blockIdx.x;
    const int dt = (int)(b % tl.n_dt);
    b /= tl.n_dt;
    const int ot = (int)(b % tl.n_ot);
    const int64_t m = b / tl.n_ot;               // grid: n_particles x n_ot x n_dt workgroups
    const int dl = tid % TD;
    const int d = dt * TD + dl;
    const int dg = d < a.n_dir ? d : a.n_dir - 1;
    const int n_blocks = (a.n_omega + W - 1) / W;
    const int ob = ot * tl.ob + tid / TD;         // this thread's frequency block
    const bool live = d < a.n_dir && ob < n_blocks;
    const int o0 = (ob < n_blocks ? ob : n_blocks - 1) * W;
    const int kmax = a.n_omega - o0 < W ? a.n_omega - o0 : W;
    constexpr int KS = W / 2;                     // seeded frequency of the block
    const double om_seed = a.omega[o0] + (double)KS * a.domega;
    double om[DIRECT ? W : 1];
    if constexpr (DIRECT) {
#pragma unroll
        for (int k = 0; k < W; ++k) om[k] = a.omega[o0 + (k < kmax ? k : kmax - 1)];
    }
    const int ss = tid / TD;                      // set-up role: step ss of the sub-chunk
    constexpr int G = 2;
    double4* T = reinterpret_cast<double4*>(a.T) + (m * a.n_omega + o0) * a.n_dir + d;
    for (int j0 = 0; j0 < a.n_steps; j0 += kStepGroup) {
        const int j1 = a.n_steps - j0 < kStepGroup ? a.n_steps : j0 + kStepGroup;
        float4 acc[W];
#pragma unroll
        for (int k = 0; k < W; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int js = j0; js < j1; js += S) {
            const int ns = j1 - js < S ? j1 - js : S;
            // 1. the particle's states at the sub-chunk's steps (step-major SoA input)
            if (tid < ns) {
                const int64_t i = (int64_t)(js + tid) * a.n_particles + m;
#pragma unroll
                for (int f = 0; f < 9; ++f) raw[f * SMAX + tid] = load_wide<InT>(a.f[f], i);
                raw[9 * SMAX + tid] = 1.0;     // weights enter only at read-out
                raw[10 * SMAX + tid] = a.t + (double)(js + tid) * a.dt;
            }
            __syncthreads();
            // 2. one (step, direction) geometry per thread
            {
                float4 gv = make_float4(0.f, 0.f, 1.f, 0.f);
                double ph = 0.0;
                if (ss < ns)
                    particle_direction_setup<0, !DIRECT, SMAX>(raw, ss, a.dirs9 + 9 * dg, a.domega, gv, ph, a.err);
                geo[tid] = gv;
                tau[tid] = ph;
            }
            __syncthreads();
            // 3. W frequencies per step; raw is rewritten only after every thread has passed
            //    the barrier above, and geo/tau only after the next sub-chunk's first barrier
            for (int s = 0; s < ns; ++s) {
                const float4 gv = geo[s * TD + dl];
                const double ph = tau[s * TD + dl];
                // the three-term walk's sign factors sigma_k ride on A (nA = -A)
                float nA1 = 0.f, nA2 = 0.f;
                if constexpr (!DIRECT) {
                    nA1 = -gv.x;
                    nA2 = -gv.y;
                    asm volatile("" : "+v"(nA1), "+v"(nA2));
                }
                auto add = [&](int k, float xr, float xi) {
                    const float a1 = (!DIRECT && (k & 2)) ? nA1 : gv.x;
                    const float a2 = (!DIRECT && (k & 2)) ? nA2 : gv.y;
                    acc[k].x = fmaf(a1, xr, acc[k].x);
                    acc[k].y = fmaf(a1, xi, acc[k].y);
                    acc[k].z = fmaf(a2, xr, acc[k].z);
                    acc[k].w = fmaf(a2, xi, acc[k].w);
                };
                if constexpr (DIRECT) {
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        float zr, zi;
                        sincos_rev_fast(static_cast<float>(frac_rev(om[k] * ph)), zi, zr);
                        add(k, zr, zi);
                    }
                } else {
                    // the main path's three-term walk on y_k = sigma_k z_k, sigma = (+, +, -, -)
                    // by k mod 4, from the seed at frequency KS (a multiple of 4, so y_KS = z):
                    // forward from (y_KS, y_KS+1 = z w) by y_{k+1} = c_k y_k + y_{k-1}, backward
                    // from (y_KS, y_KS-1 = -c y_KS + y_KS+1) by y_{k-1} = c'_k y_k + y_{k+1};
                    // c = 2 Re(w), c_k = +c / -c and c'_k = -c / +c for even / odd k
                    static_assert(KS % 4 == 0, "the sign pattern assumes y_KS = y_KS+1 = +z");
                    float zr, zi;
                    sincos_rev_fast(static_cast<float>(frac_rev(om_seed * ph)), zi, zr);
                    const float wr = gv.z, wi = gv.w;
                    float pc = 2.f * wr, nc = -2.f * wr;
                    asm volatile("" : "+v"(pc), "+v"(nc));
                    float pr = zr, pi = zi;
                    float cr = fmaf(zr, wr, -(zi * wi)), ci = fmaf(zr, wi, zi * wr);
                    const float ybr = fmaf(nc, zr, cr), ybi = fmaf(nc, zi, ci);
                    add(KS, pr, pi);
                    add(KS + 1, cr, ci);
#pragma unroll
                    for (int k = KS + 1; k < W - 1; ++k) {
                        const float ck = (k & 1) ? nc : pc;
                        const float nr = fmaf(ck, cr, pr), ni = fmaf(ck, ci, pi);
                        pr = cr; pi = ci; cr = nr; ci = ni;
                        add(k + 1, cr, ci);
                    }
                    pr = zr; pi = zi;
                    cr = ybr; ci = ybi;
                    add(KS - 1, cr, ci);
#pragma unroll
                    for (int k = KS - 1; k > 0; --k) {
                        const float ck = (k & 1) ? pc : nc;
                        const float nr = fmaf(ck, cr, pr), ni = fmaf(ck, ci, pi);
                        pr = cr; pi = ci; cr = nr; ci = ni;
                        add(k - 1, cr, ci);
                    }
                }
            }
        }
        // 4. read-modify-write of the integrals, G loads in flight before their stores
        //    (consecutive threads hold consecutive directions: 32 B each, contiguous)
        if (live) {
            // an opaque copy of the stride keeps the W addresses from being hoisted out of
            // the step-group loop (they would stay live through the hot loop)
            int64_t stride = a.n_dir;
            asm volatile("" : "+s"(stride));
#pragma unroll
            for (int q = 0; q < W; q += G) {
                double4 t[G];
#pragma unroll
                for (int u = 0; u < G; ++u)
                    if (q + u < kmax) t[u] = T[(q + u) * stride];
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const int k = q + u;
                    if (k < kmax) {
                        t[u].x += (double)acc[k].x;
                        t[u].y += (double)acc[k].y;
                        t[u].z += (double)acc[k].z;
                        t[u].w += (double)acc[k].w;
                        T[k * stride] = t[u];
                    }
                }
            }
        }
    }
}

// I[d][k] = C |sum_m F_m(d, k) T_m(k, d)|^2 with F_m = sqrt(N_m + (N_m^2 - N_m) g) in FP64;
// g from gk[k] (1-D shape) or g3[d][k] (3-D shape).
__global__ void k_tracked_finalize(const double* __restrict__ T, const double* __restrict__ wts,
                                   const double* __restrict__ gk, const double* __restrict__ g3,
                                   int64_t n_particles, int n_dir, int n_omega, double C,
                                   double* __restrict__ I)
{
    // consecutive threads take consecutive directions, so the reads of T are contiguous
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_dir * n_omega) return;
    const int k = (int)(i / n_dir), d = (int)(i % n_dir);
    const double g = g3 ? g3[(int64_t)d * n_omega + k] : gk[k];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int64_t m = 0; m < n_particles; ++m) {
        const double N = wts[m];
        const double F = sqrt(fmax(N + (N * N - N) * g, 0.0));
        const double* t = T + ((m * n_omega + k) * n_dir + d) * 4;
        s0 += F * t[0]; s1 += F * t[1]; s2 += F * t[2]; s3 += F * t[3];
    }
    I[(int64_t)d * n_omega + k] = C * (s0 * s0 + s1 * s1 + s2 * s2 + s3 * s3);
}

// S[p] += sum over splits of part[s][p] for every grid point p (four components: S1r,
// S1i, S2r, S2i), in split order, in FP64.  One thread per point reads 16 B per split with
// kFoldUnroll loads in flight (the partials are read once: non-temporal loads), so few
// waves keep HBM busy while the next push's accumulate holds the rest of the CUs.
constexpr int kFoldUnroll = 16;
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_fold(const f32x4* __restrict__ part, double* __restrict__ S,
                                              int splits, int64_t points)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= points) return;
    const f32x4* p = part + i;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int k = 0;
    for (; k + kFoldUnroll <= splits; k += kFoldUnroll) {
        f32x4 v[kFoldUnroll];
#pragma unroll
        for (int u = 0; u < kFoldUnroll; ++u) v[u] = __builtin_nontemporal_load(p + (int64_t)(k + u) * points);
#pragma unroll
        for (int u = 0; u < kFoldUnroll; ++u) {
            a0 += (double)v[u].x;
            a1 += (double)v[u].y;
            a2 += (double)v[u].z;
            a3 += (double)v[u].w;
        }
    }
    for (; k < splits; ++k) {
        const f32x4 v = __builtin_nontemporal_load(p + (int64_t)k * points);
        a0 += (double)v.x;
        a1 += (double)v.y;
        a2 += (double)v.z;
        a3 += (double)v.w;
    }
    double2* s2 = reinterpret_cast<double2*>(S) + 2 * i;
    double2 lo = s2[0], hi = s2[1];
    lo.x += a0;
    lo.y += a1;
    hi.x += a2;
    hi.y += a3;
    s2[0] = lo;
    s2[1] = hi;
}

// Batched fold: for every (grid, tile) job and every in-grid point of the tile, add the
// listed segments' partial values (in list order, FP64) into the grid's S.
__global__ void k_fold_batch(const int32_t* __restrict__ n_jobs_dev, const FoldJob* __restrict__ jobs,
                             const int32_t* __restrict__ seg_list, const float4* __restrict__ seg_part,
                             int TD, int TO)
{
    const int n_jobs = *n_jobs_dev;
    const int64_t per_job = (int64_t)TD * TO;
    const int64_t total = per_job * n_jobs;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int jb = (int)(idx / per_job);
        const int e = (int)(idx % per_job);
        const FoldJob fj = jobs[jb];
        const int og = fj.tw * TO + e / TD;
        const int dg = fj.td * TD + e % TD;
        if (og >= fj.n_omega || dg >= fj.n_dir) continue;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int k = fj.list_begin; k < fj.list_end; ++k) {
            const float4 v = seg_part[(int64_t)seg_list[k] * per_job + e];
            a0 += (double)v.x; a1 += (double)v.y; a2 += (double)v.z; a3 += (double)v.w;
        }
        double* S = fj.S + ((int64_t)og * fj.n_dir + dg) * 4;
        S[0] += a0; S[1] += a1; S[2] += a2; S[3] += a3;
    }
}

// I[d][k] = C * (|S1|^2 + |S2|^2), S layout [omega][dir][4].
__global__ void k_finalize(const double* __restrict__ S, double* __restrict__ I, int n_dir,
                           int n_omega, double C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_dir * n_omega) return;
    const int d = (int)(i / n_omega), k = (int)(i % n_omega);
    const double* s = S + ((int64_t)k * n_dir + d) * 4;
    I[i] = C * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + s[3] * s[3]);
}

// Cartesian complex spectrum out[((d*n_omega + k)*3 + c)*2 + {re, im}] = e1_c S1 + e2_c S2.
__global__ void k_cartesian(const double* __restrict__ S, const double* __restrict__ dirs9,
                            double* __restrict__ out, int n_dir, int n_omega)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_dir * n_omega) return;
    const int d = (int)(i / n_omega), k = (int)(i % n_omega);
    const double* s = S + ((int64_t)k * n_dir + d) * 4;
    const double* e = dirs9 + 9 * d;
    for (int c = 0; c < 3; ++c) {
        out[(i * 3 + c) * 2 + 0] = e[3 + c] * s[0] + e[6 + c] * s[2];
        out[(i * 3 + c) * 2 + 1] = e[3 + c] * s[1] + e[6 + c] * s[3];
    }
}

__global__ void k_fill(double* p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_int(int* p, int64_t n, int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// out[4i..4i+3] = hardware sin/cos and library sin/cos of 2*pi*in[i].
__global__ void k_trig_probe(const float* in, float* out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s, c, s2, c2;
    sincos_rev_fast(in[i], s, c);
    sincos_rev_accurate(in[i], s2, c2);
    out[4 * i + 0] = s;
    out[4 * i + 1] = c;
    out[4 * i + 2] = s2;
    out[4 * i + 3] = c2;
}

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_fold_batch(const int32_t* n_jobs_dev, const FoldJob* jobs, int max_jobs,
                             const int32_t* seg_list, const float* seg_part, int td, int to, hipStream_t st)
{
    if (max_jobs <= 0) return hipSuccess;
    const int64_t total = (int64_t)max_jobs * td * to;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fold_batch, dim3(blocks), dim3(256), 0, st, n_jobs_dev, jobs, seg_list,
                       reinterpret_cast<const float4*>(seg_part), td, to);
    return hipGetLastError();
}

hipError_t launch_fold(const float* part, double* S, int splits, int64_t count, hipStream_t st,
                       hipEvent_t ev_start, hipEvent_t ev_stop)
{
    int64_t points = count / 4;
    if (points <= 0) return hipSuccess;
    const f32x4* p4 = reinterpret_cast<const f32x4*>(part);
    if (ev_start || ev_stop) {
        void* args[] = {&p4, &S, &splits, &points};
        return hipExtLaunchKernel(reinterpret_cast<const void*>(k_fold), dim3(grid1d(points, 256)), dim3(256), args,
                                  0, st, ev_start, ev_stop, 0);
    }
    hipLaunchKernelGGL(k_fold, dim3(grid1d(points, 256)), dim3(256), 0, st, p4, S, splits, points);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* S, double* I, int n_dir, int n_omega, double C,
                           hipStream_t st)
{
    const int64_t n = (int64_t)n_dir * n_omega;
    hipLaunchKernelGGL(k_finalize, dim3(grid1d(n, 256)), dim3(256), 0, st, S, I, n_dir, n_omega, C);
    return hipGetLastError();
}

hipError_t launch_cartesian(const double* S, const double* dirs9, double* out, int n_dir,
                            int n_omega, hipStream_t st)
{
    const int64_t n = (int64_t)n_dir * n_omega;
    hipLaunchKernelGGL(k_cartesian, dim3(grid1d(n, 256)), dim3(256), 0, st, S, dirs9, out, n_dir,
                       n_omega);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid1d(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3(grid1d(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

int tracked_step_group() { return kStepGroup; }

template <int NT>
hipError_t launch_tracked_nt(const TrackedArgs& a, int dtype, bool direct, hipStream_t st)
{
    const TrackedTiling tl = tracked_tiling(a.n_dir, a.n_omega, NT);
    const int64_t blocks = a.n_particles * tl.n_dt * tl.n_ot;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks);
    const dim3 block(NT);
    if (dtype == 0) {
        if (direct) hipLaunchKernelGGL((k_tracked_accumulate<float, true, NT>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_tracked_accumulate<float, false, NT>), grid, block, 0, st, a);
    } else {
        if (direct) hipLaunchKernelGGL((k_tracked_accumulate<double, true, NT>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_tracked_accumulate<double, false, NT>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_tracked_accumulate(const TrackedArgs& a, int dtype, bool direct, hipStream_t st)
{
    if (a.n_particles <= 0 || a.n_steps <= 0 || a.n_dir <= 0 || a.n_omega <= 0) return hipSuccess;
    return a.n_steps == 1 ? launch_tracked_nt<kTrackThreadsOneStep>(a, dtype, direct, st)
                          : launch_tracked_nt<kTrackThreads>(a, dtype, direct, st);
}

hipError_t launch_tracked_finalize(const double* T, const double* wts, const double* gk, const double* g3,
                                   int64_t n_particles, int n_dir, int n_omega, double C, double* I,
                                   hipStream_t st)
{
    const int64_t n = (int64_t)n_dir * n_omega;
    hipLaunchKernelGGL(k_tracked_finalize, dim3(grid1d(n, 256)), dim3(256), 0, st, T, wts, gk, g3, n_particles,
                       n_dir, n_omega, C, I);
    return hipGetLastError();
}

hipError_t launch_trig_probe(const float* in, float* out, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trig_probe, dim3(grid1d(n, 256)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

}  // namespace rad
