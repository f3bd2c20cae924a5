// gfx950 kernels of the in-situ macro-particle radiation sum (arXiv:1802.03972, Eq. 13).
//
// Work decomposition of the accumulate kernel
// -------------------------------------------
// One update is one (macro-particle m, direction n, frequency omega) term
//     S(n, omega) += F_m(omega) * A_m(n) * exp(i omega tau_m(n)),   tau = t - n.r/c.
// * A lane owns ONE direction and W consecutive frequencies; its W complex spectrum
//   entries live in registers for the whole launch.
// * Since A = n x [...] is normal to n, it is stored in a fixed per-direction basis
//   (e1, e2) of the plane normal to n: two real components instead of three, and the
//   spectrum holds two complex components.  |S|^2 is unchanged and the Cartesian
//   spectrum is e1*S1 + e2*S2.
// * A workgroup owns a tile of TD directions x TO frequencies and a contiguous range of
//   particles (its split).  Particles stream through LDS in chunks of kChunk:
//     1. coalesced SoA load of the chunk into LDS (widened to FP64);
//     2. per (particle, direction) geometry in FP64 -- 1 - beta.n without cancellation,
//        A in the (e1, e2) basis, tau/(2 pi), the rotation w = exp(i domega tau) --
//        shared by the workgroup's TO frequencies;
//     3. per (particle, frequency) form-factor weight F = sqrt(N (1-g) + N^2 g) (Eq. 12),
//        shared by the workgroup's TD directions;
//     4. the hot loop: per particle, each lane seeds z = exp(i omega_first tau) from the
//        FP64 phase (reduced to [0, 1) revolutions before leaving FP64), then walks its W
//        frequencies with z <- z*w (uniform omega grid), scaling by F and accumulating.
//        10 FP32 VALU operations per update: 2 (scale) + 4 (two complex FMAs) + 4 (rotate).
// * At the end each workgroup writes its FP32 partial tile; a fold kernel adds the splits
//   in a fixed order in FP64 into the grid's FP64 accumulator (deterministic).

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "rad_internal.h"

namespace rad {

namespace {

constexpr double kInvC = 1.0 / 299792458.0;          // 1/c [s/m]
constexpr double kInv2Pi = 0.15915494309189533577;   // 1/(2 pi)

// sin and cos of 2*pi*r, r in revolutions (the hardware transcendental takes revolutions).
__device__ __forceinline__ void sincos_rev_fast(float r, float& s, float& c)
{
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}

// Library sin/cos(pi x) (few-ulp accurate); used where the result is reused many times.
__device__ __forceinline__ void sincos_rev_accurate(float r, float& s, float& c)
{
    sincospif(2.0f * r, &s, &c);
}

__device__ __forceinline__ void flag_error(int* err)
{
    atomicOr(err, 1);
}

template <typename InT>
__device__ __forceinline__ double load_wide(const void* p, int64_t i)
{
    return static_cast<double>(static_cast<const InT*>(p)[i]);
}

// Per (particle, direction) geometry.  Writes A1, A2 (FP32), w = exp(i domega tau) and
// tau/(2 pi) (FP64).
template <int PREC, bool WANT_W, int P = kChunk>
__device__ __forceinline__ void particle_direction_setup(const double* __restrict__ raw, int m,
                                                         const double* __restrict__ dv,
                                                         double domega, float4& geo,
                                                         double& ph_out, int* err)
{
    const double x = raw[0 * P + m], y = raw[1 * P + m], z = raw[2 * P + m];
    const double bx = raw[3 * P + m], by = raw[4 * P + m], bz = raw[5 * P + m];
    const double dbx = raw[6 * P + m], dby = raw[7 * P + m], dbz = raw[8 * P + m];
    const double N = raw[9 * P + m], t = raw[10 * P + m];
    const double nx = dv[0], ny = dv[1], nz = dv[2];
    const double e1x = dv[3], e1y = dv[4], e1z = dv[5];
    const double e2x = dv[6], e2y = dv[7], e2z = dv[8];
    float A1, A2, wr, wi;
    double ph;
    bool bad;
    if constexpr (PREC == 0) {
        // A = [(n - beta)(n.dbeta) - dbeta (1 - beta.n)] / (1 - beta.n)^2, projected on e1, e2
        // (n.e = 0 removes the n term).  FP64 keeps 1 - beta.n ~ 1/(2 gamma^2) accurate.
        const double D = 1.0 - (bx * nx + by * ny + bz * nz);
        const double nbd = nx * dbx + ny * dby + nz * dbz;
        const double b1 = bx * e1x + by * e1y + bz * e1z;
        const double b2 = bx * e2x + by * e2y + bz * e2z;
        const double q1 = dbx * e1x + dby * e1y + dbz * e1z;
        const double q2 = dbx * e2x + dby * e2y + dbz * e2z;
        // D^2 >= ~1e-13 is a normal FP32 number; A is kept in FP32, so an FP32 reciprocal
        // (about 1 ulp) of the FP64 D^2 loses nothing that matters.
        const float inv = __builtin_amdgcn_rcpf(static_cast<float>(D * D));
        A1 = -static_cast<float>(b1 * nbd + q1 * D) * inv;
        A2 = -static_cast<float>(b2 * nbd + q2 * D) * inv;
        const double tau = t - (nx * x + ny * y + nz * z) * kInvC;
        ph = tau * kInv2Pi;
        wr = 1.f;
        wi = 0.f;
        if constexpr (WANT_W) {
            double rw = domega * ph;
            rw -= floor(rw);
            sincos_rev_fast(static_cast<float>(rw), wi, wr);
        }
        bad = !(D > 0.0) || !(N >= 0.0) || !isfinite(N) || !isfinite(ph) || !isfinite(A1) ||
              !isfinite(A2);
    } else {
        // All-FP32 variant (precision study): same formulas on FP32-rounded values.
        const float fx = (float)x, fy = (float)y, fz = (float)z;
        const float fbx = (float)bx, fby = (float)by, fbz = (float)bz;
        const float fdbx = (float)dbx, fdby = (float)dby, fdbz = (float)dbz;
        const float fnx = (float)nx, fny = (float)ny, fnz = (float)nz;
        const float f1x = (float)e1x, f1y = (float)e1y, f1z = (float)e1z;
        const float f2x = (float)e2x, f2y = (float)e2y, f2z = (float)e2z;
        const float D = 1.0f - (fbx * fnx + fby * fny + fbz * fnz);
        const float nbd = fnx * fdbx + fny * fdby + fnz * fdbz;
        const float b1 = fbx * f1x + fby * f1y + fbz * f1z;
        const float b2 = fbx * f2x + fby * f2y + fbz * f2z;
        const float q1 = fdbx * f1x + fdby * f1y + fdbz * f1z;
        const float q2 = fdbx * f2x + fdby * f2y + fdbz * f2z;
        const float inv = 1.0f / (D * D);
        A1 = -(b1 * nbd + q1 * D) * inv;
        A2 = -(b2 * nbd + q2 * D) * inv;
        const float tau = (float)t - (fnx * fx + fny * fy + fnz * fz) * (float)kInvC;
        const float phf = tau * (float)kInv2Pi;
        wr = 1.f;
        wi = 0.f;
        if constexpr (WANT_W) {
            float rw = (float)domega * phf;
            rw -= floorf(rw);
            sincos_rev_fast(rw, wi, wr);
        }
        ph = (double)phf;
        bad = !(D > 0.0f) || !(N >= 0.0) || !isfinite(N) || !isfinite(phf) || !isfinite(A1) ||
              !isfinite(A2);
    }
    if (bad) flag_error(err);
    geo = make_float4(A1, A2, wr, wi);
    ph_out = ph;
}

// Accumulate chunks [c_begin, c_end) of `j` into the tile (td, tw) and write the FP32
// partial tile: element (omega o, direction d) of the tile goes to out[o * row + d] (as
// (S1r, S1i, S2r, S2i)) when it lies inside the grid.  Every thread of the workgroup must
// call this with the same arguments; LDS is reused chunk by chunk.
template <typename InT, int PREC, int W, int DPW, int V>
__device__ __forceinline__ void accumulate_range(const Job& j, int td, int tw, int64_t c_begin,
                                                 int64_t c_end, float4* __restrict__ out, int row,
                                                 float4* smem4)
{
    constexpr int P = kChunk;
    constexpr int SUBS = 64 / DPW;
    constexpr int TD = DPW;
    static_assert(W % 4 == 0, "W must be a multiple of 4");

    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int waves = nt >> 6;
    const int TO = waves * SUBS * W;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int dl = lane % DPW;
    const int ob = wave * SUBS + lane / DPW;

    float4* geo = smem4;                                             // [P][TD]
    double* taus = reinterpret_cast<double*>(geo + P * TD);          // [P][TD]
    double* raw = taus + P * TD;                                     // [11][P]
    float2* nw = reinterpret_cast<float2*>(raw + 11 * P);            // [P]: (N, N^2) in FP32
    float* ff = reinterpret_cast<float*>(nw + P);                    // [P][TO]

    constexpr bool DIRECT = (V & kVarDirect) != 0;
    constexpr bool SHAPE3 = (V & kVarShape3) != 0;
    const int d = td * TD + dl;
    const int o_first = tw * TO + ob * W;
    const double om_first = j.omega[o_first < j.n_omega ? o_first : j.n_omega - 1];
    // explicit frequencies (direct phase) and direction-dependent shape factors of this lane
    double om[DIRECT ? W : 1];
    float gl[SHAPE3 ? W : 1];
    {
        const int dc = d < j.n_dir ? d : j.n_dir - 1;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int oc = o_first + k < j.n_omega ? o_first + k : j.n_omega - 1;
            if constexpr (DIRECT) om[k] = j.omega[oc];
            if constexpr (SHAPE3) gl[k] = j.g3[(int64_t)dc * j.n_omega + oc];
        }
    }

    float s1r[W], s1i[W], s2r[W], s2i[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        s1r[k] = 0.f; s1i[k] = 0.f; s2r[k] = 0.f; s2i[k] = 0.f;
    }

    for (int64_t c = c_begin; c < c_end; ++c) {
        // 1. stage the chunk (SoA, coalesced), widened to FP64, plus the step time.
        if (tid < P) {
            const int64_t i = j.i_begin + c * P + tid;
            const bool ok = i < j.i_end;
            const int64_t ii = ok ? i : j.i_begin;
#pragma unroll
            for (int f = 0; f < 10; ++f) raw[f * P + tid] = ok ? load_wide<InT>(j.f[f], ii) : 0.0;
            // step = ii / n_per_step without a 64-bit integer division: the FP64 quotient of
            // two integers below 2^53 is within one of the true one; correct it exactly.
            int64_t step = 0;
            if (j.i_end > j.n_per_step) {
                step = (int64_t)floor((double)ii / (double)j.n_per_step);
                if (step * j.n_per_step > ii) --step;
                else if ((step + 1) * j.n_per_step <= ii) ++step;
            }
            raw[10 * P + tid] = ok ? j.t0 + (double)step * j.dt : 0.0;
            const float N = ok ? (float)raw[9 * P + tid] : 0.f;
            nw[tid] = make_float2(N, N * N);
        }
        __syncthreads();
        // 2. per (particle, direction) geometry.
        for (int i = tid; i < P * TD; i += nt) {
            const int m = i / TD;
            int dg = td * TD + (i % TD);
            dg = dg < j.n_dir ? dg : j.n_dir - 1;
            float4 gv;
            double ph;
            particle_direction_setup<PREC, !DIRECT>(raw, m, j.dirs9 + 9 * dg, j.domega, gv, ph, j.err);
            geo[i] = gv;
            taus[i] = ph;
        }
        // 3. per (particle, frequency) form-factor weight F = sqrt(N^2 g + N (1 - g)) (Eq. 12),
        //    FP32; frequencies outside the grid get F = 0 and contribute nothing.
        for (int o = tid; o < (SHAPE3 ? 0 : TO); o += nt) {
            const int og = tw * TO + o;
            float2 g = make_float2(0.f, 0.f);
            if (og < j.n_omega) g = j.gtab[og];
            float* dst = ff + o;
#pragma unroll 8
            for (int m = 0; m < P; ++m, dst += TO) {
                const float2 N = nw[m];
                *dst = __builtin_amdgcn_sqrtf(fmaf(N.y, g.x, N.x * g.y));
            }
        }
        __syncthreads();
        // 4. hot loop.
        for (int m = 0; m < P; ++m) {
            const float4 gm = geo[m * TD + dl];
            const double ph = taus[m * TD + dl];
            float zr = 1.f, zi = 0.f;
            if constexpr (!DIRECT) {
                if constexpr (PREC == 0) {
                    double rv = om_first * ph;
                    rv -= floor(rv);
                    sincos_rev_fast(static_cast<float>(rv), zi, zr);
                } else {
                    float rv = (float)om_first * (float)ph;
                    rv -= floorf(rv);
                    sincos_rev_fast(rv, zi, zr);
                }
            }
            const float A1 = gm.x, A2 = gm.y, wr = gm.z, wi = gm.w;
            const float4* fq = reinterpret_cast<const float4*>(ff + m * TO + ob * W);
            float Nm = 0.f, NN1 = 0.f;
            if constexpr (SHAPE3) {
                const float2 Nv = nw[m];
                Nm = Nv.x;
                NN1 = Nv.y - Nv.x;   // N^2 - N
            }
#pragma unroll
            for (int q = 0; q < W / 4; ++q) {
                float Fv[4];
                if constexpr (SHAPE3) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)   // F^2 = N + (N^2 - N) g(n, omega) (Eq. 12)
                        Fv[u] = __builtin_amdgcn_sqrtf(fmaxf(fmaf(NN1, gl[4 * q + u], Nm), 0.f));
                } else {
                    const float4 F4 = fq[q];
                    Fv[0] = F4.x; Fv[1] = F4.y; Fv[2] = F4.z; Fv[3] = F4.w;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = 4 * q + u;
                    if constexpr (DIRECT) {
                        // explicit frequency list: each term's phase from the FP64 product,
                        // reduced to [0, 1) revolutions before leaving FP64
                        if constexpr (PREC == 0) {
                            double rv = om[k] * ph;
                            rv -= floor(rv);
                            sincos_rev_fast(static_cast<float>(rv), zi, zr);
                        } else {
                            float rv = (float)om[k] * (float)ph;
                            rv -= floorf(rv);
                            sincos_rev_fast(rv, zi, zr);
                        }
                    }
                    const float ur = Fv[u] * zr;
                    const float ui = Fv[u] * zi;
                    s1r[k] = fmaf(A1, ur, s1r[k]);
                    s1i[k] = fmaf(A1, ui, s1i[k]);
                    s2r[k] = fmaf(A2, ur, s2r[k]);
                    s2i[k] = fmaf(A2, ui, s2i[k]);
                    if constexpr (!DIRECT) {
                        const float nr = fmaf(zr, wr, -(zi * wi));
                        const float ni = fmaf(zr, wi, zi * wr);
                        zr = nr;
                        zi = ni;
                    }
                }
            }
        }
        __syncthreads();
    }

    // 5. partial tile (coalesced over directions).
    if (d < j.n_dir) {
        const int o_loc = ob * W;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (o_first + k < j.n_omega)
                out[(int64_t)(o_loc + k) * row + dl] = make_float4(s1r[k], s1i[k], s2r[k], s2i[k]);
        }
    }
}

template <typename InT, int PREC, int W, int DPW, int V>
__global__ void __launch_bounds__(512) k_accumulate(AccArgs a)
{
    extern __shared__ float4 smem4[];
    constexpr int TD = DPW;
    const int TO = (blockDim.x >> 6) * (64 / DPW) * W;
    const int ntiles = a.job.tiles_d * a.job.tiles_w;
    const int tile = blockIdx.x % ntiles;
    const int split = blockIdx.x / ntiles;
    const int td = tile % a.job.tiles_d;
    const int tw = tile / a.job.tiles_d;
    const int64_t n_local = a.job.i_end - a.job.i_begin;
    const int64_t nchunks = (n_local + kChunk - 1) / kChunk;
    const int64_t c_begin = (int64_t)split * a.chunks_per_split;
    int64_t c_end = c_begin + a.chunks_per_split;
    if (c_end > nchunks) c_end = nchunks;
    // partial layout [split][omega][dir]
    float4* out = reinterpret_cast<float4*>(a.part) +
                  ((int64_t)split * a.job.n_omega + (int64_t)tw * TO) * a.job.n_dir + td * TD;
    accumulate_range<InT, PREC, W, DPW, V>(a.job, td, tw, c_begin, c_end, out, a.job.n_dir, smem4);
}

// Persistent batched accumulate: block r processes segments [wg_seg_begin[r], wg_seg_begin[r+1]),
// each a chunk range of one (item, tile); segment s writes its partial tile [TO][TD] at
// seg_part + s * TO * TD (float4 units).
template <typename InT, int PREC, int W, int DPW, int V>
__global__ void __launch_bounds__(512) k_accumulate_batch(const Job* __restrict__ items,
                                                          const int32_t* __restrict__ wg_seg_begin,
                                                          const BatchSeg* __restrict__ segs,
                                                          float* seg_part)
{
    extern __shared__ float4 smem4[];
    constexpr int TD = DPW;
    const int TO = (blockDim.x >> 6) * (64 / DPW) * W;
    const int s0 = wg_seg_begin[blockIdx.x], s1 = wg_seg_begin[blockIdx.x + 1];
    for (int s = s0; s < s1; ++s) {
        const BatchSeg sg = segs[s];
        const Job j = items[sg.item];
        const int td = sg.tile % j.tiles_d;
        const int tw = sg.tile / j.tiles_d;
        float4* out = reinterpret_cast<float4*>(seg_part) + (int64_t)s * TO * TD;
        accumulate_range<InT, PREC, W, DPW, V>(j, td, tw, sg.c_begin, sg.c_end, out, TD, smem4);
    }
}

// ---------------------------------------------------------------------------------------
// Post-processing variant: tracked particles keep their own time integral
// T_m(n, omega) = sum_j A_{j,m}(n) exp(i omega tau_{j,m}) (no form factor) in FP64,
// layout [m][omega][dir][4]; the form factor is applied only when the spectrum is read.
// One thread per (particle, direction, block of W frequencies); geometry in FP64 as in the
// main path; the block's frequencies follow the same rotation recurrence (or, for explicit
// frequency lists, the per-term FP64 phase).
// ---------------------------------------------------------------------------------------
template <typename InT, bool DIRECT>
__global__ void __launch_bounds__(256) k_tracked_accumulate(TrackedArgs a)
{
    constexpr int W = 16;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n_blocks = (a.n_omega + W - 1) / W;
    const int d = (int)(idx % a.n_dir);
    const int64_t rest = idx / a.n_dir;
    const int ob = (int)(rest % n_blocks);
    const int64_t m = rest / n_blocks;
    if (m >= a.n_particles) return;
    double raw[11];
#pragma unroll
    for (int f = 0; f < 9; ++f) raw[f] = load_wide<InT>(a.f[f], m);
    raw[9] = 1.0;      // weights enter only at read-out; the weight field is never read
    raw[10] = a.t;
    float4 gv;
    double ph;
    particle_direction_setup<0, !DIRECT, 1>(raw, 0, a.dirs9 + 9 * d, a.domega, gv, ph, a.err);
    const int o0 = ob * W;
    float zr = 1.f, zi = 0.f;
    if constexpr (!DIRECT) {
        double rv = a.omega[o0] * ph;
        rv -= floor(rv);
        sincos_rev_fast(static_cast<float>(rv), zi, zr);
    }
    double* T = a.T + ((m * a.n_omega + o0) * a.n_dir + d) * 4;
    for (int k = 0; k < W && o0 + k < a.n_omega; ++k, T += (int64_t)a.n_dir * 4) {
        if constexpr (DIRECT) {
            double rv = a.omega[o0 + k] * ph;
            rv -= floor(rv);
            sincos_rev_fast(static_cast<float>(rv), zi, zr);
        }
        T[0] += (double)(gv.x * zr);
        T[1] += (double)(gv.x * zi);
        T[2] += (double)(gv.y * zr);
        T[3] += (double)(gv.y * zi);
        if constexpr (!DIRECT) {
            const float nr = fmaf(zr, gv.z, -(zi * gv.w));
            const float ni = fmaf(zr, gv.w, zi * gv.z);
            zr = nr;
            zi = ni;
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
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_dir * n_omega) return;
    const int d = (int)(i / n_omega), k = (int)(i % n_omega);
    const double g = g3 ? g3[(int64_t)d * n_omega + k] : gk[k];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int64_t m = 0; m < n_particles; ++m) {
        const double N = wts[m];
        const double F = sqrt(fmax(N + (N * N - N) * g, 0.0));
        const double* t = T + ((m * n_omega + k) * n_dir + d) * 4;
        s0 += F * t[0]; s1 += F * t[1]; s2 += F * t[2]; s3 += F * t[3];
    }
    I[i] = C * (s0 * s0 + s1 * s1 + s2 * s2 + s3 * s3);
}

// S[i] += sum over splits of part[s][i], in split order, in FP64.
__global__ void k_fold(const float* __restrict__ part, double* __restrict__ S, int splits,
                       int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += (double)part[(int64_t)k * count + i];
    S[i] += s;
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

template <typename InT, int PREC, int W, int DPW, int V>
hipError_t launch_acc_t(const AccArgs& a, const LaunchShape& s, int n_blocks, hipStream_t st)
{
    auto kern = k_accumulate<InT, PREC, W, DPW, V>;
    const size_t lds = acc_lds_bytes(s);
    static size_t lds_allowed = 64 * 1024;  // per instantiation; the attribute is process-wide
    if (lds > lds_allowed) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_allowed = lds;
    }
    hipLaunchKernelGGL(kern, dim3(n_blocks), dim3(64 * s.waves), lds, st, a);
    return hipGetLastError();
}

struct BatchArgs {
    const Job* items;
    const int32_t* wg_seg_begin;
    const BatchSeg* segs;
    float* seg_part;
    bool prepare_only;   // only set the kernel's LDS attribute (done before a graph capture)
};

template <typename InT, int PREC, int W, int DPW, int V>
hipError_t launch_batch_t(const BatchArgs& b, const LaunchShape& s, int n_blocks, hipStream_t st)
{
    auto kern = k_accumulate_batch<InT, PREC, W, DPW, V>;
    const size_t lds = acc_lds_bytes(s);
    static size_t lds_allowed = 64 * 1024;
    if (lds > lds_allowed) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_allowed = lds;
    }
    if (b.prepare_only) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(n_blocks), dim3(64 * s.waves), lds, st, b.items, b.wg_seg_begin,
                       b.segs, b.seg_part);
    return hipGetLastError();
}

// Dispatch on the launch shape; Fn<W, DPW>::run(...) is the templated launcher.
template <typename InT, int PREC, typename A>
hipError_t dispatch_shape(const A& a, const LaunchShape& s, int n_blocks, hipStream_t st)
{
#define RAD_SHAPE_CASE(WW, DD, VV)                                                    \
    if (s.w_per_lane == WW && s.dir_per_wave == DD && s.variant == VV) {              \
        if constexpr (std::is_same<A, AccArgs>::value)                                \
            return launch_acc_t<InT, PREC, WW, DD, VV>(a, s, n_blocks, st);           \
        else                                                                          \
            return launch_batch_t<InT, PREC, WW, DD, VV>(a, s, n_blocks, st);         \
    }
    RAD_SHAPE_CASE(32, 64, 0)
    RAD_SHAPE_CASE(32, 32, 0)
    RAD_SHAPE_CASE(32, 16, 0)
    RAD_SHAPE_CASE(16, 64, 0)
    RAD_SHAPE_CASE(16, 32, 0)
    RAD_SHAPE_CASE(16, 16, 0)
    // explicit frequency lists and 3-D shapes: 16 frequencies per lane (register budget)
    RAD_SHAPE_CASE(16, 64, 1)
    RAD_SHAPE_CASE(16, 32, 1)
    RAD_SHAPE_CASE(16, 16, 1)
    RAD_SHAPE_CASE(16, 64, 2)
    RAD_SHAPE_CASE(16, 32, 2)
    RAD_SHAPE_CASE(16, 16, 2)
    RAD_SHAPE_CASE(16, 64, 3)
    RAD_SHAPE_CASE(16, 32, 3)
    RAD_SHAPE_CASE(16, 16, 3)
#undef RAD_SHAPE_CASE
    return hipErrorInvalidValue;
}

template <typename A>
hipError_t dispatch_all(const A& a, int dtype, int precision, const LaunchShape& s, int n_blocks,
                        hipStream_t st)
{
    if (dtype == 0) {
        return precision == 0 ? dispatch_shape<float, 0>(a, s, n_blocks, st)
                              : dispatch_shape<float, 1>(a, s, n_blocks, st);
    }
    return precision == 0 ? dispatch_shape<double, 0>(a, s, n_blocks, st)
                          : dispatch_shape<double, 1>(a, s, n_blocks, st);
}

}  // namespace

hipError_t launch_accumulate(const AccArgs& a, int dtype, int precision, const LaunchShape& s,
                             int n_blocks, hipStream_t st)
{
    return dispatch_all(a, dtype, precision, s, n_blocks, st);
}

hipError_t launch_accumulate_batch(const Job* items, const int32_t* wg_seg_begin, const BatchSeg* segs,
                                   float* seg_part, int dtype, int precision,
                                   const LaunchShape& s, int n_blocks, hipStream_t st)
{
    const BatchArgs b{items, wg_seg_begin, segs, seg_part, false};
    return dispatch_all(b, dtype, precision, s, n_blocks, st);
}

hipError_t prepare_accumulate_batch(int dtype, int precision, const LaunchShape& s)
{
    const BatchArgs b{nullptr, nullptr, nullptr, nullptr, true};
    return dispatch_all(b, dtype, precision, s, 0, nullptr);
}

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

hipError_t launch_fold(const float* part, double* S, int splits, int64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold, dim3(grid1d(count, 256)), dim3(256), 0, st, part, S, splits, count);
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

hipError_t launch_tracked_accumulate(const TrackedArgs& a, int dtype, bool direct, hipStream_t st)
{
    const int64_t n_blocks = (a.n_omega + 15) / 16;
    const int64_t threads = a.n_particles * n_blocks * a.n_dir;
    if (threads <= 0) return hipSuccess;
    const dim3 grid(grid1d(threads, 256));
    if (dtype == 0) {
        if (direct) hipLaunchKernelGGL((k_tracked_accumulate<float, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_tracked_accumulate<float, false>), grid, dim3(256), 0, st, a);
    } else {
        if (direct) hipLaunchKernelGGL((k_tracked_accumulate<double, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_tracked_accumulate<double, false>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError();
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
