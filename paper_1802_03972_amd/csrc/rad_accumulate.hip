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
//     4. the hot loop: per particle, each lane seeds z = exp(i omega tau) at the middle
//        frequency of its block from the FP64 phase (reduced to [0, 1) revolutions before
//        leaving FP64), then walks its W frequencies forward and backward from it, scaling
//        by F and accumulating.  With 16 frequencies per lane on uniform steps (grid-wide
//        or per block) the walk is the three-term recurrence z_{k+1} = 2 cos(theta) z_k -
//        z_{k-1}: 8 FP32 VALU operations per update, 2 (scale) + 4 (two complex
//        multiply-adds) + 2 (recurrence).  32-frequency lanes walk by complex products with
//        w: 10 per update (4 for the rotation).
// * At the end each workgroup writes its FP32 partial tile; a fold kernel adds the splits
//   in a fixed order in FP64 into the grid's FP64 accumulator (deterministic).

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "rad_device.h"
#include "rad_internal.h"

namespace rad {

namespace {


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
    constexpr bool BSTEP = (V & kVarBlockStep) != 0;
    static_assert(!(DIRECT && BSTEP), "a frequency list is either direct or block-stepped");
    static_assert(!BSTEP || W == kBlockW, "block steps are defined per 16 frequencies");
    // uniform steps (grid-wide or per block), FP64 geometry, 16 frequencies per lane: the
    // walk is the three-term recurrence from the mid-block seed (at most 8 steps from it)
    constexpr bool TT = !DIRECT && (W == 16) && (PREC == 0);
    const int d = td * TD + dl;
    const int o_first = tw * TO + ob * W;
    const double om_first = gload(j.omega, o_first < j.n_omega ? o_first : j.n_omega - 1);
    // piecewise-uniform list: this lane's block spacing (the lane's frequencies are one block)
    double bstep = 0.0;
    if constexpr (BSTEP) bstep = gload(j.bstep, (o_first < j.n_omega ? o_first : j.n_omega - 1) / kBlockW);
    // The lane's W frequencies are walked from one FP64-seeded frequency with the rotation
    // w = exp(i domega tau).  The seed is the middle of the block (index KS = W/2, on the
    // block's own progression), and the walk goes forward and backward from it, so no
    // frequency is more than W/2 steps from its seed (the rounding of w, or of 2 Re(w),
    // enters once per step).
    constexpr int KS = DIRECT ? 0 : W / 2;
    const double om_seed = om_first + (double)KS * (BSTEP ? bstep : j.domega);
    // explicit frequencies (direct phase) and direction-dependent shape factors of this lane
    double om[DIRECT ? W : 1];
    float gl[SHAPE3 ? W : 1];
    {
        const int dc = d < j.n_dir ? d : j.n_dir - 1;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int oc = o_first + k < j.n_omega ? o_first + k : j.n_omega - 1;
            if constexpr (DIRECT) om[k] = gload(j.omega, oc);
            if constexpr (SHAPE3) gl[k] = gload(j.g3, (int64_t)dc * j.n_omega + oc);
        }
    }

    float s1r[W], s1i[W], s2r[W], s2i[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        s1r[k] = 0.f; s1i[k] = 0.f; s2r[k] = 0.f; s2i[k] = 0.f;
    }

    for (int64_t c = c_begin; c < c_end; ++c) {
        // Stages 1-3 gate the workgroup's barriers: their waves get issue priority over the
        // hot loops of other workgroups on the CU (measured +2 %).  The hot loop itself runs
        // one level above the default.
        __builtin_amdgcn_s_setprio(3);
        // The set-up's per-thread offsets are derived from an opaque copy of the thread
        // index in every chunk, so the compiler recomputes them (a few integer adds) instead
        // of keeping them live across the hot loop, where the 4W accumulators leave no room
        // for them (they were spilled to scratch memory).
        int tc = threadIdx.x;
        asm volatile("" : "+v"(tc));
        // 1. stage the chunk (SoA, coalesced), widened to FP64, plus the step time.
        if (tc < P) {
            const int64_t i = j.i_begin + c * P + tc;
            const bool ok = i < j.i_end;
            const int64_t ii = ok ? i : j.i_begin;
#pragma unroll
            for (int f = 0; f < 10; ++f) raw[f * P + tc] = ok ? load_wide<InT>(j.f[f], ii) : 0.0;
            // step = ii / n_per_step without a 64-bit integer division: the FP64 quotient of
            // two integers below 2^53 is within one of the true one; correct it exactly.
            int64_t step = 0;
            if (j.i_end > j.n_per_step) {
                step = (int64_t)floor((double)ii / (double)j.n_per_step);
                if (step * j.n_per_step > ii) --step;
                else if ((step + 1) * j.n_per_step <= ii) ++step;
            }
            raw[10 * P + tc] = ok ? j.t0 + (double)step * j.dt : 0.0;
            const float N = ok ? (float)raw[9 * P + tc] : 0.f;
            nw[tc] = make_float2(N, N * N);
        }
        __syncthreads();
        // 2. per (particle, direction) geometry.
        for (int i = tc; i < P * TD; i += nt) {
            const int m = i / TD;
            int dg = td * TD + (i % TD);
            dg = dg < j.n_dir ? dg : j.n_dir - 1;
            float4 gv;
            double ph;
            particle_direction_setup<PREC, !DIRECT && !BSTEP>(raw, m, j.dirs9 + 9 * dg, j.domega, gv, ph, j.err);
            geo[i] = gv;
            taus[i] = ph;
        }
        // 3. per (particle, frequency) form-factor weight F = sqrt(N^2 g + N (1 - g)) (Eq. 12),
        //    FP32; frequencies outside the grid get F = 0 and contribute nothing.
        for (int o = tc; o < (SHAPE3 ? 0 : TO); o += nt) {
            const int og = tw * TO + o;
            float2 g = make_float2(0.f, 0.f);
            if (og < j.n_omega) {
                const float* gt = reinterpret_cast<const float*>(j.gtab);
                g = make_float2(gload(gt, 2 * (int64_t)og), gload(gt, 2 * (int64_t)og + 1));
            }
            float* dst = ff + o;
#pragma unroll 8
            for (int m = 0; m < P; ++m, dst += TO) {
                const float2 N = nw[m];
                const float Fo = __builtin_amdgcn_sqrtf(fmaf(N.y, g.x, N.x * g.y));
                *dst = (TT && (o & 2)) ? -Fo : Fo;   // sigma_k of the three-term walk
            }
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(1);
        // 4. hot loop.
        for (int m = 0; m < P; ++m) {
            const float4 gm = geo[m * TD + dl];
            const double ph = taus[m * TD + dl];
            float zr = 1.f, zi = 0.f;
            if constexpr (!DIRECT) {
                if constexpr (PREC == 0) {
                    sincos_rev_fast(static_cast<float>(frac_rev(om_seed * ph)), zi, zr);
                } else {
                    float rv = (float)om_seed * (float)ph;
                    rv -= floorf(rv);
                    sincos_rev_fast(rv, zi, zr);
                }
            }
            const float A1 = gm.x, A2 = gm.y;
            float wr = gm.z, wi = gm.w;
            if constexpr (BSTEP) {
                // the block's own rotation exp(i bstep tau), from the FP64 phase
                if constexpr (PREC == 0) {
                    sincos_rev_f64(frac_rev(bstep * ph), wi, wr);
                } else {
                    float rw = (float)bstep * (float)ph;
                    rw -= floorf(rw);
                    sincos_rev_fast(rw, wi, wr);
                }
            }
            const float4* fq = reinterpret_cast<const float4*>(ff + m * TO + ob * W);
            float Nm = 0.f, NN1 = 0.f;
            if constexpr (SHAPE3) {
                const float2 Nv = nw[m];
                Nm = Nv.x;
                NN1 = Nv.y - Nv.x;   // N^2 - N
            }
            // the lane's weights for frequencies 4q .. 4q+3
            auto weights = [&](int q, float (&Fv)[4]) {
                if constexpr (SHAPE3) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {   // F^2 = N + (N^2 - N) g(n, omega) (Eq. 12)
                        Fv[u] = __builtin_amdgcn_sqrtf(fmaxf(fmaf(NN1, gl[4 * q + u], Nm), 0.f));
                    }
                } else {
                    const float4 F4 = fq[q];
                    Fv[0] = F4.x; Fv[1] = F4.y; Fv[2] = F4.z; Fv[3] = F4.w;
                }
            };
            // The three-term walk's sign factors sigma_k (below) ride on the F table; a
            // per-update F (cubic cells) has no table, so there they ride on A instead.
            float nA1 = 0.f, nA2 = 0.f;
            if constexpr (TT && SHAPE3) {
                nA1 = -A1;
                nA2 = -A2;
                asm volatile("" : "+v"(nA1), "+v"(nA2));
            }
            // S(k) += F A exp(i omega_k tau): 2 products and 4 multiply-adds
            auto add = [&](int k, float F, float xr, float xi) {
                const float ur = F * xr, ui = F * xi;
                const float a1 = (TT && SHAPE3 && (k & 2)) ? nA1 : A1;
                const float a2 = (TT && SHAPE3 && (k & 2)) ? nA2 : A2;
                s1r[k] = fmaf(a1, ur, s1r[k]);
                s1i[k] = fmaf(a1, ui, s1i[k]);
                s2r[k] = fmaf(a2, ur, s2r[k]);
                s2i[k] = fmaf(a2, ui, s2i[k]);
            };
            if constexpr (DIRECT) {
                // explicit frequency list: each term's phase from the FP64 product, reduced to
                // [0, 1) revolutions before leaving FP64
#pragma unroll
                for (int q = 0; q < W / 4; ++q) {
                    float Fv[4];
                    weights(q, Fv);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int k = 4 * q + u;
                        if constexpr (PREC == 0) {
                            sincos_rev_fast(static_cast<float>(frac_rev(om[k] * ph)), zi, zr);
                        } else {
                            float rv = (float)om[k] * (float)ph;
                            rv -= floorf(rv);
                            sincos_rev_fast(rv, zi, zr);
                        }
                        add(k, Fv[u], zr, zi);
                    }
                }
            } else if constexpr (TT) {
                // z_{k+1} = c z_k - z_{k-1} with c = 2 cos(theta) = 2 Re(w), theta = domega tau,
                // forward from (z_8, z_9 = z_8 w) and backward from (z_8, z_7 = c z_8 - z_9).
                // To make every step one multiply-add per component without a negation the
                // lane walks y_k = sigma_k z_k, sigma = (+, +, -, -) by k mod 4 (the F table
                // holds sigma_k F_k, or A is negated, so the accumulated term is F_k A z_k):
                //   forward   y_{k+1} = c_k y_k + y_{k-1},  c_k = +c (k even), -c (k odd);
                //   backward  y_{k-1} = c'_k y_k + y_{k+1}, c'_k = -c (k even), +c (k odd).
                // Accuracy: a perturbation e of one step reaches m steps later as
                // e sin(m theta) / sin(theta), at most m e in size, so the rounding of c
                // (about 2^-23) and of each step gives at most ~m^2 ulps after m <= 7 steps
                // -- a few 1e-6 of |z| = 1, also for theta near 0 or pi.  The mid-block seed
                // (short walks) and the accurate w keep this close to the product walk's
                // error; a 15-step walk from one end of the block, or a hardware-quality
                // cos(theta), would lose one to two more decimal digits.
                // +c and -c each in a register of their own, so that every step is a VOP2
                // multiply-add (no negation modifier, which needs the longer VOP3 form)
                float pc = 2.f * wr, nc = -2.f * wr;
                asm volatile("" : "+v"(pc), "+v"(nc));
                float Fh[16];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float Fv[4];
                    weights(q, Fv);
#pragma unroll
                    for (int u = 0; u < 4; ++u) Fh[4 * q + u] = Fv[u];
                }
                // forward: (pr, pi) = y_{k-1}, (cr, ci) = y_k
                float pr = zr, pi = zi;                                          // y8
                float cr = fmaf(zr, wr, -(zi * wi)), ci = fmaf(zr, wi, zi * wr); // y9 = z w
                // y7 = -z_7 = -(c z_8 - z_9) = -c y8 + y9: one multiply-add per component
                const float y7r = fmaf(nc, zr, cr), y7i = fmaf(nc, zi, ci);
                add(8, Fh[8], pr, pi);
                add(9, Fh[9], cr, ci);
#pragma unroll
                for (int k = 9; k < 15; ++k) {
                    const float ck = (k & 1) ? nc : pc;
                    const float nr = fmaf(ck, cr, pr), ni = fmaf(ck, ci, pi);
                    pr = cr; pi = ci; cr = nr; ci = ni;
                    add(k + 1, Fh[k + 1], cr, ci);
                }
                // backward: (pr, pi) = y_{k+1}, (cr, ci) = y_k
                pr = zr; pi = zi;
                cr = y7r; ci = y7i;
                add(7, Fh[7], cr, ci);
#pragma unroll
                for (int k = 7; k > 0; --k) {
                    const float ck = (k & 1) ? pc : nc;
                    const float nr = fmaf(ck, cr, pr), ni = fmaf(ck, ci, pi);
                    pr = cr; pi = ci; cr = nr; ci = ni;
                    add(k - 1, Fh[k - 1], cr, ci);
                }
            } else {
                // Uniform steps (or a block's own step): z_{k+1} = z_k w forward from the seed
                // and z_{k-1} = z_k conj(w) backward from it -- complex products, two products
                // and two multiply-adds per frequency, whose error grows by about one rounding
                // of w per product.  Used where the three-term walk is not: 32 frequencies
                // per lane (walks of 16 steps) and the FP32 geometry variant (whose w comes
                // from the hardware sin/cos).  The opaque negation keeps every operation a
                // VOP2 product or multiply-add without source modifiers.
                float nwi = -wi;
                asm volatile("" : "+v"(nwi));
                float fr = zr, fi = zi;
#pragma unroll
                for (int q = KS / 4; q < W / 4; ++q) {
                    float Fv[4];
                    weights(q, Fv);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int k = 4 * q + u;
                        add(k, Fv[u], fr, fi);
                        if (k + 1 < W) {
                            const float nr = fmaf(fr, wr, fi * nwi), ni = fmaf(fr, wi, fi * wr);
                            fr = nr;
                            fi = ni;
                        }
                    }
                }
                float br = zr, bi = zi;
#pragma unroll
                for (int q = KS / 4 - 1; q >= 0; --q) {
                    float Fv[4];
                    weights(q, Fv);
#pragma unroll
                    for (int u = 3; u >= 0; --u) {
                        const float nr = fmaf(br, wr, bi * wi), ni = fmaf(bi, wr, br * nwi);
                        br = nr;
                        bi = ni;
                        add(4 * q + u, Fv[u], br, bi);
                    }
                }
            }
        }
        __syncthreads();
    }

    // 5. partial tile (coalesced over directions); the lane's place in it is recomputed
    //    from an opaque thread index for the same reason as the set-up's offsets.
    int te = threadIdx.x;
    asm volatile("" : "+v"(te));
    const int dl_e = (te & 63) % DPW;
    const int o_loc = ((te >> 6) * SUBS + (te & 63) / DPW) * W;
    if (td * TD + dl_e < j.n_dir) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (tw * TO + o_loc + k < j.n_omega)
                out[(int64_t)(o_loc + k) * row + dl_e] = make_float4(s1r[k], s1i[k], s2r[k], s2i[k]);
        }
    }
}

// Block b runs on XCD b % 8; return its rank in XCD-major order: XCD 0's blocks first,
// then XCD 1's, ...  For n blocks, XCD x holds n / 8 blocks, plus one if x < n % 8.
__device__ __forceinline__ int xcd_major_id(int b, int n)
{
    constexpr int kXcd = 8;
    const int per = n / kXcd, rem = n % kXcd;
    const int x = b % kXcd, i = b / kXcd;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Waves per SIMD the 16-frequency walk kernels (uniform grid, per-block step) are
// compiled for: 4 caps them at 128 VGPRs, so four waves share a SIMD (the issue rate of
// this VALU-bound loop grows with resident waves; they fit without spills because the
// set-up offsets are recomputed per chunk).  The other kernels keep the default for
// 512-thread workgroups.
#ifndef RAD_W16_WAVES
#define RAD_W16_WAVES 4
#endif
#ifndef RAD_W16V_WAVES
#define RAD_W16V_WAVES 2
#endif
#ifndef RAD_W32_WAVES
#define RAD_W32_WAVES 2
#endif
constexpr int min_waves(int W, int V)
{
    return W == 32 ? RAD_W32_WAVES : ((V == 0 || V == kVarBlockStep) ? RAD_W16_WAVES : RAD_W16V_WAVES);
}

template <typename InT, int PREC, int W, int DPW, int V>
__global__ void __launch_bounds__(512, min_waves(W, V)) k_accumulate(AccArgs a)
{
    extern __shared__ float4 smem4[];
    constexpr int TD = DPW;
    const int TO = (blockDim.x >> 6) * (64 / DPW) * W;
    const int ntiles = a.job.tiles_d * a.job.tiles_w;
    // Workgroups are handed to the 8 XCDs round-robin; renumber them so that consecutive
    // virtual ids -- the tiles of one particle split, which read the same particle chunk --
    // run on one XCD and share its L2 (a bijection on [0, gridDim.x) whatever the policy).
    const int v = xcd_major_id(blockIdx.x, gridDim.x);
    const int tile = v % ntiles;
    const int split = v / ntiles;
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
__global__ void __launch_bounds__(512, min_waves(W, V)) k_accumulate_batch(const Job* __restrict__ items,
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

// Raises `kern`'s dynamic-LDS limit to `lds` bytes on the current device if it needs more
// than the default 64 KiB.  The attribute is set per device; `allowed` caches, per device
// ordinal, the largest limit already set (safe for concurrent callers: at worst two of them
// set the same attribute).
constexpr int kMaxDevices = 64;
inline hipError_t allow_lds(const void* kern, size_t lds, std::atomic<size_t>* allowed)
{
    if (lds <= 64 * 1024) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const bool cached = dev >= 0 && dev < kMaxDevices;
    if (cached && lds <= allowed[dev].load(std::memory_order_acquire)) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess || !cached) return e;
    size_t cur = allowed[dev].load(std::memory_order_relaxed);
    while (cur < lds && !allowed[dev].compare_exchange_weak(cur, lds, std::memory_order_release)) {
    }
    return hipSuccess;
}

template <typename InT, int PREC, int W, int DPW, int V>
hipError_t launch_acc_t(const AccArgs& a, const LaunchShape& s, int n_blocks, hipStream_t st,
                        hipEvent_t ev_start, hipEvent_t ev_stop)
{
    auto kern = k_accumulate<InT, PREC, W, DPW, V>;
    const size_t lds = acc_lds_bytes(s);
    static std::atomic<size_t> lds_allowed[kMaxDevices] = {};   // per instantiation and device
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds, lds_allowed);
    if (e != hipSuccess) return e;
    if (ev_start || ev_stop) {
        AccArgs arg = a;
        void* args[] = {&arg};
        return hipExtLaunchKernel(reinterpret_cast<const void*>(kern), dim3(n_blocks), dim3(64 * s.waves), args, lds,
                                  st, ev_start, ev_stop, 0);
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
    static std::atomic<size_t> lds_allowed[kMaxDevices] = {};   // per instantiation and device
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds, lds_allowed);
    if (e != hipSuccess) return e;
    if (b.prepare_only) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(n_blocks), dim3(64 * s.waves), lds, st, b.items, b.wg_seg_begin,
                       b.segs, b.seg_part);
    return hipGetLastError();
}

// Dispatch on the launch shape to the templated launchers.
template <typename InT, int PREC, typename A>
hipError_t dispatch_shape(const A& a, const LaunchShape& s, int n_blocks, hipStream_t st, hipEvent_t ev0,
                          hipEvent_t ev1)
{
#define RAD_SHAPE_CASE(WW, DD, VV)                                                    \
    if (s.w_per_lane == WW && s.dir_per_wave == DD && s.variant == VV) {              \
        if constexpr (std::is_same<A, AccArgs>::value)                                \
            return launch_acc_t<InT, PREC, WW, DD, VV>(a, s, n_blocks, st, ev0, ev1); \
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
    RAD_SHAPE_CASE(16, 64, 4)
    RAD_SHAPE_CASE(16, 32, 4)
    RAD_SHAPE_CASE(16, 16, 4)
    RAD_SHAPE_CASE(16, 64, 6)
    RAD_SHAPE_CASE(16, 32, 6)
    RAD_SHAPE_CASE(16, 16, 6)
#undef RAD_SHAPE_CASE
    return hipErrorInvalidValue;
}

template <typename A>
hipError_t dispatch_all(const A& a, int dtype, int precision, const LaunchShape& s, int n_blocks,
                        hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    if (dtype == 0) {
        return precision == 0 ? dispatch_shape<float, 0>(a, s, n_blocks, st, ev0, ev1)
                              : dispatch_shape<float, 1>(a, s, n_blocks, st, ev0, ev1);
    }
    return precision == 0 ? dispatch_shape<double, 0>(a, s, n_blocks, st, ev0, ev1)
                          : dispatch_shape<double, 1>(a, s, n_blocks, st, ev0, ev1);
}

}  // namespace

hipError_t launch_accumulate(const AccArgs& a, int dtype, int precision, const LaunchShape& s,
                             int n_blocks, hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop)
{
    return dispatch_all(a, dtype, precision, s, n_blocks, st, ev_start, ev_stop);
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

}  // namespace rad
