// Device helpers shared by the accumulate kernels and the auxiliary kernels: physical
// constants, the revolutions-based sin/cos, input widening and the per (particle,
// direction) geometry of Eq. 1 (radiation amplitude and retarded phase).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rad_internal.h"

namespace rad {

namespace {

constexpr double kInvC = 1.0 / 299792458.0;          // 1/c [s/m]
constexpr double kInv2Pi = 0.15915494309189533577;   // 1/(2 pi)

// Fractional part x - floor(x) of an FP64 phase in revolutions (one v_fract_f64; the
// result lies in [0, 1], and 1 is the same angle as 0).
__device__ __forceinline__ double frac_rev(double x) { return __builtin_amdgcn_fract(x); }

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

// exp(2 pi i r) for a phase r in revolutions held in FP64 (r in [0, 1]): sin/cos of the
// FP32-rounded r, corrected to first order for that rounding (the FP32 argument alone is
// off by up to 3e-8 revolutions, 1.9e-7 rad).  ACCURATE selects the library sin/cos
// (about 4e-8 absolute error measured) over the hardware one (about 1.1e-7).
template <bool ACCURATE = false>
__device__ __forceinline__ void sincos_rev_f64(double r, float& s, float& c)
{
    const float rh = static_cast<float>(r);
    float sh, ch;
    if constexpr (ACCURATE) sincos_rev_accurate(rh, sh, ch);
    else sincos_rev_fast(rh, sh, ch);
    const float d = static_cast<float>(r - static_cast<double>(rh)) * 6.28318530717958648f;
    s = fmaf(ch, d, sh);
    c = fmaf(-sh, d, ch);
}



__device__ __forceinline__ void flag_error(int* err)
{
    atomicOr(err, 1);
}

// Reads p[i] from device (global) memory.  A pointer that reaches a kernel inside a
// structure loaded from memory (the batched kernel's per-item jobs) is generic to the
// compiler, which then emits flat loads; a flat load also counts against the LDS wait
// counter, so every LDS wait of the set-up stages would wait for the HBM reads too.  The
// cast states the address space (a no-op for pointers that are kernel arguments).  T is
// a scalar type (vector class types cannot be copied out of another address space).
template <typename T>
__device__ __forceinline__ T gload(const T* p, int64_t i)
{
    return ((const __attribute__((address_space(1))) T*)p)[i];
}

template <typename InT>
__device__ __forceinline__ double load_wide(const void* p, int64_t i)
{
    return static_cast<double>(gload(static_cast<const InT*>(p), i));
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
    const double nx = gload(dv, 0), ny = gload(dv, 1), nz = gload(dv, 2);
    const double e1x = gload(dv, 3), e1y = gload(dv, 4), e1z = gload(dv, 5);
    const double e2x = gload(dv, 6), e2y = gload(dv, 7), e2z = gload(dv, 8);
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
        // w is reused by every product of a lane's walk (its angle error grows once per
        // product) and is shared by all the frequencies of a workgroup: accurate sin/cos
        if constexpr (WANT_W) sincos_rev_f64<true>(frac_rev(domega * ph), wi, wr);
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

}  // namespace

}  // namespace rad
