// Internal interface between the host runtime and the gfx950 kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rad {

// Particles staged per workgroup chunk (one LDS round).
constexpr int kChunk = 32;

// Arguments of the accumulate kernel.  Pointers are device addresses.
struct AccArgs {
    const void* f[10];      // x, y, z, bx, by, bz, dbx, dby, dbz, w (element type = kernel InT)
    int64_t i_begin;        // first particle index of this launch (into f[])
    int64_t i_end;          // one past the last
    int64_t n_per_step;     // particles per time step (step of element i = i / n_per_step)
    double t0, dt;          // t_j = t0 + j * dt
    const double* dirs9;    // [n_dir][9]: n, e1, e2 (e1, e2 span the plane normal to n)
    const double* omega;    // [n_omega]
    const float2* gtab;     // [n_omega]: (g, 1 - g) of the shape
    double domega;
    float* part;            // [splits][n_omega][n_dir][4] per-workgroup partial sums
    int* err;               // sticky data-error flag
    int32_t n_dir, n_omega;
    int32_t tiles_d, tiles_w;
    int32_t splits;
    int64_t chunks_per_split;
};

struct LaunchShape {
    int w_per_lane;    // 16 | 32
    int dir_per_wave;  // 16 | 32 | 64
    int waves;         // 1..8
};

inline int tile_dirs(const LaunchShape& s) { return s.dir_per_wave; }
inline int tile_omegas(const LaunchShape& s) { return s.waves * (64 / s.dir_per_wave) * s.w_per_lane; }
inline size_t acc_lds_bytes(const LaunchShape& s)
{
    const size_t td = tile_dirs(s), to = tile_omegas(s);
    return kChunk * td * 16 + kChunk * td * 8 + 11 * kChunk * 8 + kChunk * to * 4;
}

// Launchers (stream-ordered, return hipError_t).
hipError_t launch_accumulate(const AccArgs& a, int dtype, int precision, const LaunchShape& s,
                             int n_blocks, hipStream_t st);
hipError_t launch_fold(const float* part, double* S, int splits, int64_t count, hipStream_t st);
hipError_t launch_finalize(const double* S, double* I, int n_dir, int n_omega, double C,
                           hipStream_t st);
hipError_t launch_cartesian(const double* S, const double* dirs9, double* out, int n_dir,
                            int n_omega, hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st);
hipError_t launch_trig_probe(const float* in, float* out, int n, hipStream_t st);

}  // namespace rad
