// Internal interface between the host runtime and the gfx950 kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rad {

// Particles staged per workgroup chunk (one LDS round).
#ifndef RAD_CHUNK
#define RAD_CHUNK 32
#endif
constexpr int kChunk = RAD_CHUNK;

// One accumulation source: a particle range of one grid (one push, or one batch item).
struct Job {
    const void* f[10];      // x, y, z, bx, by, bz, dbx, dby, dbz, w (element type = kernel InT)
    int64_t i_begin;        // first particle index (into f[])
    int64_t i_end;          // one past the last
    int64_t n_per_step;     // particles per time step (step of element i = i / n_per_step)
    double t0, dt;          // t_j = t0 + j * dt
    const double* dirs9;    // [n_dir][9]: n, e1, e2 (e1, e2 span the plane normal to n)
    const double* omega;    // [n_omega]
    const float2* gtab;     // [n_omega]: (g, 1 - g) of a 1-D shape
    const float* g3;        // [n_dir][n_omega]: g of a 3-D (direction-dependent) shape, or null
    const double* bstep;    // [ceil(n_omega / 16)]: spacing inside each 16-frequency block of a
                            // piecewise-uniform frequency list, or null
    double domega;          // uniform spacing (unused for explicit frequency lists)
    int32_t n_dir, n_omega;
    int32_t tiles_d, tiles_w;
    int* err;               // sticky data-error flag of the grid
};

// Kernel variant bits: how the phase is advanced along the lane's frequencies and where
// the form factor comes from.
constexpr int kVarDirect = 1;   // explicit frequency list: phase from FP64 per term (no walk)
constexpr int kVarShape3 = 2;   // direction-dependent shape factor g(n, omega)
constexpr int kVarBlockStep = 4;  // piecewise-uniform list: frequency walk with a per-block step
// Frequencies per block of a piecewise-uniform list (= frequencies per lane of the variants).
constexpr int kBlockW = 16;

// Arguments of the per-grid accumulate kernel: block b handles tile b % ntiles of split
// b / ntiles, i.e. chunks [split * chunks_per_split, +chunks_per_split) of the job.
struct AccArgs {
    Job job;
    float* part;            // [splits][n_omega][n_dir][4] per-workgroup partial sums
    int32_t splits;
    int64_t chunks_per_split;
};

// Batched launch: every workgroup walks its own list of segments; a segment is a chunk
// range of one (item, tile) and owns one partial tile [TO][TD][4] in the segment buffer.
struct BatchSeg {
    int32_t item;
    int32_t tile;
    int64_t c_begin, c_end;
};

// Fold of one (grid, tile): sum of the listed segments' partial tiles into S.
struct FoldJob {
    double* S;              // grid accumulator, layout [n_omega][n_dir][4]
    int32_t n_dir, n_omega;
    int32_t td, tw;
    int32_t list_begin, list_end;   // into the segment index list
};

// Post-processing variant: one step of tracked particles into per-particle integrals.
struct TrackedArgs {
    const void* f[10];      // x, y, z, bx, by, bz, dbx, dby, dbz, w (w is not used);
                            // n_steps x n_particles elements, step-major
    int64_t n_particles;
    double t;               // time of the first step
    double dt;              // step of the time grid (t_j = t + j dt)
    int32_t n_steps;
    const double* dirs9;
    const double* omega;
    double domega;
    double* T;              // [n_particles][n_omega][n_dir][4] FP64
    int* err;
    int32_t n_dir, n_omega;
};

struct LaunchShape {
    int w_per_lane;    // 16 | 32 (16 only for variant != 0)
    int dir_per_wave;  // 16 | 32 | 64
    int waves;         // 1..8
    int variant = 0;   // kVarDirect | kVarShape3 | kVarBlockStep bits
};

inline int tile_dirs(const LaunchShape& s) { return s.dir_per_wave; }
inline int tile_omegas(const LaunchShape& s) { return s.waves * (64 / s.dir_per_wave) * s.w_per_lane; }
inline size_t acc_lds_bytes(const LaunchShape& s)
{
    const size_t td = tile_dirs(s), to = tile_omegas(s);
    return kChunk * td * 16 + kChunk * td * 8 + 11 * kChunk * 8 + kChunk * 8 + kChunk * to * 4;
}

// Sets the calling thread's message returned by rad_last_error().
void set_last_error(const char* msg);

// Launchers (stream-ordered, return hipError_t).  Non-null ev_start / ev_stop are stamped
// with the kernel's own start and end (hipExtLaunchKernel: no separate marker packets on
// the stream, so timing does not slow the launch sequence down).
hipError_t launch_accumulate(const AccArgs& a, int dtype, int precision, const LaunchShape& s,
                             int n_blocks, hipStream_t st, hipEvent_t ev_start = nullptr,
                             hipEvent_t ev_stop = nullptr);
// count = 4 * grid points (FP32 values per split); part is 16-byte aligned.
hipError_t launch_fold(const float* part, double* S, int splits, int64_t count, hipStream_t st,
                       hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t launch_accumulate_batch(const Job* items, const int32_t* wg_seg_begin, const BatchSeg* segs,
                                   float* seg_part, int dtype, int precision,
                                   const LaunchShape& s, int n_blocks, hipStream_t st);
// Kernel attributes only (no launch), so that a later stream capture records launches only.
hipError_t prepare_accumulate_batch(int dtype, int precision, const LaunchShape& s);
// n_jobs is read on the device (from n_jobs_dev) so that a captured graph can be replayed
// with different plans; the grid is sized for max_jobs.
hipError_t launch_fold_batch(const int32_t* n_jobs_dev, const FoldJob* jobs, int max_jobs,
                             const int32_t* seg_list, const float* seg_part, int td, int to, hipStream_t st);
hipError_t launch_finalize(const double* S, double* I, int n_dir, int n_omega, double C,
                           hipStream_t st);
hipError_t launch_cartesian(const double* S, const double* dirs9, double* out, int n_dir,
                            int n_omega, hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st);
hipError_t launch_trig_probe(const float* in, float* out, int n, hipStream_t st);
hipError_t launch_tracked_accumulate(const TrackedArgs& a, int dtype, bool direct, hipStream_t st);
hipError_t launch_tracked_finalize(const double* T, const double* wts, const double* gk, const double* g3,
                                   int64_t n_particles, int n_dir, int n_omega, double C, double* I,
                                   hipStream_t st);

}  // namespace rad
