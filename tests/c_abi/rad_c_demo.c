/*
 * End-to-end use of the C ABI (include/rad.h) with no Python and no torch: the HIP runtime
 * for device memory, librad.so for everything else.  Test harness for the GPU tests.
 *
 * usage: rad_c_demo IN OUT n_particles n_steps n_dir n_omega omega0 domega dt shape shape_len
 *   IN : raw float64, the 10 particle fields (x y z bx by bz dbx dby dbz w), each
 *        n_steps * n_particles values step-major, followed by n_dir * 3 direction values
 *   OUT: raw float64, the n_dir x n_omega spectrum
 * Pushes step by step (rad_push_step) on a stream of its own, then reads the spectrum.
 * Exit status 0 on success; a failed call prints rad_last_error() and exits 1.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "rad.h"

#define CHECK_RAD(call)                                                           \
    do {                                                                          \
        int rc_ = (call);                                                         \
        if (rc_ != RAD_OK) {                                                      \
            fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, rad_last_error()); \
            return 1;                                                             \
        }                                                                         \
    } while (0)
#define CHECK_HIP(call)                                                           \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));      \
            return 1;                                                             \
        }                                                                         \
    } while (0)

int main(int argc, char** argv)
{
    if (argc != 12) {
        fprintf(stderr, "usage: %s IN OUT n_particles n_steps n_dir n_omega omega0 domega dt shape shape_len\n", argv[0]);
        return 2;
    }
    const long n = atol(argv[3]);
    const int steps = atoi(argv[4]), n_dir = atoi(argv[5]), n_omega = atoi(argv[6]);
    const double omega0 = atof(argv[7]), domega = atof(argv[8]), dt = atof(argv[9]);
    const int shape = atoi(argv[10]);
    const double shape_len = atof(argv[11]);
    if (n < 1 || steps < 1 || n_dir < 1 || n_omega < 1) return 2;
    const size_t per_field = (size_t)n * steps;
    double* host = (double*)malloc(sizeof(double) * (10 * per_field + 3 * (size_t)n_dir));
    double* I = (double*)malloc(sizeof(double) * (size_t)n_dir * n_omega);
    if (!host || !I) return 1;
    FILE* f = fopen(argv[1], "rb");
    if (!f || fread(host, sizeof(double), 10 * per_field + 3 * (size_t)n_dir, f) != 10 * per_field + 3 * (size_t)n_dir) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 1;
    }
    fclose(f);

    double* dev = NULL;
    CHECK_HIP(hipMalloc((void**)&dev, sizeof(double) * 10 * per_field));
    CHECK_HIP(hipMemcpy(dev, host, sizeof(double) * 10 * per_field, hipMemcpyHostToDevice));
    hipStream_t stream;
    CHECK_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));

    rad_grid_desc d;
    d.n_dir = n_dir;
    d.dirs = host + 10 * per_field;
    d.omega0 = omega0;
    d.domega = domega;
    d.n_omega = n_omega;
    d.shape = shape;
    d.shape_len = shape_len;
    d.dt = dt;
    d.precision = RAD_PHASE_F64;
    d.device = 0;
    d.omegas = NULL;
    rad_grid* g = NULL;
    CHECK_RAD(rad_create_grid(&g, &d));
    for (int j = 0; j < steps; ++j) {
        rad_particles p;
        p.dtype = RAD_F64;
        const double* base = dev + (size_t)j * n;
        p.x = base;
        p.y = base + per_field;
        p.z = base + 2 * per_field;
        p.bx = base + 3 * per_field;
        p.by = base + 4 * per_field;
        p.bz = base + 5 * per_field;
        p.dbx = base + 6 * per_field;
        p.dby = base + 7 * per_field;
        p.dbz = base + 8 * per_field;
        p.w = base + 9 * per_field;
        CHECK_RAD(rad_push_step(g, (double)j * dt, n, &p, stream));
    }
    CHECK_RAD(rad_spectrum(g, I, stream));
    CHECK_RAD(rad_destroy_grid(g));
    CHECK_HIP(hipStreamDestroy(stream));
    CHECK_HIP(hipFree(dev));

    f = fopen(argv[2], "wb");
    if (!f || fwrite(I, sizeof(double), (size_t)n_dir * n_omega, f) != (size_t)n_dir * n_omega) {
        fprintf(stderr, "cannot write %s\n", argv[2]);
        return 1;
    }
    fclose(f);
    free(host);
    free(I);
    printf("rad_c_demo: %ld particles x %d steps, %d x %d grid\n", n, steps, n_dir, n_omega);
    return 0;
}
