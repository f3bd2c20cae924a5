/*
 * rad.h - C ABI of the MI355X (gfx950) in-situ radiation-spectrum library.
 *
 * Computes, on the GPU, the spectrally resolved far-field radiation of PIC
 * macro-particles with the form-factor weighting of Pausch et al., arXiv:1802.03972:
 *
 *   d^2I/(dOmega domega)(n, omega) =
 *       C * | sum_j sum_m F_m(omega) A_{j,m}(n) exp(i omega (t_j - n.r_{j,m}/c)) |^2      (Eq. 13)
 *
 *   A = n x [(n - beta) x dbeta/dt] / (1 - beta.n)^2                                       (Eq. 1)
 *   F_m(omega) = sqrt( N_m + (N_m^2 - N_m) g(omega) )                                      (Eqs. 11-12)
 *   g = |F~(omega)|^2 of the normalised macro-particle shape                               (Table 1)
 *   C = (q_e dt)^2 / (16 pi^3 eps0 c)   [J s / sr]
 *
 * The inner sum over macro-particles is accumulated step by step into a
 * device-resident complex spectrum (the in-situ evaluation of Sec. 3.3), so memory is
 * independent of the number of steps and particles.  |.|^2 is taken only when the
 * spectrum is read.
 *
 * Conventions for every call:
 *  - Return value: RAD_OK (0) or a negative RAD_ERR_* code; on error a message is
 *    available from rad_last_error() (per calling thread) and outputs are untouched.
 *  - `stream` is a hipStream_t passed as void*; NULL means the device's null stream.
 *    All work is stream-ordered.  Calls on one grid come from one host thread at a time.
 *    The library orders every update of a grid's accumulator itself (a push's fold runs
 *    on the caller's stream after the grid's previous fold; batched folds, resets and
 *    device read-outs wait for the last fold and become the new last write, which later
 *    calls on other streams wait for), so pushes, resets and read-outs may be issued on
 *    different streams and take effect in the order they are issued.
 *  - Device pointers are plain device addresses on the grid's device, caller-owned.
 *  - Units are SI: r [m], beta [1], dbeta/dt [1/s], N [electrons, real >= 0],
 *    t and dt [s], omega [rad/s], shape length [m].
 */
#ifndef RAD_H
#define RAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define RAD_OK               0
#define RAD_ERR_INVALID_ARG (-1) /* a host-side argument check failed                   */
#define RAD_ERR_OOM         (-2) /* device allocation failed                            */
#define RAD_ERR_DEVICE      (-3) /* a HIP runtime call failed                           */
#define RAD_ERR_BAD_DATA    (-4) /* device saw non-finite data, N < 0 or 1 - beta.n <= 0 */
#define RAD_ERR_QUEUE_FULL  (-5) /* serving: request queue at capacity                  */

/* ---- macro-particle shapes (Table 1; normalised so that g(0) = 1) ---- */
#define RAD_SHAPE_POINT 0 /* g = 1 (all radiation coherent)                        */
#define RAD_SHAPE_CIC   1 /* g = sinc^2(omega L / 2c), sinc(x) = sin(x)/x, L = cell  */
#define RAD_SHAPE_TSC   2 /* g = sinc^4(omega L / 2c)                                */
#define RAD_SHAPE_QSC   3 /* g = sinc^6(omega L / 2c)                                */
#define RAD_SHAPE_GAUSS 4 /* g = exp(-omega^2 L^2 / c^2), rho ~ exp(-x^2 / 2 L^2)      */
/* Direction-dependent shapes of a cubic cell of side L (separable in x, y, z):
 * g(n, omega) = prod_c sinc^(2p)(omega n_c L / 2c), p = 1 (CIC), 2 (TSC), 3 (QSC).  For
 * n along an axis they reduce to the 1-D shapes above. */
#define RAD_SHAPE_CIC3D 5
#define RAD_SHAPE_TSC3D 6
#define RAD_SHAPE_QSC3D 7

/* ---- arithmetic modes ---- */
#define RAD_PHASE_F64 0 /* default: geometry and phase t - n.r/c in FP64, FP32 update */
#define RAD_ALL_F32   1 /* everything in FP32 (precision study only)                 */

/* ---- particle element types ---- */
#define RAD_F32 0
#define RAD_F64 1

typedef struct rad_grid rad_grid;

/* Observation grid of one spectrum (Eq. 13 is evaluated on every (n, omega) pair). */
typedef struct rad_grid_desc {
    int32_t n_dir;       /* number of directions, >= 1                                  */
    const double* dirs;  /* HOST pointer, n_dir x 3 unit vectors (|n| within 1e-6 of 1);
                            copied at creation                                          */
    double omega0;       /* first frequency [rad/s], >= 0 (ignored with `omegas`)       */
    double domega;       /* uniform spacing [rad/s], >= 0; omega_k = omega0 + k*domega  */
    int32_t n_omega;     /* number of frequencies, >= 1                                 */
    int32_t shape;       /* RAD_SHAPE_*                                                  */
    double shape_len;    /* cell width (CIC/TSC/QSC) or sigma (GAUSS) [m], > 0 unless POINT */
    double dt;           /* time step of Eq. 13 [s], > 0 (enters the prefactor only)   */
    int32_t precision;   /* RAD_PHASE_F64 or RAD_ALL_F32                                 */
    int32_t device;      /* HIP device ordinal                                          */
    const double* omegas;/* optional HOST list of n_omega frequencies [rad/s] (finite, >= 0,
                            any spacing, e.g. logarithmic); NULL: the uniform grid above.
                            The list is classified at creation (rad_grid_variant):
                            uniform to a few FP64 ulps -> the uniform grid; every aligned
                            block of 16 entries an arithmetic progression (piecewise-
                            uniform) -> the frequency walk with a per-block step;
                            otherwise each term's phase is evaluated from FP64.  Lists
                            that are not uniform use 16 frequencies per lane            */
} rad_grid_desc;

/* One batch of macro-particles, structure of arrays, all fields the same type. */
typedef struct rad_particles {
    int32_t dtype;                 /* RAD_F32 or RAD_F64                               */
    const void *x, *y, *z;         /* position r [m]                                   */
    const void *bx, *by, *bz;      /* velocity beta = v/c                              */
    const void *dbx, *dby, *dbz;   /* dbeta/dt [1/s]                                   */
    const void *w;                 /* weighting N (electrons per macro-particle)       */
} rad_particles;

/* Create a grid: the observation points (n, omega) on which Eq. 13 (Sec. 3.3) is
 * evaluated -- every direction n of the far-field sum of Eq. 1 (Sec. 2) paired with every
 * frequency omega -- with the macro-particle shape whose normalised Table 1 factor g(omega)
 * enters F_m of Eqs. 11-12.  Copies the directions, builds the frequency and shape tables
 * and a zeroed FP64 accumulator of the complex sum on `d->device`.  Host-side argument
 * errors return RAD_ERR_INVALID_ARG, device allocation failures RAD_ERR_OOM, other HIP
 * failures RAD_ERR_DEVICE; *out is written only on success. */
int rad_create_grid(rad_grid** out, const rad_grid_desc* d);

/* Release a grid.  Waits for the grid's device to finish outstanding work first.
 * NULL is accepted (no-op). */
int rad_destroy_grid(rad_grid* g);

/* Zero the accumulated spectrum and clear the sticky data-error flag (stream-ordered). */
int rad_reset(rad_grid* g, void* stream);

/* Add one time step (Eq. 13 inner sum at t_j = t): for every (n, omega) of the grid,
 * S += sum_{m<n_particles} F_m(omega) A_m(n) exp(i omega (t - n.r_m / c)).
 * Particle arrays are device pointers of length n_particles and must stay valid until
 * the stream passes this call.  n_particles == 0 is a no-op.  Data checked on the
 * device (non-finite values, N < 0, 1 - beta.n <= 0) set a sticky flag that the next
 * rad_spectrum / rad_spectrum_complex / rad_get_state reports as RAD_ERR_BAD_DATA.
 * Phase accuracy: the phase omega (t - n.r/c) / 2 pi is formed in FP64 and reduced to
 * [0, 1) revolutions, so its absolute error is about 1.1e-16 of its size; for 1e-7
 * revolutions at omega = 1e20 rad/s keep |t - n.r/c| below ~30 ps.  The spectrum does
 * not change when one constant is added to every t (it multiplies S by a common phase),
 * so callers may subtract a reference time from all steps' t. */
int rad_push_step(rad_grid* g, double t, int64_t n_particles, const rad_particles* p,
                  void* stream);

/* Add n_steps consecutive steps at t_j = t0 + j*dt (dt of the grid), j = 0..n_steps-1.
 * Arrays hold n_steps * n_particles elements, step-major (element j*n_particles + m).
 * Same ownership and error behaviour as rad_push_step. */
int rad_push_steps(rad_grid* g, double t0, int32_t n_steps, int64_t n_particles,
                   const rad_particles* p, void* stream);

/* ---- push without device allocation -------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, ownership, ordering and
 * result as rad_push_step, but the call allocates nothing (no hipMalloc or hipFree, no
 * events or streams): the accumulate kernel's FP32 partial sums go to a fixed device
 * array inside the library, RAD_NOALLOC_SCRATCH_BYTES on each GPU (reserved when the
 * library's code is loaded on that GPU, held until the process ends), and the fold into
 * the grid's accumulator runs on `stream` right after the accumulate.  The grid itself
 * comes from rad_create_grid as usual.
 * Limits: a grid needs 16 * n_dir * n_omega bytes of scratch per particle split; grids of
 * more than RAD_NOALLOC_SCRATCH_BYTES / 16 points are rejected with RAD_ERR_INVALID_ARG,
 * and a push uses at most RAD_NOALLOC_SCRATCH_BYTES / (16 * n_dir * n_omega) splits at a
 * time (more launches for long pushes; the result then differs from rad_push_step's only
 * by FP32 rounding of the partial sums).  Kernel timing (rad_profile_*) does not cover it.
 * All calls on one GPU share the scratch and leave their partial sums in it: calls that
 * can overlap on one GPU (issued on different streams with no ordering between them)
 * race and give wrong results; order them on one stream.
 * Under HIP stream capture the call records no event and waits on none, so the captured
 * kernels carry no ordering against the grid's other work: capture after that work has
 * completed and replay on the stream that issues the grid's other calls. */
#define RAD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int rad_push_step_noalloc(rad_grid* g, double t, int64_t n_particles, const rad_particles* p,
                          void* stream);

/* Read d^2I/(dOmega domega) [J s/sr] into I_host (HOST, n_dir x n_omega doubles,
 * row-major by direction): the squared modulus of the accumulated complex sum of Eq. 13
 * (Sec. 3.3) times its prefactor, read as C = (q_e dt)^2 / (16 pi^3 eps0 c) -- the
 * rectangle-rule dt of the time integral inside the square, which is what makes Eq. 13
 * consistent in units with Eq. 1 (the printed prefactor has dt and q_e outside it).
 * Synchronises `stream`.  Non-destructive: accumulation may continue afterwards.  Returns
 * RAD_ERR_BAD_DATA (and writes nothing) if the flag is set. */
int rad_spectrum(rad_grid* g, double* I_host, void* stream);

/* Same as rad_spectrum (Eq. 13's C |.|^2) into a DEVICE buffer of n_dir x n_omega
 * doubles, without synchronising; the data-error flag is not checked.  Later pushes and
 * resets of the grid, on any stream, take effect only after this read-out. */
int rad_spectrum_device(rad_grid* g, double* I_dev, void* stream);

/* Read the complex spectrum S(n, omega) -- the vector sum inside |.|^2 of Eq. 13
 * (Sec. 3.3), without the prefactor C -- into S_host (HOST, n_dir x n_omega x 3 complex,
 * Cartesian components, interleaved re/im: index ((d*n_omega + k)*3 + c)*2).
 * Synchronises `stream`.  Returns RAD_ERR_BAD_DATA (and writes nothing) if the flag is set. */
int rad_spectrum_complex(rad_grid* g, double* S_host, void* stream);

/* Number of doubles in the opaque accumulator state of this grid. */
size_t rad_state_size(const rad_grid* g);

/* Copy the accumulator state to / from HOST memory (rad_state_size doubles).  A state
 * taken from one grid may be loaded into any grid with the same n_dir and n_omega.
 * Both synchronise `stream`.  Used for checkpoint / resume. */
int rad_get_state(rad_grid* g, double* state_host, void* stream);
int rad_set_state(rad_grid* g, const double* state_host, void* stream);

/* Per-thread message of the last failed call on this thread ("" if none). */
const char* rad_last_error(void);

/* Launch shape used by the accumulate kernel of a grid.
 *   w_per_lane : frequencies held per lane (16 or 32)
 *   dir_per_wave: directions per wavefront (16, 32 or 64)
 *   waves      : wavefronts per workgroup (1..8)
 *   wg_per_cu  : workgroups per compute unit in one launch (1..16): a push is cut into
 *                CUs * wg_per_cu / tiles particle splits (the hardware runs as many of
 *                them at once as registers and LDS allow)
 * rad_set_tile validates and applies it to later pushes. */
typedef struct rad_tile {
    int32_t w_per_lane;
    int32_t dir_per_wave;
    int32_t waves;
    int32_t wg_per_cu;
} rad_tile;
int rad_get_tile(const rad_grid* g, rad_tile* t);
int rad_set_tile(rad_grid* g, const rad_tile* t);

/* Kernel variant chosen for a grid at creation, as bits (or a negative code):
 *   1  explicit frequency list, per-term FP64 phase
 *   2  direction-dependent (cubic-cell) shape factor
 *   4  piecewise-uniform frequency list, frequency walk with a per-block step
 * 0 is the uniform frequency grid with a 1-D shape.  Launch-shape tables key on it. */
int rad_grid_variant(const rad_grid* g);

/* Kernel timing of one grid.  rad_profile_enable(g, k) with k >= 1 times every k-th
 * accumulate launch of the grid and the fold launch that follows it (1: every launch; 0
 * stops timing): the launches carry HIP start and stop events stamped by the launch itself
 * on its own stream (hipExtLaunchKernel; no marker packets between launches; each timed
 * launch still costs a few microseconds).  rad_profile_read waits for the recorded events,
 * returns the totals of the timed launches since the last read (or enable) and clears
 * them. */
typedef struct rad_profile_stats {
    int64_t launches;        /* accumulate launches timed                               */
    int64_t updates;         /* particle x direction x frequency terms in those launches */
    double accumulate_ms;    /* summed accumulate kernel time [ms]                      */
    double fold_ms;          /* summed fold kernel time [ms]                            */
} rad_profile_stats;
int rad_profile_enable(rad_grid* g, int enable);
int rad_profile_read(rad_grid* g, rad_profile_stats* out);

/* ---- several grids in one persistent launch ------------------------------------ */

/* One unit of batched work: n_steps consecutive steps (t_j = t0 + j*dt of the grid) of
 * n_particles macro-particles each, accumulated into `grid` exactly as rad_push_steps
 * would (arrays of n_steps * n_particles elements, step-major, device pointers). */
typedef struct rad_batch_item {
    rad_grid* grid;
    double t0;
    int32_t n_steps;
    int64_t n_particles;
    rad_particles p;
} rad_batch_item;

typedef struct rad_batcher rad_batcher;

/* A batcher owns the device work plan and the partial-sum scratch of batched launches on
 * `device`.  max_items bounds the items of one rad_batcher_push. */
int rad_batcher_create(rad_batcher** out, int32_t device, int32_t max_items);
int rad_batcher_destroy(rad_batcher* b);

/* Accumulate every item into its grid with one persistent launch: the (item, tile,
 * particle-chunk) iterations of all items are cut into equal contiguous ranges, one per
 * workgroup, so bunches of very different sizes share the device evenly; then one fold
 * launch adds the per-range partial tiles (fixed order, FP64) into each grid.  The result
 * equals that of pushing each item on its own, up to FP32 rounding of the partial sums.
 * Requirements: all grids on the batcher's device with the same precision mode, all items
 * of one particle dtype; grid shapes may differ.  The launch shape is the batcher's own
 * (rad_batcher_set_tile), independent of the grids' single-push tiles.  Several items may
 * target the same grid.  Stream-ordered; the host blocks only to recycle a plan buffer
 * used two calls earlier.  Calls on one batcher must be ordered on one stream. */
int rad_batcher_push(rad_batcher* b, const rad_batch_item* items, int32_t n_items, void* stream);

/* Launch shape of the batched kernel; NULL restores the default (the built-in heuristic
 * for the first item's grid shape, chosen at each push).  wg_per_cu sets the number of
 * workgroups (ranges) per compute unit of the persistent launch. */
int rad_batcher_set_tile(rad_batcher* b, const rad_tile* t);
int rad_batcher_get_tile(rad_batcher* b, rad_tile* t);

/* Graph mode: the batcher lays every plan out with fixed capacities (max_items items,
 * one range per workgroup of the whole device) and replays a hipGraph captured once per
 * launch configuration -- upload of the plan from pinned host memory, the persistent
 * accumulate launch and the fold -- instead of issuing the three operations each push.
 * A plan that does not fit the capacities (more than 16 tiles per item on average) is
 * launched directly.  If capture fails the batcher falls back to direct launches. */
int rad_batcher_set_graph(rad_batcher* b, int enable);
/* Captured graphs held, graph replays issued, capture failures. */
int rad_batcher_graph_stats(rad_batcher* b, int64_t* graphs, int64_t* launches, int64_t* failures);

/* Kernel timing of a batcher's launches (same semantics as rad_profile_*; in graph mode
 * a replay is timed as a whole and reported as accumulate time). */
int rad_batcher_profile_enable(rad_batcher* b, int enable);
int rad_batcher_profile_read(rad_batcher* b, rad_profile_stats* out);

/* ---- serving loop: continuous batching of per-step chunks of many bunches -------- */

typedef struct rad_server rad_server;

typedef struct rad_server_config {
    int32_t device;
    size_t hbm_budget;      /* bytes of device memory for admitted chunks (>= 1 MiB)      */
    int32_t max_batch;      /* chunks per batched launch (>= 1)                            */
    int32_t max_inflight;   /* batched launches queued on the device at once (1 or 2;
                               larger values are treated as 2)                             */
    int32_t max_admitted;   /* chunks admitted (copying or copied) but not yet launched    */
    int64_t max_pending;    /* chunks submitted but not yet admitted; beyond it submit
                               returns RAD_ERR_QUEUE_FULL                                  */
    int32_t poll_us;        /* scheduler wake-up period when nothing moves [us] (>= 1)     */
    int32_t use_graph;      /* 1: replay captured graphs for the batched launches          */
} rad_server_config;

/* Per-chunk timeline on the server clock [s since creation] and the launch it rode in. */
typedef struct rad_chunk_stats {
    double t_submit, t_admit, t_launch, t_complete;
    int32_t batch_size;
    int32_t status;          /* RAD_OK or the first error the server met */
    int64_t batch_id;        /* 1, 2, ... in launch order: chunks with the same id shared
                                one batched launch */
} rad_chunk_stats;

typedef struct rad_server_counters {
    int64_t submitted, admitted, chunks_launched, batches, completed;
    int64_t pending;           /* waiting for admission (backlog)       */
    int64_t admitted_waiting;  /* admitted, not yet launched            */
    int64_t inflight_batches;
    size_t pool_used;          /* bytes of the HBM budget in use        */
    double now;                /* server clock [s]                      */
} rad_server_counters;

/* Start a server with its own scheduler thread, copy and compute streams (default
 * priority) and a device chunk pool of hbm_budget bytes on cfg->device. */
int rad_server_create(rad_server** out, const rad_server_config* cfg);

/* Queue one chunk: n particles of one time step t of `grid`, given in HOST memory (SoA,
 * one dtype).  The host arrays must stay valid and unchanged until the chunk completes.
 * Admission is in arrival order, when the chunk's device footprint (10 fields, 256-byte
 * aligned) fits in the free part of the budget; the server then copies it, batches it with
 * every other copied chunk (any bunch) into one batched persistent launch, and releases
 * its bytes when the launch completes.  Never drops a chunk; a chunk larger than the whole
 * budget is rejected (RAD_ERR_INVALID_ARG).  Chunks of one grid may be in flight together.
 * While a server runs, other calls on its grids must wait for rad_server_drain. */
int rad_server_submit(rad_server* s, rad_grid* grid, double t, int64_t n, const rad_particles* host_p,
                      uint64_t* ticket);

/* 1 and the chunk's stats if the chunk completed (the ticket is then retired), 0 if not
 * yet, negative on error. */
int rad_server_poll(rad_server* s, uint64_t ticket, rad_chunk_stats* st);

/* Block until the chunk completes; 1 on success (ticket retired) or a negative code. */
int rad_server_wait(rad_server* s, uint64_t ticket, rad_chunk_stats* st);

/* Block until every submitted chunk has completed. */
int rad_server_drain(rad_server* s);

int rad_server_counters_read(rad_server* s, rad_server_counters* out);

/* Launch shape of the server's batched launches (as rad_batcher_set_tile; NULL restores
 * the library default) and the shape in use (RAD_ERR_INVALID_ARG while the default
 * applies).  Takes effect from the next batch. */
int rad_server_set_tile(rad_server* s, const rad_tile* t);
int rad_server_get_tile(rad_server* s, rad_tile* t);

/* Kernel timing of the server's batched launches (as rad_batcher_profile_*: events on
 * the server's compute stream around each launch; with graph replays, around the whole
 * replay).  rad_server_profile_read waits for the recorded events. */
int rad_server_profile_enable(rad_server* s, int enable);
int rad_server_profile_read(rad_server* s, rad_profile_stats* out);

/* Drain, stop the scheduler thread and free the server (not its grids). */
int rad_server_destroy(rad_server* s);

/* ---- post-processing variant: tracked particles -------------------------------- */

/* For a small set of tracked particles (same particles, same order, every step) the
 * device keeps each particle's own time integral T_m(n, omega) = sum_j A_{j,m}(n) chi_{j,m}
 * in FP64 (n_particles x n_dir x n_omega x 2 complex numbers), and the form factor is
 * applied only when the spectrum is read (the post-processing alternative of Sec. 3.3):
 *   I = C | sum_m F_m(omega) T_m(n, omega) |^2,  F_m = sqrt(N_m + (N_m^2 - N_m) g).
 * With constant weights this equals the in-situ sum; weights and shape may be changed
 * between read-outs without recomputing.  Memory grows with the number of particles,
 * which is why this is meant for test-particle sets only. */
typedef struct rad_tracked rad_tracked;

/* Grid fields of `d` (directions, frequencies or frequency list, dt, device) are used;
 * the shape fields are ignored (chosen at read-out); precision must be RAD_PHASE_F64. */
int rad_tracked_create(rad_tracked** out, const rad_grid_desc* d, int64_t n_particles);
int rad_tracked_destroy(rad_tracked* tr);
int rad_tracked_reset(rad_tracked* tr, void* stream);

/* One step at time t; device arrays of n_particles elements (the weight field is not
 * read and may be NULL).  Stream-ordered; data errors set the sticky flag reported at read-out. */
int rad_tracked_push_step(rad_tracked* tr, double t, const rad_particles* p, void* stream);

/* n_steps steps at t0 + j dt (dt of the descriptor), device arrays of n_steps x
 * n_particles elements, step-major.  Up to rad_tracked_step_group() steps are summed in
 * FP32 registers before each update of the FP64 integrals, which cuts their HBM traffic by
 * that factor. */
int rad_tracked_push_steps(rad_tracked* tr, double t0, int32_t n_steps, const rad_particles* p, void* stream);

/* Steps summed in registers per read-modify-write of the integrals (128). */
int rad_tracked_step_group(void);

/* Spectrum with the given HOST weights (n_particles, >= 0) and shape applied now;
 * I_host: n_dir x n_omega doubles.  Synchronises `stream`. */
int rad_tracked_spectrum(rad_tracked* tr, const double* weights_host, int32_t shape, double shape_len,
                         double* I_host, void* stream);

/* Library and device facts: compute-unit count of `device`, or a negative code. */
int rad_device_cus(int32_t device);



#ifdef __cplusplus
}
#endif

#endif /* RAD_H */
