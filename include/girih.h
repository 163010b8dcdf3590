/*
 * girih.h — C ABI of the MI355X (gfx950) multi-threaded wavefront diamond
 * (MWD) stencil library.
 *
 * The operation (paper: Section "Background / Cache blocking" and Listings
 * 1-4): T Jacobi steps u^{t+1} = F(u^t) of one of four 3-D stencils on a
 * structured grid with a fixed Dirichlet halo of width R (the stencil radius),
 * using two solution buffers whose roles swap after each step.  The blocked
 * algorithm (Section "Approach", the MWD listing) reorders the point updates
 * with diamond tiles in (t, y) and a wavefront along z, several threads per
 * tile; it reaches exactly the result of the naive sweep.
 *
 * Conventions
 *  - All pointers to grid data are DEVICE pointers (HIP) owned by the caller;
 *    the library never frees them.  Host pointers are only the small
 *    descriptor structs, coefficient scalars and output arguments.
 *  - Layout: element (k, j, i) — z, y, x, x fastest — with k in [-h, nz+h),
 *    j in [-h, ny+h), i in [-h, nx+h) lives at element offset
 *    ((k+h)*pitch_y + (j+h))*pitch_x + (i+h); pitch_x >= nx+2h,
 *    pitch_y >= ny+2h.  h must equal the stencil radius (1 or 4).
 *  - Element type: double (GIRIH_F64) or float (GIRIH_F32); all arithmetic of
 *    the sweep is done in that type, in the listing's left-to-right order,
 *    without fused multiply-add.
 *  - Every function returns 0 (GIRIH_OK) or a negative error code; nothing
 *    is launched when an argument is rejected.  girih_strerror() names codes.
 *  - A plan may be used by one host thread / one stream at a time.
 */
#ifndef GIRIH_H
#define GIRIH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GIRIH_OK 0
#define GIRIH_E_INVALID (-1)     /* bad argument (null pointer, size, halo, pitch, T < 0, ...) */
#define GIRIH_E_UNSUPPORTED (-2) /* valid request the library has no kernel for */
#define GIRIH_E_LDS (-3)         /* tile parameters exceed the on-chip budget */
#define GIRIH_E_HIP (-4)         /* a HIP runtime call failed */
#define GIRIH_E_NOMEM (-5)       /* device or host allocation failed */
#define GIRIH_E_NOGPU (-6)       /* no usable gfx950 device */
#define GIRIH_E_SCRATCH (-7)     /* grid larger than girih_run_noalloc's fixed scratch */
#define GIRIH_E_STALL (-8)       /* a bounded device wait of variants 1-3 gave up (girih_check) */

/* Stencils (paper Listings 1-4; the 25-point constant stencil is the
 * first-order Jacobi form of Listing 3's bracketed term, the leapfrog one is
 * Listing 3 as printed). */
typedef enum {
    GIRIH_7PT_CONST = 0,  /* c0, c1 scalars                         */
    GIRIH_7PT_VAR = 1,    /* 7 coefficient arrays C0..C6            */
    GIRIH_25PT_CONST = 2, /* c0..c4 scalars, radius 4               */
    GIRIH_25PT_VAR = 3,   /* 13 coefficient arrays C00..C12, R = 4  */
    GIRIH_25PT_LEAPFROG = 4, /* c0..c4 scalars and 1 array C, R = 4:
                             * u^{t+1} = (2u^t - u^{t-1}) + C*(bracket of u^t);
                             * buf1 holds u^{t-1} = u^{-1} on entry (its
                             * interior is read), buf0 holds u^0 */
    GIRIH_27PT_BOX = 5      /* c0..c3 scalars, R = 1: the 27-point box stencil
                             * (Section "Handling other stencil types"),
                             * ((c0*V + c1*F) + c2*E) + c3*K with F, E, K the
                             * sums of the 6 face, 12 edge and 8 corner
                             * neighbours, each in lexicographic order of the
                             * offset (dz, dy, dx); blocked at Dw = 8
                             * (FP32 also 12), wavefront depth 1, row
                             * launches */
} girih_stencil;

typedef enum { GIRIH_F64 = 0, GIRIH_F32 = 1 } girih_dtype;

typedef enum {
    GIRIH_NAIVE = 0, /* T launches of one full-domain Jacobi step              */
    GIRIH_MWD = 1    /* diamond rows: one launch per row of diamond tiles      */
} girih_algo;
/* GIRIH_MWD exists for every stencil, in the diamond shapes compiled for it
 * (girih_candidates); girih_plan returns GIRIH_E_UNSUPPORTED for a shape that
 * was not compiled.  For the second-order-in-time stencil a level also reads
 * the level two below it at its own cell.  For the box stencil a level reads
 * the level below at three planes of the neighbouring rows: its levels are
 * skewed by two planes along z, and a stage row holds those three planes. */

/* Grid descriptor, in elements. */
typedef struct girih_grid {
    int64_t nx, ny, nz; /* interior points                      */
    int32_t halo;       /* must equal the stencil radius         */
    int64_t pitch_x;    /* >= nx + 2*halo (0 = nx + 2*halo)      */
    int64_t pitch_y;    /* >= ny + 2*halo (0 = ny + 2*halo)      */
} girih_grid;

/* Tile parameters (paper, Section "Auto-tuning": diamond width, wavefront
 * width, threads along x/y/z).  Zero fields are filled with defaults.
 *  MWD:   diamond_width  Dw, multiple of 2R (of 4 when R = 1);
 *         wavefront_depth N_F, z-planes per wavefront step (1; 2 for the
 *                        shapes compiled with it, girih_candidates);
 *         tile_x         x cells one workgroup owns and stores;
 *         threads_x      threads along x per diamond row = 64 * waves along x;
 *         cells_per_lane x cells each of those threads holds (1, 2, 4): a row
 *                        of the workgroup spans threads_x * cells_per_lane
 *                        cells, owned tile plus the recomputed halo;
 *         threads_y      row pairs = waves along y (filled in: Dw/2);
 *         tile_y, tile_z filled in: Dw and nz;
 *         variant        two bits.  Bit 0, schedule of the diamond rows
 *                        (paper, Section "Runtime system"): 0 = one launch
 *                        per row (the stream orders the rows); 1 = one
 *                        launch of a workgroup per tile of every row, in
 *                        row order, each tile starting once the tiles of
 *                        the previous row it depends on are done.  Bit 1,
 *                        synchronisation of the waves of a tile (paper,
 *                        Section "Multi-core wavefront temporal blocking"):
 *                        0 = workgroup barriers in every wavefront step;
 *                        1 = relaxed: each wave waits only for the waves
 *                        whose stage rows it reads or that read its own.
 *                        Either bit needs a shape compiled with it
 *                        (girih_candidates lists them).
 *         With diamond_width, cells_per_lane, threads_x, wavefront_depth
 *         and variant all zero, the library's default plan for the stencil
 *         and precision is taken: its shape, depth and schedule (bit 0 set
 *         for the 25-point constant and 7-point variable stencils in FP64,
 *         where it measured faster).
 *  NAIVE: variant        0 = x/y neighbours through the caches (any block
 *                        of at most 256 threads, threads_x a multiple of 64),
 *                        1 = each plane's x/y neighbourhood staged in an LDS
 *                        tile (threads_x = 64, threads_y = 4, 8 or 16); for
 *                        GIRIH_27PT_BOX, 1 = register columns: each wave of
 *                        64 lanes holds cells_per_lane (2, 4 or 8) rows along
 *                        y of three planes, takes x neighbours from the
 *                        neighbouring lanes and stores 62 x cells per row
 *                        (threads_x = 64, threads_y = 2 or 4; tile_x and
 *                        tile_y are filled in: 62 and threads_y *
 *                        cells_per_lane),
 *                        2 = register columns for GIRIH_7PT_CONST and
 *                        GIRIH_25PT_CONST: each wave holds cells_per_lane
 *                        (2, 4 or 8) rows of the 2R+1 planes of their
 *                        z-window and the 2R rows beside them, takes x
 *                        neighbours from the neighbouring lanes and stores
 *                        64 - 2R x cells per row (same block shapes; tile_x
 *                        = 64 - 2R);
 *         threads_x, threads_y  block shape (x lanes, y rows);
 *         tile_z         z planes each thread marches.
 *         All zero: variant 1 with 64 x 16 threads and z chunks of up to
 *         128 planes; in FP32 for GIRIH_7PT_CONST and GIRIH_25PT_CONST
 *         variant 2 with 64 x 2 threads of 4 and 8 rows and up to 12 planes;
 *         for the box stencil variant 1 with 64 x 2 threads of 8 rows and up
 *         to 32 planes (FP64) or of 4 rows and up to 12 planes (FP32); fewer
 *         planes per chunk on small grids. */
typedef struct girih_params {
    int32_t diamond_width;
    int32_t wavefront_depth;
    int32_t tile_x;
    int32_t tile_y;
    int32_t tile_z;
    int32_t threads_x;
    int32_t threads_y;
    int32_t variant;
    int32_t cells_per_lane;
} girih_params;

typedef struct girih_plan_s* girih_plan_t;

/* Create a plan (paper, Section "Auto-tuning": the user selects the stencil
 * type and grid size).  const_coefs: host array of c0,c1 (7-point constant)
 * or c0..c4 (25-point constant) in double precision — rounded once to float
 * for GIRIH_F32 plans; NULL for variable-coefficient stencils.  params: NULL
 * or a struct whose zero fields take defaults.  Validates everything
 * (including the on-chip budget of the tile) and allocates nothing on the
 * device. */
int girih_plan(girih_plan_t* out, girih_stencil stencil, girih_dtype dtype, const girih_grid* grid,
               const double* const_coefs, girih_algo algo, const girih_params* params);

/* Run T time steps on the caller's buffers, asynchronously on hip_stream
 * (a hipStream_t; NULL = default stream).
 *  buf0: u^0 including its halo.  buf1: same size; its halo is overwritten
 *  with buf0's, its interior is never read.  Both interiors are clobbered.
 *  coef_arrays: host array of n_coef DEVICE pointers (7 for 7-point variable,
 *  13 for 25-point variable, same layout as the field; halos never read), or
 *  NULL with n_coef = 0.
 *  On return *result_index = T % 2: the result is the interior of that buffer.
 *  MWD plans use two plan-owned scratch arrays of the same size, allocated on
 *  the first run (GIRIH_E_NOMEM if that fails) and freed by girih_destroy. */
int girih_run(girih_plan_t plan, void* buf0, void* buf1, const void* const* coef_arrays, int32_t n_coef,
              int64_t T, void* hip_stream, int32_t* result_index);

/* girih_run for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * sweep, arguments, result and errors as girih_run, but the memory it needs
 * beside the caller's buffers -- for MWD plans the pair of grid-sized arrays
 * and the halo flag -- lives in a fixed device array of the library instead
 * of plan-owned allocations.  It calls no hipMalloc, hipFree or other
 * allocating routine, and records no launch timing.
 *  Limit: each array of the grid (pitches and halos included) at most
 *  64 MiB (e.g. 200^3 FP64, 250^3 FP32); larger MWD grids return
 *  GIRIH_E_SCRATCH before anything is launched.  NAIVE plans need no
 *  scratch and have no limit.
 *  The fixed array exists once per device for the life of the process and
 *  is shared by every call on that device: calls that overlap on one device
 *  (other streams, other threads) race and must be serialised by the caller.
 *  Nothing in it needs to start at zero (each run initialises what it
 *  reads).  Plans with variant bit 0 set run with one launch per diamond
 *  row here (the fixed array has no room for the schedule's completion
 *  marks). */
int girih_run_noalloc(girih_plan_t plan, void* buf0, void* buf1, const void* const* coef_arrays, int32_t n_coef,
                      int64_t T, void* hip_stream, int32_t* result_index);

/* Runs of variants 1-3 wait on the device: the dependency-driven schedule
 * for the tiles a tile depends on, relaxed synchronisation for the waves of
 * a tile.  The waits cannot deadlock (tiles start in row order; a wave waits
 * only on earlier phases of other waves), and each is bounded anyway: after
 * `polls` polls (default 2^20) a wait gives up, records the failure and
 * goes on, so the launch always ends; the result is then wrong.
 * girih_check synchronises hip_stream and returns GIRIH_E_STALL if a wait of
 * the plan's last run gave up, GIRIH_OK otherwise. */
int girih_set_wait_limit(girih_plan_t plan, uint32_t polls);
int girih_check(girih_plan_t plan, void* hip_stream);

/* Auto-tuner (paper, Section "Auto-tuning").  Allocates and initialises its
 * own arrays of the plan's grid (freed before return), times candidates with
 * HIP events on hip_stream, and writes the best parameters into *best and
 * the plan.  A candidate is timed on the problem itself: back-to-back runs of
 * the plan's T-step schedule (every diamond row, the clipped first and last
 * rows included), the number of runs doubled while a measurement lasts less
 * than 50 ms, until two consecutive measurements agree within 3 %
 * (girih_adaptive_time) or the candidate's share of max_seconds is spent.
 *  mode: GIRIH_TUNE_EXHAUSTIVE  every feasible candidate
 *        GIRIH_TUNE_HILLCLIMB   per thread shape, local search over Dw and
 *                               the x tile (the paper's search)
 *        GIRIH_TUNE_MODEL       only the candidates given by
 *                               girih_tune_set_candidates (e.g. the top-k of
 *                               a learned cost model), in that order
 *  T: steps the tuned run will take (part of the problem, >= 1; 0 gives
 *  GIRIH_E_INVALID).  Each measured candidate is appended to the plan's log
 *  (girih_tune_log); GIRIH_E_UNSUPPORTED if no candidate ran. */
#define GIRIH_TUNE_EXHAUSTIVE 0
#define GIRIH_TUNE_HILLCLIMB 1
#define GIRIH_TUNE_MODEL 2
int girih_tune(girih_plan_t plan, int32_t mode, int64_t T, double max_seconds, void* hip_stream,
               girih_params* best, double* best_glups);

/* The tuner's search and its adaptive test length with a caller-supplied
 * measurement: the same code girih_tune runs, for other measurement backends
 * (a cost model, another device, a recorded table) and for testing the
 * search without a GPU.  Neither touches the device.
 *
 * girih_tune_search: measure(candidate, ctx) returns GLUP/s (<= 0: the
 * candidate failed).  mode GIRIH_TUNE_EXHAUSTIVE or GIRIH_TUNE_MODEL measures
 * the list in order until max_seconds is spent (at least one); HILLCLIMB
 * searches per thread shape (threads_x, cells_per_lane) from the median
 * diamond width and widest x tile of the smallest wavefront depth, moving to
 * the best improving neighbour (next diamond width or wavefront depth up or
 * down, at its widest x tile; next x tile up or down) until none improves.
 * Every candidate is measured at most once.  Outputs: *best_index into cands
 * (-1 if none measured > 0), *best_glups, *n_measured (any may be NULL).
 * GIRIH_E_UNSUPPORTED if no candidate measured > 0.
 *
 * girih_adaptive_time: time_fn(reps, ctx) returns the seconds of reps
 * back-to-back runs (negative: failure, GIRIH_E_HIP).  reps starts at 1 and
 * doubles while a measurement is shorter than min_seconds; the per-run time
 * is accepted when two consecutive measurements agree within tol (relative),
 * or after max_seconds or max_tries measurements (the last one is taken). */
typedef double (*girih_measure_fn)(const girih_params* candidate, void* ctx);
typedef double (*girih_time_fn)(int64_t reps, void* ctx);
int girih_tune_search(const girih_params* cands, int32_t n, int32_t mode, girih_measure_fn measure, void* ctx,
                      double max_seconds, int32_t* best_index, double* best_glups, int32_t* n_measured);
int girih_adaptive_time(girih_time_fn time_fn, void* ctx, double tol, double min_seconds, double max_seconds,
                        int32_t max_tries, double* seconds_per_run, int64_t* reps, int32_t* tries);

/* Candidate list for GIRIH_TUNE_MODEL (copied).  n <= 4096. */
int girih_tune_set_candidates(girih_plan_t plan, const girih_params* cands, int32_t n);

/* Enumerate the feasible MWD candidates of the plan's problem: writes up to
 * cap parameter sets into out (may be NULL to count) and their count to *n. */
int girih_candidates(girih_plan_t plan, girih_params* out, int32_t cap, int32_t* n);

/* The user's on-chip budget (paper, Section "Auto-tuning": the user gives the
 * cache size, and candidates whose cache block does not fit it are pruned):
 * MWD candidates whose workgroup needs more than `bytes` of LDS are left out
 * of girih_candidates and of the exhaustive and hill-climbing searches.
 * 0 (the default) = the CU's own 160 KiB, which every compiled shape fits.
 * Negative: GIRIH_E_INVALID. */
int girih_set_lds_budget(girih_plan_t plan, int64_t bytes);

/* One measured tuner candidate. */
typedef struct girih_tune_record {
    girih_params params;
    int64_t lds_bytes;      /* LDS of the candidate's workgroup            */
    int64_t steps;          /* time steps of the final measurement          */
    double seconds;         /* time of the final measurement                */
    double glups;           /* giga lattice updates per second              */
    int32_t repeats;        /* measurements taken before it was accepted    */
    int32_t status;         /* 0 = measured, <0 = error code                */
} girih_tune_record;

/* Copy up to cap records of the plan's tuner log; *n = total count. */
int girih_tune_log(girih_plan_t plan, girih_tune_record* out, int32_t cap, int32_t* n);

/* Resolved parameters, LDS bytes per workgroup, and the algorithmic code
 * balance in bytes per lattice update: for MWD the paper's blocked code
 * balance B_C (Section "Memory traffic model", both equations, scaled to the
 * element size: 2 * size * R * [(2Dw - 2R) + (N_D*Dw + 2R)] / Dw^2, with N_D
 * = 2 + n_coef domain-sized streams read); the redundant x-halo that
 * x-chunking reads on top of it is not included; for NAIVE the streaming
 * (2 + n_coef) * size, plus one more stream (u^{t-1}) for the
 * second-order-in-time stencil. */
int girih_plan_info(girih_plan_t plan, girih_params* params, int64_t* lds_bytes, double* model_bytes_per_lup);

/* Change the parameters of an existing plan (validated like girih_plan). */
int girih_plan_set_params(girih_plan_t plan, const girih_params* params);

/* Launch timing (diagnostics, used by the benchmark's roofline figure).
 * With timing enabled, girih_run brackets every sweep-kernel launch (one per
 * diamond row for MWD, one per step for NAIVE; not the halo copies) with a
 * pair of HIP events on hip_stream.  girih_timing waits for the last event of
 * the most recent run and returns the number of such launches and the sum of
 * their durations in milliseconds (0 launches if timing is off).  The tuner's
 * own test runs are not recorded. */
int girih_set_timing(girih_plan_t plan, int32_t enable);
int girih_timing(girih_plan_t plan, int32_t* n_launches, double* kernel_ms);

void girih_destroy(girih_plan_t plan);

const char* girih_strerror(int code);

/* Error norms of a result against a reference, accumulated in double
 * precision over the interior (dtype_a, dtype_b: element types of a and b,
 * same grid layout): out[0] = sqrt(sum (a-b)^2), out[1] = sqrt(sum b^2),
 * out[2] = max |a-b|, out[3] = number of bitwise-different elements (only
 * meaningful when both types are equal).  Synchronises hip_stream. */
int girih_error_norms(const girih_grid* grid, girih_dtype dtype_a, const void* a, girih_dtype dtype_b,
                      const void* b, void* hip_stream, double out[4]);

/* Cost model of the tuner: a fully connected network in FP32 that predicts
 * the log throughput of a tuner candidate from its features (the feature list
 * is in paper_1510_04995_amd/costmodel.py).  Not from the paper: it
 * proposes candidates to the paper's auto-tuner (Section "Auto-tuning"),
 * which measures them (GIRIH_TUNE_MODEL).
 *
 * Network: n_in inputs -> n_layers hidden layers of n_hidden units, each
 * z = W a + b followed by ReLU -> one linear output.  Parameters: one flat FP32
 * DEVICE array, layer by layer (first hidden layer first, output layer last):
 * W (fan_out x fan_in, row-major) then b (fan_out).  Inputs x: n x n_in,
 * row-major, device.  All buffers are caller-owned device memory; work is a
 * scratch array of at least girih_mlp_work_count floats.  Sums run in a fixed
 * order.  Asynchronous on hip_stream.  Errors: GIRIH_E_INVALID for null
 * pointers, sizes out of range (n_in, n_hidden <= 4096, 1 <= n_layers <= 16,
 * n >= 1) or a short work array; GIRIH_E_HIP for a failed launch. */
int girih_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_layers, int64_t* count);
int girih_mlp_work_count(int32_t n_in, int32_t n_hidden, int32_t n_layers, int32_t n, int64_t* count);
/* y[i] = network(x[i]) for i < n (y: n floats, device). */
int girih_mlp_forward(const float* params, int32_t n_in, int32_t n_hidden, int32_t n_layers, const float* x,
                      int32_t n, float* y, float* work, int64_t work_len, void* hip_stream);
/* loss = (1/n) sum_i (network(x[i]) - target[i])^2 (one float, device) and its
 * gradient with respect to every parameter (grad: param_count floats, device),
 * by back-propagation. */
int girih_mlp_loss_grad(const float* params, int32_t n_in, int32_t n_hidden, int32_t n_layers, const float* x,
                        const float* target, int32_t n, float* loss, float* grad, float* work, int64_t work_len,
                        void* hip_stream);
/* One Adam step (Kingma and Ba) on count parameters: m and v are the first and
 * second moment arrays (device, zero before step 1), step >= 1:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
int girih_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t count, float lr, float beta1,
                   float beta2, float eps, int32_t step, void* hip_stream);

/* Library version string. */
const char* girih_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GIRIH_H */
