/*
 * ewald.h -- C ABI of the MI355X spectral Ewald library for the triply
 * periodic Stokeslet sum.
 *
 * The library evaluates, for N particles x_i in an orthorhombic periodic box
 * B = [0,L1) x [0,L2) x [0,L3) with forces f_i,
 *
 *     u(x_i) = sum_j sum_p' G(x_i - x_j + p) f_j,   G(r) = I/|r| + r r^T/|r|^3,
 *
 * (Sec. 2, eq. (potentials) and the Stokeslet below it; targets = sources;
 * coincident points skipped; no 1/(8 pi mu) factor), with Hasimoto's Ewald
 * split into a near field (P2P, Sec. 2.1 eq. (g-near)) and a far field
 * evaluated on a uniform grid (P2G, FFT, CNV, IFFT, G2P: Sec. 2.2, eq. (p2g),
 * (sca), (g2p), with Ghat^F of eq. (GFk)), plus the self-term correction
 * -(4 xi / sqrt(pi)) f_i.  The k = 0 Fourier mode is dropped (Hasimoto's
 * convention: a net force is balanced by a mean pressure gradient).
 *
 * Conventions shared by every entry point:
 *  - Arrays x, f, u are structure-of-arrays (3, n) FP64 in DEVICE memory:
 *    component d of particle i is at [d*n + i].  They are owned by the caller.
 *  - `workspace` is caller-owned device memory of at least
 *    ewald_workspace_bytes(plan, n) bytes, 256-byte aligned.  A plan owns only
 *    small read-only tables, so one plan can serve concurrent evaluations on
 *    different streams as long as each uses its own workspace.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Evaluation entry
 *    points only enqueue work on it: they allocate nothing, do not
 *    synchronise, and return before the device has finished.  Device faults
 *    surface at the caller's next synchronisation.
 *  - Return values: EWALD_OK (0) or a negative ewald_status; the message of
 *    the last failure on the calling thread is returned by ewald_last_error().
 *    All argument checks happen before anything is enqueued.  The library
 *    never aborts or prints.
 *  - Positions outside [0, L) are wrapped periodically.  n = 0 is a no-op.
 */
#ifndef EWALD_H
#define EWALD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ewald_plan_s* ewald_plan_t;

typedef enum {
    EWALD_OK = 0,
    EWALD_EINVAL = -1,       /* bad argument, size or parameter */
    EWALD_ENOMEM = -2,       /* workspace too small, or a plan table allocation failed */
    EWALD_EHIP = -3,         /* a HIP runtime call failed */
    EWALD_EUNSUPPORTED = -4  /* valid request outside what this build implements */
} ewald_status;

/* Precision modes (low byte of ewald_params.precision) and flags (OR'd in). */
enum {
    EWALD_FP64 = 0,      /* every step in FP64 */
    EWALD_FP32_BULK = 1, /* the pair formula of P2P, the window weights of P2G and G2P and (for
                            tol >= 1e-6) the grid, FFT, CNV input/output and IFFT in FP32.  P2G
                            computes its sums in FP64 and stores them to the FP32 grid; below
                            tol 1e-6 the grid and its transforms stay FP64 (the FP32 round trip
                            through the 3D FFT alone leaves ~2e-7 relative error).  Positions,
                            the cutoff test, the Fourier-space scaling, the k = 0 and self
                            terms and the final sum are FP64, and every sum over pairs or
                            stencil points accumulates in FP64 */
    EWALD_FLAG_P2P_FP64_ACC = 1 << 8, /* deprecated, no effect: the near-field sums are always
                                         accumulated in FP64 (in FP32 bulk too: FP64 LDS
                                         atomics are fast on gfx950, FP32 ones are not) */
    EWALD_FLAG_STAGE_TIMERS = 1 << 9, /* record per-stage HIP events (see ewald_stage_ms); the
                                         events belong to the plan, so overlapping evaluations
                                         of one timed plan on several streams time nothing
                                         meaningful: time one evaluation at a time */
    EWALD_FLAG_WINDOW_KB = 1 << 10,   /* truncated Kaiser-Bessel window (Sec. 2.2) instead of the
                                         Gaussian: w0(d) = I0(beta sqrt(1 - (2d/(P h))^2)) / I0(beta) */
    EWALD_FLAG_DETERMINISTIC = 1 << 11, /* bitwise reproducible results for the same inputs on the
                                          same device: P2P evaluates every pair from both sides
                                          (about 1.5x the P2P time) and sums in a fixed order; the
                                          particles of every grid cell are ordered by input index
                                          whatever the cell's size.  Without it each pair is
                                          evaluated once and its two contributions are added with
                                          atomics, so repeated evaluations agree to rounding
                                          (~1e-16 relative), not bitwise */
    EWALD_FLAG_STRESSLET = 1 << 12,    /* the plan also evaluates stresslet (double-layer) sources
                                          with ewald_eval_combined: its workspace holds the sorted
                                          source tensors and a 9-component grid.  Not combinable
                                          with EWALD_FLAG_DETERMINISTIC (EWALD_EUNSUPPORTED) */
    EWALD_FLAG_CHECK_INPUTS = 1 << 13  /* debug mode: every evaluation first counts the
                                          non-finite values of its inputs on the device and
                                          returns EWALD_EINVAL, with nothing else enqueued, if
                                          there are any.  The check waits for the stream (the
                                          evaluation calls then synchronise) */
};

/*
 * Plan parameters.  Any parameter given as <= 0 is derived from `tol`
 * following the error split of Sec. 2.4 (eq. (ese), each error term held to
 * tol/3): xi from the grid spacing (E^F), r_c from xi (E^N), the window
 * support P and shape from the window's error model.  When grid, xi and r_c
 * are all left to derive, every power-of-two grid is resolved this way and the
 * one with the smallest predicted device time for n_max particles is taken
 * (the plan cost model, Sec. 2.4's parameter choice made by measured cost);
 * when xi or r_c is given, the grid is the coarsest that resolves xi.
 */
typedef struct {
    double box[3];       /* L1, L2, L3 > 0: orthorhombic, triply periodic */
    double xi;           /* Ewald split parameter; <= 0: derive */
    double r_c;          /* near-field cutoff radius; <= 0: derive */
    int32_t grid[3];     /* M1, M2, M3: powers of two in [8, 512]; any <= 0: derive */
    int32_t P;           /* window support in grid points per dimension: even, 4..16; <= 0: derive */
    double tol;          /* target relative RMS error, in [1e-12, 1e-2] */
    int32_t precision;   /* EWALD_FP64 or EWALD_FP32_BULK, OR'd with EWALD_FLAG_* */
    int32_t reserved;    /* must be 0 */
    int64_t n_max;       /* largest n this plan will evaluate (sizes workspace queries) */
    double window_shape; /* Gaussian: shape m, w0(d) = exp(-2 m^2 d^2 / (P h)^2); Kaiser-Bessel:
                            beta / P; <= 0: derive */
} ewald_params;

/* Everything a plan resolved (returned by ewald_plan_get_info). */
typedef struct {
    ewald_params params;      /* every field resolved */
    double h[3];              /* grid spacing L_d / M_d */
    double err_near;          /* predicted near-field RMS error term E^N (eq. (ese)) */
    double err_far;           /* predicted Fourier truncation term E^F (eq. (ese)) */
    double err_window;        /* predicted window error (window model of the plan's window) */
    int32_t tile;             /* P2P cell edge, in grid cells */
    int32_t n_tiles[3];       /* P2P cells per dimension */
    int32_t stencil[3];       /* P2P neighbour half-width, in cells */
    int32_t fourier_fp64;     /* 1 when the grid, FFT, CNV and IFFT are FP64, 0 for FP32 */
    int64_t workspace_bytes;  /* ewald_workspace_bytes(plan, n_max) */
    double predicted_ms;      /* device time of one evaluation of n_max particles predicted by
                                 the plan cost model (uniform particles; MI355X-calibrated) */
    double self_coef;         /* c of the self term -c f_i: c = 4 xi / sqrt(pi), the limit of
                                 G - G^N at r = 0 (so u = u_near + u_far - c f) */
    int64_t grid_bytes;       /* bytes of the grid ewald_spread and ewald_far_grid write:
                                 3 M1 M2 M3 elements of 8 bytes when fourier_fp64, else 4 */
} ewald_plan_info;

/* Create a plan (host call; allocates the plan's small device tables on the
 * current device).  Fails with EWALD_EINVAL for: box <= 0, tol outside its
 * range, a grid entry that is not a power of two in [8, 512], odd P or P
 * outside 4..16, r_c above the smallest box side or below one grid spacing,
 * n_max < 0, a non-zero reserved field. */
int ewald_plan_create(const ewald_params* params, ewald_plan_t* plan_out);

/* Resolve parameters exactly as ewald_plan_create would, without creating a plan or
 * touching the device (host only); fills *info, including workspace_bytes for n_max.
 * Same validation errors as ewald_plan_create. */
int ewald_resolve(const ewald_params* params, ewald_plan_info* info);

/* Copy the resolved parameters of `plan` into *info. */
int ewald_plan_get_info(ewald_plan_t plan, ewald_plan_info* info);

/* Free the plan's tables and events.  No evaluation using it may be in flight. */
int ewald_plan_destroy(ewald_plan_t plan);

/* Workspace bytes ewald_eval needs for n particles (negative status on error). */
int64_t ewald_workspace_bytes(ewald_plan_t plan, int64_t n);

/*
 * Full evaluation u = u^N + u^F - (4 xi/sqrt(pi)) f (Algorithm "se": P2P,
 * P2G, FFT, CNV, IFFT, G2P, SUM).  x, f: (3, n) FP64 device inputs; u: (3, n)
 * FP64 device output, fully overwritten.  Errors: EWALD_EINVAL for a null
 * pointer with n > 0, n < 0 or n > n_max; EWALD_ENOMEM when workspace_bytes
 * is below ewald_workspace_bytes(plan, n); EWALD_EHIP if a launch fails.
 */
int ewald_eval(ewald_plan_t plan, int64_t n, const double* x, const double* f, double* u,
               void* workspace, int64_t workspace_bytes, void* stream);

/* Bytes of the device array that serves as ewald_eval_noalloc's workspace (64 MiB). */
#define EWALD_NOALLOC_MAX_WORKSPACE ((int64_t)64 << 20)

/*
 * ewald_eval for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same evaluation and kernels,
 * with the workspace taken from an array of EWALD_NOALLOC_MAX_WORKSPACE bytes that the
 * library holds on each device (set up when the first plan is created on that device, and
 * kept until the process ends).  Allocates nothing.  The caller still passes x, f and u
 * (device, (3, n) FP64).  Errors as ewald_eval, plus EWALD_ENOMEM (nothing enqueued) when
 * ewald_workspace_bytes(plan, n) exceeds EWALD_NOALLOC_MAX_WORKSPACE, and EWALD_EINVAL
 * when the current device is not the plan's.  Every call on one device uses the same
 * array: calls that overlap on a device (other streams, other threads) race and give
 * wrong results; serialise them.  Each call initialises what it reads of the array.
 */
int ewald_eval_noalloc(ewald_plan_t plan, int64_t n, const double* x, const double* f, double* u, void* stream);

/*
 * Combined single and double layer sources (Sec. 2.3, "Combined single and double
 * layers"): every particle j carries a force f_j and two vectors q_j, n_j, and
 *   u(x_i) = sum_j sum_p' [ G(x_i - x_j + p) f_j + T(x_i - x_j + p) (q_j n_j^T) ]
 * with the stresslet T_abc(r) = -6 r_a r_b r_c / |r|^5 (component a of T (q n^T) is
 * sum_bc T_abc q_b n_c).  Split like the Stokeslet: T^N in P2P, That^F (the same
 * screening (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)}) through P2G (force + the 6 independent
 * components of (q n^T + n q^T)/2, T being symmetric), FFT, CNV (9 -> 3 components),
 * IFFT and G2P; T^F is odd, so there is no stresslet self term.  x, f, q, nrm: (3, n) FP64
 * device inputs; u: (3, n) FP64 device output.  The plan must carry
 * EWALD_FLAG_STRESSLET (else EWALD_EINVAL); other errors as ewald_eval.  The split
 * parameters are those of the Stokeslet error model.
 */
int ewald_eval_combined(ewald_plan_t plan, int64_t n, const double* x, const double* f, const double* q,
                        const double* nrm, double* u, void* workspace, int64_t workspace_bytes, void* stream);

/* Near and far parts of ewald_eval_combined (as ewald_eval_parts). */
int ewald_eval_combined_parts(ewald_plan_t plan, int64_t n, const double* x, const double* f, const double* q,
                              const double* nrm, double* u_near, double* u_far, void* workspace,
                              int64_t workspace_bytes, void* stream);

/*
 * ewald_eval with the near field (P2P) on a second stream: P2P does not depend on P2G or the
 * FFTs (Sec. 6.5 notes that they can overlap), so after the sort `stream` records
 * `fork_event`, `near_stream` waits for it and runs P2P, then records `join_event`, for which
 * `stream` waits before G2P; P2G, FFT, CNV and IFFT run on `stream` meanwhile.  When the call
 * returns, all work is ordered before later work on `stream` (near_stream carries nothing
 * after join_event).  The caller owns both streams and both events (hipEvent_t, e.g. created
 * with hipEventDisableTiming); concurrent evaluations need their own streams, events and
 * workspaces.  Same results and arguments as ewald_eval; EWALD_EINVAL for null or equal
 * streams or null events with n > 0.  With EWALD_FLAG_STAGE_TIMERS, ewald_stage_ms reports
 * P2P and P2G each from the fork and G2P from the later of the join and the far field.
 */
int ewald_eval_overlap(ewald_plan_t plan, int64_t n, const double* x, const double* f, double* u,
                       void* workspace, int64_t workspace_bytes, void* stream, void* near_stream,
                       void* fork_event, void* join_event);

/* Most systems one ewald_eval_batch call evaluates. */
#define EWALD_MAX_BATCH 64

/*
 * Batched evaluation of `count` independent systems that share the plan (box, tolerance,
 * parameters): system r is the particles [offsets[r], offsets[r+1]) of x, f and u, each
 * (3, offsets[count]) FP64 device arrays, and is summed over its own periodic images only
 * (Algorithm "se" per system).  One launch sequence serves all systems, so small systems
 * cost little more than one (the serving loop groups small requests this way).  `offsets`
 * is a host array of count + 1 non-decreasing entries, offsets[0] = 0, each system at most
 * the plan's n_max particles (offsets[count] may exceed it).  The workspace must hold
 * ewald_workspace_bytes_batch(plan, count, offsets) bytes.  Errors as ewald_eval, plus
 * EWALD_EINVAL for count outside [1, EWALD_MAX_BATCH] or bad offsets, and
 * EWALD_EUNSUPPORTED for stresslet plans.
 */
int ewald_eval_batch(ewald_plan_t plan, int32_t count, const int64_t* offsets, const double* x, const double* f,
                     double* u, void* workspace, int64_t workspace_bytes, void* stream);

/* Workspace bytes of ewald_eval_batch for these systems (negative status on error). */
int64_t ewald_workspace_bytes_batch(ewald_plan_t plan, int32_t count, const int64_t* offsets);

/*
 * Diagnostic split of ewald_eval: u_near = the P2P sum (Sec. 2.1,
 * eq. (potentials-near)) and u_far = the interpolated far field u^F_h
 * (eq. (g2p)), both (3, n) FP64 device arrays in the caller's particle order,
 * so that u = u_near + u_far - (4 xi/sqrt(pi)) f.  Same kernels, same
 * arguments and errors as ewald_eval.
 */
int ewald_eval_parts(ewald_plan_t plan, int64_t n, const double* x, const double* f,
                     double* u_near, double* u_far, void* workspace, int64_t workspace_bytes,
                     void* stream);

/*
 * Diagnostic: the P2G grid phi (eq. (p2g), no h^3 factor) as (3, M1, M2, M3)
 * row-major (M3 fastest).  Element type: double when ewald_plan_info.fourier_fp64
 * is 1 (every FP64 plan, and FP32-bulk plans below tol 1e-6), else float.  `grid`
 * is caller-owned device memory of grid_bytes bytes; EWALD_ENOMEM (nothing
 * enqueued) when grid_bytes is below ewald_plan_info.grid_bytes.  Other errors as
 * ewald_eval.
 */
int ewald_spread(ewald_plan_t plan, int64_t n, const double* x, const double* f, void* grid,
                 int64_t grid_bytes, void* workspace, int64_t workspace_bytes, void* stream);

/*
 * Diagnostic: the real grid that G2P interpolates, after P2G, FFT, CNV
 * (eq. (sca)) and IFFT, stored as h1 h2 h3 * v(g_l) of eq. (g2p) (the h^3
 * factor and the inverse-DFT normalisation are folded into CNV); layout, element
 * type, size check and errors as for ewald_spread.
 */
int ewald_far_grid(ewald_plan_t plan, int64_t n, const double* x, const double* f, void* grid,
                   int64_t grid_bytes, void* workspace, int64_t workspace_bytes, void* stream);

/*
 * Diagnostic for measurement: the exact number of ordered pairs (i, j), i != j, over all
 * periodic images p with 0 < |x_i - x_j + p| < r_c -- the pairs the near-field sum of
 * Sec. 2.1 (eq. (potentials-near)) runs over -- written to `count`, one uint64_t in
 * device memory (overwritten; n = 0 writes 0).  Runs the sort and a count-only pass of the
 * one-sided P2P over the same cell walk; computes no pair formula.  Arguments and errors
 * otherwise as ewald_eval (f is read by the sort).
 */
int ewald_count_pairs(ewald_plan_t plan, int64_t n, const double* x, const double* f, uint64_t* count,
                      void* workspace, int64_t workspace_bytes, void* stream);

/*
 * Per-stage device times (ms) of the last evaluation made with this plan when
 * it was created with EWALD_FLAG_STAGE_TIMERS; valid once that evaluation's
 * stream has been synchronised.  Stages, in order: 0 bin/sort, 1 P2P, 2 P2G,
 * 3 FFT+CNV+IFFT, 4 G2P+self+sum+unsort, 5 total.  Writes min(count, 6)
 * values; returns the number written or a negative status.
 */
int ewald_stage_ms(ewald_plan_t plan, float* ms, int32_t count);

/*
 * Failure injection for tests of error handling: the next `count` evaluation calls made on
 * the calling thread (any ewald_eval* entry point, ewald_spread, ewald_far_grid,
 * ewald_count_pairs) return EWALD_EHIP after their argument checks, with nothing enqueued,
 * as a failed launch would.  count = 0 disarms.  Returns EWALD_OK, or EWALD_EINVAL for
 * count < 0.
 */
int ewald_debug_fail_next(int32_t count);

/* Message describing the last failure on the calling thread ("" if none). */
const char* ewald_last_error(void);

/* Library version string. */
const char* ewald_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EWALD_H */
