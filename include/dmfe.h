/*
 * dmfe.h -- C-ABI of the MI355X-native solver for the two-time dynamical
 * mean-field equations (DMFE) of the mixed spherical p-spin model
 * (DYNAMITE, arXiv 2604.06309).
 *
 * The model (Sec. 2.1): covariance f(q) = sum_p a_p^2 q^p / 2, temperature T,
 * initial inverse temperature beta0 (0 = random start), memory kernels
 * K = f''(C) R and D = f'(C), forcing F_C = beta0 f'(C(t,0)) C(t',0),
 * Lagrange multiplier mu(t) and energy E(t).
 *
 * Two discretisations:
 *  - DMFE_UNIFORM: equidistant grid in t and t' (the O(N^3) baseline of
 *    Sec. 2.3), classical RK4 with trapezoid history integrals;
 *  - DMFE_ADAPTIVE: the paper's method (Sec. 3): fixed grid in theta = t'/t
 *    (eq. theta, alpha = 0), s-point index-Lagrange interpolation in theta and
 *    cubic Hermite interpolation in t (Sec. 3.3), quadrature sums of eq. (int)
 *    with quintic-spline weights (Sec. 3.4), Dormand-Prince 5(4) then
 *    SSPRK(10,4) with the 1-norm error control of Sec. 3.5, and
 *    sparsification of the stored history (Sec. 3.6).
 *
 * Conventions for every entry point:
 *  - return value: DMFE_OK (0), DMFE_DONE (1, t reached t_max) or a negative
 *    error code; no C++ exception crosses this boundary;
 *  - all floating point is IEEE double unless stated;
 *  - "device" pointers are HIP device addresses on the handle's device;
 *    "host" pointers are ordinary process memory;
 *  - work is ordered on the handle's stream; calls that return data to the
 *    host synchronise that stream before returning;
 *  - one handle must not be used by two host threads at the same time.
 */
#ifndef DMFE_H
#define DMFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmfe_status;

/* Opaque solver handle. */
typedef struct dmfe_handle dmfe_handle;

enum {
    DMFE_OK = 0,
    DMFE_DONE = 1,                /* t >= t_max after the call */
    DMFE_ERR_INVALID = -1,        /* bad parameters or arguments */
    DMFE_ERR_NOMEM = -2,          /* device or host allocation failed, or workspace too small */
    DMFE_ERR_CAPACITY = -3,       /* history full (M = M_cap) and a sparsification pass freed nothing */
    DMFE_ERR_STEP_UNDERFLOW = -4, /* the step size fell below dt_min (Appendix B) */
    DMFE_ERR_NONFINITE = -5,      /* the RK error estimate is NaN or Inf */
    DMFE_ERR_DEVICE = -6,         /* a HIP call failed; dmfe_last_error() has the text */
    DMFE_ERR_UNSUPPORTED = -7,    /* valid but not implemented here (e.g. grid_alpha != 0) */
    DMFE_ERR_BUFFER = -8          /* destination buffer too small; needed_bytes says how much */
};

enum { DMFE_UNIFORM = 0, DMFE_ADAPTIVE = 1 };
enum { DMFE_FP64 = 0, DMFE_FP32_COMP = 1 };
enum { DMFE_SCHEME_DP5 = 0, DMFE_SCHEME_SSPRK104 = 1 };
enum { DMFE_MAX_TERMS = 8, DMFE_MAX_P = 16 };
/* theta-interpolation schemes (Sec. 3.3) */
enum {
    DMFE_INTERP_INDEX_LAGRANGE = 0, /* Lagrange on the equidistant index coordinate (default) */
    DMFE_INTERP_THETA_LAGRANGE = 1, /* Lagrange on theta itself */
    DMFE_INTERP_INDEX_FH = 2,       /* Floater-Hormann rational interpolation on the index coordinate */
    DMFE_INTERP_THETA_FH = 3        /* Floater-Hormann on theta */
};

/*
 * Problem statement (Sec. 2.1, 3.2, 3.5, Appendix B).
 *   n_terms, p[], a2[]  f(q) = sum_k a2[k] q^p[k] / 2, 2 <= p[k] <= DMFE_MAX_P, a2[k] >= 0
 *   T, beta0            bath temperature, inverse temperature of the initial state
 *   t_max               largest simulated time; sets gamma = -W_{-1}(-1/t_max) (needs t_max > e)
 *   mode                DMFE_UNIFORM or DMFE_ADAPTIVE
 *   precision           DMFE_FP64 (only value accepted by DMFE_UNIFORM) or DMFE_FP32_COMP:
 *                       the history (C, R and their t-derivatives) is stored in FP32 and
 *                       widened to FP64 as it is read; all arithmetic, mu, the RK error,
 *                       the controller and the sparsification decision stay FP64.  The
 *                       sparsification residual of an FP32 history has a bound on the
 *                       FP32 rounding of the stored values subtracted (never below 0).
 * uniform mode:
 *   h, N                step and number of steps (t_max is ignored)
 * adaptive mode:
 *   L                   theta-grid length (2s <= L <= 16384)
 *   M_cap               history capacity in slices (0 means L): 16 <= M_cap <= 65536 (above about
 *                       17.1K stored slices with an FP64 history, 16.7K with FP32, the history-integral
 *                       kernel reads their times from global memory instead of LDS); <= 16384 in the
 *                       serving pool
 *   eps                 tolerance on the 1-norm RK error (Sec. 3.5); sparsification drops
 *                       a slice whose residual is below eps/10 (Sec. 3.6)
 *   dt0, dt_min         first step and smallest allowed step
 *   s                   theta stencil size (even, 4 <= s <= 16; 0 means 10)
 *   auto_passes         sparsification passes run when M reaches M_cap (0 means 1)
 *   grid_alpha, grid_delta  flattening parameters of eq. (theta); only alpha = 0 is supported
 *   scheme_policy       0: DP5 until its stability boundary, then SSPRK(10,4) (default);
 *                       1: SSPRK(10,4) from the start; 2: DP5 only
 *   theta_interp        DMFE_INTERP_*: how a value between theta-grid nodes is formed from
 *                       the s stencil nodes around it (Sec. 3.3).  The stencil is the
 *                       same for every scheme: nodes base..base+s-1, base = floor(x) -
 *                       (s-1)/2 clamped to [0, L-s], x the continuous index of the target.
 *                       Theta schemes difference theta below 1/2 and 1 - theta above.
 *   fh_d                Floater-Hormann blending degree d (0 <= d <= s-1; read by the FH
 *                       schemes only): rational, no real poles, exact on polynomials of
 *                       degree d; d = s-1 is the polynomial interpolant
 *   log_r               1: interpolate log R and the scaled derivative (dR/dt)/R with the
 *                       same rules in theta and in t and exponentiate; a target any of whose
 *                       stencil values of R is <= 0 interpolates R itself (Appendix A).
 *                       The sparsification residual stays the integral of R's Hermite
 *                       interpolant.
 * The serving pool admits the default stencil only (s = 10, index Lagrange, log_r = 0).
 */
typedef struct dmfe_params {
    int32_t n_terms;
    int32_t p[DMFE_MAX_TERMS];
    double a2[DMFE_MAX_TERMS];
    double T;
    double beta0;
    double t_max;
    int32_t mode;
    int32_t precision;
    double h;
    int64_t N;
    int32_t L;
    int32_t M_cap;
    double eps;
    double dt0;
    double dt_min;
    int32_t s;
    int32_t auto_passes;
    double grid_alpha;
    double grid_delta;
    int32_t scheme_policy;
    int32_t theta_interp;
    int32_t fh_d;
    int32_t log_r;
} dmfe_params;

/*
 * Device resources.  `stream` is a hipStream_t (NULL: the null stream).
 * `workspace`, if not NULL, is caller-owned device memory of at least
 * dmfe_footprint() bytes that the handle uses instead of allocating; the
 * handle never frees it and the caller keeps it alive until dmfe_destroy().
 */
typedef struct dmfe_resources {
    int32_t device;
    int32_t reserved0;
    void *stream;
    void *workspace;
    size_t workspace_bytes;
} dmfe_resources;

/* Counters and state after dmfe_step / dmfe_get_info. */
typedef struct dmfe_step_info {
    int64_t accepted;       /* accepted steps since create */
    int64_t rejected;       /* rejected steps (each one reverts, Sec. 3.5) */
    int64_t reverts;        /* slices dropped by reverts */
    int64_t sparsify_calls; /* sparsification passes run */
    int64_t removed;        /* slices removed by sparsification */
    int64_t rhs_evals;      /* right-hand-side evaluations (stages) */
    int64_t M;              /* stored slices (uniform mode: stored rows) */
    int32_t scheme;         /* DMFE_SCHEME_* in use */
    int32_t nb_valid;       /* leading stored slices that carry their d/dt (M, or M-1 when the newest
                               slice's derivative is formed at the next step's first stage) */
    double t;               /* current time */
    double dt;              /* next step size */
    double eps_rk;          /* error estimate of the last step */
} dmfe_step_info;

/* Fields for dmfe_read. */
typedef enum dmfe_field {
    DMFE_F_T_GRID = 0,  /* t_n of stored slices, [count]                                  */
    DMFE_F_THETA = 1,   /* theta_i, [L] (first/count index the grid)                      */
    DMFE_F_THETA_C = 2, /* 1 - theta_i evaluated without cancellation, [L]                */
    DMFE_F_NU = 3,      /* quadrature weights nu_i, [L]                                   */
    DMFE_F_C = 4,       /* C(t_n, theta_i t_n), [count][L]; uniform: packed rows n, C[n][0..n] */
    DMFE_F_R = 5,       /* R(t_n, theta_i t_n), [count][L]; uniform: packed rows           */
    DMFE_F_DC = 6,      /* d/dt C(t, theta_i t) at t_n (adaptive only), [count][L]        */
    DMFE_F_DR = 7,      /* d/dt R(t, theta_i t) at t_n (adaptive only), [count][L]        */
    DMFE_F_ENERGY = 8,  /* E(t_n), [count]                                                 */
    DMFE_F_MU = 9       /* mu(t_n), [count]                                                */
} dmfe_field;

/*
 * Bytes of device memory the handle needs for these parameters (host only, no
 * device call).  Infrastructure, not a step of the method: it sizes a caller
 * workspace and the serving pool's admission test.  The bulk is the history of
 * Sec. 3.2 (M_cap + 1 slices of C, R and their t-derivatives: 32 bytes per
 * point in FP64, 16 with an FP32 history) plus O(L) arrays.  Errors:
 * DMFE_ERR_INVALID / DMFE_ERR_UNSUPPORTED as dmfe_create would return them.
 */
dmfe_status dmfe_footprint(const dmfe_params *params, size_t *bytes);

/*
 * Create a solver: validates params, computes the run-constant grid data on the
 * host (gamma, theta, nu), takes or allocates device memory and sets the
 * initial slice C(0,0) = R(0,0^-) = 1 (Sec. 2.2).  *out receives the handle.
 */
dmfe_status dmfe_create(const dmfe_params *params, const dmfe_resources *res, dmfe_handle **out);

/*
 * Advance until t >= min(t_target, t_max) (uniform mode: until n h >= t_target
 * or n = N) or until max_steps steps (accepted + rejected) were taken.
 * Adaptive mode follows Sec. 3.5: each step evaluates the right-hand side of
 * Sec. 3.3-3.4 at every stage of Dormand-Prince 5(4) (SSPRK(10,4) once dt
 * reaches DP5's real-axis stability limit), forms the 1-norm error estimate
 * over all grid points and both fields, and accepts (dt x 0.9 when
 * eps < err <= 2 eps, x 1.01 when err < eps/2) or rejects (err > 2 eps: the
 * last min(10, M-1) slices are dropped and dt halved).  An accepted step
 * appends the new slice to the history (Sec. 3.2).  Sparsification (Sec. 3.6,
 * as dmfe_sparsify) runs automatically when the history reaches M_cap.
 * Uniform mode: classical RK4 steps of the trapezoid scheme of Sec. 2.3.
 * info (host, may be NULL) receives the counters and state.
 * Returns DMFE_OK, DMFE_DONE once t >= t_max (adaptive) or n = N (uniform),
 * DMFE_ERR_CAPACITY, DMFE_ERR_STEP_UNDERFLOW (dt < dt_min), DMFE_ERR_NONFINITE
 * or DMFE_ERR_DEVICE; on an error the handle keeps the last accepted state.
 */
dmfe_status dmfe_step(dmfe_handle *h, double t_target, int64_t max_steps, dmfe_step_info *info);

/*
 * Run `passes` sparsification passes over the stored history (Sec. 3.6):
 * for each candidate slice n = 1..M-12 (the first slice and the revert window
 * of the last eleven are kept) the residual eps_n = sum_i |Delta^C| + |Delta^R|
 * of the Hermite integrals over [t_{n-1}, t_{n+1}] with and without n is
 * formed on the device; a greedy sweep drops n when eps_n < eps/10 and then
 * skips n+1.  *removed (may be NULL) receives the number of slices dropped.
 */
dmfe_status dmfe_sparsify(dmfe_handle *h, int32_t passes, int64_t *removed);

/*
 * Copy `count` entries starting at `first` of a field into dst (device memory
 * if dst_on_device, else host; caller-owned, dst_bytes long).  Infrastructure,
 * not a step of the method: it exposes the stored history of Sec. 3.2 (t_n,
 * C, R and their t-derivatives, in logical slice order, as FP64 whatever the
 * storage precision) and the observables E(t_n), mu(t_n) of Sec. 2.1 formed
 * from the stored slices.  With dst == NULL only *needed_bytes is set.
 * Returns DMFE_ERR_BUFFER if dst_bytes is too small, DMFE_ERR_INVALID if the
 * range is outside the stored data.  Synchronises the handle's stream.
 */
dmfe_status dmfe_read(dmfe_handle *h, int32_t field, int64_t first, int64_t count, void *dst, size_t dst_bytes,
                      int32_t dst_on_device, size_t *needed_bytes);

/* Current counters and state (no device synchronisation beyond the stream's). */
dmfe_status dmfe_get_info(dmfe_handle *h, dmfe_step_info *info);

/*
 * Replace the stored history (adaptive mode).  t_hist[M] strictly increasing
 * with t_hist[0] = 0; C, R, dC, dR are [M][L] row-major (host or device as
 * src_on_device says); slices 0..nb-1 carry valid d/dt (nb = M or M-1).  The
 * state becomes slice M-1.  dt and scheme set the controller (dt <= 0 keeps
 * the current one).  Used to resume a run and to feed synthetic histories.
 */
dmfe_status dmfe_set_history(dmfe_handle *h, int64_t M, int64_t nb, const double *t_hist, const double *C,
                             const double *R, const double *dC, const double *dR, int32_t src_on_device,
                             double dt, int32_t scheme);

/*
 * One evaluation of the right-hand side on the theta grid (the hot path,
 * Sec. 3.3-3.4): d/dt C(t, theta_j t) and d/dt R(t, theta_j t) for all j at
 * stage time t >= t_{nb-1}, for the stage slice (yC, yR) [L] on the stored
 * history with slices 0..nb-1 carrying valid d/dt.  yC, yR, outC, outR are
 * device pointers.  Row L-1 (the diagonal) is pinned: outC[L-1] = outR[L-1] = 0
 * and the values computed there are returned in diag[2] (host, may be NULL).
 * mu (host, may be NULL) receives mu(t).  The history is not modified.
 */
dmfe_status dmfe_rhs(dmfe_handle *h, double t, const double *yC, const double *yR, int64_t nb, double *outC,
                     double *outR, double *mu, double *diag);

/*
 * For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): dmfe_rhs with the same
 * arguments, results and errors, but every transient buffer of the evaluation
 * (the interleaved stage slice, its history-format copy and log mirror, the
 * right-hand side before it is split into outC/outR, mu, E and the diagonal
 * values) is taken from one static device array of the library instead of the
 * handle's workspace.  No device or host memory is allocated and no timing
 * events are recorded.  The array holds a grid of at most 16384 points (about
 * 1.3 MB per device, kept until the process ends): DMFE_ERR_INVALID for a
 * larger L.  All calls on one device share its array and leave their contents
 * in it: calls that overlap in time on one device (two streams or two host
 * threads) race and must be serialised by the caller.
 */
dmfe_status dmfe_rhs_noalloc(dmfe_handle *h, double t, const double *yC, const double *yR, int64_t nb,
                             double *outC, double *outR, double *mu, double *diag);

void dmfe_destroy(dmfe_handle *h);

/*
 * Per-kernel timing with HIP events recorded on the handle's stream around
 * every launch of the timed kernels (enable = 1 starts and zeroes the
 * counters, 0 stops).  Kernel ids: DMFE_K_HIST_INTEGRAL (the history-integral
 * kernel), DMFE_K_STAGE_PREP (mu, E), DMFE_K_RK (stage combination and error
 * norm), DMFE_K_SPARSIFY (sparsification residual).  dmfe_timing_read returns
 * the number of timed launches, their summed duration in milliseconds, and
 * the summed number of stored slices the launches read (history-integral
 * kernel: slices with a stored derivative; others: 0).
 */
enum { DMFE_K_HIST_INTEGRAL = 0, DMFE_K_STAGE_PREP = 1, DMFE_K_RK = 2, DMFE_K_SPARSIFY = 3, DMFE_K_COUNT = 4 };
dmfe_status dmfe_timing(dmfe_handle *h, int32_t enable);
/* Which kernels dmfe_timing times: bit k of mask for kernel id k (default: all).
 * Each timed launch adds two event records to the stream, about 5% of an RK
 * step at L = 4096 when every kernel is timed; timing the history-integral
 * kernel alone costs a third of that.  Infrastructure, not a step of the
 * method.  Returns DMFE_ERR_INVALID for bits outside the kernel ids. */
dmfe_status dmfe_timing_select(dmfe_handle *h, uint32_t mask);
dmfe_status dmfe_timing_read(dmfe_handle *h, int32_t kernel, int64_t *launches, double *total_ms,
                             int64_t *slices_read);

/* Static text for a status code. */
const char *dmfe_status_string(dmfe_status s);

/* Text of the last HIP failure seen by any handle in this thread ("" if none). */
const char *dmfe_last_error(void);

/*
 * Human-readable parameter record of a solve (Appendix A: each run records
 * what reproduces it).  One "key = value" line per item: the library's source
 * revision and compiler, the HIP runtime and device, the process command line,
 * every field of dmfe_params, the grid-generation values (gamma, the grid
 * parameters) and the solve's current state and counters.
 * buf (host memory, cap bytes, may be NULL when cap is 0) receives the text
 * with a terminating NUL; *needed (if not NULL) the bytes that requires.
 * DMFE_ERR_BUFFER when cap is too small (buf untouched); DMFE_ERR_INVALID for
 * a NULL handle.  Reads host state only: no device work is enqueued.
 */
dmfe_status dmfe_param_record(const dmfe_handle *h, char *buf, size_t cap, size_t *needed);

/* ---------------------------------------------------------------- checkpoint and resume
 * Long solves (Sec. 4: runs to t ~ 1e7) survive restarts.  A checkpoint holds
 * the parameters (the solve's record), the controller state and counters, the
 * stored history in logical order, the FP64 state y(t) and, for DP5, the last
 * stage derivative it reuses, so a restored handle continues bitwise as the
 * saved one would have.  Adaptive mode only (DMFE_ERR_UNSUPPORTED otherwise).
 */

/* Save h's state to the file `path` (host string).  The device state is copied
 * to host memory before the call returns (the handle may step on at once);
 * with async != 0 the file is written by a background thread.  At most one
 * write is in flight per handle: a save first waits for the previous one and
 * returns its error, if any.  Not allowed while a pool steps the handle.
 * Errors: DMFE_ERR_INVALID (bad arguments, file cannot be written),
 * DMFE_ERR_DEVICE. */
dmfe_status dmfe_checkpoint_save(dmfe_handle *h, const char *path, int32_t async);
/* Wait for h's checkpoint write in flight, if any; returns its status. */
dmfe_status dmfe_checkpoint_wait(dmfe_handle *h);
/* Create a handle from the checkpoint file `path` on the device and stream of
 * `res` (as dmfe_create; a caller workspace must be at least dmfe_footprint of
 * the saved parameters).  DMFE_ERR_INVALID if the file is missing, of another
 * format or version, inconsistent, truncated or fails its checksum. */
dmfe_status dmfe_checkpoint_load(const char *path, const dmfe_resources *res, dmfe_handle **out);

/*
 * Compressed snapshot for post-processing (Appendix A): the history at reduced
 * resolution, for analyses that do not need all of it.  Kept: every
 * slice_stride-th stored slice and the newest, every theta_stride-th grid node
 * and theta = 1 (strides >= 1).  Written (host byte order):
 *   magic "DMFESNP1", uint32 version 1, uint32 header bytes,
 *   int64 L, M, theta_stride, slice_stride, L_kept, M_kept, uint64 record bytes,
 *   the parameter record text (dmfe_param_record, with its NUL),
 *   theta[L_kept] f64, t[M_kept] f64, E[M_kept] f64, mu[M_kept] f64,
 *   C[M_kept][L_kept] f32, R[M_kept][L_kept] f32 (rounded from the stored values).
 * Adaptive mode only (DMFE_ERR_UNSUPPORTED otherwise); DMFE_ERR_INVALID for bad
 * strides, a step in flight or an unwritable path.  Synchronous: the call
 * returns after the file is closed.
 */
dmfe_status dmfe_snapshot_save(dmfe_handle *h, const char *path, int32_t theta_stride, int32_t slice_stride);

/* ---------------------------------------------------------------- serving pool
 * Many solves (a parameter sweep: different T, a_p, t_max, L) stepped
 * together on one device.  Requests queue on submit and are admitted while a
 * slot is free and their footprint (dmfe_footprint) fits in the pool's arena;
 * admitted solves keep their history resident and advance together, one RK
 * stage evaluation per tick (DP5's first stage, the last stage of the step
 * before, takes none: its second runs in the same tick), each phase of a tick
 * being one batched launch over all of them (uneven L and M per solve).  Finished solves keep their memory until
 * dmfe_pool_release, so results can be read; released memory admits queued
 * requests.  All solves of a pool use the same history precision and s = 10.
 */
typedef struct dmfe_pool dmfe_pool;

typedef struct dmfe_pool_params {
    int32_t max_instances; /* admitted solves at most (1..4096) */
    int32_t reserved0;
    size_t max_bytes;      /* arena bytes used, 0: all of res->workspace_bytes */
} dmfe_pool_params;

typedef struct dmfe_pool_stats {
    int32_t running;             /* admitted and not finished */
    int32_t queued;              /* submitted, not yet admitted */
    int32_t finished_unreleased; /* finished, memory still held */
    int32_t reserved0;
    int64_t ticks;               /* stage ticks run so far */
    size_t bytes_free;
    size_t bytes_total;
} dmfe_pool_stats;

typedef struct dmfe_pool_times {
    int32_t status;   /* DMFE_DONE when the solve reached its t_max, else its error code */
    int32_t done;     /* 1 once finished */
    double queue_s;   /* submit -> admit */
    double service_s; /* admit -> done (or now) */
    double total_s;   /* submit -> done (or now): time to solution */
} dmfe_pool_times;

/* res->workspace (device memory, caller-owned, res->workspace_bytes bytes) is the
 * arena; res->stream orders all work of the pool. */
dmfe_status dmfe_pool_create(const dmfe_pool_params *pp, const dmfe_resources *res, dmfe_pool **out);
/* Queue a solve (adaptive mode); *request_id identifies it.  DMFE_ERR_NOMEM if it
 * can never fit, DMFE_ERR_UNSUPPORTED for a stencil other than the default (s != 10, theta_interp
 * != DMFE_INTERP_INDEX_LAGRANGE or log_r != 0) or a precision other than the pool's. */
dmfe_status dmfe_pool_submit(dmfe_pool *pool, const dmfe_params *params, uint64_t *request_id);
/* Run up to max_ticks stage ticks (returns early when nothing is running and
 * nothing can be admitted); stats may be NULL. */
dmfe_status dmfe_pool_run(dmfe_pool *pool, int64_t max_ticks, dmfe_pool_stats *stats);
/* Ids of solves finished since the last poll (up to cap). */
dmfe_status dmfe_pool_poll(dmfe_pool *pool, uint64_t *done_ids, int32_t cap, int32_t *n_done);
/* State and timings of an admitted or finished solve (info, times may be NULL). */
dmfe_status dmfe_pool_result(dmfe_pool *pool, uint64_t request_id, dmfe_step_info *info, dmfe_pool_times *times);
/* dmfe_read on an admitted or finished solve. */
dmfe_status dmfe_pool_read(dmfe_pool *pool, uint64_t request_id, int32_t field, int64_t first, int64_t count, void *dst,
                           size_t dst_bytes, int32_t dst_on_device, size_t *needed_bytes);
/* dmfe_set_history on an admitted, running solve that is between two steps (a
 * solve is admitted by dmfe_pool_run, also with max_ticks = 0): resumes a solve
 * from a stored history inside the pool.  DMFE_ERR_INVALID for an unknown,
 * queued or finished solve, or one whose step is in flight. */
dmfe_status dmfe_pool_set_history(dmfe_pool *pool, uint64_t request_id, int64_t M, int64_t nb, const double *t_hist,
                                  const double *C, const double *R, const double *dC, const double *dR,
                                  int32_t src_on_device, double dt, int32_t scheme);
/* Free a finished solve's memory. */
dmfe_status dmfe_pool_release(dmfe_pool *pool, uint64_t request_id);
void dmfe_pool_destroy(dmfe_pool *pool);

/* ---------------------------------------------------------------- host-only helpers
 * These run on the host without touching a device; they expose the
 * run-constant precompute and the scalar control logic the solver uses. */

/*
 * theta_i, 1 - theta_i and nu_i for the grid of these params (adaptive mode):
 * eq. (theta) at alpha = 0 with gamma = -W_{-1}(-1/t_max), and the integrals
 * of the not-a-knot quintic interpolating spline (Sec. 3.4).  Arrays of L
 * doubles (host).  *gamma (may be NULL) receives gamma.
 */
dmfe_status dmfe_grid(const dmfe_params *params, double *theta, double *theta_c, double *nu, double *gamma);

/*
 * Controller of Sec. 3.5 as a pure function of the last error estimate.
 * In: eps_rk, and *st (dt, scheme, M = stored slices before the step).
 * Out: *accepted (1/0), *n_revert (slices to drop when rejected) and the
 * updated *st (dt, scheme).  Rules: reject if eps_rk > 2 eps (revert
 * min(10, M-1) slices, halve dt); else accept and scale dt by 0.9 if
 * eps_rk > eps, by 1.01 if eps_rk < eps/2; DP5 switches to SSPRK(10,4) once
 * dt * 4 sqrt(f''(1)) reaches its real-axis stability limit, halving dt;
 * under SSPRK(10,4) dt is capped at its own real-axis limit.
 */
typedef struct dmfe_control {
    double eps;
    double dt;
    double dt_min;
    double rho; /* 4 sqrt(f''(1)), the spectral bound of Sec. 3.5 */
    int64_t M;
    int32_t scheme;
    int32_t policy;
} dmfe_control;

dmfe_status dmfe_control_update(dmfe_control *st, double eps_rk, int32_t *accepted, int32_t *n_revert);

/*
 * Greedy selection of one sparsification pass (Sec. 3.6) on host residuals:
 * candidates n = 1..last; drop[n] = 1 when eps_n[n] < thr and n-1 was not
 * dropped.  drop has M entries (host).  *removed receives the count.
 */
dmfe_status dmfe_sparsify_select(const double *eps_n, int64_t M, int64_t last, double thr, uint8_t *drop,
                                 int64_t *removed);

#ifdef __cplusplus
}
#endif

#endif /* DMFE_H */
