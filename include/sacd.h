/*
 * sacd.h -- C ABI of the MI355X (gfx950) implementation of Saturating
 * Coordinate Descent (SaCD) for sparse nonnegative CP factorization of a
 * 3-way tensor.
 *
 * Paper: Balasubramaniam, Nayak, Yuen, "Efficient Nonnegative Tensor
 * Factorization via Saturating Coordinate Descent", ACM TKDD 2020
 * (arXiv 2003.03572).  Problem (Sec. 3, eq. ntf): given a sparse tensor X of
 * size I0 x I1 x I2 with observed set Omega, find nonnegative factors
 * A0 (I0 x R), A1 (I1 x R), A2 (I2 x R) minimising ||X - [[A0, A1, A2]]||^2
 * (eq. 6), unobserved cells counting as zeros.  The library runs Algorithm 1:
 * for every outer iteration, one sweep of each mode 0, 1, 2.
 *
 * Conventions for every call
 *   - Device pointers are plain HIP device addresses on the device that was
 *     current when the tensor was created.  Host pointers are marked "host".
 *   - Streams are hipStream_t values passed as void*.  NULL means "the
 *     library creates its own non-blocking stream" (the null stream cannot be
 *     captured into the graphs the library uses).
 *   - Calls never throw; they return a sacd_status.  sacd_last_error()
 *     returns a message for the last failing call on the calling thread.
 *   - A tensor or model is used by one host thread at a time.  All GPU work
 *     of a model is ordered on its stream; calls that return results to the
 *     host synchronise that stream.
 *   - Factors are FP32, row-major, R columns (unpadded) at the boundary.
 */
#ifndef SACD_H
#define SACD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SACD_OK = 0,
  SACD_ERR_INVALID_ARG = -1,  /* bad size, mode, rank, pointer or option */
  SACD_ERR_OUT_OF_RANGE = -2, /* a coordinate is outside dims */
  SACD_ERR_NO_MEMORY = -3,    /* device allocation failed */
  SACD_ERR_BAD_STATE = -4,    /* call not valid in the object's state */
  SACD_ERR_DEVICE = -5,       /* a HIP runtime call failed */
  SACD_ERR_NUMERIC = -6       /* NaN/Inf input, or ||X|| = 0 where a fit is asked */
} sacd_status;

/* Arithmetic of the dense R x R products (Gram matrices and A_n * H).
 * FP32: everything in FP32 (objective in FP64).  MIXED_BF16: the Grams that
 * form H and the product A_n * H on BF16 MFMA with FP32 accumulation; MTTKRP
 * and updates stay FP32; the objective (eq. 6) is formed in FP64 from Grams of
 * FP32 operands, so the reported objective and fit are those of the factors
 * as they are. */
typedef enum { SACD_PREC_FP32 = 0, SACD_PREC_MIXED_BF16 = 1 } sacd_precision;

/* Update of the selected elements (eq. 13).  GS: each selected element takes
 * the exact one-variable minimiser with the gradient refreshed for the
 * elements of its row already moved in this sweep (the refresh of g_qr that
 * Lemma 2 calls for).  JACOBI: every selected element moves by the step
 * computed from the sweep's snapshot gradient. */
typedef enum { SACD_UPDATE_GS = 0, SACD_UPDATE_JACOBI = 1 } sacd_update;

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns a device pointer (256-byte aligned) or NULL; release frees it.
 * When the pointer passed to sacd_create_tensor is NULL the library uses
 * hipMalloc / hipFree. */
typedef struct sacd_allocator {
  void *(*alloc)(size_t bytes, void *user);
  void (*release)(void *ptr, void *user);
  void *user;
} sacd_allocator;

typedef struct sacd_tensor sacd_tensor; /* opaque, library-owned */
typedef struct sacd_model sacd_model;   /* opaque, library-owned */

/* Per-sweep statistics of one mode (host struct). */
typedef struct sacd_sweep_stats {
  int64_t k;          /* sweeps of this mode done so far (Alg. 1 loop counter) */
  double lipschitz;   /* L = ||H||_F of the last sweep (Alg. 1) */
  double ti;          /* total importance of the last sweep (eq. 25) */
  int32_t flip;       /* 1 if the last sweep used eq. 27 (ti grew) */
  int64_t n_selected; /* |E|: elements selected in the last sweep */
  double objective;   /* eq. 6 after the last sweep of this mode (FP64) */
} sacd_sweep_stats;

/* ------------------------------------------------------------------------ */
/* Tensor                                                                    */
/* ------------------------------------------------------------------------ */

/* Ingest a sparse tensor (Sec. 3: observed set Omega and its slices
 * Omega^U_q, Omega^V_p, Omega^W_s).
 *   dims  host, 3 mode lengths, each in [1, 2^31 - 1]; the bit widths of
 *         (I0 - 1, I1 - 1, I2 - 1) must sum to at most 64.
 *   nnz   number of entries, in [0, 2^31 - 1].
 *   idx   device, nnz x 3 int32, row-major, 0-based coordinates.
 *   vals  device, nnz float32.
 *   alloc optional device allocator (NULL: hipMalloc).
 *   stream hipStream_t or NULL (see conventions).
 *   out   host, receives the tensor handle.
 * The library copies the data; the caller keeps ownership of idx / vals.
 * Entries with equal coordinates are merged by FP32 addition in input order.
 * For each mode n the entries are sorted by (i_n, i_a, i_b), a < b the other
 * modes, and slice pointers are built.  Synchronises the stream once.
 * Errors: INVALID_ARG (sizes, NULL pointers), OUT_OF_RANGE (a coordinate not
 * in [0, dims)), NUMERIC (NaN/Inf value), NO_MEMORY, DEVICE. */
sacd_status sacd_create_tensor(const int64_t dims[3], int64_t nnz, const int32_t *idx,
                               const float *vals, const sacd_allocator *alloc, void *stream,
                               sacd_tensor **out);

/* dims (host, 3), nnz after merging, ||X||^2 (FP64) and the device bytes the
 * tensor holds.  Any output pointer may be NULL. */
sacd_status sacd_tensor_info(const sacd_tensor *t, int64_t dims[3], int64_t *nnz, double *norm2,
                             int64_t *device_bytes);

/* Export mode `mode`'s sorted entries: coords device nnz x 3 int32 holding
 * (i_n, i_a, i_b); vals device nnz float32; ptr device (dims[mode] + 1)
 * int64 slice offsets.  Any pointer may be NULL.  Synchronises. */
sacd_status sacd_tensor_mode_coo(const sacd_tensor *t, int32_t mode, int32_t *coords, float *vals,
                                 int64_t *ptr);

/* Release the tensor.  While models built on it are alive, the release is
 * deferred until the last of them is destroyed. */
void sacd_destroy_tensor(sacd_tensor *t);

/* ------------------------------------------------------------------------ */
/* Model                                                                     */
/* ------------------------------------------------------------------------ */

/* Create a model of rank R in [1, 128] over tensor t (Alg. 1 inputs: tensor,
 * randomly initialised factors, rank).  The cap of 128 is this library's: the
 * element kernels keep a block's rows of A_n and the R x R matrix H in LDS,
 * and at R = 256 H alone (256 KB in FP32) exceeds a CU's 160 KB.  Factors A0, A1, A2 are filled in that
 * order, row-major with R columns, from consecutive outputs of SplitMix64
 * seeded with `seed`, each output x mapped to (x >> 40) * 2^-24 in [0, 1).
 * Z = empty (no sweep done).  The tensor must outlive the model.
 * Errors: INVALID_ARG, NO_MEMORY, DEVICE. */
sacd_status sacd_init_factors(sacd_tensor *t, int32_t R, uint64_t seed, sacd_precision prec,
                              sacd_update update, sacd_model **out);

/* A model in the column-at-a-time form (Sec. 4.4, Alg. 2: the MTTKRP formed a
 * column block at a time, as the paper's "sparse tensor times vector" column
 * form does one column at a time): every sweep forms M in blocks of
 * column_block columns -- once for the importances of all elements (whose
 * total ti, eq. 25, is needed before any update), and once more per block,
 * in ascending column order, right before the Gauss-Seidel steps of that
 * block's selected elements -- so the model holds an I_n x column_block block
 * of M instead of three I_n x R buffers (and no per-element selection record
 * unless diagnostics are on).  The sweeps compute what sacd_init_factors'
 * models compute (same selection rule and steps; sums in another order), at
 * the cost of two passes over the entries per column block.  FP32,
 * Gauss-Seidel; other arguments as sacd_init_factors.  column_block in
 * {1, 2, 4, 8, 16}, else INVALID_ARG.  Kernel timing (sacd_time_kernel) is
 * not available for such a model (BAD_STATE); sacd_iterate_timed's MTTKRP
 * interval covers both passes. */
sacd_status sacd_init_factors_columns(sacd_tensor *t, int32_t R, uint64_t seed, int32_t column_block,
                                      sacd_model **out);

/* Enqueue one SaCD sweep of mode `mode` in {0, 1, 2} (Alg. 1 body for one
 * factor matrix: MTTKRP, H and L, gradient and importance eq. 14 / eq. 20,
 * total importance eq. 25, selection eq. 24 / eq. 27, update eq. 11-13,
 * Gram and objective).  Asynchronous.  Errors: INVALID_ARG, DEVICE. */
sacd_status sacd_sweep(sacd_model *m, int32_t mode);

/* Enqueue `n_iters` outer iterations (sweeps of modes 0, 1, 2 each) as
 * replays of one captured HIP graph.  Asynchronous. */
sacd_status sacd_iterate(sacd_model *m, int32_t n_iters);

/* Objective eq. 6 after the most recent sweep (FP64) and fit
 * 1 - sqrt(max(f, 0)) / ||X||.  Before any sweep, the objective of the
 * initial factors.  Synchronises.  NUMERIC if ||X|| = 0 (f is still set). */
sacd_status sacd_fit(sacd_model *m, double *fit, double *objective);

/* Outer loop of Alg. 1: run iterations until, after iteration k >= 2 of
 * this call, |fit_k - fit_{k-1}| < tol * |fit_{k-1}|, or max_iter
 * iterations.  Per-mode sweep counters persist across calls.  Synchronises
 * once per iteration.  Outputs may be NULL. */
sacd_status sacd_run_until(sacd_model *m, double tol, int32_t max_iter, int32_t *iters_done,
                           double *final_fit);

/* Copy factor `mode` out to / in from device memory (I_n x R row-major
 * FP32).  set_factor rejects negative or non-finite values (NUMERIC) and
 * recomputes that mode's Gram matrix.  Synchronises. */
sacd_status sacd_get_factor(const sacd_model *m, int32_t mode, float *dst);
sacd_status sacd_set_factor(sacd_model *m, int32_t mode, const float *src);

/* Accuracy of the factorization (Sec. 6, evaluation criteria).
 * sacd_rmse: eq. 30, sqrt(sum (x - x_hat)^2 / n) over n entries, usually
 * held out of the factorised tensor.  idx: device, n x 3 int32 0-based
 * coordinates; vals: device, n f32.  x_hat (eq. 5) is formed from the FP32
 * factors in FP64.  OUT_OF_RANGE if a coordinate is outside dims; n = 0
 * gives 0.  Synchronises.
 * sacd_pd: pattern distinctiveness (eq. pd) of the columns of factor `mode`
 * (the paper uses the last factor): the cosine similarity of every column
 * pair i < r, averaged over the pairs; pairs with a zero column are left out
 * (no pair left: 0).  Computed from the factor's Gram matrix.  Synchronises. */
sacd_status sacd_rmse(sacd_model *m, int64_t n, const int32_t *idx, const float *vals, double *rmse);
sacd_status sacd_pd(const sacd_model *m, int32_t mode, double *pd);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sacd_rmse
 * without any allocation and without synchronising.  The same kernel runs on
 * the model's stream with its scratch (1024 per-block partial sums, their
 * total, a counter and a flag: 8.4 KiB) in a static device array of the
 * library, one copy per device, kept until the process ends.
 *   idx, vals  device, as for sacd_rmse; n in [0, 2^31 - 1] (larger n:
 *              INVALID_ARG, nothing launched).
 *   out        device, 2 doubles written asynchronously: out[0] the RMSE
 *              (0 for n = 0; NaN if a coordinate is outside dims), out[1] 1.0
 *              if a coordinate was outside dims, else 0.0.
 * Every call on one device shares that device's scratch: calls that overlap
 * on one GPU (other streams, other threads, other models) race and must be
 * ordered by the caller.  Errors: INVALID_ARG, DEVICE. */
sacd_status sacd_rmse_static(const sacd_model *m, int64_t n, const int32_t *idx, const float *vals, double *out);

/* Selection state of one mode, for checkpoint / resume: zprev device
 * I_n x R FP32 (importance of the last sweep, Z^{k-1} of Alg. 1), ti_prev
 * (host, eq. 26) and k (host, sweeps done; k = 0 means Z is empty).
 * Synchronises.  Any pointer of get_state may be NULL. */
sacd_status sacd_get_state(const sacd_model *m, int32_t mode, float *zprev, double *ti_prev,
                           int64_t *k);
sacd_status sacd_set_state(sacd_model *m, int32_t mode, const float *zprev, double ti_prev,
                           int64_t k);

/* Statistics of the last sweep of `mode` (host struct).  Synchronises. */
sacd_status sacd_get_stats(const sacd_model *m, int32_t mode, sacd_sweep_stats *out);

/* Per-column counts |e_r| of the last sweep of `mode`: counts (host, R
 * int64) receives, for every column r, the number of elements of column r
 * selected for update (Alg. 1, the column-wise element update of Sec. 4.3 and
 * Alg. 2); their sum is n_selected of sacd_get_stats.  Zeros before the first
 * sweep of the mode.  Synchronises.  Errors: INVALID_ARG (NULL, mode), DEVICE. */
sacd_status sacd_get_column_counts(const sacd_model *m, int32_t mode, int64_t *counts);

/* Diagnostics of the last sweep of `mode`, for parity tests:
 *   mttkrp     device I_n x R FP32, the MTTKRP M of eq. 9;
 *   selection  device I_n x R uint8, 1 where the element was selected
 *              (recorded only while diagnostics are enabled, else zeros);
 *   gram       host R x R FP64, A_n^T A_n after the sweep.
 * Any pointer may be NULL.  Synchronises. */
sacd_status sacd_get_diagnostics(const sacd_model *m, int32_t mode, float *mttkrp,
                                 uint8_t *selection, double *gram);
/* Enable (1) or disable (0) recording of the selection mask. */
sacd_status sacd_set_diagnostics(sacd_model *m, int32_t enable);

/* Time kernel `which` (0 = MTTKRP main kernel, 1 = selection/update kernel,
 * 2 = importance kernel) of mode `mode` on the model's stream with HIP
 * events: `reps` back-to-back launches on the current state; the average
 * milliseconds per launch go to *avg_ms (host).  The kernels re-run on
 * unchanged inputs, so the model state is not advanced by MTTKRP / importance
 * timing; timing the update kernel does change the factors.  Synchronises. */
sacd_status sacd_time_kernel(sacd_model *m, int32_t which, int32_t mode, int32_t reps,
                             float *avg_ms);

/* Measurement support.  sacd_timing_prepare creates the HIP events for
 * n_iters timed iterations (no sweep runs).  sacd_iterate_timed runs n_iters
 * outer iterations -- the same kernels, on the same stream, advancing the
 * model exactly like sacd_iterate(m, n_iters), but enqueued launch by launch
 * instead of replayed from the graph, with an event recorded right before
 * and right after each MTTKRP launch and after each sweep's last kernel --
 * waits for them, and writes the MTTKRP kernel duration of iteration i, mode
 * n (milliseconds) to mttkrp_ms[3 i + n] and, when sweep_ms is not NULL, the
 * duration of that whole sweep to sweep_ms[3 i + n] (host arrays of 3 n_iters
 * floats).  BAD_STATE if events for fewer than n_iters iterations were
 * prepared.  The events live as long as the model. */
sacd_status sacd_timing_prepare(sacd_model *m, int32_t n_iters);
sacd_status sacd_iterate_timed(sacd_model *m, int32_t n_iters, float *mttkrp_ms, float *sweep_ms);

/* Algorithmic HBM bytes of one launch of kernel `which` (as in
 * sacd_time_kernel) for mode `mode` at the model's shapes (host). */
sacd_status sacd_kernel_bytes(const sacd_model *m, int32_t which, int32_t mode, double *bytes);

/* Device bytes held by the model (factors, importances, MTTKRP, scratch). */
sacd_status sacd_model_bytes(const sacd_model *m, int64_t *bytes);

void sacd_destroy_model(sacd_model *m);

/* ------------------------------------------------------------------------
 * Serving: many independent jobs resident on one GPU.
 *
 * A server holds factorization jobs (a tensor, a rank, a seed) of uneven size.
 * Requests are queued by sacd_server_submit and admitted first come first
 * served while the device bytes of the running jobs plus the new job's upper
 * bound (sacd_job_bytes: resident + transient ingest bytes) stay within the
 * budget and a slot is free.  Each sacd_server_step runs one outer iteration
 * (Alg. 1: sweeps of modes 0, 1, 2) of every running job and admits what fits
 * while it runs (uploads and ingests on a stream the server owns; the
 * admitted jobs iterate from the next step, or in this step when no job was
 * running).  The iteration uses persistent job-batched kernels -- per mode and per padded rank one
 * launch of each sweep kernel covers all jobs, its blocks looping over the
 * jobs' work items -- replayed from a HIP graph while the
 * set of running jobs is unchanged, and retires the jobs that met the
 * stopping rule of sacd_run_until (relative fit change < tol after at least
 * two iterations, or max_iter).  A job's arithmetic is the same as when it
 * runs alone (sacd_init_factors + sacd_run_until with the same arguments):
 * results are bit-identical alone and in the mix.  Updates are Gauss-Seidel.
 * The server's iterations run on its stream, admissions on a second stream
 * it creates; calls synchronise both. */
typedef struct sacd_server sacd_server;

typedef struct {
  int64_t budget_bytes;     /* device bytes the running jobs may hold */
  int32_t max_slots;        /* running jobs at most */
  int32_t max_iter;         /* outer iterations per job at most */
  double tol;               /* relative fit change that stops a job */
  sacd_precision precision; /* arithmetic of every job */
  int32_t use_graphs;       /* 1: replay unchanged job sets from a HIP graph */
} sacd_server_config;

enum { SACD_JOB_QUEUED = 0, SACD_JOB_RUNNING = 1, SACD_JOB_DONE = 2, SACD_JOB_FAILED = 3, SACD_JOB_CANCELLED = 4 };

typedef struct {
  int32_t running, queued;
  int64_t bytes_in_use, peak_bytes;
  int64_t steps, graph_builds, graph_launches, eager_launches;
  /* host wall seconds spent admitting jobs, building launch tables, running
   * iterations (launch to the objectives read back) and retiring jobs */
  double sec_admit, sec_tables, sec_iterate, sec_retire;
} sacd_server_stats_t;

/* Upper bounds of the device bytes of a job of this shape and precision
 * (host only, no GPU call): *resident while it runs, *transient extra during
 * its ingest.  Errors: INVALID_ARG (sizes, rank, precision). */
sacd_status sacd_job_bytes(const int64_t dims[3], int64_t nnz, int32_t R, sacd_precision prec,
                           int64_t *resident, int64_t *transient);
/* alloc, stream: as for sacd_create_tensor (every job's buffers come from
 * alloc; all work runs on the stream). */
sacd_status sacd_server_create(const sacd_server_config *cfg, const sacd_allocator *alloc, void *stream,
                               sacd_server **out);
/* Queue a job.  idx (nnz x 3 int32, 0-based) and vals (nnz f32) are HOST
 * arrays, copied at once.  NO_MEMORY if the job's bound exceeds the whole
 * budget.  *ticket identifies the job in later calls. */
sacd_status sacd_server_submit(sacd_server *s, const int64_t dims[3], int64_t nnz, const int32_t *idx,
                               const float *vals, int32_t R, uint64_t seed, int64_t *ticket);
/* Iterate every running job once while admitting what fits, retire finished
 * ones, then add the admitted jobs to the running set.  A job whose
 * objective turns non-finite fails there (state FAILED, status NUMERIC, its
 * memory freed, no result); the other jobs run on unchanged. */
sacd_status sacd_server_step(sacd_server *s, int32_t *n_running, int32_t *n_queued);
/* Tickets that finished (done or failed) in the last step: the first
 * min(cap, *n) are written to tickets (host). */
sacd_status sacd_server_finished(const sacd_server *s, int64_t *tickets, int32_t cap, int32_t *n);
/* State (SACD_JOB_*), iterations done, fit and objective of a job; a failed
 * job returns the status its admission failed with. */
sacd_status sacd_server_poll(const sacd_server *s, int64_t ticket, int32_t *state, int32_t *iters,
                             double *fit, double *objective);
/* Factor `mode` of a done job into dst (HOST, I_n x R row-major f32). */
sacd_status sacd_server_result(const sacd_server *s, int64_t ticket, int32_t mode, float *dst);
/* Forget a done, failed or cancelled job's result. */
sacd_status sacd_server_release(sacd_server *s, int64_t ticket);
/* Cancel a queued or running job (between steps): it leaves the queue, or
 * stops and frees its device memory at once; state CANCELLED, no result; the
 * other jobs run on unchanged.  Errors: INVALID_ARG (unknown ticket),
 * BAD_STATE (the job has already finished). */
sacd_status sacd_server_cancel(sacd_server *s, int64_t ticket);
/* Set the budget of later admissions to budget_bytes (at most the budget the
 * server was created with).  Running jobs keep their memory even above a
 * lowered budget; no job is admitted until the running jobs' bytes plus its
 * bound fit.  Queued jobs whose bound alone exceeds the new budget fail
 * (status NO_MEMORY), as sacd_server_submit refuses such jobs.  Errors:
 * INVALID_ARG (budget not in (0, creation budget]). */
sacd_status sacd_server_set_budget(sacd_server *s, int64_t budget_bytes);
sacd_status sacd_server_stats(const sacd_server *s, sacd_server_stats_t *out);
void sacd_server_destroy(sacd_server *s);

/* ------------------------------------------------------------------------ */
/* N-way tensors                                                             */
/* ------------------------------------------------------------------------ */

/* Sec. 3 defines nonnegative CP factorization for a tensor of any number of
 * modes N; the paper derives the sweep for three.  For N modes each sweep of
 * mode n is the same Alg. 1 body with the Khatri-Rao product of the N - 1
 * other factors in the MTTKRP (eq. 9: M[i_n, r] = sum over the entries of the
 * slice of x times the product of the other factors' rows at column r) and H
 * the Hadamard product of the N - 1 other Gram matrices (eq. 10); the
 * objective (eq. 6) is ||X||^2 - 2 <X, Xhat> + the sum over the Hadamard
 * product of all N Grams.  FP32 arithmetic, Gauss-Seidel updates (as
 * SACD_UPDATE_GS), objective in FP64; every convention of the three-way calls
 * holds unless stated.  An outer iteration is one sweep of each mode
 * 0, ..., N - 1. */
typedef struct sacd_ntensor sacd_ntensor; /* opaque, library-owned */
typedef struct sacd_nmodel sacd_nmodel;   /* opaque, library-owned */

/* Ingest an N-way sparse tensor.
 *   N     number of modes, in [2, 8].
 *   dims  host, N mode lengths, each in [1, 2^31 - 1]; the bit widths of
 *         (I_n - 1) must sum to at most 64.
 *   nnz   in [0, 2^31 - 1]; idx device nnz x N int32 (row-major, 0-based);
 *         vals device nnz float32.
 *   alloc, stream, out: as sacd_create_tensor.
 * Duplicates merged by FP32 addition in input order.  For each mode n the
 * entries are sorted by (i_n, then the other indices in increasing mode
 * order) and slice pointers built.  Errors: INVALID_ARG, OUT_OF_RANGE,
 * NUMERIC (NaN/Inf value), NO_MEMORY, DEVICE. */
sacd_status sacd_create_ntensor(int32_t N, const int64_t *dims, int64_t nnz, const int32_t *idx,
                                const float *vals, const sacd_allocator *alloc, void *stream,
                                sacd_ntensor **out);
/* N, dims (host, N), nnz after merging, ||X||^2, device bytes; any output
 * may be NULL. */
sacd_status sacd_ntensor_info(const sacd_ntensor *t, int32_t *N, int64_t *dims, int64_t *nnz,
                              double *norm2, int64_t *device_bytes);
/* Mode `mode`'s sorted entries: coords device nnz x N int32 (i_n, then the
 * other indices in increasing mode order), vals device nnz float32, ptr
 * device (dims[mode] + 1) int64.  Any pointer may be NULL.  Synchronises. */
sacd_status sacd_ntensor_mode_coo(const sacd_ntensor *t, int32_t mode, int32_t *coords, float *vals,
                                  int64_t *ptr);
/* Deferred while models built on the tensor are alive. */
void sacd_destroy_ntensor(sacd_ntensor *t);

/* Model of rank R in [1, 128]; factors A_0, ..., A_{N-1} filled in that order
 * from consecutive SplitMix64 outputs as sacd_init_factors does.  Errors:
 * INVALID_ARG, NO_MEMORY, DEVICE. */
sacd_status sacd_init_nfactors(sacd_ntensor *t, int32_t R, uint64_t seed, sacd_nmodel **out);
/* One sweep of mode `mode` in [0, N) (asynchronous). */
sacd_status sacd_nsweep(sacd_nmodel *m, int32_t mode);
/* n_iters outer iterations replayed from one captured HIP graph (asynchronous). */
sacd_status sacd_niterate(sacd_nmodel *m, int32_t n_iters);
/* n_iters outer iterations enqueued launch by launch with events around
 * each MTTKRP launch and at each sweep's end; waits, then writes the MTTKRP
 * milliseconds of iteration i, mode n to mttkrp_ms[N i + n] and (if sweep_ms
 * is not NULL) the sweep's to sweep_ms[N i + n] (host, N n_iters floats).
 * n_iters in [1, 100000]. */
sacd_status sacd_niterate_timed(sacd_nmodel *m, int32_t n_iters, float *mttkrp_ms, float *sweep_ms);
/* As sacd_fit / sacd_run_until (the objective is read after mode N - 1). */
sacd_status sacd_nfit(sacd_nmodel *m, double *fit, double *objective);
sacd_status sacd_nrun_until(sacd_nmodel *m, double tol, int32_t max_iter, int32_t *iters_done,
                            double *final_fit);
/* As sacd_get_factor / sacd_set_factor / sacd_get_state / sacd_set_state /
 * sacd_get_stats / sacd_get_column_counts / sacd_get_diagnostics /
 * sacd_set_diagnostics, for mode in [0, N). */
sacd_status sacd_get_nfactor(const sacd_nmodel *m, int32_t mode, float *dst);
sacd_status sacd_set_nfactor(sacd_nmodel *m, int32_t mode, const float *src);
sacd_status sacd_get_nstate(const sacd_nmodel *m, int32_t mode, float *zprev, double *ti_prev,
                            int64_t *k);
sacd_status sacd_set_nstate(sacd_nmodel *m, int32_t mode, const float *zprev, double ti_prev,
                            int64_t k);
sacd_status sacd_get_nstats(const sacd_nmodel *m, int32_t mode, sacd_sweep_stats *out);
sacd_status sacd_get_ncolumn_counts(const sacd_nmodel *m, int32_t mode, int64_t *counts);
sacd_status sacd_get_ndiagnostics(const sacd_nmodel *m, int32_t mode, float *mttkrp,
                                  uint8_t *selection, double *gram);
sacd_status sacd_set_ndiagnostics(sacd_nmodel *m, int32_t enable);
/* Device bytes held by the model. */
sacd_status sacd_nmodel_bytes(const sacd_nmodel *m, int64_t *bytes);
void sacd_destroy_nmodel(sacd_nmodel *m);

/* ------------------------------------------------------------------------ */
/* Misc                                                                      */
/* ------------------------------------------------------------------------ */
const char *sacd_status_string(sacd_status s);
const char *sacd_last_error(void);
/* Library version, e.g. "0.1.0". */
const char *sacd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SACD_H */
