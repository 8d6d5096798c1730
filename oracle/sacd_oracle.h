/*
 * sacd_oracle.h -- plain FP64 CPU oracle of Saturating Coordinate Descent (SaCD)
 * for sparse nonnegative CP factorization of a 3-way tensor.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * Paper: Balasubramaniam, Nayak, Yuen, "Efficient Nonnegative Tensor
 * Factorization via Saturating Coordinate Descent", ACM TKDD 2020
 * (arXiv 2003.03572).  Every function below cites the passage it follows.
 *
 * Conventions
 *   - dims[3] = (I0, I1, I2) = (Q, P, S) in the paper's notation (Table of
 *     Symbols); mode n's factor A_n is I_n x R, row-major, FP64.
 *   - For mode n the two other modes are a < b.
 *   - Return codes: 0 ok, -1 invalid argument, -2 index out of range,
 *     -3 out of memory, -4 bad state, -6 non-finite value.
 */
#ifndef SACD_ORACLE_H
#define SACD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_tensor ora_tensor;
typedef struct ora_model ora_model;

/* Sparse tensor (Sec. 3, observed set Omega).  idx is nnz x 3, 0-based.
 * Duplicate coordinates are merged by FP32 addition in input order. */
int ora_tensor_create(const int64_t dims[3], int64_t nnz, const int32_t *idx,
                      const float *vals, ora_tensor **out);
void ora_tensor_destroy(ora_tensor *t);
int64_t ora_tensor_nnz(const ora_tensor *t);
double ora_tensor_norm2(const ora_tensor *t);
/* Mode-n sorted coordinates: coords is nnz x 3 holding (i_n, i_a, i_b) in
 * lexicographic order; ptr has dims[mode]+1 entries (slice Omega^n_i is
 * ptr[i]..ptr[i+1]). */
int ora_tensor_mode_coo(const ora_tensor *t, int mode, int32_t *coords,
                        float *vals, int64_t *ptr);

/* Sparse MTTKRP (eq. 9 first term; Sec. 4.4 column form):
 * M[i_n, r] = sum over Omega of x * A_a[i_a, r] * A_b[i_b, r]. */
int ora_mttkrp(const ora_tensor *t, int mode, int R, const double *A0,
               const double *A1, const double *A2, double *M);

/* Column r of the MTTKRP of `mode` alone (Sec. 4.4, the column form of FSaCD:
 * m_r[i_n] = sum over the slice Omega^n_{i_n} of x * A_a[i_a, r] * A_b[i_b, r],
 * a sparse tensor times vector product per column): m has dims[mode] entries. */
int ora_sttvp(const ora_tensor *t, int mode, int R, int r, const double *A0, const double *A1,
              const double *A2, double *m);

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): writes the first `count`
 * outputs of the generator seeded with `seed`. */
void ora_splitmix64(uint64_t seed, int64_t count, uint64_t *out);

/* Single-coordinate pieces, exposed for the pins. */
double ora_cd_delta(double a, double g, double h);          /* eq. 11-12 */
double ora_importance(double g, double delta, double L);    /* eq. 20 */
int ora_select(int64_t k, double z, double zprev, int flip); /* eq. 24-27, Alg. 1 */

enum { ORA_UPDATE_GS = 0, ORA_UPDATE_JACOBI = 1 };

/* Model: factors initialised from SplitMix64(seed): A_0, A_1, A_2 in that
 * order, row-major with R columns, each output x mapped to (x >> 40) * 2^-24. */
int ora_model_create(const ora_tensor *t, int R, uint64_t seed, int update_rule,
                     ora_model **out);
void ora_model_destroy(ora_model *m);
int ora_model_get_factor(const ora_model *m, int mode, double *dst);
int ora_model_set_factor(ora_model *m, int mode, const double *src);
/* Selection state of one mode: previous importances Z^{k-1} (I_n x R), the
 * previous total importance ti^{k-1} and the per-mode sweep counter k.
 * set_state takes the given Z^{k-1} as exact (its tie band is zero). */
int ora_model_get_state(const ora_model *m, int mode, double *zprev,
                        double *ti_prev, int64_t *k);
int ora_model_set_state(ora_model *m, int mode, const double *zprev,
                        double ti_prev, int64_t k);
/* force_flip: -1 = decide from ti (normal), 0 / 1 = force the eq. 27 branch
 * off / on (used to enumerate both outcomes at a total-importance tie). */
void ora_model_force_flip(ora_model *m, int force_flip);
/* Column-at-a-time form (Sec. 4.4, Alg. 2): cb >= 1 makes every later sweep
 * compute the MTTKRP cb columns at a time by ora_sttvp, once for the
 * importances and again, block by block in ascending column order, right
 * before the update of those columns, so that M is never needed whole; cb = 0
 * (default) is the row form.  Gauss-Seidel only (the update of a column uses
 * the current values of the earlier columns, as in the row form, so both forms
 * give the same sweep).  INVALID_ARG for cb < 0 or the Jacobi rule. */
int ora_model_set_columns(ora_model *m, int cb);

/* Relative width tau of the tie band (default 1e-6), see ora_sweep_band. */
void ora_model_set_tie_tol(ora_model *m, double tau);

/* Threads of the oracle's parallel loops (OpenMP; loops whose iterations are
 * independent, so every result is bit-identical for any thread count).
 * n < 1 leaves the count unchanged.  Returns the count now in use (1 when
 * built without OpenMP). */
int ora_set_threads(int n);

/* One SaCD sweep of mode n (Alg. 1 body for one factor matrix). */
int ora_sweep(ora_model *m, int mode);

/* Record of the last sweep of `mode`.  Any pointer may be NULL.
 * M, G0, z (I_n x R), sel (uint8 I_n x R), H (R x R), scalars: L, ti, flip,
 * ti_prev (the ti^{k-1} the selection compared with), f (objective after the
 * sweep), nsel, inner <M, A_n>, model sum (G0 * G1 * G2). */
int ora_sweep_info(const ora_model *m, int mode, double *M, double *G0,
                   double *z, uint8_t *sel, double *H,
                   double *scalars /* [L, ti, flip, ti_prev, f, nsel, inner, model] */);

/* Tie band of the last sweep of `mode` (a diagnostic of the oracle, not part
 * of the method).  The selection turns the sign of a difference of rounded
 * values into a decision; where an implementation in lower precision may
 * take either decision, both are correct.  For every element:
 *   band   tau (|dz/dg| T + (L/2) d^2) + (tau T / h)^2 (h + L/2): how far
 *          z moves when its gradient g carries an error of tau T, T = |M| +
 *          sum_s |A_s H_sr| the terms g is formed from (eq. 14), d the step
 *          (eq. 11-12); (L/2) d^2 covers the rounding of that term of z
 *          (eq. 20), the last term (interior steps and zero-gradient ties
 *          only) the second-order move of z near g = 0.
 *   kind   0 decided (margin outside the band), 1 exact zero (z and Z^{k-1}
 *          structurally zero: decided), 2 zero-gradient tie (a = 0 and
 *          |g| <= tau T: the step is zero or not by the sign of g),
 *          3 margin tie (|margin| <= band + band of Z^{k-1}).
 * scalars: [band_ti = sum band + sum band of Z^{k-1}, tie_global (k >= 2 and
 *           |ti - ti^{k-1}| <= band_ti), n_exact_zero, n_zero_grad,
 *           n_margin]. */
int ora_sweep_band(const ora_model *m, int mode, double *band, uint8_t *kind,
                   double *scalars /* [5] */);

/* Undo the last sweep of `mode`: restore the factor, its Gram matrix, Z^{k-1},
 * ti^{k-1}, k and the tie band of Z^{k-1} to their values before that sweep
 * (used to re-run a sweep with the other eq. 27 branch at a tie of the total
 * importance).  BAD_STATE if the mode has not been swept since its state was
 * last set. */
int ora_sweep_undo(ora_model *m, int mode);

/* The update (step 9 of ora_sweep) of row q of the last sweep of `mode`
 * under the decisions sel (R bytes, 1 = selected), from the state before that
 * sweep: the oracle's row for any valid choice at tie elements. */
int ora_row_outcome(const ora_model *m, int mode, int64_t q, const uint8_t *sel, double *out);

/* Objective eq. 6 (full-tensor least squares) and fit 1 - sqrt(f)/||X||. */
double ora_objective(const ora_model *m);
int ora_fit(const ora_model *m, double *fit, double *f);

/* Accuracy of a factorization (Sec. 6, evaluation criteria).
 * ora_rmse: eq. 30, the root mean square error of the model on n entries
 * (idx: n x 3 coordinates, vals: observed values), typically held out of the
 * factorised tensor; n = 0 gives 0.  ERANGE for a coordinate outside dims.
 * ora_pd: pattern distinctiveness of the columns of factor `mode`: the
 * cosine similarity of every column pair i < r (eq. pd), averaged (the paper
 * lists the pairs without saying how they are combined; the mean is the
 * reading taken).  Pairs with a zero column are left out; no pair gives 0. */
int ora_rmse(const ora_model *m, int64_t n, const int32_t *idx, const float *vals, double *rmse);
int ora_pd(const ora_model *m, int mode, double *pd);

/* Outer loop of Alg. 1: iterations of sweep(0), sweep(1), sweep(2); stops
 * after iteration k >= 2 when |fit_k - fit_{k-1}| < tol * |fit_{k-1}|, or at
 * max_iter.  fit_trace (may be NULL) receives one fit per iteration. */
int ora_run_until(ora_model *m, double tol, int max_iter, int *iters_done,
                  double *final_fit, double *fit_trace);

#ifdef __cplusplus
}
#endif
#endif
