/*
 * sacd_oracle_n.h -- plain FP64 CPU oracle of SaCD for N-way tensors.
 *
 * TEST INFRASTRUCTURE ONLY (as sacd_oracle.h): it checks the GPU library and
 * shares nothing with it.
 *
 * The paper defines nonnegative tensor factorization for N modes (Sec. 3,
 * eq. ntf) and derives the sweep for three; for N modes the steps are the
 * same with the Khatri-Rao product of the N - 1 other factors in the MTTKRP
 * (eq. 9) and the Hadamard product of their N - 1 Gram matrices as H
 * (eq. 10).  Mode n's factor A_n is I_n x R, row-major, FP64.  Return codes as
 * in sacd_oracle.h.  N in [2, 8].
 */
#ifndef SACD_ORACLE_N_H
#define SACD_ORACLE_N_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oran_tensor oran_tensor;
typedef struct oran_model oran_model;

/* idx: nnz x N, 0-based.  Duplicates merged by FP32 addition in input order. */
int oran_tensor_create(int N, const int64_t *dims, int64_t nnz, const int32_t *idx, const float *vals,
                       oran_tensor **out);
void oran_tensor_destroy(oran_tensor *t);
int64_t oran_tensor_nnz(const oran_tensor *t);
double oran_tensor_norm2(const oran_tensor *t);
/* Mode-n sorted entries: coords nnz x N holding (i_n, then the other indices
 * in increasing mode order), lexicographic; ptr dims[mode] + 1 slice offsets. */
int oran_tensor_mode_coo(const oran_tensor *t, int mode, int32_t *coords, float *vals, int64_t *ptr);

/* M[i_n, r] = sum over Omega of x * prod_{m != n} A_m[i_m, r]  (eq. 9). */
int oran_mttkrp(const oran_tensor *t, int mode, int R, const double *const *A, double *M);

/* Factors from SplitMix64(seed): A_0, ..., A_{N-1} in that order, row-major,
 * each output x mapped to (x >> 40) * 2^-24 (as the 3-way oracle). */
int oran_model_create(const oran_tensor *t, int R, uint64_t seed, oran_model **out);
void oran_model_destroy(oran_model *m);
int oran_model_get_factor(const oran_model *m, int mode, double *dst);
int oran_model_set_factor(oran_model *m, int mode, const double *src);
int oran_model_get_state(const oran_model *m, int mode, double *zprev, double *ti_prev, int64_t *k);
int oran_model_set_state(oran_model *m, int mode, const double *zprev, double ti_prev, int64_t k);

/* One sweep of mode n (Alg. 1 body; Gauss-Seidel reading as the 3-way oracle). */
int oran_sweep(oran_model *m, int mode);
/* Record of the last sweep of `mode` (any pointer may be NULL): M, z (I_n x R),
 * sel (uint8), H (R x R), scalars [L, ti, flip, ti_prev, f, nsel, <M, A_n>,
 * sum of the Hadamard product of all Grams]. */
int oran_sweep_info(const oran_model *m, int mode, double *M, double *z, uint8_t *sel, double *H,
                    double *scalars);
/* Tie band of the last sweep of `mode` (a diagnostic of the tests, as
 * ora_sweep_band): band (I_n x R), kind (0 decided, 1 exact zero, 2
 * zero-gradient tie, 3 margin tie), scalars [band of ti, global tie,
 * exact zeros, zero-gradient ties, margin ties].  set_state clears the band
 * of the Z^{k-1} it sets. */
int oran_sweep_band(const oran_model *m, int mode, double *band, uint8_t *kind, double *scalars);
/* Row q of the last sweep of `mode` updated (step 9) under the decisions
 * sel (R bytes) instead of the oracle's own: out (R doubles). */
int oran_row_outcome(const oran_model *m, int mode, int64_t q, const uint8_t *sel, double *out);
/* eq. 6 for the current factors: ||X||^2 - 2 <X, Xhat> + sum_rs (prod_m Gram_m)_rs. */
double oran_objective(const oran_model *m);

#ifdef __cplusplus
}
#endif
#endif
