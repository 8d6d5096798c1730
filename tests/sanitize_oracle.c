/* Driver of the oracle's C code for a sanitizer build (AddressSanitizer and
 * UndefinedBehaviorSanitizer): every entry point of the three-way and N-way
 * oracles on small seeded tensors, including duplicate coordinates, empty
 * slices, the Jacobi rule, the column form, the tie band, undo, row outcomes
 * and the accuracy measures.  Exits non-zero on any error status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/sacd_oracle.h"
#include "../oracle/sacd_oracle_n.h"

#define CHECK(expr)                                                    \
  do {                                                                 \
    int rc_ = (expr);                                                  \
    if (rc_ != 0) {                                                    \
      fprintf(stderr, "%s:%d: %s returned %d\n", __FILE__, __LINE__, #expr, rc_); \
      exit(1);                                                         \
    }                                                                  \
  } while (0)

static uint64_t lcg = 12345;
static uint32_t next_u32(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(lcg >> 33);
}

static void three_way(int update_rule, int columns) {
  const int64_t dims[3] = {7, 5, 9};
  const int64_t nnz = 120;  /* with repeats: merged by the oracle */
  int32_t *idx = malloc(sizeof(int32_t) * 3 * nnz);
  float *vals = malloc(sizeof(float) * nnz);
  for (int64_t e = 0; e < nnz; ++e) {
    idx[3 * e + 0] = (int32_t)(next_u32() % 6); /* slice 6 of mode 0 stays empty */
    idx[3 * e + 1] = (int32_t)(next_u32() % dims[1]);
    idx[3 * e + 2] = (int32_t)(next_u32() % dims[2]);
    vals[e] = 1.0f + (float)(next_u32() % 5);
  }
  ora_tensor *t = NULL;
  CHECK(ora_tensor_create(dims, nnz, idx, vals, &t));
  const int64_t u = ora_tensor_nnz(t);
  const int R = 4;
  for (int n = 0; n < 3; ++n) {
    int32_t *coords = malloc(sizeof(int32_t) * 3 * u);
    float *v = malloc(sizeof(float) * u);
    int64_t *ptr = malloc(sizeof(int64_t) * (dims[n] + 1));
    CHECK(ora_tensor_mode_coo(t, n, coords, v, ptr));
    free(coords);
    free(v);
    free(ptr);
  }
  ora_model *m = NULL;
  CHECK(ora_model_create(t, R, 7, update_rule, &m));
  if (columns) CHECK(ora_model_set_columns(m, 2));
  double *A[3], *M = malloc(sizeof(double) * 9 * R), *col = malloc(sizeof(double) * 9);
  for (int n = 0; n < 3; ++n) {
    A[n] = malloc(sizeof(double) * dims[n] * R);
    CHECK(ora_model_get_factor(m, n, A[n]));
  }
  for (int n = 0; n < 3; ++n) {
    CHECK(ora_mttkrp(t, n, R, A[0], A[1], A[2], M));
    for (int r = 0; r < R; ++r) CHECK(ora_sttvp(t, n, R, r, A[0], A[1], A[2], col));
  }
  for (int it = 0; it < 4; ++it)
    for (int n = 0; n < 3; ++n) {
      CHECK(ora_sweep(m, n));
      const int64_t I = dims[n];
      double *G0 = malloc(sizeof(double) * I * R), *z = malloc(sizeof(double) * I * R);
      double *Mi = malloc(sizeof(double) * I * R), *H = malloc(sizeof(double) * R * R);
      double *band = malloc(sizeof(double) * I * R), sc[8], bs[5], row[4];
      uint8_t *sel = malloc(I * R), *kind = malloc(I * R);
      CHECK(ora_sweep_info(m, n, Mi, G0, z, sel, H, sc));
      CHECK(ora_sweep_band(m, n, band, kind, bs));
      for (int64_t q = 0; q < I; ++q) CHECK(ora_row_outcome(m, n, q, sel + q * R, row));
      if (it == 2) {
        double *zp = malloc(sizeof(double) * I * R), tp;
        int64_t k;
        CHECK(ora_sweep_undo(m, n));
        CHECK(ora_model_get_state(m, n, zp, &tp, &k));
        CHECK(ora_model_set_state(m, n, zp, tp, k));
        CHECK(ora_sweep(m, n));
        free(zp);
      }
      free(G0);
      free(z);
      free(Mi);
      free(H);
      free(band);
      free(sel);
      free(kind);
    }
  double fit, f, rmse, pd;
  CHECK(ora_fit(m, &fit, &f));
  (void)ora_objective(m);
  CHECK(ora_rmse(m, nnz, idx, vals, &rmse));
  CHECK(ora_pd(m, 2, &pd));
  int iters;
  double trace[20];
  CHECK(ora_run_until(m, 1e-4, 20, &iters, &fit, trace));
  ora_model_force_flip(m, 1);
  CHECK(ora_sweep(m, 0));
  for (int n = 0; n < 3; ++n) free(A[n]);
  free(M);
  free(col);
  ora_model_destroy(m);
  ora_tensor_destroy(t);
  free(idx);
  free(vals);
}

static void n_way(void) {
  const int N = 4;
  const int64_t dims[4] = {5, 4, 6, 3};
  const int64_t nnz = 90;
  int32_t *idx = malloc(sizeof(int32_t) * N * nnz);
  float *vals = malloc(sizeof(float) * nnz);
  for (int64_t e = 0; e < nnz; ++e) {
    for (int k = 0; k < N; ++k) idx[N * e + k] = (int32_t)(next_u32() % dims[k]);
    vals[e] = 1.0f + (float)(next_u32() % 5);
  }
  oran_tensor *t = NULL;
  CHECK(oran_tensor_create(N, dims, nnz, idx, vals, &t));
  const int64_t u = oran_tensor_nnz(t);
  const int R = 3;
  oran_model *m = NULL;
  CHECK(oran_model_create(t, R, 11, &m));
  double *A[4];
  for (int n = 0; n < N; ++n) {
    A[n] = malloc(sizeof(double) * dims[n] * R);
    CHECK(oran_model_get_factor(m, n, A[n]));
  }
  for (int n = 0; n < N; ++n) {
    double *M = malloc(sizeof(double) * dims[n] * R);
    int32_t *coords = malloc(sizeof(int32_t) * N * u);
    float *v = malloc(sizeof(float) * u);
    int64_t *ptr = malloc(sizeof(int64_t) * (dims[n] + 1));
    CHECK(oran_mttkrp(t, n, R, (const double *const *)A, M));
    CHECK(oran_tensor_mode_coo(t, n, coords, v, ptr));
    free(M);
    free(coords);
    free(v);
    free(ptr);
  }
  for (int it = 0; it < 3; ++it)
    for (int n = 0; n < N; ++n) {
      CHECK(oran_sweep(m, n));
      const int64_t I = dims[n];
      double *Mi = malloc(sizeof(double) * I * R), *z = malloc(sizeof(double) * I * R);
      double *H = malloc(sizeof(double) * R * R), *band = malloc(sizeof(double) * I * R);
      double sc[16], bs[5], row[3];
      uint8_t *sel = malloc(I * R), *kind = malloc(I * R);
      CHECK(oran_sweep_info(m, n, Mi, z, sel, H, sc));
      CHECK(oran_sweep_band(m, n, band, kind, bs));
      for (int64_t q = 0; q < I; ++q) CHECK(oran_row_outcome(m, n, q, sel + q * R, row));
      free(Mi);
      free(z);
      free(H);
      free(band);
      free(sel);
      free(kind);
    }
  (void)oran_objective(m);
  for (int n = 0; n < N; ++n) free(A[n]);
  oran_model_destroy(m);
  oran_tensor_destroy(t);
  free(idx);
  free(vals);
}

int main(void) {
  three_way(ORA_UPDATE_GS, 0);
  three_way(ORA_UPDATE_JACOBI, 0);
  three_way(ORA_UPDATE_GS, 1);
  n_way();
  printf("sanitized oracle run ok\n");
  return 0;
}
