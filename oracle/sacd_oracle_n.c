/*
 * sacd_oracle_n.c -- plain FP64 CPU oracle of SaCD for N-way tensors (see
 * sacd_oracle_n.h).  TEST INFRASTRUCTURE ONLY.
 *
 * The steps of ora_sweep (sacd_oracle.c) for N modes: the MTTKRP multiplies
 * the N - 1 other factors' rows (eq. 9 with the Khatri-Rao product of all the
 * other factors) and H is the Hadamard product of their N - 1 Gram matrices
 * (eq. 10); importance, selection and the Gauss-Seidel update are those of
 * the three-way sweep.
 */
#include "sacd_oracle_n.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ERANGE (-2)
#define ORA_ENOMEM (-3)
#define ORA_ENUMERIC (-6)
#define NMAX 8

struct oran_tensor {
  int N;
  int64_t dims[NMAX];
  int64_t nnz;
  int32_t *coords[NMAX]; /* mode-n sorted: nnz x N, (i_n, others in increasing mode order) */
  float *vals[NMAX];
  int64_t *ptr[NMAX];
  double norm2;
};

typedef struct {
  int32_t c[NMAX];
  int64_t pos;
  float v;
} oran_entry;

static int g_sort_n; /* key length of the comparison below */

static int cmp_entry(const void *pa, const void *pb) {
  const oran_entry *a = (const oran_entry *)pa, *b = (const oran_entry *)pb;
  for (int k = 0; k < g_sort_n; ++k) {
    if (a->c[k] < b->c[k]) return -1;
    if (a->c[k] > b->c[k]) return 1;
  }
  return (a->pos > b->pos) - (a->pos < b->pos);
}

void oran_tensor_destroy(oran_tensor *t) {
  if (!t) return;
  for (int n = 0; n < t->N; ++n) {
    free(t->coords[n]);
    free(t->vals[n]);
    free(t->ptr[n]);
  }
  free(t);
}

int oran_tensor_create(int N, const int64_t *dims, int64_t nnz, const int32_t *idx, const float *vals,
                       oran_tensor **out) {
  if (N < 2 || N > NMAX || !dims || !out || nnz < 0 || (nnz > 0 && (!idx || !vals))) return ORA_EINVAL;
  for (int n = 0; n < N; ++n)
    if (dims[n] < 1 || dims[n] > INT32_MAX) return ORA_EINVAL;
  for (int64_t p = 0; p < nnz; ++p) {
    for (int n = 0; n < N; ++n)
      if (idx[N * p + n] < 0 || idx[N * p + n] >= dims[n]) return ORA_ERANGE;
    if (!isfinite(vals[p])) return ORA_ENUMERIC;
  }
  oran_tensor *t = (oran_tensor *)calloc(1, sizeof(oran_tensor));
  if (!t) return ORA_ENOMEM;
  t->N = N;
  memcpy(t->dims, dims, (size_t)N * sizeof(int64_t));
  oran_entry *e = (oran_entry *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(oran_entry));
  if (!e) { oran_tensor_destroy(t); return ORA_ENOMEM; }
  for (int64_t p = 0; p < nnz; ++p) {
    for (int n = 0; n < N; ++n) e[p].c[n] = idx[N * p + n];
    e[p].pos = p;
    e[p].v = vals[p];
  }
  /* merge duplicates: sort by (i_0, ..., i_{N-1}, input position) */
  g_sort_n = N;
  qsort(e, (size_t)nnz, sizeof(oran_entry), cmp_entry);
  int64_t u = 0;
  for (int64_t p = 0; p < nnz; ++p) {
    if (u > 0 && memcmp(e[u - 1].c, e[p].c, (size_t)N * sizeof(int32_t)) == 0)
      e[u - 1].v = e[u - 1].v + e[p].v; /* FP32, input order */
    else
      e[u++] = e[p];
  }
  t->nnz = u;
  double n2 = 0.0;
  for (int64_t p = 0; p < u; ++p) n2 += (double)e[p].v * (double)e[p].v;
  t->norm2 = n2;
  for (int n = 0; n < N; ++n) {
    oran_entry *s = (oran_entry *)malloc((size_t)(u > 0 ? u : 1) * sizeof(oran_entry));
    t->coords[n] = (int32_t *)malloc((size_t)(u > 0 ? u : 1) * N * sizeof(int32_t));
    t->vals[n] = (float *)malloc((size_t)(u > 0 ? u : 1) * sizeof(float));
    t->ptr[n] = (int64_t *)calloc((size_t)dims[n] + 1, sizeof(int64_t));
    if (!s || !t->coords[n] || !t->vals[n] || !t->ptr[n]) {
      free(s); free(e); oran_tensor_destroy(t); return ORA_ENOMEM;
    }
    for (int64_t p = 0; p < u; ++p) {
      int k = 0;
      s[p].c[k++] = e[p].c[n];
      for (int m = 0; m < N; ++m)
        if (m != n) s[p].c[k++] = e[p].c[m];
      s[p].pos = p;
      s[p].v = e[p].v;
    }
    qsort(s, (size_t)u, sizeof(oran_entry), cmp_entry);
    for (int64_t p = 0; p < u; ++p) {
      for (int k = 0; k < N; ++k) t->coords[n][N * p + k] = s[p].c[k];
      t->vals[n][p] = s[p].v;
      t->ptr[n][s[p].c[0] + 1] += 1;
    }
    for (int64_t i = 0; i < dims[n]; ++i) t->ptr[n][i + 1] += t->ptr[n][i];
    free(s);
  }
  free(e);
  *out = t;
  return ORA_OK;
}

int64_t oran_tensor_nnz(const oran_tensor *t) { return t ? t->nnz : -1; }
double oran_tensor_norm2(const oran_tensor *t) { return t ? t->norm2 : -1.0; }

int oran_tensor_mode_coo(const oran_tensor *t, int mode, int32_t *coords, float *vals, int64_t *ptr) {
  if (!t || mode < 0 || mode >= t->N) return ORA_EINVAL;
  if (coords) memcpy(coords, t->coords[mode], (size_t)t->nnz * t->N * sizeof(int32_t));
  if (vals) memcpy(vals, t->vals[mode], (size_t)t->nnz * sizeof(float));
  if (ptr) memcpy(ptr, t->ptr[mode], (size_t)(t->dims[mode] + 1) * sizeof(int64_t));
  return ORA_OK;
}

/* eq. 9 for N modes: the product of the N - 1 other rows, entry by entry. */
int oran_mttkrp(const oran_tensor *t, int mode, int R, const double *const *A, double *M) {
  if (!t || mode < 0 || mode >= t->N || R < 1 || !A || !M) return ORA_EINVAL;
  const int N = t->N;
  int other[NMAX];
  for (int m = 0, k = 0; m < N; ++m)
    if (m != mode) other[k++] = m;
  memset(M, 0, (size_t)t->dims[mode] * R * sizeof(double));
  const int32_t *c = t->coords[mode];
  for (int64_t p = 0; p < t->nnz; ++p) {
    const int64_t in = c[N * p];
    const double x = (double)t->vals[mode][p];
    for (int r = 0; r < R; ++r) {
      double prod = x;
      for (int k = 0; k < N - 1; ++k) prod *= A[other[k]][(int64_t)c[N * p + 1 + k] * R + r];
      M[in * R + r] += prod;
    }
  }
  return ORA_OK;
}

static void gram(const double *A, int64_t I, int R, double *G) {
  for (int r = 0; r < R; ++r)
    for (int s = 0; s < R; ++s) {
      double acc = 0.0;
      for (int64_t q = 0; q < I; ++q) acc += A[q * R + r] * A[q * R + s];
      G[r * R + s] = acc;
    }
}

struct oran_model {
  const oran_tensor *t;
  int R;
  double *A[NMAX], *G[NMAX], *zprev[NMAX];
  double ti_prev[NMAX];
  int64_t k[NMAX];
  double *M[NMAX], *z[NMAX], *H[NMAX];
  uint8_t *sel[NMAX];
  double info[NMAX][8];
  /* diagnostics of the tests (no step of the method reads them): the factor
   * and Z^{k-1} the last sweep started from, its gradient G0, and the tie
   * band of its importances (as in the three-way oracle) */
  double *A_prev[NMAX], *G0[NMAX], *zprev_used[NMAX], *band[NMAX], *band_used[NMAX];
  uint8_t *kind[NMAX];
  double band_info[NMAX][5];
  double tau;
};

void oran_model_destroy(oran_model *m) {
  if (!m) return;
  for (int n = 0; n < m->t->N; ++n) {
    free(m->A[n]); free(m->G[n]); free(m->zprev[n]); free(m->M[n]);
    free(m->z[n]); free(m->H[n]); free(m->sel[n]);
    free(m->A_prev[n]); free(m->G0[n]); free(m->zprev_used[n]); free(m->band[n]);
    free(m->band_used[n]); free(m->kind[n]);
  }
  free(m);
}

int oran_model_create(const oran_tensor *t, int R, uint64_t seed, oran_model **out) {
  if (!t || !out || R < 1 || R > 1024) return ORA_EINVAL;
  oran_model *m = (oran_model *)calloc(1, sizeof(oran_model));
  if (!m) return ORA_ENOMEM;
  m->t = t;
  m->R = R;
  m->tau = 1e-6;
  uint64_t state = seed; /* SplitMix64 (Steele, Lea, Flood 2014), outputs in factor order */
  for (int n = 0; n < t->N; ++n) {
    const size_t IR = (size_t)t->dims[n] * R;
    m->A[n] = (double *)malloc(IR * sizeof(double));
    m->G[n] = (double *)malloc((size_t)R * R * sizeof(double));
    m->zprev[n] = (double *)calloc(IR, sizeof(double));
    m->M[n] = (double *)calloc(IR, sizeof(double));
    m->z[n] = (double *)calloc(IR, sizeof(double));
    m->H[n] = (double *)calloc((size_t)R * R, sizeof(double));
    m->sel[n] = (uint8_t *)calloc(IR, 1);
    m->A_prev[n] = (double *)calloc(IR > 0 ? IR : 1, sizeof(double));
    m->G0[n] = (double *)calloc(IR > 0 ? IR : 1, sizeof(double));
    m->zprev_used[n] = (double *)calloc(IR > 0 ? IR : 1, sizeof(double));
    m->band[n] = (double *)calloc(IR > 0 ? IR : 1, sizeof(double));
    m->band_used[n] = (double *)calloc(IR > 0 ? IR : 1, sizeof(double));
    m->kind[n] = (uint8_t *)calloc(IR > 0 ? IR : 1, 1);
    if (!m->A[n] || !m->G[n] || !m->zprev[n] || !m->M[n] || !m->z[n] || !m->H[n] || !m->sel[n] ||
        !m->A_prev[n] || !m->G0[n] || !m->zprev_used[n] || !m->band[n] || !m->band_used[n] || !m->kind[n]) {
      oran_model_destroy(m);
      return ORA_ENOMEM;
    }
    for (size_t i = 0; i < IR; ++i) {
      state += 0x9E3779B97F4A7C15ULL;
      uint64_t z = state;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
      z ^= z >> 31;
      m->A[n][i] = (double)(z >> 40) * (1.0 / 16777216.0);
    }
    gram(m->A[n], t->dims[n], R, m->G[n]);
  }
  *out = m;
  return ORA_OK;
}

int oran_model_get_factor(const oran_model *m, int mode, double *dst) {
  if (!m || mode < 0 || mode >= m->t->N || !dst) return ORA_EINVAL;
  memcpy(dst, m->A[mode], (size_t)m->t->dims[mode] * m->R * sizeof(double));
  return ORA_OK;
}

int oran_model_set_factor(oran_model *m, int mode, const double *src) {
  if (!m || mode < 0 || mode >= m->t->N || !src) return ORA_EINVAL;
  memcpy(m->A[mode], src, (size_t)m->t->dims[mode] * m->R * sizeof(double));
  gram(m->A[mode], m->t->dims[mode], m->R, m->G[mode]);
  return ORA_OK;
}

int oran_model_get_state(const oran_model *m, int mode, double *zprev, double *ti_prev, int64_t *k) {
  if (!m || mode < 0 || mode >= m->t->N) return ORA_EINVAL;
  if (zprev) memcpy(zprev, m->zprev[mode], (size_t)m->t->dims[mode] * m->R * sizeof(double));
  if (ti_prev) *ti_prev = m->ti_prev[mode];
  if (k) *k = m->k[mode];
  return ORA_OK;
}

int oran_model_set_state(oran_model *m, int mode, const double *zprev, double ti_prev, int64_t k) {
  if (!m || mode < 0 || mode >= m->t->N || k < 0) return ORA_EINVAL;
  const size_t IR = (size_t)m->t->dims[mode] * m->R;
  if (zprev) memcpy(m->zprev[mode], zprev, IR * sizeof(double));
  memset(m->band[mode], 0, IR * sizeof(double)); /* a Z^{k-1} from outside carries no band */
  m->ti_prev[mode] = ti_prev;
  m->k[mode] = k;
  return ORA_OK;
}

double oran_objective(const oran_model *m) {
  const oran_tensor *t = m->t;
  const int N = t->N, R = m->R;
  double inner = 0.0;
  for (int64_t p = 0; p < t->nnz; ++p) {
    /* mode-0 sorted copy: (i_0, i_1, ..., i_{N-1}) */
    const int32_t *c = &t->coords[0][N * p];
    double xhat = 0.0;
    for (int r = 0; r < R; ++r) {
      double prod = 1.0;
      for (int n = 0; n < N; ++n) prod *= m->A[n][(int64_t)c[n] * R + r];
      xhat += prod;
    }
    inner += (double)t->vals[0][p] * xhat;
  }
  double model = 0.0;
  for (int i = 0; i < R * R; ++i) {
    double prod = 1.0;
    for (int n = 0; n < N; ++n) prod *= m->G[n][i];
    model += prod;
  }
  return t->norm2 - 2.0 * inner + model;
}

static double cd_step(double a, double g, double h) {
  /* eq. 11-12: Newton step of one variable, clipped at zero; 0 where h = 0 */
  if (!(h > 0.0)) return 0.0;
  const double u = a - g / h;
  return (u > 0.0 ? u : 0.0) - a;
}

/* Tie band of the last sweep of `mode`, as the three-way oracle records it
 * (a diagnostic of the tests): the change of z (eq. 20) that a relative
 * error tau in the terms of its gradient causes, to first order (|dz/dg| T)
 * plus, for an interior or zero-gradient element, the second-order term
 * (tau T / h)^2 (h + L/2); the element's kind from the margin of its
 * selection (z, or z - Z^{k-1}) against that band plus the band of Z^{k-1}. */
static void record_tie_band(oran_model *m, int mode) {
  const int R = m->R;
  const int64_t I = m->t->dims[mode];
  const size_t IR = (size_t)I * R;
  const double tau = m->tau, L = m->info[mode][0];
  const int64_t k = m->k[mode];
  const double *A = m->A_prev[mode], *H = m->H[mode], *M = m->M[mode], *G0 = m->G0[mode];
  const double *z = m->z[mode], *zp = m->zprev_used[mode];
  double *band = m->band[mode], *band_used = m->band_used[mode];
  uint8_t *kind = m->kind[mode];
  memcpy(band_used, band, IR * sizeof(double));
  double sum_band = 0.0, sum_used = 0.0;
  int64_t n_zero = 0, n_grad = 0, n_margin = 0;
  for (int64_t q = 0; q < I; ++q)
    for (int r = 0; r < R; ++r) {
      const int64_t e = q * R + r;
      const double h = H[r * R + r];
      double T = fabs(M[e]);
      for (int s = 0; s < R; ++s) T += fabs(A[q * R + s] * H[s * R + r]);
      const double d = cd_step(A[e], G0[e], h);
      const int interior = h > 0.0 && A[e] - G0[e] / h > 0.0;
      const double dzdg = fabs(d) + (interior ? (fabs(G0[e]) + L * fabs(d)) / h : 0.0);
      double bz = tau * (dzdg * T + 0.5 * L * d * d);
      const int zero_grad = A[e] == 0.0 && h > 0.0 && T > 0.0 && fabs(G0[e]) <= tau * T;
      if (interior || zero_grad) {
        const double dd = tau * T / h;
        bz += dd * dd * (h + 0.5 * L);
      }
      band[e] = bz;
      const double margin = (k <= 1) ? z[e] : z[e] - zp[e];
      const double width = (k <= 1) ? bz : bz + band_used[e];
      if (zero_grad) {
        kind[e] = 2;
        ++n_grad;
      } else if (width > 0.0 && fabs(margin) <= width) {
        kind[e] = 3;
        ++n_margin;
      } else if (margin == 0.0) {
        kind[e] = 1;
        ++n_zero;
      } else {
        kind[e] = 0;
      }
      sum_band += bz;
      sum_used += band_used[e];
    }
  const double band_ti = sum_band + sum_used;
  m->band_info[mode][0] = band_ti;
  m->band_info[mode][1] = (k >= 2 && fabs(m->info[mode][1] - m->info[mode][3]) <= band_ti) ? 1.0 : 0.0;
  m->band_info[mode][2] = (double)n_zero;
  m->band_info[mode][3] = (double)n_grad;
  m->band_info[mode][4] = (double)n_margin;
}

int oran_sweep_band(const oran_model *m, int mode, double *band, uint8_t *kind, double *scalars) {
  if (!m || mode < 0 || mode >= m->t->N) return ORA_EINVAL;
  const size_t IR = (size_t)m->t->dims[mode] * m->R;
  if (band) memcpy(band, m->band[mode], IR * sizeof(double));
  if (kind) memcpy(kind, m->kind[mode], IR);
  if (scalars) memcpy(scalars, m->band_info[mode], sizeof(m->band_info[mode]));
  return ORA_OK;
}

int oran_row_outcome(const oran_model *m, int mode, int64_t q, const uint8_t *sel, double *out) {
  if (!m || mode < 0 || mode >= m->t->N || !sel || !out) return ORA_EINVAL;
  const int R = m->R;
  if (q < 0 || q >= m->t->dims[mode]) return ORA_ERANGE;
  const double *H = m->H[mode], *Mq = m->M[mode] + q * R;
  memcpy(out, m->A_prev[mode] + q * R, (size_t)R * sizeof(double));
  for (int r = 0; r < R; ++r) {
    const double h = H[r * R + r];
    if (!sel[r] || !(h > 0.0)) continue;
    double g = -Mq[r];
    for (int s = 0; s < R; ++s) g += out[s] * H[s * R + r];
    const double u = out[r] - g / h;
    out[r] = u > 0.0 ? u : 0.0;
  }
  return ORA_OK;
}

/* The steps of ora_sweep (sacd_oracle.c) with N - 1 other factors. */
int oran_sweep(oran_model *m, int mode) {
  if (!m || mode < 0 || mode >= m->t->N) return ORA_EINVAL;
  const oran_tensor *t = m->t;
  const int N = t->N, R = m->R;
  const int64_t I = t->dims[mode];
  const size_t IR = (size_t)I * R;
  double *A = m->A[mode], *H = m->H[mode], *M = m->M[mode], *z = m->z[mode], *zprev = m->zprev[mode];
  uint8_t *sel = m->sel[mode];
  memcpy(m->A_prev[mode], A, IR * sizeof(double));
  memcpy(m->zprev_used[mode], zprev, IR * sizeof(double));
  /* 1 */
  m->k[mode] += 1;
  const int64_t k = m->k[mode];
  /* 2: H = Hadamard product of the other modes' Grams (eq. 10), L = ||H||_F */
  double L2 = 0.0;
  for (int i = 0; i < R * R; ++i) {
    double h = 1.0;
    for (int n = 0; n < N; ++n)
      if (n != mode) h *= m->G[n][i];
    H[i] = h;
    L2 += h * h;
  }
  const double L = sqrt(L2);
  /* 3 */
  oran_mttkrp(t, mode, R, (const double *const *)m->A, M);
  /* 4, 5: G0 = -M + A H, step, importance */
  double *G0 = m->G0[mode];
  for (int64_t q = 0; q < I; ++q)
    for (int r = 0; r < R; ++r) {
      double ah = 0.0;
      for (int s = 0; s < R; ++s) ah += A[q * R + s] * H[s * R + r];
      const int64_t e = q * R + r;
      G0[e] = -M[e] + ah;
      const double h = H[r * R + r];
      double d = 0.0;
      if (h > 0.0) {
        const double u = A[e] - G0[e] / h;
        d = (u > 0.0 ? u : 0.0) - A[e];
      }
      z[e] = -(G0[e] * d) - 0.5 * L * d * d;
    }
  /* 6 */
  double ti = 0.0;
  for (size_t e = 0; e < IR; ++e) ti += z[e];
  /* 7 */
  const int flip = k >= 2 && ti > m->ti_prev[mode];
  int64_t nsel = 0;
  for (size_t e = 0; e < IR; ++e) {
    const double sp = k <= 1 ? z[e] : (flip ? zprev[e] - z[e] : z[e] - zprev[e]);
    sel[e] = sp > 0.0;
    nsel += sel[e];
  }
  /* 8 */
  const double ti_used = m->ti_prev[mode];
  memcpy(zprev, z, IR * sizeof(double));
  m->ti_prev[mode] = ti;
  /* 9: Gauss-Seidel within each row */
  for (int64_t q = 0; q < I; ++q) {
    double *a = A + q * R;
    for (int r = 0; r < R; ++r) {
      const double h = H[r * R + r];
      if (!sel[q * R + r] || !(h > 0.0)) continue;
      double g = -M[q * R + r];
      for (int s = 0; s < R; ++s) g += a[s] * H[s * R + r];
      const double u = a[r] - g / h;
      a[r] = u > 0.0 ? u : 0.0;
    }
  }
  /* 10, 11 */
  gram(A, I, R, m->G[mode]);
  double inner = 0.0;
  for (size_t e = 0; e < IR; ++e) inner += M[e] * A[e];
  double model = 0.0;
  for (int i = 0; i < R * R; ++i) {
    double prod = 1.0;
    for (int n = 0; n < N; ++n) prod *= m->G[n][i];
    model += prod;
  }
  m->info[mode][0] = L;
  m->info[mode][1] = ti;
  m->info[mode][2] = flip;
  m->info[mode][3] = ti_used;
  m->info[mode][4] = t->norm2 - 2.0 * inner + model;
  m->info[mode][5] = (double)nsel;
  m->info[mode][6] = inner;
  m->info[mode][7] = model;
  record_tie_band(m, mode);
  return ORA_OK;
}

int oran_sweep_info(const oran_model *m, int mode, double *M, double *z, uint8_t *sel, double *H,
                    double *scalars) {
  if (!m || mode < 0 || mode >= m->t->N) return ORA_EINVAL;
  const size_t IR = (size_t)m->t->dims[mode] * m->R;
  if (M) memcpy(M, m->M[mode], IR * sizeof(double));
  if (z) memcpy(z, m->z[mode], IR * sizeof(double));
  if (sel) memcpy(sel, m->sel[mode], IR);
  if (H) memcpy(H, m->H[mode], (size_t)m->R * m->R * sizeof(double));
  if (scalars) memcpy(scalars, m->info[mode], sizeof(m->info[mode]));
  return ORA_OK;
}
