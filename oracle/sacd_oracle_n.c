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
  double info[NMAX][6];
};

void oran_model_destroy(oran_model *m) {
  if (!m) return;
  for (int n = 0; n < m->t->N; ++n) {
    free(m->A[n]); free(m->G[n]); free(m->zprev[n]); free(m->M[n]);
    free(m->z[n]); free(m->H[n]); free(m->sel[n]);
  }
  free(m);
}

int oran_model_create(const oran_tensor *t, int R, uint64_t seed, oran_model **out) {
  if (!t || !out || R < 1 || R > 1024) return ORA_EINVAL;
  oran_model *m = (oran_model *)calloc(1, sizeof(oran_model));
  if (!m) return ORA_ENOMEM;
  m->t = t;
  m->R = R;
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
    if (!m->A[n] || !m->G[n] || !m->zprev[n] || !m->M[n] || !m->z[n] || !m->H[n] || !m->sel[n]) {
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
  if (zprev) memcpy(m->zprev[mode], zprev, (size_t)m->t->dims[mode] * m->R * sizeof(double));
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

/* The steps of ora_sweep (sacd_oracle.c) with N - 1 other factors. */
int oran_sweep(oran_model *m, int mode) {
  if (!m || mode < 0 || mode >= m->t->N) return ORA_EINVAL;
  const oran_tensor *t = m->t;
  const int N = t->N, R = m->R;
  const int64_t I = t->dims[mode];
  const size_t IR = (size_t)I * R;
  double *A = m->A[mode], *H = m->H[mode], *M = m->M[mode], *z = m->z[mode], *zprev = m->zprev[mode];
  uint8_t *sel = m->sel[mode];
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
  double *G0 = (double *)malloc((IR > 0 ? IR : 1) * sizeof(double));
  if (!G0) return ORA_ENOMEM;
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
  free(G0);
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
