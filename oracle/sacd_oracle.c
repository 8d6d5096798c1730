/*
 * sacd_oracle.c -- plain FP64 CPU oracle of SaCD (see sacd_oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  Nothing in the GPU library links it.
 *
 * Written to be read against the paper, not to be fast: plain loops, FP64
 * arithmetic, the steps of Algorithm 1 in the paper's order.  Readings of the
 * paper where its text is ambiguous are marked "Reading:".
 *
 * Loops whose iterations are independent (rows, slices, Gram entries) carry an
 * OpenMP "parallel for" so that the oracle can also be timed on all host
 * cores.  No loop that adds across iterations is parallelised: every sum is
 * formed in the same order for any thread count, so results are bit-identical
 * with 1 or many threads.
 */
#include "sacd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ERANGE (-2)
#define ORA_ENOMEM (-3)
#define ORA_ESTATE (-4)
#define ORA_ENUMERIC (-6)

/* ------------------------------------------------------------------------ */
/* Tensor: the observed set Omega with its per-mode slices (Sec. 3).         */
/* ------------------------------------------------------------------------ */

struct ora_tensor {
  int64_t dims[3];
  int64_t nnz;
  /* mode-n sorted copy: coords[n] is nnz x 3 holding (i_n, i_a, i_b) */
  int32_t *coords[3];
  float *vals[3];
  int64_t *ptr[3];
  double norm2; /* ||X||^2 over the stored (merged) values */
};

typedef struct {
  int32_t c[3]; /* key in comparison order */
  int64_t pos;  /* input position, makes the order total (stable) */
  float v;
} ora_entry;

static int cmp_entry(const void *pa, const void *pb) {
  const ora_entry *a = (const ora_entry *)pa, *b = (const ora_entry *)pb;
  for (int k = 0; k < 3; ++k) {
    if (a->c[k] < b->c[k]) return -1;
    if (a->c[k] > b->c[k]) return 1;
  }
  if (a->pos < b->pos) return -1;
  if (a->pos > b->pos) return 1;
  return 0;
}

/* The two other modes of `mode`, in increasing order. */
static void other_modes(int mode, int *a, int *b) {
  if (mode == 0) { *a = 1; *b = 2; }
  else if (mode == 1) { *a = 0; *b = 2; }
  else { *a = 0; *b = 1; }
}

void ora_tensor_destroy(ora_tensor *t) {
  if (!t) return;
  for (int n = 0; n < 3; ++n) {
    free(t->coords[n]);
    free(t->vals[n]);
    free(t->ptr[n]);
  }
  free(t);
}

int ora_tensor_create(const int64_t dims[3], int64_t nnz, const int32_t *idx,
                      const float *vals, ora_tensor **out) {
  if (!dims || !out || nnz < 0 || (nnz > 0 && (!idx || !vals))) return ORA_EINVAL;
  for (int n = 0; n < 3; ++n)
    if (dims[n] < 1 || dims[n] > INT32_MAX) return ORA_EINVAL;
  for (int64_t p = 0; p < nnz; ++p) {
    for (int n = 0; n < 3; ++n)
      if (idx[3 * p + n] < 0 || idx[3 * p + n] >= dims[n]) return ORA_ERANGE;
    if (!isfinite(vals[p])) return ORA_ENUMERIC;
  }
  ora_tensor *t = (ora_tensor *)calloc(1, sizeof(ora_tensor));
  if (!t) return ORA_ENOMEM;
  memcpy(t->dims, dims, sizeof(t->dims));

  /* Merge duplicate coordinates: sort by (i0, i1, i2, input position) and add
   * the values of equal coordinates in FP32, in input order. */
  ora_entry *e = (ora_entry *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(ora_entry));
  if (!e) { ora_tensor_destroy(t); return ORA_ENOMEM; }
  for (int64_t p = 0; p < nnz; ++p) {
    e[p].c[0] = idx[3 * p + 0];
    e[p].c[1] = idx[3 * p + 1];
    e[p].c[2] = idx[3 * p + 2];
    e[p].pos = p;
    e[p].v = vals[p];
  }
  qsort(e, (size_t)nnz, sizeof(ora_entry), cmp_entry);
  int64_t u = 0;
  for (int64_t p = 0; p < nnz; ++p) {
    if (u > 0 && e[u - 1].c[0] == e[p].c[0] && e[u - 1].c[1] == e[p].c[1] &&
        e[u - 1].c[2] == e[p].c[2]) {
      e[u - 1].v = e[u - 1].v + e[p].v; /* FP32 addition, input order */
    } else {
      e[u++] = e[p];
    }
  }
  t->nnz = u;
  double n2 = 0.0;
  for (int64_t p = 0; p < u; ++p) n2 += (double)e[p].v * (double)e[p].v;
  t->norm2 = n2;

  /* Per-mode copies sorted by (i_n, i_a, i_b), a < b, with slice pointers. */
  for (int n = 0; n < 3; ++n) {
    int a, b;
    other_modes(n, &a, &b);
    ora_entry *s = (ora_entry *)malloc((size_t)(u > 0 ? u : 1) * sizeof(ora_entry));
    t->coords[n] = (int32_t *)malloc((size_t)(u > 0 ? u : 1) * 3 * sizeof(int32_t));
    t->vals[n] = (float *)malloc((size_t)(u > 0 ? u : 1) * sizeof(float));
    t->ptr[n] = (int64_t *)calloc((size_t)dims[n] + 1, sizeof(int64_t));
    if (!s || !t->coords[n] || !t->vals[n] || !t->ptr[n]) {
      free(s); free(e); ora_tensor_destroy(t); return ORA_ENOMEM;
    }
    for (int64_t p = 0; p < u; ++p) {
      /* e[] holds (i0, i1, i2); reorder to (i_n, i_a, i_b) */
      int32_t full[3] = {e[p].c[0], e[p].c[1], e[p].c[2]};
      s[p].c[0] = full[n];
      s[p].c[1] = full[a];
      s[p].c[2] = full[b];
      s[p].pos = p;
      s[p].v = e[p].v;
    }
    qsort(s, (size_t)u, sizeof(ora_entry), cmp_entry);
    for (int64_t p = 0; p < u; ++p) {
      t->coords[n][3 * p + 0] = s[p].c[0];
      t->coords[n][3 * p + 1] = s[p].c[1];
      t->coords[n][3 * p + 2] = s[p].c[2];
      t->vals[n][p] = s[p].v;
      t->ptr[n][s[p].c[0] + 1] += 1; /* count slice sizes */
    }
    for (int64_t i = 0; i < dims[n]; ++i) t->ptr[n][i + 1] += t->ptr[n][i];
    free(s);
  }
  free(e);
  *out = t;
  return ORA_OK;
}

int64_t ora_tensor_nnz(const ora_tensor *t) { return t ? t->nnz : -1; }
double ora_tensor_norm2(const ora_tensor *t) { return t ? t->norm2 : -1.0; }

int ora_tensor_mode_coo(const ora_tensor *t, int mode, int32_t *coords,
                        float *vals, int64_t *ptr) {
  if (!t || mode < 0 || mode > 2) return ORA_EINVAL;
  if (coords) memcpy(coords, t->coords[mode], (size_t)t->nnz * 3 * sizeof(int32_t));
  if (vals) memcpy(vals, t->vals[mode], (size_t)t->nnz * sizeof(float));
  if (ptr) memcpy(ptr, t->ptr[mode], (size_t)(t->dims[mode] + 1) * sizeof(int64_t));
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* MTTKRP: the first term of the gradient, eq. 9, in the sparse column form  */
/* of Sec. 4.4 (m_r = sum over the slice of x * (product of the other two    */
/* factors' r-th entries)).  Loops over Omega; no Khatri-Rao product is      */
/* formed.                                                                   */
/* ------------------------------------------------------------------------ */
int ora_mttkrp(const ora_tensor *t, int mode, int R, const double *A0,
               const double *A1, const double *A2, double *M) {
  if (!t || mode < 0 || mode > 2 || R < 1 || !M) return ORA_EINVAL;
  const double *F[3] = {A0, A1, A2};
  int a, b;
  other_modes(mode, &a, &b);
  if (!F[a] || !F[b]) return ORA_EINVAL;
  memset(M, 0, (size_t)t->dims[mode] * (size_t)R * sizeof(double));
  const int32_t *c = t->coords[mode];
  const float *v = t->vals[mode];
  const int64_t *ptr = t->ptr[mode];
  /* slice by slice (row i_n of M only receives its slice's entries, which
   * are added in their sorted order) */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < t->dims[mode]; ++i) {
    for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
      const int64_t ia = c[3 * p + 1], ib = c[3 * p + 2];
      const double x = (double)v[p];
      for (int r = 0; r < R; ++r)
        M[i * R + r] += x * F[a][ia * R + r] * F[b][ib * R + r];
    }
  }
  return ORA_OK;
}

/* Column r of the MTTKRP (Sec. 4.4): one pass over the slices with column r
 * of the two other factors only. */
int ora_sttvp(const ora_tensor *t, int mode, int R, int r, const double *A0, const double *A1,
              const double *A2, double *m) {
  if (!t || mode < 0 || mode > 2 || R < 1 || r < 0 || r >= R || !m) return ORA_EINVAL;
  const double *F[3] = {A0, A1, A2};
  int a, b;
  other_modes(mode, &a, &b);
  if (!F[a] || !F[b]) return ORA_EINVAL;
  const int32_t *c = t->coords[mode];
  const float *v = t->vals[mode];
  const int64_t *ptr = t->ptr[mode];
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < t->dims[mode]; ++i) {
    double s = 0.0;
    for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
      s += (double)v[p] * F[a][(int64_t)c[3 * p + 1] * R + r] * F[b][(int64_t)c[3 * p + 2] * R + r];
    m[i] = s;
  }
  return ORA_OK;
}

/* Gram matrix A^T A (R x R). */
static void gram(const double *A, int64_t I, int R, double *G) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int r = 0; r < R; ++r)
    for (int s = 0; s < R; ++s) {
      double acc = 0.0;
      for (int64_t q = 0; q < I; ++q) acc += A[q * R + r] * A[q * R + s];
      G[r * R + s] = acc;
    }
}

int ora_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Random initialisation (Alg. 1 input "randomly initialised factors").      */
/* ------------------------------------------------------------------------ */
void ora_splitmix64(uint64_t seed, int64_t count, uint64_t *out) {
  uint64_t state = seed;
  for (int64_t i = 0; i < count; ++i) {
    state += 0x9E3779B97F4A7C15ULL;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    out[i] = z ^ (z >> 31);
  }
}

/* ------------------------------------------------------------------------ */
/* One-coordinate pieces.                                                    */
/* ------------------------------------------------------------------------ */

/* eq. 11 gives the Newton step g/h; eq. 12 projects it so the updated value
 * stays nonnegative; the returned step is the change applied by eq. 13.
 * Reading: a dead column (h = 0) has g = 0 and no defined step; it is 0. */
double ora_cd_delta(double a, double g, double h) {
  if (!(h > 0.0)) return 0.0;
  double u = a - g / h;
  return (u > 0.0 ? u : 0.0) - a;
}

/* eq. 20: Lipschitz element importance, with the step of eq. 12. */
double ora_importance(double g, double delta, double L) {
  return -(g * delta) - 0.5 * L * delta * delta;
}


/* Alg. 1 selection.  First sweep: update iff z > 0.  Later sweeps: the
 * saturation point is z - zprev (eq. 24), or zprev - z when the total
 * importance grew (eq. 27); update iff it is > 0.  Comparisons are strict. */
int ora_select(int64_t k, double z, double zprev, int flip) {
  if (k <= 1) return z > 0.0;
  const double sp = flip ? (zprev - z) : (z - zprev);
  return sp > 0.0;
}

/* ------------------------------------------------------------------------ */
/* Model and the SaCD sweep (Algorithm 1).                                   */
/* ------------------------------------------------------------------------ */

struct ora_model {
  const ora_tensor *t;
  int R;
  int update_rule;
  int cb; /* column-at-a-time form: columns per block (0: row form) */
  int force_flip;
  double tau;
  /* state of Alg. 1 */
  double *A[3];
  double *G[3];      /* Gram matrices A_n^T A_n */
  double *zprev[3];  /* Z^{k-1} */
  double ti_prev[3]; /* ti^{k-1} */
  int64_t k[3];
  /* record of the last sweep of each mode (for the tests) */
  double *M[3], *G0[3], *z[3];
  uint8_t *sel[3];
  double *H[3];
  double info[3][8];
  double *A_prev[3];     /* factor before the sweep */
  double *zprev_used[3]; /* Z^{k-1} the selection compared with */
  int undo_ok[3];        /* the record above holds the state before the last sweep */
  /* tie band (diagnostics, see ora_sweep_band) */
  double *band[3];       /* band of z of the last sweep */
  double *band_used[3];  /* band of the Z^{k-1} that sweep compared with */
  uint8_t *kind[3];
  double band_info[3][5];
};

void ora_model_destroy(ora_model *m) {
  if (!m) return;
  for (int n = 0; n < 3; ++n) {
    free(m->A[n]); free(m->G[n]); free(m->zprev[n]);
    free(m->M[n]); free(m->G0[n]); free(m->z[n]);
    free(m->sel[n]); free(m->H[n]); free(m->A_prev[n]);
    free(m->zprev_used[n]); free(m->band[n]); free(m->band_used[n]);
    free(m->kind[n]);
  }
  free(m);
}

int ora_model_create(const ora_tensor *t, int R, uint64_t seed, int update_rule,
                     ora_model **out) {
  if (!t || !out || R < 1 || R > 1024) return ORA_EINVAL;
  if (update_rule != ORA_UPDATE_GS && update_rule != ORA_UPDATE_JACOBI) return ORA_EINVAL;
  ora_model *m = (ora_model *)calloc(1, sizeof(ora_model));
  if (!m) return ORA_ENOMEM;
  m->t = t;
  m->R = R;
  m->update_rule = update_rule;
  m->force_flip = -1;
  m->tau = 1e-6;
  int64_t total = 0;
  for (int n = 0; n < 3; ++n) total += t->dims[n] * R;
  uint64_t *raw = (uint64_t *)malloc((size_t)total * sizeof(uint64_t));
  if (!raw) { ora_model_destroy(m); return ORA_ENOMEM; }
  ora_splitmix64(seed, total, raw);
  int64_t off = 0;
  for (int n = 0; n < 3; ++n) {
    const size_t IR = (size_t)t->dims[n] * (size_t)R;
    m->A[n] = (double *)malloc(IR * sizeof(double));
    m->G[n] = (double *)malloc((size_t)R * R * sizeof(double));
    m->zprev[n] = (double *)calloc(IR, sizeof(double));
    m->M[n] = (double *)calloc(IR, sizeof(double));
    m->G0[n] = (double *)calloc(IR, sizeof(double));
    m->z[n] = (double *)calloc(IR, sizeof(double));
    m->sel[n] = (uint8_t *)calloc(IR, 1);
    m->H[n] = (double *)calloc((size_t)R * R, sizeof(double));
    m->A_prev[n] = (double *)calloc(IR, sizeof(double));
    m->zprev_used[n] = (double *)calloc(IR, sizeof(double));
    m->band[n] = (double *)calloc(IR, sizeof(double));
    m->band_used[n] = (double *)calloc(IR, sizeof(double));
    m->kind[n] = (uint8_t *)calloc(IR, 1);
    if (!m->A[n] || !m->G[n] || !m->zprev[n] || !m->M[n] || !m->G0[n] || !m->z[n] ||
        !m->sel[n] || !m->H[n] || !m->A_prev[n] || !m->zprev_used[n] || !m->band[n] ||
        !m->band_used[n] || !m->kind[n]) {
      free(raw); ora_model_destroy(m); return ORA_ENOMEM;
    }
    for (size_t i = 0; i < IR; ++i)
      m->A[n][i] = (double)(raw[off + (int64_t)i] >> 40) * (1.0 / 16777216.0);
    off += (int64_t)IR;
    gram(m->A[n], t->dims[n], R, m->G[n]);
    m->ti_prev[n] = 0.0;
    m->k[n] = 0;
  }
  free(raw);
  *out = m;
  return ORA_OK;
}

int ora_model_get_factor(const ora_model *m, int mode, double *dst) {
  if (!m || mode < 0 || mode > 2 || !dst) return ORA_EINVAL;
  memcpy(dst, m->A[mode], (size_t)m->t->dims[mode] * m->R * sizeof(double));
  return ORA_OK;
}

int ora_model_set_factor(ora_model *m, int mode, const double *src) {
  if (!m || mode < 0 || mode > 2 || !src) return ORA_EINVAL;
  const size_t IR = (size_t)m->t->dims[mode] * m->R;
  for (size_t i = 0; i < IR; ++i)
    if (!isfinite(src[i])) return ORA_ENUMERIC;
  memcpy(m->A[mode], src, IR * sizeof(double));
  gram(m->A[mode], m->t->dims[mode], m->R, m->G[mode]);
  return ORA_OK;
}

int ora_model_get_state(const ora_model *m, int mode, double *zprev,
                        double *ti_prev, int64_t *k) {
  if (!m || mode < 0 || mode > 2) return ORA_EINVAL;
  if (zprev) memcpy(zprev, m->zprev[mode], (size_t)m->t->dims[mode] * m->R * sizeof(double));
  if (ti_prev) *ti_prev = m->ti_prev[mode];
  if (k) *k = m->k[mode];
  return ORA_OK;
}

int ora_model_set_state(ora_model *m, int mode, const double *zprev,
                        double ti_prev, int64_t k) {
  if (!m || mode < 0 || mode > 2 || k < 0) return ORA_EINVAL;
  const size_t IR = (size_t)m->t->dims[mode] * m->R;
  if (zprev) memcpy(m->zprev[mode], zprev, IR * sizeof(double));
  memset(m->band[mode], 0, IR * sizeof(double)); /* the given Z^{k-1} is exact */
  m->ti_prev[mode] = ti_prev;
  m->k[mode] = k;
  m->undo_ok[mode] = 0;
  return ORA_OK;
}

int ora_model_set_columns(ora_model *m, int cb) {
  if (!m || cb < 0 || (cb > 0 && m->update_rule != ORA_UPDATE_GS)) return ORA_EINVAL;
  m->cb = cb;
  return ORA_OK;
}

void ora_model_force_flip(ora_model *m, int force_flip) {
  if (m) m->force_flip = force_flip;
}

void ora_model_set_tie_tol(ora_model *m, double tau) {
  if (m) m->tau = tau;
}

/* ||X - [[A0, A1, A2]]||^2 (eq. 6) for the current factors, evaluated as
 * ||X||^2 - 2 <X, Xhat> + ||Xhat||^2 with <X, Xhat> summed over Omega (eq. 8)
 * and ||Xhat||^2 = sum_rs (G0 * G1 * G2)_rs. */
double ora_objective(const ora_model *m) {
  const ora_tensor *t = m->t;
  const int R = m->R;
  double inner = 0.0;
  for (int64_t p = 0; p < t->nnz; ++p) {
    const int32_t *c = &t->coords[0][3 * p]; /* (i0, i1, i2) */
    double xhat = 0.0;
    for (int r = 0; r < R; ++r)
      xhat += m->A[0][(int64_t)c[0] * R + r] * m->A[1][(int64_t)c[1] * R + r] *
              m->A[2][(int64_t)c[2] * R + r];
    inner += (double)t->vals[0][p] * xhat;
  }
  double model = 0.0;
  for (int i = 0; i < R * R; ++i) model += m->G[0][i] * m->G[1][i] * m->G[2][i];
  return t->norm2 - 2.0 * inner + model;
}

int ora_fit(const ora_model *m, double *fit, double *f) {
  if (!m) return ORA_EINVAL;
  const double obj = ora_objective(m);
  if (f) *f = obj;
  if (!(m->t->norm2 > 0.0)) return ORA_ENUMERIC;
  if (fit) *fit = 1.0 - sqrt(obj > 0.0 ? obj : 0.0) / sqrt(m->t->norm2);
  return ORA_OK;
}

/* eq. 30 on the given entries: sqrt(sum (x - xhat)^2 / n), xhat from eq. 5. */
int ora_rmse(const ora_model *m, int64_t n, const int32_t *idx, const float *vals, double *rmse) {
  if (!m || !rmse || n < 0 || (n > 0 && (!idx || !vals))) return ORA_EINVAL;
  const int R = m->R;
  double se = 0.0;
  for (int64_t p = 0; p < n; ++p) {
    for (int k = 0; k < 3; ++k)
      if (idx[3 * p + k] < 0 || idx[3 * p + k] >= m->t->dims[k]) return ORA_ERANGE;
    double xhat = 0.0;
    for (int r = 0; r < R; ++r)
      xhat += m->A[0][(int64_t)idx[3 * p] * R + r] * m->A[1][(int64_t)idx[3 * p + 1] * R + r] *
              m->A[2][(int64_t)idx[3 * p + 2] * R + r];
    const double e = (double)vals[p] - xhat;
    se += e * e;
  }
  *rmse = n > 0 ? sqrt(se / (double)n) : 0.0;
  return ORA_OK;
}

/* eq. pd: cosine similarity of columns i < r of factor `mode`, averaged. */
int ora_pd(const ora_model *m, int mode, double *pd) {
  if (!m || !pd || mode < 0 || mode > 2) return ORA_EINVAL;
  const int R = m->R;
  const int64_t I = m->t->dims[mode];
  const double *A = m->A[mode];
  double sum = 0.0;
  int64_t pairs = 0;
  for (int i = 0; i < R; ++i)
    for (int r = i + 1; r < R; ++r) {
      double dot = 0.0, ni = 0.0, nr = 0.0;
      for (int64_t q = 0; q < I; ++q) {
        dot += A[q * R + i] * A[q * R + r];
        ni += A[q * R + i] * A[q * R + i];
        nr += A[q * R + r] * A[q * R + r];
      }
      if (ni > 0.0 && nr > 0.0) {
        sum += dot / (sqrt(ni) * sqrt(nr));
        ++pairs;
      }
    }
  *pd = pairs > 0 ? sum / (double)pairs : 0.0;
  return ORA_OK;
}

/* Update of one row's selected elements (step 9 below).  a: the row (R
 * values, updated in place); sel: decisions; M, delta: the row's MTTKRP and
 * snapshot steps; H: R x R. */
static void update_row(double *a, const uint8_t *sel, const double *M, const double *delta,
                       const double *H, int R, int rule) {
  if (rule == ORA_UPDATE_GS) {
    for (int r = 0; r < R; ++r) {
      const double h = H[r * R + r];
      if (!sel[r] || !(h > 0.0)) continue;
      double g = -M[r];
      for (int s = 0; s < R; ++s) g += a[s] * H[s * R + r];
      const double u = a[r] - g / h;
      a[r] = u > 0.0 ? u : 0.0;
    }
  } else {
    for (int r = 0; r < R; ++r)
      if (sel[r]) a[r] += delta[r];
  }
}

static void record_tie_band(ora_model *m, int mode);

/*
 * One sweep of mode n: the body of Alg. 1 for one factor matrix.
 *
 *  1. k_n += 1 (the loop counter of Alg. 1, kept per mode).
 *  2. H = Gram_a * Gram_b (eq. 10 / its mode-2, mode-3 analogues) and
 *     L = ||H|| (Alg. 1; the norm is the Frobenius norm, Table of Symbols).
 *  3. M = sparse MTTKRP (eq. 9 first term).
 *  4. G0 = -M + A_n H, the gradient computed once per sweep (eq. 9, eq. 14).
 *  5. For every element: step delta (eq. 11-12) and importance z (eq. 20).
 *  6. Total importance ti = sum z over all elements (eq. 25).
 *  7. Selection (Alg. 1, eq. 24 / eq. 27).
 *  8. Z^{k-1} <- z for every element, ti^{k-1} <- ti (Alg. 1; eq. 26).
 *  9. Update of the selected elements by eq. 13.
 *     Reading (Gauss-Seidel): the selection uses the snapshot gradient G0,
 *     while each selected update uses the one-variable gradient refreshed
 *     for the elements of the same row already updated in this sweep; the
 *     paper's Lemma 2 states that only g_qr itself has to be refreshed for
 *     the update of u_qr, and Sec. 4.4 computes the gradient column by column
 *     during the column-wise update.  Rows are independent, so the
 *     column-major order of the paper and the row-wise order used here give
 *     the same result.  The literal Jacobi form (every selected element moves
 *     by its snapshot step) is kept as ORA_UPDATE_JACOBI.
 * 10. Gram_n = A_n^T A_n.
 * 11. f = ||X||^2 - 2 <M, A_n> + sum (Gram_0 * Gram_1 * Gram_2), which equals
 *     eq. 6 because M does not depend on A_n.
 * The tie band of the sweep is recorded afterwards (not a step of Alg. 1).
 */
int ora_sweep(ora_model *m, int mode) {
  if (!m || mode < 0 || mode > 2) return ORA_EINVAL;
  const ora_tensor *t = m->t;
  const int R = m->R;
  const int64_t I = t->dims[mode];
  const size_t IR = (size_t)I * R;
  int a, b;
  other_modes(mode, &a, &b);
  double *A = m->A[mode];
  double *H = m->H[mode];
  double *M = m->M[mode];
  double *G0 = m->G0[mode];
  double *z = m->z[mode];
  double *zprev = m->zprev[mode];
  uint8_t *sel = m->sel[mode];
  double *delta = (double *)malloc((IR > 0 ? IR : 1) * sizeof(double));
  if (!delta) return ORA_ENOMEM;
  memcpy(m->A_prev[mode], A, IR * sizeof(double));

  /* 1 */
  m->k[mode] += 1;
  const int64_t k = m->k[mode];

  /* 2 */
  double L2 = 0.0;
  for (int i = 0; i < R * R; ++i) {
    H[i] = m->G[a][i] * m->G[b][i];
    L2 += H[i] * H[i];
  }
  const double L = sqrt(L2);

  /* 3 (in the column form, the MTTKRP column by column: Sec. 4.4) */
  double *col = NULL;
  if (m->cb > 0) {
    col = (double *)malloc((size_t)(I > 0 ? I : 1) * sizeof(double));
    if (!col) { free(delta); return ORA_ENOMEM; }
    for (int r = 0; r < R; ++r) {
      ora_sttvp(t, mode, R, r, m->A[0], m->A[1], m->A[2], col);
      for (int64_t q = 0; q < I; ++q) M[q * R + r] = col[q];
    }
  } else {
    ora_mttkrp(t, mode, R, m->A[0], m->A[1], m->A[2], M);
  }

  /* 4, 5 */
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < I; ++q) {
    for (int r = 0; r < R; ++r) {
      double ah = 0.0;
      for (int s = 0; s < R; ++s) ah += A[q * R + s] * H[s * R + r];
      const int64_t e = q * R + r;
      G0[e] = -M[e] + ah;
      delta[e] = ora_cd_delta(A[e], G0[e], H[r * R + r]);
      z[e] = ora_importance(G0[e], delta[e], L);
    }
  }

  /* 6 */
  double ti = 0.0;
  for (size_t e = 0; e < IR; ++e) ti += z[e];

  /* 7 */
  int flip = 0;
  if (k >= 2) {
    flip = ti > m->ti_prev[mode]; /* "more than" (eq. 27 condition) */
    if (m->force_flip == 0 || m->force_flip == 1) flip = m->force_flip;
  }
  int64_t nsel = 0;
  for (size_t e = 0; e < IR; ++e) {
    sel[e] = (uint8_t)ora_select(k, z[e], zprev[e], flip);
    nsel += sel[e];
  }

  /* 8 */
  const double ti_used = m->ti_prev[mode];
  memcpy(m->zprev_used[mode], zprev, IR * sizeof(double));
  memcpy(zprev, z, IR * sizeof(double));
  m->ti_prev[mode] = ti;

  /* 9 */
  if (m->cb > 0) {
    /* column form: block by block in ascending column order, the block's
     * columns of M computed again (M is not kept between the two passes),
     * then each selected element of the block updated with the gradient of
     * the row's current values -- the same element steps, in the same order
     * per row, as update_row */
    for (int c0 = 0; c0 < R; c0 += m->cb) {
      const int c1 = c0 + m->cb < R ? c0 + m->cb : R;
      for (int r = c0; r < c1; ++r) {
        ora_sttvp(t, mode, R, r, m->A[0], m->A[1], m->A[2], col);
        for (int64_t q = 0; q < I; ++q) M[q * R + r] = col[q];
      }
#pragma omp parallel for schedule(static)
      for (int64_t q = 0; q < I; ++q) {
        double *a = A + q * R;
        for (int r = c0; r < c1; ++r) {
          const double h = H[r * R + r];
          if (!sel[q * R + r] || !(h > 0.0)) continue;
          double g = -M[q * R + r];
          for (int s2 = 0; s2 < R; ++s2) g += a[s2] * H[s2 * R + r];
          const double u = a[r] - g / h;
          a[r] = u > 0.0 ? u : 0.0;
        }
      }
    }
    free(col);
  } else {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < I; ++q)
      update_row(A + q * R, sel + q * R, M + q * R, delta + q * R, H, R, m->update_rule);
  }
  free(delta);

  /* 10 */
  gram(A, I, R, m->G[mode]);

  /* 11 */
  double inner = 0.0;
  for (size_t e = 0; e < IR; ++e) inner += M[e] * A[e];
  double model = 0.0;
  for (int i = 0; i < R * R; ++i) model += m->G[0][i] * m->G[1][i] * m->G[2][i];
  const double f = t->norm2 - 2.0 * inner + model;

  m->info[mode][0] = L;
  m->info[mode][1] = ti;
  m->info[mode][2] = (double)flip;
  m->info[mode][3] = ti_used;
  m->info[mode][4] = f;
  m->info[mode][5] = (double)nsel;
  m->info[mode][6] = inner;
  m->info[mode][7] = model;
  record_tie_band(m, mode);
  m->undo_ok[mode] = 1;
  return ORA_OK;
}

int ora_sweep_undo(ora_model *m, int mode) {
  if (!m || mode < 0 || mode > 2) return ORA_EINVAL;
  if (!m->undo_ok[mode]) return ORA_ESTATE;
  const int64_t I = m->t->dims[mode];
  const size_t IR = (size_t)I * m->R;
  memcpy(m->A[mode], m->A_prev[mode], IR * sizeof(double));
  gram(m->A[mode], I, m->R, m->G[mode]);
  memcpy(m->zprev[mode], m->zprev_used[mode], IR * sizeof(double));
  memcpy(m->band[mode], m->band_used[mode], IR * sizeof(double));
  m->ti_prev[mode] = m->info[mode][3];
  m->k[mode] -= 1;
  m->undo_ok[mode] = 0;
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Tie band (diagnostics of the tests; no step of the method reads it).      */
/* ------------------------------------------------------------------------ */

/* See ora_sweep_band in the header.  Sensitivity of z = -g d - (L/2) d^2
 * (eq. 20) to its gradient g: with a clipped step (d = -a, eq. 12) dz/dg = a
 * = |d|; with an interior one (d = -g/h, eq. 11) dz/dg = -d + g/h + L d/h, so
 * |dz/dg| <= 2|d| + L|d|/h.  An interior z is quadratic in g, and near
 * g = 0 its first-order term vanishes: an error e of g moves the step by up
 * to |e|/h, so z may move by (tau T / h)^2 (h + L/2) as well; that
 * second-order term is added to the band of every interior step.  A clipped
 * step is linear in g (and exactly zero when a = 0), so it has none.  A
 * zero-gradient tie (a = 0, g within tau T of zero) has z = 0 on one side of
 * zero and that interior step on the other. */
static void record_tie_band(ora_model *m, int mode) {
  const int R = m->R;
  const int64_t I = m->t->dims[mode];
  const size_t IR = (size_t)I * R;
  const double tau = m->tau, L = m->info[mode][0];
  const int64_t k = m->k[mode];
  const double *A = m->A_prev[mode], *H = m->H[mode], *M = m->M[mode], *G0 = m->G0[mode];
  const double *z = m->z[mode], *zp = m->zprev_used[mode];
  double *band = m->band[mode], *band_used = m->band_used[mode];
  uint8_t *kind = m->kind[mode];
  memcpy(band_used, band, IR * sizeof(double)); /* band of the Z^{k-1} just used */
  double sum_band = 0.0, sum_used = 0.0;
  int64_t n_zero = 0, n_grad = 0, n_margin = 0;
  for (int64_t q = 0; q < I; ++q) {
    for (int r = 0; r < R; ++r) {
      const int64_t e = q * R + r;
      const double h = H[r * R + r];
      double T = fabs(M[e]);
      for (int s = 0; s < R; ++s) T += fabs(A[q * R + s] * H[s * R + r]);
      const double d = ora_cd_delta(A[e], G0[e], h);
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
  }
  const double band_ti = sum_band + sum_used;
  m->band_info[mode][0] = band_ti;
  m->band_info[mode][1] = (k >= 2 && fabs(m->info[mode][1] - m->info[mode][3]) <= band_ti) ? 1.0 : 0.0;
  m->band_info[mode][2] = (double)n_zero;
  m->band_info[mode][3] = (double)n_grad;
  m->band_info[mode][4] = (double)n_margin;
}

int ora_sweep_band(const ora_model *m, int mode, double *band, uint8_t *kind, double *scalars) {
  if (!m || mode < 0 || mode > 2) return ORA_EINVAL;
  const size_t IR = (size_t)m->t->dims[mode] * m->R;
  if (band) memcpy(band, m->band[mode], IR * sizeof(double));
  if (kind) memcpy(kind, m->kind[mode], IR);
  if (scalars) memcpy(scalars, m->band_info[mode], sizeof(m->band_info[mode]));
  return ORA_OK;
}

/* Step 9 for one row of the last sweep of `mode` under the given decisions:
 * a decision inside the tie band may go either way, and rows are independent
 * in step 9, so this is the oracle's row for any valid set of decisions. */
int ora_row_outcome(const ora_model *m, int mode, int64_t q, const uint8_t *sel, double *out) {
  if (!m || mode < 0 || mode > 2 || !sel || !out) return ORA_EINVAL;
  const int R = m->R;
  if (q < 0 || q >= m->t->dims[mode]) return ORA_ERANGE;
  const double *a_prev = m->A_prev[mode] + q * R;
  const double *G0 = m->G0[mode] + q * R;
  const double *H = m->H[mode];
  double *delta = (double *)malloc((size_t)R * sizeof(double));
  if (!delta) return ORA_ENOMEM;
  for (int r = 0; r < R; ++r) delta[r] = ora_cd_delta(a_prev[r], G0[r], H[r * R + r]);
  memcpy(out, a_prev, (size_t)R * sizeof(double));
  update_row(out, sel, m->M[mode] + q * R, delta, H, R, m->update_rule);
  free(delta);
  return ORA_OK;
}

int ora_sweep_info(const ora_model *m, int mode, double *M, double *G0,
                   double *z, uint8_t *sel, double *H, double *scalars) {
  if (!m || mode < 0 || mode > 2) return ORA_EINVAL;
  const size_t IR = (size_t)m->t->dims[mode] * m->R;
  if (M) memcpy(M, m->M[mode], IR * sizeof(double));
  if (G0) memcpy(G0, m->G0[mode], IR * sizeof(double));
  if (z) memcpy(z, m->z[mode], IR * sizeof(double));
  if (sel) memcpy(sel, m->sel[mode], IR);
  if (H) memcpy(H, m->H[mode], (size_t)m->R * m->R * sizeof(double));
  if (scalars) memcpy(scalars, m->info[mode], sizeof(m->info[mode]));
  return ORA_OK;
}

int ora_run_until(ora_model *m, double tol, int max_iter, int *iters_done,
                  double *final_fit, double *fit_trace) {
  if (!m || max_iter < 1 || !(tol >= 0.0)) return ORA_EINVAL;
  if (!(m->t->norm2 > 0.0)) return ORA_ENUMERIC;
  double prev = 0.0, fit = 0.0;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    for (int n = 0; n < 3; ++n) {
      int rc = ora_sweep(m, n);
      if (rc) return rc;
    }
    const double f = m->info[2][4];
    fit = 1.0 - sqrt(f > 0.0 ? f : 0.0) / sqrt(m->t->norm2);
    if (fit_trace) fit_trace[it - 1] = fit;
    if (it >= 2 && fabs(fit - prev) < tol * fabs(prev)) break;
    prev = fit;
  }
  if (it > max_iter) it = max_iter;
  if (iters_done) *iters_done = it;
  if (final_fit) *final_fit = fit;
  return ORA_OK;
}
