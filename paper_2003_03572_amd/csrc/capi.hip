// capi.hip -- host runtime of libsacd: the C ABI declared in include/sacd.h.
//
// Owns the device buffers of tensors and models, orders all work on the
// object's stream, captures one outer iteration (three mode sweeps) as a HIP
// graph for replay, and turns every failure into a sacd_status plus a
// thread-local message.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/sacd.h"
#include "common.hpp"

using namespace sacd;

namespace {

thread_local char g_err[512] = "";

sacd_status fail(sacd_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return fail(_e == hipErrorOutOfMemory ? SACD_ERR_NO_MEMORY : SACD_ERR_DEVICE,      \
                  "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
  } while (0)

#define SACD_TRY(expr)                 \
  do {                                 \
    sacd_status _s = (expr);           \
    if (_s != SACD_OK) return _s;      \
  } while (0)

int bits_for(int64_t n) {  // bits needed to hold the values 0 .. n-1
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  return b;
}

void other_modes(int n, int *a, int *b) {
  *a = (n == 0) ? 1 : 0;
  *b = (n == 2) ? 1 : 2;
}

// Device memory owner: caller's allocator if given, else hipMalloc.
struct DevAlloc {
  sacd_allocator alloc{};
  bool custom = false;
  std::vector<void *> blocks;
  int64_t bytes = 0;

  sacd_status get(size_t n, void **out) {
    if (n == 0) n = 16;
    n = (n + 255) & ~(size_t)255;
    void *p = nullptr;
    if (custom) {
      p = alloc.alloc(n, alloc.user);
      if (!p) return fail(SACD_ERR_NO_MEMORY, "allocator returned NULL for %zu bytes", n);
    } else {
      hipError_t e = hipMalloc(&p, n);
      if (e != hipSuccess) return fail(SACD_ERR_NO_MEMORY, "hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
    }
    blocks.push_back(p);
    bytes += (int64_t)n;
    *out = p;
    return SACD_OK;
  }
  template <typename T>
  sacd_status get_t(size_t count, T **out) {
    void *p = nullptr;
    SACD_TRY(get(count * sizeof(T), &p));
    *out = (T *)p;
    return SACD_OK;
  }
  void release(void *p) {
    for (size_t i = 0; i < blocks.size(); ++i)
      if (blocks[i] == p) {
        if (custom) alloc.release(p, alloc.user);
        else (void)hipFree(p);
        blocks.erase(blocks.begin() + i);
        return;
      }
  }
  void release_all() {
    for (void *p : blocks) {
      if (custom) alloc.release(p, alloc.user);
      else (void)hipFree(p);
    }
    blocks.clear();
  }
};

// Small pinned host buffers (64 bytes each) for scalar read-backs, carved
// from process-wide 64 KB slabs that live until the process ends:
// hipHostMalloc / hipHostFree cost milliseconds and synchronise the device,
// too much to pay per model when jobs come and go.
struct PinnedPool {
  std::mutex mu;
  std::vector<double *> free_list;
};

PinnedPool &pinned_pool() {
  static PinnedPool *p = new PinnedPool();  // never destroyed: slabs outlive every model
  return *p;
}

sacd_status pinned_get(double **out) {
  PinnedPool &P = pinned_pool();
  std::lock_guard<std::mutex> lock(P.mu);
  if (P.free_list.empty()) {
    char *slab = nullptr;
    HIP_TRY(hipHostMalloc((void **)&slab, 65536, hipHostMallocDefault));
    for (int i = 0; i < 1024; ++i) P.free_list.push_back((double *)(slab + 64 * i));
  }
  *out = P.free_list.back();
  P.free_list.pop_back();
  return SACD_OK;
}

void pinned_put(double *p) {
  if (!p) return;
  PinnedPool &P = pinned_pool();
  std::lock_guard<std::mutex> lock(P.mu);
  P.free_list.push_back(p);
}

}  // namespace

struct sacd_tensor {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevAlloc mem;
  int64_t dims[3] = {0, 0, 0};
  long long nnz = 0;
  KeyLayout lay[3];
  unsigned long long *keys[3] = {nullptr, nullptr, nullptr};
  float *vals[3] = {nullptr, nullptr, nullptr};
  int *ptr[3] = {nullptr, nullptr, nullptr};
  std::vector<int> hptr[3];  // host copy of the slice pointers
  double norm2 = 0.0;
  int nmodels = 0;              // live models built on this tensor
  bool destroy_pending = false;  // destroyed by the caller while models were live
};

struct sacd_model {
  sacd_tensor *t = nullptr;
  hipStream_t s = nullptr;
  DevAlloc mem;
  int R = 0, RP = 0;
  sacd_precision prec = SACD_PREC_FP32;
  sacd_update upd = SACD_UPDATE_GS;
  bool diag = false;
  float *A[3] = {}, *Z[3] = {}, *M[3] = {}, *H[3] = {};
  double *G64[3] = {};
  // mixed form: the objective's Grams (FP32 operands) beside the BF16 ones
  // that form H; in the FP32 form G64o[n] == G64[n]
  double *G64o[3] = {};
  float *gpart_obj = nullptr;
  HInfo *hinfo[3] = {};
  ModeState *st = nullptr;  // 3 entries
  long long *colcnt[3] = {};
  uint8_t *selmask[3] = {};
  float *part = nullptr, *gpart = nullptr;
  double *mpart = nullptr;
  unsigned *gcounter = nullptr;
  double *ti_part = nullptr, *inner_part = nullptr;
  int *cnt_part = nullptr, *flag = nullptr;
  double *full_part = nullptr, *full_out = nullptr;
  unsigned *full_cnt = nullptr;
  int full_nparts = 0;
  int nparts[3] = {0, 0, 0};
  MttkrpPlan plan[3];
  int lds_cols[3] = {0, 0, 0};  // MTTKRP form per mode: A_b staged in LDS slabs of this many columns (0: plain)
  // tiled MTTKRP form of a mode (see tiled_mode): the mode's entries in
  // (i_n, i_b tile, i_a, i_b) order, and the block table of the LDS kernel
  unsigned long long *tkeys[3] = {};
  float *tvals[3] = {};
  int4 *btab[3] = {};
  int nbt[3] = {0, 0, 0};
  // column-at-a-time form: cb columns of M at a time (0: the row form, M held whole)
  int cb = 0;
  float *Mb = nullptr, *upart = nullptr;
  unsigned *bits = nullptr;
  double *colpart = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  // measurement: events recorded around the MTTKRP launches and at the end of
  // every sweep (9 per iteration)
  std::vector<hipEvent_t> tev;
  double *h_pinned = nullptr;
  bool counted = false;  // included in t->nmodels
  int last_mode = -1;  // mode of the most recent sweep, -1: objective must be recomputed
  bool dirty = true;   // factors changed outside a sweep
};

namespace {

sacd_status enter(int dev) {
  (void)hipGetLastError();  // drop an error left by an unrelated earlier call
  HIP_TRY(hipSetDevice(dev));
  return SACD_OK;
}

sacd_status make_stream(void *stream, hipStream_t *out, bool *own) {
  if (stream) {
    *out = (hipStream_t)stream;
    *own = false;
  } else {
    HIP_TRY(hipStreamCreateWithFlags(out, hipStreamNonBlocking));
    *own = true;
  }
  return SACD_OK;
}

// ---------------------------------------------------------------- sweep ----

// Kernel arguments of mode n of one model (also the per-job entries of the
// job-batched launches).
MttkrpArgs mttkrp_args(const sacd_model *m, int n) {
  const sacd_tensor *t = m->t;
  int a, b;
  other_modes(n, &a, &b);
  MttkrpArgs x;
  x.keys = m->tkeys[n] ? m->tkeys[n] : t->keys[n];
  x.vals = m->tvals[n] ? m->tvals[n] : t->vals[n];
  x.units = m->plan[n].units;
  x.nunits = m->plan[n].nunits;
  x.lay = t->lay[n];
  x.Aa = m->A[a];
  x.Ab = m->A[b];
  x.M = m->M[n];
  x.part = m->part;
  return x;
}

FixArgs fix_args(const sacd_model *m, int n) {
  int a, b;
  other_modes(n, &a, &b);
  FixArgs x;
  x.longs = m->plan[n].longs;
  x.nlong = m->plan[n].nlong;
  x.nbig = m->plan[n].nbig;
  x.part = m->part;
  x.M = m->M[n];
  x.Ga = m->G64[a];
  x.Gb = m->G64[b];
  x.H = m->H[n];
  x.hinfo = m->hinfo[n];
  x.st = m->st + n;
  return x;
}

ImpArgs imp_args(const sacd_model *m, int n) {
  ImpArgs x;
  x.I = (int)m->t->dims[n];
  x.A = m->A[n];
  x.M = m->M[n];
  x.H = m->H[n];
  x.hi = m->hinfo[n];
  x.ti_part = m->ti_part;
  x.st = m->st + n;
  return x;
}

UpdArgs upd_args(const sacd_model *m, int n) {
  UpdArgs x;
  x.I = (int)m->t->dims[n];
  x.A = m->A[n];
  x.M = m->M[n];
  x.Z = m->Z[n];
  x.H = m->H[n];
  x.hi = m->hinfo[n];
  x.st = m->st + n;
  x.gpart = m->gpart;
  x.gpart_obj = m->gpart_obj;
  x.inner_part = m->inner_part;
  x.cnt_part = m->cnt_part;
  x.selmask = m->selmask[n];
  return x;
}

// with_f: the sweep form (Gram, counts, <M, A_n>, objective); otherwise the
// Gram of a factor set from outside (partials from k_gram_partial).
GramArgs gram_args(const sacd_model *m, int n, bool with_f) {
  int a, b;
  other_modes(n, &a, &b);
  GramArgs x;
  x.nparts = m->nparts[n];
  x.gpart = m->gpart;
  x.mpart = m->mpart;
  x.Gn = m->G64[n];
  x.Ga = with_f ? m->G64[a] : nullptr;
  x.Gb = with_f ? m->G64[b] : nullptr;
  x.gpart_obj = m->gpart_obj;
  x.Gn_obj = m->gpart_obj ? m->G64o[n] : nullptr;
  x.Ga_obj = m->gpart_obj && with_f ? m->G64o[a] : nullptr;
  x.Gb_obj = m->gpart_obj && with_f ? m->G64o[b] : nullptr;
  x.inner_part = with_f ? m->inner_part : nullptr;
  x.cnt_part = with_f ? m->cnt_part : nullptr;
  x.colcnt = with_f ? m->colcnt[n] : nullptr;
  x.normX2 = with_f ? m->t->norm2 : 0.0;
  x.with_f = with_f ? 1 : 0;
  x.counter = m->gcounter;
  x.st = m->st + n;
  return x;
}

bool is_bf16(const sacd_model *m) { return m->prec == SACD_PREC_MIXED_BF16; }

// The MTTKRP of mode n: the LDS-staged form when A_b has few enough rows
// (the same M as the plain form, bit for bit), the tiled form when the mode
// has a tiled copy, else the plain form.
hipError_t launch_mode_mttkrp(const sacd_model *m, int n, hipStream_t s) {
  int a, b;
  other_modes(n, &a, &b);
  if (m->btab[n])
    return launch_mttkrp_lds(m->RP, 64, mttkrp_args(m, n), (int)m->t->dims[b], m->btab[n], m->nbt[n], s);
  if (m->lds_cols[n] > 0)
    return launch_mttkrp_lds(m->RP, m->lds_cols[n], mttkrp_args(m, n), (int)m->t->dims[b], nullptr, 0, s);
  return launch_mttkrp(m->RP, mttkrp_args(m, n), s);
}

// One sweep of mode n in the column-at-a-time form (Sec. 4.4): H and L; pass A
// over the column blocks (M_b, importances, both decisions, Z); ti and the
// eq. 27 branch; pass B (M_b again, Gauss-Seidel steps of the selected
// elements, <M, A_n>); counts; Gram and objective.  mark (optional): events
// before pass A, after pass B and at the end.
sacd_status enqueue_sweep_columns(sacd_model *m, int n, const hipEvent_t *mark) {
  hipStream_t s = m->s;
  const int I = (int)m->t->dims[n], RP = m->RP, CB = m->cb;
  const int Rc = (m->R + CB - 1) / CB * CB;  // columns swept; the others are zero padding
  const int ncb = Rc / CB, nrb = col_row_blocks(I);
  FixArgs fx = fix_args(m, n);
  fx.nlong = 0;  // H, L and the diagonal only: no split slices of a whole M to add
  fx.nbig = 0;
  HIP_TRY(launch_mttkrp_fix(RP, fx, s));
  if (mark) HIP_TRY(hipEventRecord(mark[0], s));
  HIP_TRY(launch_zero_words(m->bits, (int)(((long long)I * RP + 15) / 16), s));
  MttkrpArgs ma = mttkrp_args(m, n);
  ma.M = nullptr;
  ma.part = m->upart;
  const MttkrpPlan &pl = m->plan[n];
  ColArgs ca;
  ca.I = I;
  ca.RP = RP;
  ca.CB = CB;
  ca.A = m->A[n];
  ca.Mb = m->Mb;
  ca.H = m->H[n];
  ca.hi = m->hinfo[n];
  ca.st = m->st + n;
  ca.Z = m->Z[n];
  ca.bits = m->bits;
  ca.part = m->colpart;
  ca.cnt_part = m->cnt_part;
  ca.selmask = m->diag ? m->selmask[n] : nullptr;
  ca.Mdiag = m->diag ? m->M[n] : nullptr;
  // M_b is shared by the modes and the column blocks, and the rows of empty
  // slices are never written by the MTTKRP: it is cleared before each block
  const int mb_words = I * CB;
  for (int b = 0; b < ncb; ++b) {
    HIP_TRY(launch_zero_words((unsigned *)m->Mb, mb_words, s));
    HIP_TRY(launch_sttvp(CB, ma, RP, b * CB, pl.uslot, pl.ulongs, pl.nulong, m->Mb, s));
    ca.c0 = b * CB;
    ca.part_off = b * nrb;
    HIP_TRY(launch_col_importance(CB, ca, s));
  }
  HIP_TRY(launch_col_decide(m->colpart, ncb * nrb, m->st + n, s));
  for (int b = 0; b < ncb; ++b) {
    HIP_TRY(launch_zero_words((unsigned *)m->Mb, mb_words, s));
    HIP_TRY(launch_sttvp(CB, ma, RP, b * CB, pl.uslot, pl.ulongs, pl.nulong, m->Mb, s));
    ca.c0 = b * CB;
    ca.part_off = b * nrb;
    HIP_TRY(launch_col_update(CB, ca, s));
  }
  if (mark) HIP_TRY(hipEventRecord(mark[1], s));
  HIP_TRY(launch_col_finish(m->colpart, ncb * nrb, m->cnt_part, nrb, RP, Rc, m->colcnt[n], m->st + n, s));
  HIP_TRY(launch_gram_partial(RP, false, I, m->A[n], m->gpart, nullptr, s));
  GramArgs g = gram_args(m, n, true);
  g.inner_part = nullptr;  // <M, A_n>, the counts and |E| come from k_col_finish
  g.cnt_part = nullptr;
  g.colcnt = nullptr;
  HIP_TRY(launch_gram_final(RP, g, s));
  if (mark) HIP_TRY(hipEventRecord(mark[2], s));
  return SACD_OK;
}

// Enqueues one sweep of mode n on the model's stream.  mark (optional): three
// events recorded right before and right after the MTTKRP launch and after the
// sweep's last kernel.
sacd_status enqueue_sweep(sacd_model *m, int n, const hipEvent_t *mark = nullptr) {
  if (m->cb > 0) return enqueue_sweep_columns(m, n, mark);
  hipStream_t s = m->s;
  const bool bf = is_bf16(m);
  if (mark) HIP_TRY(hipEventRecord(mark[0], s));
  HIP_TRY(launch_mode_mttkrp(m, n, s));
  if (mark) HIP_TRY(hipEventRecord(mark[1], s));
  HIP_TRY(launch_mttkrp_fix(m->RP, fix_args(m, n), s));
  HIP_TRY(launch_importance(m->RP, bf, imp_args(m, n), s));
  HIP_TRY(launch_select_update(m->RP, (int)m->upd, m->diag, bf, upd_args(m, n), s));
  HIP_TRY(launch_gram_final(m->RP, gram_args(m, n, true), s));
  if (mark) HIP_TRY(hipEventRecord(mark[2], s));
  return SACD_OK;
}

sacd_status recompute_gram(sacd_model *m, int n) {
  const int I = (int)m->t->dims[n];
  HIP_TRY(launch_gram_partial(m->RP, is_bf16(m), I, m->A[n], m->gpart, m->gpart_obj, m->s));
  HIP_TRY(launch_gram_final(m->RP, gram_args(m, n, false), m->s));
  return SACD_OK;
}

void drop_graph(sacd_model *m) {
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->gexec = nullptr;
  m->graph = nullptr;
}

// Captures one iteration (sweeps of modes 0, 1, 2) into an executable graph.
sacd_status capture_iteration(sacd_model *m, hipGraph_t *graph, hipGraphExec_t *exec) {
  HIP_TRY(hipStreamBeginCapture(m->s, hipStreamCaptureModeThreadLocal));
  sacd_status st = SACD_OK;
  for (int n = 0; n < 3 && st == SACD_OK; ++n) st = enqueue_sweep(m, n);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(m->s, &g);
  if (st != SACD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(SACD_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t ge = nullptr;
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(SACD_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  *graph = g;
  *exec = ge;
  return SACD_OK;
}

sacd_status ensure_graph(sacd_model *m) {
  if (m->gexec) return SACD_OK;
  return capture_iteration(m, &m->graph, &m->gexec);
}

sacd_status read_state(const sacd_model *m, int n, ModeState *out) {
  HIP_TRY(hipMemcpyAsync(out, m->st + n, sizeof(ModeState), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

// Objective of the current factors from scratch (no sweep information).
sacd_status objective_full(sacd_model *m, double *f) {
  sacd_tensor *t = m->t;
  const int RP = m->RP;
  HIP_TRY(launch_inner_full(t->keys[0], t->vals[0], t->nnz, t->lay[0], RP, m->A[0], m->A[1], m->A[2],
                            m->full_part, m->full_nparts, m->full_out, m->full_cnt, m->s));
  std::vector<double> G((size_t)3 * RP * RP);
  double inner = 0.0;
  for (int n = 0; n < 3; ++n)
    HIP_TRY(hipMemcpyAsync(G.data() + (size_t)n * RP * RP, m->G64o[n], sizeof(double) * RP * RP,
                           hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipMemcpyAsync(&inner, m->full_out, sizeof(double), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  double model = 0.0;
  for (int i = 0; i < RP * RP; ++i)
    model += G[i] * G[(size_t)RP * RP + i] * G[(size_t)2 * RP * RP + i];
  *f = t->norm2 - 2.0 * inner + model;
  return SACD_OK;
}

// ---------------------------------------------------------------- static scratch --
// The allocation-free entry point (sacd_rmse_static) keeps its scratch -- the
// per-block partial sums of the squared errors, their total, the arrival
// counter and the out-of-range flag -- in the file-scope device array
// `scratch` below, one copy per device, instead of the model's buffers.  Host
// code never passes the array's name to a kernel or a copy (on the host it is
// only a stand-in): the array's device address is looked up once per device
// with hipGetSymbolAddress and kept in g_scratch_ptr.

constexpr int kStaticParts = 1024;                       // partial sums: one per block, at most
constexpr long long kStaticMaxEntries = 2147483647LL;    // entries per call, at most
constexpr size_t kStaticScratchBytes = (size_t)kStaticParts * 8 + 256;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current.  Looked up
// once per device (at model set-up, else at the entry point's first call).
sacd_status static_scratch(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SACD_ERR_DEVICE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SACD_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SACD_OK;
}

sacd_status check_mode(const sacd_model *m, int32_t mode) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  if (mode < 0 || mode > 2) return fail(SACD_ERR_INVALID_ARG, "mode %d not in {0, 1, 2}", mode);
  return SACD_OK;
}

}  // namespace

extern "C" {

const char *sacd_version(void) { return "0.1.0"; }

const char *sacd_last_error(void) { return g_err; }

const char *sacd_status_string(sacd_status s) {
  switch (s) {
    case SACD_OK: return "ok";
    case SACD_ERR_INVALID_ARG: return "invalid argument";
    case SACD_ERR_OUT_OF_RANGE: return "index out of range";
    case SACD_ERR_NO_MEMORY: return "out of device memory";
    case SACD_ERR_BAD_STATE: return "bad state";
    case SACD_ERR_DEVICE: return "device error";
    case SACD_ERR_NUMERIC: return "non-finite or degenerate value";
  }
  return "unknown status";
}

// ------------------------------------------------------------------ tensor --

// Partial slots of the units of split slices (w == -2 on entry): consecutive
// units of one split slice inside one block (of upb units, or as block_of
// gives) form a run, whose
// sum the MTTKRP kernel writes to one slot; the runs are numbered slice by
// slice, and *longs gets (slice, first slot, slots, 0) per split slice.
// Sets each such unit's w to its run's slot; returns the number of slots.
static int number_runs(std::vector<int4> &units, int upb, std::vector<int4> *longs,
                       const std::vector<int> *block_of = nullptr);

// The fix-up's order of the split slices: those with more than kFixSmall
// slots first (a block each), then the others (a lane group each); returns
// how many are big.
static int order_longs(std::vector<int4> *longs) {
  std::stable_partition(longs->begin(), longs->end(), [](const int4 &l) { return l.z > kFixSmall; });
  return (int)std::count_if(longs->begin(), longs->end(), [](const int4 &l) { return l.z > kFixSmall; });
}

static int number_runs(std::vector<int4> &units, int upb, std::vector<int4> *longs,
                       const std::vector<int> *block_of) {
  std::vector<int> run_of(units.size(), -1);
  std::vector<int> run_slice;
  auto blk = [&](size_t u) { return block_of ? (size_t)(*block_of)[u] : u / (size_t)upb; };
  for (size_t u = 0; u < units.size(); ++u) {
    if (units[u].w != -2) continue;
    const bool cont = u > 0 && units[u - 1].w == -2 && units[u - 1].x == units[u].x && blk(u - 1) == blk(u);
    if (cont) {
      run_of[u] = run_of[u - 1];
    } else {
      run_of[u] = (int)run_slice.size();
      run_slice.push_back(units[u].x);
    }
  }
  std::vector<int> order(run_slice.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return run_slice[a] < run_slice[b]; });
  std::vector<int> slot_of(run_slice.size());
  longs->clear();
  for (size_t k = 0; k < order.size(); ++k) {
    const int r = run_slice[order[k]];
    slot_of[order[k]] = (int)k;
    if (longs->empty() || longs->back().x != r) longs->push_back(make_int4(r, (int)k, 0, 0));
    longs->back().z += 1;
  }
  for (size_t u = 0; u < units.size(); ++u)
    if (units[u].w == -2) units[u].w = slot_of[run_of[u]];
  return (int)run_slice.size();
}

// Work plan of mode m for the MTTKRP kernels: each slice cut into segments
// of at most kSegment entries, ordered by length (longest first, stable);
// unit u runs in block u / upb.  Segments of a split slice that sit next to
// each other in one block form a run that shares one partial slot; the slots
// of a slice are numbered consecutively.
// Host arrays whose uploads may still be in flight on a stream, kept until
// the stream has passed them (the destructor waits, also on an error
// return), so that a model's plans take one wait instead of one per mode.
struct HostHold {
  hipStream_t s = nullptr;
  std::vector<std::vector<int4>> v4;
  std::vector<std::vector<int>> v1;
  ~HostHold() {
    if (s && (!v4.empty() || !v1.empty())) (void)hipStreamSynchronize(s);
  }
};

static sacd_status build_plan(const sacd_tensor *t, int m, int upb, DevAlloc &mem, MttkrpPlan *out,
                              HostHold *hold) {
  const std::vector<int> &ptr = t->hptr[m];
  const int I = (int)t->dims[m];
  std::vector<int4> units;
  std::vector<char> split;
  for (int r = 0; r < I; ++r) {
    const int len = ptr[r + 1] - ptr[r];
    if (len == 0) continue;
    if (len <= kSegment) {
      units.push_back(make_int4(r, ptr[r], len, -1));
      continue;
    }
    const int nseg = (len + kSegment - 1) / kSegment;
    for (int q = 0; q < nseg; ++q) {
      const int b = ptr[r] + q * kSegment;
      const int l = (q == nseg - 1) ? ptr[r + 1] - b : kSegment;
      units.push_back(make_int4(r, b, l, -2));  // -2: segment of a split slice
    }
  }
  // Full-length segments first, ordered by the range of A_a rows they gather
  // (kGatherBuckets coarse buckets of i_a; within a bucket by slice and
  // position), so the work in flight together reuses a small part of A_a from
  // cache; then every shorter unit, longest first.
  {
    std::vector<int> pos;
    for (const int4 &u : units)
      if (u.z == kSegment) pos.push_back(u.y);
    std::vector<unsigned long long> first_key(pos.size());
    if (!pos.empty()) {
      int *dpos = nullptr;
      unsigned long long *dkey = nullptr;
      DevAlloc tmp;
      tmp.alloc = mem.alloc;
      tmp.custom = mem.custom;
      SACD_TRY(tmp.get_t(pos.size(), &dpos));
      SACD_TRY(tmp.get_t(pos.size(), &dkey));
      HIP_TRY(hipMemcpyAsync(dpos, pos.data(), sizeof(int) * pos.size(), hipMemcpyHostToDevice, t->stream));
      HIP_TRY(launch_gather_keys(t->keys[m], dpos, (int)pos.size(), dkey, t->stream));
      HIP_TRY(hipMemcpyAsync(first_key.data(), dkey, sizeof(unsigned long long) * pos.size(),
                             hipMemcpyDeviceToHost, t->stream));
      HIP_TRY(hipStreamSynchronize(t->stream));
      tmp.release_all();
    }
    int a, b;
    other_modes(m, &a, &b);
    const long long Ia = t->dims[a];
    std::vector<std::pair<long long, int4>> full;
    std::vector<int4> rest;
    size_t k = 0;
    for (const int4 &u : units) {
      if (u.z == kSegment) {
        const long long ia = (long long)((first_key[k++] >> t->lay[m].sh_a) & t->lay[m].mask_a);
        full.push_back({ia * kGatherBuckets / Ia, u});
      } else {
        rest.push_back(u);
      }
    }
    std::stable_sort(full.begin(), full.end(), [](const std::pair<long long, int4> &x,
                                                  const std::pair<long long, int4> &y) {
      if (x.first != y.first) return x.first < y.first;
      if (x.second.x != y.second.x) return x.second.x < y.second.x;
      return x.second.y < y.second.y;
    });
    std::stable_sort(rest.begin(), rest.end(), [](const int4 &x, const int4 &y) { return x.z > y.z; });
    units.clear();
    for (const auto &f : full) units.push_back(f.second);
    for (const int4 &u : rest) units.push_back(u);
  }
  std::vector<int4> longs;
  const int nslots = number_runs(units, upb, &longs);
  const int nbig = order_longs(&longs);
  // one slot per unit of a split slice, numbered slice by slice in entry order
  std::vector<int> uslot(units.size(), -1);
  std::vector<int4> ulongs;
  {
    std::vector<int> su;
    for (size_t u = 0; u < units.size(); ++u)
      if (units[u].w >= 0) su.push_back((int)u);
    std::stable_sort(su.begin(), su.end(), [&](int x, int y) {
      if (units[x].x != units[y].x) return units[x].x < units[y].x;
      return units[x].y < units[y].y;
    });
    for (size_t k = 0; k < su.size(); ++k) {
      uslot[su[k]] = (int)k;
      if (ulongs.empty() || ulongs.back().x != units[su[k]].x) ulongs.push_back(make_int4(units[su[k]].x, (int)k, 0, 0));
      ulongs.back().z += 1;
    }
  }
  MttkrpPlan p;
  p.nnz = t->nnz;
  p.nunits = (int)units.size();
  p.nlong = (int)longs.size();
  p.nbig = nbig;
  p.nslots = nslots;
  int4 *du = nullptr, *dl = nullptr, *dul = nullptr;
  int *dus = nullptr;
  SACD_TRY(mem.get_t(units.size() + 1, &du));
  SACD_TRY(mem.get_t(longs.size() + 1, &dl));
  SACD_TRY(mem.get_t(units.size() + 1, &dus));
  SACD_TRY(mem.get_t(ulongs.size() + 1, &dul));
  if (!units.empty()) {
    HIP_TRY(hipMemcpyAsync(du, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice, t->stream));
    HIP_TRY(hipMemcpyAsync(dus, uslot.data(), sizeof(int) * units.size(), hipMemcpyHostToDevice, t->stream));
  }
  if (!longs.empty())
    HIP_TRY(hipMemcpyAsync(dl, longs.data(), sizeof(int4) * longs.size(), hipMemcpyHostToDevice, t->stream));
  if (!ulongs.empty())
    HIP_TRY(hipMemcpyAsync(dul, ulongs.data(), sizeof(int4) * ulongs.size(), hipMemcpyHostToDevice, t->stream));
  p.units = du;
  p.longs = dl;
  p.uslot = dus;
  p.ulongs = dul;
  p.nuslots = (int)std::count_if(uslot.begin(), uslot.end(), [](int v) { return v >= 0; });
  p.nulong = (int)ulongs.size();
  *out = p;
  // the arrays move (their buffers stay where the copies read them)
  hold->v4.push_back(std::move(units));
  hold->v4.push_back(std::move(longs));
  hold->v4.push_back(std::move(ulongs));
  hold->v1.push_back(std::move(uslot));
  return SACD_OK;
}

static sacd_status create_tensor_impl(sacd_tensor *t, const int64_t dims[3], int64_t nnz,
                                      const int32_t *idx, const float *vals) {
  const hipStream_t s = t->stream;
  int bits[3];
  for (int n = 0; n < 3; ++n) bits[n] = bits_for(dims[n]);
  for (int n = 0; n < 3; ++n) {
    int a, b;
    other_modes(n, &a, &b);
    t->lay[n].sh_n = bits[a] + bits[b];
    t->lay[n].sh_a = bits[b];
    t->lay[n].mask_a = (bits[a] == 0) ? 0ull : ((1ull << bits[a]) - 1ull);
    t->lay[n].mask_b = (bits[b] == 0) ? 0ull : ((1ull << bits[b]) - 1ull);
  }
  const int total_bits = bits[0] + bits[1] + bits[2];
  const long long n = nnz;
  DevAlloc tmp;  // ingest buffers, from the tensor's allocator, released at the end
  tmp.alloc = t->mem.alloc;
  tmp.custom = t->mem.custom;
  unsigned long long *k0 = nullptr, *k1 = nullptr;
  float *v0 = nullptr, *v1 = nullptr;
  int *err = nullptr, *cnt = nullptr;
  void *temp = nullptr;
  size_t tb = radix_sort_temp_bytes(n);
  if (dedup_temp_bytes(n) > tb) tb = dedup_temp_bytes(n);
  for (int m = 0; m < 3; ++m)
    if (build_ptr_temp_bytes(n, (int)dims[m]) > tb) tb = build_ptr_temp_bytes(n, (int)dims[m]);
  if (tb < 8192) tb = 8192;  // also holds the 512 + 1 doubles of the norm reduction
  sacd_status rs = SACD_OK;
  auto cleanup = [&]() { tmp.release_all(); };
#define TMP_TRY(expr)                 \
  do {                                \
    rs = (expr);                      \
    if (rs != SACD_OK) {              \
      cleanup();                      \
      return rs;                      \
    }                                 \
  } while (0)
#define TMP_HIP(expr)                                                                          \
  do {                                                                                         \
    hipError_t _e = (expr);                                                                    \
    if (_e != hipSuccess) {                                                                    \
      cleanup();                                                                               \
      return fail(SACD_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));            \
    }                                                                                          \
  } while (0)
  TMP_TRY(tmp.get_t(n > 0 ? n : 1, &k0));
  TMP_TRY(tmp.get_t(n > 0 ? n : 1, &k1));
  TMP_TRY(tmp.get_t(n > 0 ? n : 1, &v0));
  TMP_TRY(tmp.get_t(n > 0 ? n : 1, &v1));
  TMP_TRY(tmp.get_t(4, &err));
  TMP_TRY(tmp.get_t(4, &cnt));
  TMP_TRY(tmp.get(tb, &temp));
  TMP_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
  TMP_HIP(launch_make_keys0(idx, vals, n, dims, t->lay[0], k0, v0, err, s));
  // mode 0: stable sort by the full key, then merge duplicates; the error
  // flags and the count of distinct entries are read back together (with a
  // flag set, the sort and merge ran on keys that are discarded)
  bool in_alt = false;
  TMP_HIP(radix_sort_pairs(k0, v0, k1, v1, n, 0, total_bits, temp, s, &in_alt));
  unsigned long long *ks = in_alt ? k1 : k0;
  float *vs = in_alt ? v1 : v0;
  unsigned long long *kd = in_alt ? k0 : k1;  // free pair of buffers
  float *vd = in_alt ? v0 : v1;
  TMP_HIP(dedup_sorted(ks, vs, n, kd, vd, cnt, temp, s));
  int herr = 0, hcnt = 0;
  TMP_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  TMP_HIP(hipMemcpyAsync(&hcnt, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
  TMP_HIP(hipStreamSynchronize(s));
  if (herr & 1) {
    cleanup();
    return fail(SACD_ERR_OUT_OF_RANGE, "a coordinate is outside dims (%lld, %lld, %lld)",
                (long long)dims[0], (long long)dims[1], (long long)dims[2]);
  }
  if (herr & 2) {
    cleanup();
    return fail(SACD_ERR_NUMERIC, "a value is NaN or Inf");
  }
  const long long u = hcnt;
  t->nnz = u;
  for (int m = 0; m < 3; ++m) {
    TMP_TRY(t->mem.get_t((size_t)u + kKeySlack, &t->keys[m]));
    TMP_TRY(t->mem.get_t((size_t)u + kKeySlack, &t->vals[m]));
    TMP_TRY(t->mem.get_t((size_t)dims[m] + 1, &t->ptr[m]));
    TMP_HIP(hipMemsetAsync(t->keys[m] + u, 0, sizeof(unsigned long long) * kKeySlack, s));
    TMP_HIP(hipMemsetAsync(t->vals[m] + u, 0, sizeof(float) * kKeySlack, s));
  }
  if (u > 0) {
    TMP_HIP(hipMemcpyAsync(t->keys[0], kd, sizeof(unsigned long long) * u, hipMemcpyDeviceToDevice, s));
    TMP_HIP(hipMemcpyAsync(t->vals[0], vd, sizeof(float) * u, hipMemcpyDeviceToDevice, s));
  }
  // modes 1, 2: the mode-0 order sorted stably by i_n alone is (i_n, i_a, i_b) order
  for (int m = 1; m < 3; ++m) {
    TMP_HIP(launch_rekey(t->keys[0], u, t->lay[0], m, t->lay[m], k0, s));
    if (u > 0)
      TMP_HIP(hipMemcpyAsync(v0, t->vals[0], sizeof(float) * u, hipMemcpyDeviceToDevice, s));
    bool alt = false;
    TMP_HIP(radix_sort_pairs(k0, v0, k1, v1, u, t->lay[m].sh_n, t->lay[m].sh_n + bits[m], temp, s, &alt));
    if (u > 0) {
      TMP_HIP(hipMemcpyAsync(t->keys[m], alt ? k1 : k0, sizeof(unsigned long long) * u,
                             hipMemcpyDeviceToDevice, s));
      TMP_HIP(hipMemcpyAsync(t->vals[m], alt ? v1 : v0, sizeof(float) * u, hipMemcpyDeviceToDevice, s));
    }
  }
  for (int m = 0; m < 3; ++m)
    TMP_HIP(build_ptr(t->keys[m], u, t->lay[m].sh_n, (int)dims[m], t->ptr[m], temp, s));
  for (int m = 0; m < 3; ++m) {
    t->hptr[m].resize((size_t)dims[m] + 1);
    TMP_HIP(hipMemcpyAsync(t->hptr[m].data(), t->ptr[m], sizeof(int) * ((size_t)dims[m] + 1),
                           hipMemcpyDeviceToHost, s));
  }
  // ||X||^2, read back with the slice pointers
  {
    const int nparts = 512;
    double *part = (double *)temp;  // temp holds at least 512 doubles
    double *out = part + nparts;
    TMP_HIP(launch_norm2(t->vals[0], u, part, nparts, out, s));
    TMP_HIP(hipMemcpyAsync(&t->norm2, out, sizeof(double), hipMemcpyDeviceToHost, s));
    TMP_HIP(hipStreamSynchronize(s));
  }
  cleanup();
  return SACD_OK;
#undef TMP_TRY
#undef TMP_HIP
}

sacd_status sacd_create_tensor(const int64_t dims[3], int64_t nnz, const int32_t *idx, const float *vals,
                               const sacd_allocator *alloc, void *stream, sacd_tensor **out) {
  if (!out) return fail(SACD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!dims) return fail(SACD_ERR_INVALID_ARG, "dims is NULL");
  (void)hipGetLastError();
  for (int n = 0; n < 3; ++n)
    if (dims[n] < 1 || dims[n] > 2147483647LL)
      return fail(SACD_ERR_INVALID_ARG, "dims[%d] = %lld not in [1, 2^31 - 1]", n, (long long)dims[n]);
  if (nnz < 0 || nnz > 2147483647LL) return fail(SACD_ERR_INVALID_ARG, "nnz = %lld not in [0, 2^31 - 1]", (long long)nnz);
  if (nnz > 0 && (!idx || !vals)) return fail(SACD_ERR_INVALID_ARG, "idx / vals is NULL");
  if (alloc && (!alloc->alloc || !alloc->release)) return fail(SACD_ERR_INVALID_ARG, "allocator callbacks are NULL");
  if (bits_for(dims[0]) + bits_for(dims[1]) + bits_for(dims[2]) > 64)
    return fail(SACD_ERR_INVALID_ARG, "mode lengths need more than 64 key bits");
  sacd_tensor *t = new (std::nothrow) sacd_tensor();
  if (!t) return fail(SACD_ERR_NO_MEMORY, "host allocation failed");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete t;
    return fail(SACD_ERR_DEVICE, "no HIP device");
  }
  t->dev = dev;
  for (int n = 0; n < 3; ++n) t->dims[n] = dims[n];
  if (alloc) {
    t->mem.alloc = *alloc;
    t->mem.custom = true;
  }
  sacd_status st = make_stream(stream, &t->stream, &t->own_stream);
  if (st == SACD_OK) st = create_tensor_impl(t, dims, nnz, idx, vals);
  if (st != SACD_OK) {
    sacd_destroy_tensor(t);
    return st;
  }
  *out = t;
  return SACD_OK;
}

sacd_status sacd_tensor_info(const sacd_tensor *t, int64_t dims[3], int64_t *nnz, double *norm2,
                             int64_t *device_bytes) {
  if (!t) return fail(SACD_ERR_INVALID_ARG, "tensor is NULL");
  if (dims)
    for (int n = 0; n < 3; ++n) dims[n] = t->dims[n];
  if (nnz) *nnz = t->nnz;
  if (norm2) *norm2 = t->norm2;
  if (device_bytes) *device_bytes = t->mem.bytes;
  return SACD_OK;
}

sacd_status sacd_tensor_mode_coo(const sacd_tensor *t, int32_t mode, int32_t *coords, float *vals,
                                 int64_t *ptr) {
  if (!t) return fail(SACD_ERR_INVALID_ARG, "tensor is NULL");
  if (mode < 0 || mode > 2) return fail(SACD_ERR_INVALID_ARG, "mode %d not in {0, 1, 2}", mode);
  SACD_TRY(enter(t->dev));
  HIP_TRY(launch_export_coo(t->keys[mode], t->vals[mode], t->nnz, t->lay[mode], coords, vals,
                            t->ptr[mode], (int)t->dims[mode], ptr, t->stream));
  HIP_TRY(hipStreamSynchronize(t->stream));
  return SACD_OK;
}

static void release_tensor(sacd_tensor *t) {
  (void)hipSetDevice(t->dev);
  if (t->stream) (void)hipStreamSynchronize(t->stream);
  t->mem.release_all();
  if (t->own_stream && t->stream) (void)hipStreamDestroy(t->stream);
  delete t;
}

void sacd_destroy_tensor(sacd_tensor *t) {
  if (!t) return;
  if (t->nmodels > 0) {
    t->destroy_pending = true;  // released with its last model
    return;
  }
  release_tensor(t);
}

// ------------------------------------------------------------------- model --

// The tiled MTTKRP form applies to mode n of a row-form model at RP >= 64
// when A_b (the per-entry table) is too large for the LDS kernel's whole
// table and the tensor has at least kTileMinEntries entries (smaller ones
// keep the plain form: the copy and its sort would not pay).  The bits of
// the tile field must fit the key, and the (slice, tile) pairs number at
// most kTileMaxRuns.
constexpr long long kTileMinEntries = 1ll << 20;
constexpr long long kTileMaxRuns = 1ll << 24;  // slices x tiles of a tiled mode, at most

static int tile_bits(long long Ib) { return bits_for((Ib + kTileRows - 1) / kTileRows); }

static bool tiled_mode(const int64_t dims[3], long long nnz, int RP, int cb, int n) {
  int a, b;
  other_modes(n, &a, &b);
  if (cb != 0 || RP < 64 || nnz < kTileMinEntries || mttkrp_lds_cols(RP, dims[b]) != 0) return false;
  const int tb = tile_bits(dims[b]);
  if (bits_for(dims[0]) + bits_for(dims[1]) + bits_for(dims[2]) + tb > 64) return false;
  // (slice, tile) offsets are built on the host and the device: keep them modest
  return ((long long)dims[n] << tb) <= kTileMaxRuns;
}

// Tiled copy of mode n's entries and its plan: keys in (i_n, i_b tile, i_a,
// i_b) order (a stable sort of the mode's order on (i_n, tile)); units are
// segments of at most kSegment entries of one (slice, tile) run, grouped by
// tile, tile by tile, slice by slice; a block of the LDS kernel takes up to
// its units-per-block of one tile.  A slice with more than one unit is split
// (its units' sums meet in the fix-up's slots).
static sacd_status build_tiled(sacd_model *m, int n, MttkrpPlan *out) {
  sacd_tensor *t = m->t;
  const hipStream_t s = m->s;
  const long long u = t->nnz;
  int a, b;
  other_modes(n, &a, &b);
  const int I = (int)t->dims[n];
  const long long Ib = t->dims[b];
  const int ntiles = (int)((Ib + kTileRows - 1) / kTileRows);
  const int tb = tile_bits(Ib);
  const int tsh = bits_for(kTileRows);
  const KeyLayout &lay = t->lay[n];
  const int Isup = I << tb;  // (slice, tile) pairs
  DevAlloc tmp;
  tmp.alloc = m->mem.alloc;
  tmp.custom = m->mem.custom;
  sacd_status rs = SACD_OK;
#define TL_TRY(expr)         \
  do {                       \
    rs = (expr);             \
    if (rs != SACD_OK) {     \
      tmp.release_all();     \
      return rs;             \
    }                        \
  } while (0)
#define TL_HIP(expr)                                                                \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      tmp.release_all();                                                            \
      return fail(SACD_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));  \
    }                                                                               \
  } while (0)
  unsigned long long *k0 = nullptr, *k1 = nullptr;
  float *v0 = nullptr, *v1 = nullptr;
  int *ptr = nullptr;
  void *temp = nullptr;
  const size_t tbytes = std::max(radix_sort_temp_bytes(u), build_ptr_temp_bytes(u, Isup));
  TL_TRY(tmp.get_t((size_t)u, &k0));
  TL_TRY(tmp.get_t((size_t)u, &k1));
  TL_TRY(tmp.get_t((size_t)u, &v0));
  TL_TRY(tmp.get_t((size_t)u, &v1));
  TL_TRY(tmp.get_t((size_t)Isup + 1, &ptr));
  TL_TRY(tmp.get(tbytes, &temp));
  TL_HIP(launch_tile_keys(t->keys[n], u, lay, tsh, tb, k0, s));
  TL_HIP(hipMemcpyAsync(v0, t->vals[n], sizeof(float) * u, hipMemcpyDeviceToDevice, s));
  bool alt = false;
  TL_HIP(radix_sort_pairs(k0, v0, k1, v1, u, lay.sh_n, lay.sh_n + tb + bits_for(I), temp, s, &alt));
  TL_TRY(m->mem.get_t((size_t)u + kKeySlack, &m->tkeys[n]));
  TL_TRY(m->mem.get_t((size_t)u + kKeySlack, &m->tvals[n]));
  TL_HIP(hipMemcpyAsync(m->tkeys[n], alt ? k1 : k0, sizeof(unsigned long long) * u, hipMemcpyDeviceToDevice, s));
  TL_HIP(hipMemcpyAsync(m->tvals[n], alt ? v1 : v0, sizeof(float) * u, hipMemcpyDeviceToDevice, s));
  TL_HIP(hipMemsetAsync(m->tkeys[n] + u, 0, sizeof(unsigned long long) * kKeySlack, s));
  TL_HIP(hipMemsetAsync(m->tvals[n] + u, 0, sizeof(float) * kKeySlack, s));
  // (slice, tile) run offsets: the key >> sh_n is slice * 2^tb + tile
  TL_HIP(build_ptr(m->tkeys[n], u, lay.sh_n, Isup, ptr, temp, s));
  std::vector<int> hp((size_t)Isup + 1);
  TL_HIP(hipMemcpyAsync(hp.data(), ptr, sizeof(int) * ((size_t)Isup + 1), hipMemcpyDeviceToHost, s));
  TL_HIP(hipStreamSynchronize(s));
  tmp.release_all();
#undef TL_TRY
#undef TL_HIP
  const int upb = mttkrp_lds_units_per_block(64);
  std::vector<int4> units, blocks;
  std::vector<int> block_of, units_of_slice((size_t)I, 0);
  for (int tl = 0; tl < ntiles; ++tl) {
    const int first = (int)units.size();
    for (int r = 0; r < I; ++r) {
      const int beg = hp[((size_t)r << tb) + tl], end = hp[((size_t)r << tb) + tl + 1];
      for (int q = beg; q < end; q += kSegment) {
        units.push_back(make_int4(r, q, std::min(kSegment, end - q), 0));
        units_of_slice[r] += 1;
      }
    }
    const int b0 = tl * kTileRows, rows = (int)std::min<long long>(kTileRows, Ib - b0);
    for (int u0 = first; u0 < (int)units.size(); u0 += upb) {
      const int nu = std::min(upb, (int)units.size() - u0);
      for (int k = 0; k < nu; ++k) block_of.push_back((int)blocks.size());
      blocks.push_back(make_int4(u0, nu, b0, rows));
    }
  }
  for (int4 &x : units) x.w = units_of_slice[x.x] > 1 ? -2 : -1;
  std::vector<int4> longs;
  const int nslots = number_runs(units, upb, &longs, &block_of);
  const int nbig = order_longs(&longs);
  MttkrpPlan p{};
  p.nnz = u;
  p.nunits = (int)units.size();
  p.nlong = (int)longs.size();
  p.nbig = nbig;
  p.nslots = nslots;
  int4 *du = nullptr, *dl = nullptr, *db = nullptr;
  SACD_TRY(m->mem.get_t(units.size() + 1, &du));
  SACD_TRY(m->mem.get_t(longs.size() + 1, &dl));
  SACD_TRY(m->mem.get_t(blocks.size() + 1, &db));
  if (!units.empty())
    HIP_TRY(hipMemcpyAsync(du, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice, s));
  if (!longs.empty())
    HIP_TRY(hipMemcpyAsync(dl, longs.data(), sizeof(int4) * longs.size(), hipMemcpyHostToDevice, s));
  if (!blocks.empty())
    HIP_TRY(hipMemcpyAsync(db, blocks.data(), sizeof(int4) * blocks.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  p.units = du;
  p.longs = dl;
  *out = p;
  m->btab[n] = db;
  m->nbt[n] = (int)blocks.size();
  return SACD_OK;
}

static sacd_status init_model_impl(sacd_model *m, uint64_t seed) {
  sacd_tensor *t = m->t;
  const int RP = m->RP;
  DevAlloc &A = m->mem;
  int maxI = 0;
  long long maxslots = 1;
  HostHold hold;  // plan arrays in flight until the wait at the end
  hold.s = t->stream;
  for (int n = 0; n < 3; ++n) {
    const int I = (int)t->dims[n];
    if (I > maxI) maxI = I;
    if (tiled_mode(t->dims, t->nnz, RP, m->cb, n)) {
      SACD_TRY(build_tiled(m, n, &m->plan[n]));
    } else {
      SACD_TRY(build_plan(t, n, mttkrp_units_per_block(RP), A, &m->plan[n], &hold));
      int a, b;
      other_modes(n, &a, &b);
      m->lds_cols[n] = mttkrp_lds_cols(RP, t->dims[b]);
    }
    if (m->plan[n].nslots > maxslots) maxslots = m->plan[n].nslots;
    m->nparts[n] = (I + rows_per_block(RP) - 1) / rows_per_block(RP);
    SACD_TRY(A.get_t((size_t)I * RP, &m->A[n]));
    SACD_TRY(A.get_t((size_t)I * RP, &m->Z[n]));
    if (m->cb == 0) SACD_TRY(A.get_t((size_t)I * RP, &m->M[n]));  // the column form holds I x cb only
    SACD_TRY(A.get_t((size_t)RP * RP, &m->H[n]));
    SACD_TRY(A.get_t((size_t)RP * RP, &m->G64[n]));
    if (m->prec == SACD_PREC_MIXED_BF16) SACD_TRY(A.get_t((size_t)RP * RP, &m->G64o[n]));
    else m->G64o[n] = m->G64[n];
    SACD_TRY(A.get_t(1, &m->hinfo[n]));
    SACD_TRY(A.get_t((size_t)RP, &m->colcnt[n]));
    if (m->cb == 0) SACD_TRY(A.get_t((size_t)I * RP, &m->selmask[n]));  // column form: with the diagnostics
  }
  const int maxparts = (maxI + rows_per_block(RP) - 1) / rows_per_block(RP);
  SACD_TRY(A.get_t(3, &m->st));
  SACD_TRY(A.get_t((size_t)maxslots * RP, &m->part));
  SACD_TRY(A.get_t((size_t)maxparts * RP * RP, &m->gpart));
  if (m->prec == SACD_PREC_MIXED_BF16) SACD_TRY(A.get_t((size_t)maxparts * RP * RP, &m->gpart_obj));
  // one importance partial per importance block (blocks of its own size)
  SACD_TRY(A.get_t((size_t)std::max(maxparts, importance_blocks(RP, (int)maxI)), &m->ti_part));
  SACD_TRY(A.get_t((size_t)maxparts, &m->inner_part));
  SACD_TRY(A.get_t((size_t)maxparts * RP, &m->cnt_part));
  SACD_TRY(A.get_t((size_t)gram_model_parts(RP), &m->mpart));
  if (m->cb > 0) {
    int maxus = 1, maxcp = 1;
    for (int n = 0; n < 3; ++n) {
      maxus = std::max(maxus, m->plan[n].nuslots);
      const int Rc = (m->R + m->cb - 1) / m->cb * m->cb;
      maxcp = std::max(maxcp, (Rc / m->cb) * col_row_blocks((int)t->dims[n]));
    }
    SACD_TRY(A.get_t((size_t)maxI * m->cb, &m->Mb));
    SACD_TRY(A.get_t((size_t)maxus * m->cb, &m->upart));
    SACD_TRY(A.get_t(((size_t)maxI * RP + 15) / 16, &m->bits));
    SACD_TRY(A.get_t((size_t)maxcp, &m->colpart));
  }
  SACD_TRY(A.get_t(1, &m->gcounter));
  SACD_TRY(A.get_t(4, &m->flag));
  m->full_nparts = 1024;
  SACD_TRY(A.get_t((size_t)m->full_nparts, &m->full_part));
  SACD_TRY(A.get_t(1, &m->full_out));
  SACD_TRY(A.get_t(4, &m->full_cnt));
  SACD_TRY(pinned_get(&m->h_pinned));
  hipStream_t s = m->s;
  HIP_TRY(hipMemsetAsync(m->st, 0, 3 * sizeof(ModeState), s));
  HIP_TRY(hipMemsetAsync(m->full_cnt, 0, 16, s));
  HIP_TRY(hipMemsetAsync(m->gcounter, 0, sizeof(unsigned), s));
  unsigned long long off = 0;
  for (int n = 0; n < 3; ++n) {
    const int I = (int)t->dims[n];
    HIP_TRY(launch_init_factor(m->A[n], I, m->R, RP, seed, off, s));
    off += (unsigned long long)I * m->R;
    HIP_TRY(hipMemsetAsync(m->Z[n], 0, sizeof(float) * I * RP, s));
    // empty slices are never written by the MTTKRP: their rows stay zero
    if (m->M[n]) HIP_TRY(hipMemsetAsync(m->M[n], 0, sizeof(float) * I * RP, s));
    if (m->selmask[n]) HIP_TRY(hipMemsetAsync(m->selmask[n], 0, (size_t)I * RP, s));
    HIP_TRY(hipMemsetAsync(m->colcnt[n], 0, sizeof(long long) * RP, s));
  }
  for (int n = 0; n < 3; ++n) SACD_TRY(recompute_gram(m, n));
  HIP_TRY(hipStreamSynchronize(s));
  return SACD_OK;
}

static sacd_status init_factors_impl(sacd_tensor *t, int32_t R, uint64_t seed, sacd_precision prec,
                                     sacd_update update, int32_t cb, sacd_model **out);

sacd_status sacd_init_factors(sacd_tensor *t, int32_t R, uint64_t seed, sacd_precision prec,
                              sacd_update update, sacd_model **out) {
  return init_factors_impl(t, R, seed, prec, update, 0, out);
}

sacd_status sacd_init_factors_columns(sacd_tensor *t, int32_t R, uint64_t seed, int32_t column_block,
                                      sacd_model **out) {
  if (column_block != 1 && column_block != 2 && column_block != 4 && column_block != 8 && column_block != 16) {
    if (out) *out = nullptr;
    return fail(SACD_ERR_INVALID_ARG, "column_block %d not in {1, 2, 4, 8, 16}", column_block);
  }
  return init_factors_impl(t, R, seed, SACD_PREC_FP32, SACD_UPDATE_GS, column_block, out);
}

static sacd_status init_factors_impl(sacd_tensor *t, int32_t R, uint64_t seed, sacd_precision prec,
                                     sacd_update update, int32_t cb, sacd_model **out) {
  if (!out) return fail(SACD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!t) return fail(SACD_ERR_INVALID_ARG, "tensor is NULL");
  if (R < 1 || R > kMaxRP) return fail(SACD_ERR_INVALID_ARG, "rank %d not in [1, %d]", R, kMaxRP);
  if (prec != SACD_PREC_FP32 && prec != SACD_PREC_MIXED_BF16)
    return fail(SACD_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
  if (update != SACD_UPDATE_GS && update != SACD_UPDATE_JACOBI)
    return fail(SACD_ERR_INVALID_ARG, "unknown update rule %d", (int)update);
  SACD_TRY(enter(t->dev));
  void *scratch_dev = nullptr;  // set-up of the allocation-free entry point on this device
  SACD_TRY(static_scratch(t->dev, &scratch_dev));
  sacd_model *m = new (std::nothrow) sacd_model();
  if (!m) return fail(SACD_ERR_NO_MEMORY, "host allocation failed");
  m->t = t;
  m->s = t->stream;
  m->mem.alloc = t->mem.alloc;
  m->mem.custom = t->mem.custom;
  m->R = R;
  m->RP = R <= 16 ? 16 : R <= 32 ? 32 : R <= 64 ? 64 : 128;
  m->prec = prec;
  m->upd = update;
  m->cb = cb;
  sacd_status st = init_model_impl(m, seed);
  if (st != SACD_OK) {
    sacd_destroy_model(m);
    return st;
  }
  t->nmodels++;
  m->counted = true;
  m->last_mode = -1;
  m->dirty = true;
  *out = m;
  return SACD_OK;
}

sacd_status sacd_sweep(sacd_model *m, int32_t mode) {
  SACD_TRY(check_mode(m, mode));
  SACD_TRY(enter(m->t->dev));
  SACD_TRY(enqueue_sweep(m, mode));
  m->last_mode = mode;
  m->dirty = false;
  return SACD_OK;
}

sacd_status sacd_iterate(sacd_model *m, int32_t n_iters) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  if (n_iters < 0) return fail(SACD_ERR_INVALID_ARG, "n_iters < 0");
  if (n_iters == 0) return SACD_OK;
  SACD_TRY(enter(m->t->dev));
  SACD_TRY(ensure_graph(m));
  for (int i = 0; i < n_iters; ++i) HIP_TRY(hipGraphLaunch(m->gexec, m->s));
  m->last_mode = 2;
  m->dirty = false;
  return SACD_OK;
}

sacd_status sacd_timing_prepare(sacd_model *m, int32_t n_iters) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  if (n_iters < 1 || n_iters > 100000) return fail(SACD_ERR_INVALID_ARG, "n_iters out of [1, 100000]");
  SACD_TRY(enter(m->t->dev));
  while ((int)m->tev.size() < 9 * n_iters) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    m->tev.push_back(e);
  }
  return SACD_OK;
}

sacd_status sacd_iterate_timed(sacd_model *m, int32_t n_iters, float *mttkrp_ms, float *sweep_ms) {
  if (!m || !mttkrp_ms) return fail(SACD_ERR_INVALID_ARG, "model or output is NULL");
  if (n_iters < 1 || 9 * n_iters > (int)m->tev.size())
    return fail(SACD_ERR_BAD_STATE, "sacd_timing_prepare was not called for %d iterations", (int)n_iters);
  SACD_TRY(enter(m->t->dev));
  for (int i = 0; i < n_iters; ++i)
    for (int n = 0; n < 3; ++n) SACD_TRY(enqueue_sweep(m, n, &m->tev[9 * i + 3 * n]));
  m->last_mode = 2;
  m->dirty = false;
  HIP_TRY(hipStreamSynchronize(m->s));
  for (int i = 0; i < n_iters; ++i)
    for (int n = 0; n < 3; ++n) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, m->tev[9 * i + 3 * n], m->tev[9 * i + 3 * n + 1]));
      mttkrp_ms[3 * i + n] = ms;
      if (sweep_ms) {
        HIP_TRY(hipEventElapsedTime(&ms, m->tev[9 * i + 3 * n], m->tev[9 * i + 3 * n + 2]));
        sweep_ms[3 * i + n] = ms;
      }
    }
  return SACD_OK;
}

sacd_status sacd_fit(sacd_model *m, double *fit, double *objective) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  SACD_TRY(enter(m->t->dev));
  double f = 0.0;
  if (m->last_mode < 0 || m->dirty) {
    SACD_TRY(objective_full(m, &f));
  } else {
    ModeState s;
    SACD_TRY(read_state(m, m->last_mode, &s));
    f = s.f;
  }
  if (objective) *objective = f;
  if (!(m->t->norm2 > 0.0)) return fail(SACD_ERR_NUMERIC, "||X|| = 0: the fit is undefined");
  if (fit) *fit = 1.0 - std::sqrt(f > 0.0 ? f : 0.0) / std::sqrt(m->t->norm2);
  return SACD_OK;
}

sacd_status sacd_rmse(sacd_model *m, int64_t n, const int32_t *idx, const float *vals, double *rmse) {
  if (!m || !rmse || n < 0 || (n > 0 && (!idx || !vals))) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  if (n == 0) {
    *rmse = 0.0;
    return SACD_OK;
  }
  SACD_TRY(enter(m->t->dev));
  HIP_TRY(hipMemsetAsync(m->flag, 0, sizeof(int), m->s));
  HIP_TRY(launch_sq_error(idx, vals, n, m->t->dims, m->RP, m->A[0], m->A[1], m->A[2], m->full_part,
                          m->full_nparts, m->full_out, m->full_cnt, m->flag, m->s));
  HIP_TRY(hipMemcpyAsync(m->h_pinned, m->full_out, sizeof(double), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipMemcpyAsync(m->h_pinned + 1, m->flag, sizeof(int), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  int bad = 0;
  std::memcpy(&bad, m->h_pinned + 1, sizeof(int));
  if (bad) return fail(SACD_ERR_OUT_OF_RANGE, "a coordinate is outside the tensor's dims");
  *rmse = std::sqrt(m->h_pinned[0] / (double)n);
  return SACD_OK;
}

sacd_status sacd_rmse_static(const sacd_model *m, int64_t n, const int32_t *idx, const float *vals, double *out) {
  if (!m || !out || n < 0 || (n > 0 && (!idx || !vals))) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  if (n > kStaticMaxEntries)
    return fail(SACD_ERR_INVALID_ARG, "n = %lld entries is beyond the maximum %lld of sacd_rmse_static", (long long)n,
                kStaticMaxEntries);
  SACD_TRY(enter(m->t->dev));
  void *base = nullptr;
  SACD_TRY(static_scratch(m->t->dev, &base));
  double *part = (double *)base;           // kStaticParts partial sums
  double *sum = part + kStaticParts;       // their total
  unsigned *counter = (unsigned *)(sum + 1);
  int *bad = (int *)(counter + 1);
  // the arrival counter and the flag start at zero (the array keeps the last
  // call's contents); a fill kernel, not a memset
  HIP_TRY(launch_zero_words(counter, 2, m->s));
  HIP_TRY(launch_sq_error(idx, vals, n, m->t->dims, m->RP, m->A[0], m->A[1], m->A[2], part, kStaticParts, sum,
                          counter, bad, m->s));
  HIP_TRY(launch_rmse_finish(sum, bad, n, out, m->s));
  return SACD_OK;
}

sacd_status sacd_pd(const sacd_model *m, int32_t mode, double *pd) {
  SACD_TRY(check_mode(m, mode));
  if (!pd) return fail(SACD_ERR_INVALID_ARG, "pd is NULL");
  SACD_TRY(enter(m->t->dev));
  const int RP = m->RP, R = m->R;
  std::vector<double> G((size_t)RP * RP);
  HIP_TRY(hipMemcpyAsync(G.data(), m->G64o[mode], sizeof(double) * RP * RP, hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  // cosine of columns i < r from the Gram matrix of the factor
  double sum = 0.0;
  long long pairs = 0;
  for (int i = 0; i < R; ++i)
    for (int r = i + 1; r < R; ++r) {
      const double gi = G[(size_t)i * RP + i], gr = G[(size_t)r * RP + r];
      if (gi > 0.0 && gr > 0.0) {
        sum += G[(size_t)i * RP + r] / (std::sqrt(gi) * std::sqrt(gr));
        ++pairs;
      }
    }
  *pd = pairs > 0 ? sum / (double)pairs : 0.0;
  return SACD_OK;
}

sacd_status sacd_run_until(sacd_model *m, double tol, int32_t max_iter, int32_t *iters_done,
                           double *final_fit) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  if (max_iter < 1 || !(tol >= 0.0)) return fail(SACD_ERR_INVALID_ARG, "max_iter < 1 or tol < 0");
  if (!(m->t->norm2 > 0.0)) return fail(SACD_ERR_NUMERIC, "||X|| = 0: the fit is undefined");
  SACD_TRY(enter(m->t->dev));
  SACD_TRY(ensure_graph(m));
  const double nx = std::sqrt(m->t->norm2);
  double prev = 0.0, fit = 0.0;
  int it;
  for (it = 1; it <= max_iter; ++it) {
    HIP_TRY(hipGraphLaunch(m->gexec, m->s));
    HIP_TRY(hipMemcpyAsync(m->h_pinned, &m->st[2].f, sizeof(double), hipMemcpyDeviceToHost, m->s));
    HIP_TRY(hipStreamSynchronize(m->s));
    m->last_mode = 2;
    m->dirty = false;
    const double f = m->h_pinned[0];
    fit = 1.0 - std::sqrt(f > 0.0 ? f : 0.0) / nx;
    if (it >= 2 && std::fabs(fit - prev) < tol * std::fabs(prev)) break;
    prev = fit;
  }
  if (it > max_iter) it = max_iter;
  if (iters_done) *iters_done = it;
  if (final_fit) *final_fit = fit;
  return SACD_OK;
}

sacd_status sacd_get_factor(const sacd_model *m, int32_t mode, float *dst) {
  SACD_TRY(check_mode(m, mode));
  if (!dst) return fail(SACD_ERR_INVALID_ARG, "dst is NULL");
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  HIP_TRY(launch_copy_rows(m->A[mode], m->RP, dst, m->R, I, m->R, m->R, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

sacd_status sacd_set_factor(sacd_model *m, int32_t mode, const float *src) {
  SACD_TRY(check_mode(m, mode));
  if (!src) return fail(SACD_ERR_INVALID_ARG, "src is NULL");
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  HIP_TRY(hipMemsetAsync(m->flag, 0, sizeof(int), m->s));
  HIP_TRY(launch_check_factor(src, (long long)I * m->R, m->flag, m->s));
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, m->flag, sizeof(int), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  if (hflag) return fail(SACD_ERR_NUMERIC, "factor has negative or non-finite entries");
  HIP_TRY(launch_copy_rows(src, m->R, m->A[mode], m->RP, I, m->R, m->RP, m->s));
  SACD_TRY(recompute_gram(m, mode));
  HIP_TRY(hipStreamSynchronize(m->s));
  m->dirty = true;
  return SACD_OK;
}

sacd_status sacd_get_state(const sacd_model *m, int32_t mode, float *zprev, double *ti_prev, int64_t *k) {
  SACD_TRY(check_mode(m, mode));
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  if (zprev) HIP_TRY(launch_copy_rows(m->Z[mode], m->RP, zprev, m->R, I, m->R, m->R, m->s));
  ModeState s;
  SACD_TRY(read_state(m, mode, &s));
  if (ti_prev) *ti_prev = s.ti_prev;
  if (k) *k = s.k;
  return SACD_OK;
}

sacd_status sacd_set_state(sacd_model *m, int32_t mode, const float *zprev, double ti_prev, int64_t k) {
  SACD_TRY(check_mode(m, mode));
  if (k < 0) return fail(SACD_ERR_INVALID_ARG, "k < 0");
  if (k > 0 && !zprev) return fail(SACD_ERR_INVALID_ARG, "zprev is NULL with k > 0");
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  if (zprev) HIP_TRY(launch_copy_rows(zprev, m->R, m->Z[mode], m->RP, I, m->R, m->RP, m->s));
  ModeState s;
  SACD_TRY(read_state(m, mode, &s));
  s.k = k;
  s.ti_prev = ti_prev;
  HIP_TRY(hipMemcpyAsync(m->st + mode, &s, sizeof(ModeState), hipMemcpyHostToDevice, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

sacd_status sacd_get_stats(const sacd_model *m, int32_t mode, sacd_sweep_stats *out) {
  SACD_TRY(check_mode(m, mode));
  if (!out) return fail(SACD_ERR_INVALID_ARG, "out is NULL");
  SACD_TRY(enter(m->t->dev));
  ModeState s;
  SACD_TRY(read_state(m, mode, &s));
  out->k = s.k;
  out->lipschitz = s.L;
  out->ti = s.ti;
  out->flip = s.flip;
  out->n_selected = s.nsel;
  out->objective = s.f;
  return SACD_OK;
}

sacd_status sacd_get_column_counts(const sacd_model *m, int32_t mode, int64_t *counts) {
  SACD_TRY(check_mode(m, mode));
  if (!counts) return fail(SACD_ERR_INVALID_ARG, "counts is NULL");
  SACD_TRY(enter(m->t->dev));
  std::vector<long long> c((size_t)m->RP);
  HIP_TRY(hipMemcpyAsync(c.data(), m->colcnt[mode], sizeof(long long) * m->RP, hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  for (int r = 0; r < m->R; ++r) counts[r] = (int64_t)c[(size_t)r];
  return SACD_OK;
}

sacd_status sacd_get_diagnostics(const sacd_model *m, int32_t mode, float *mttkrp, uint8_t *selection,
                                 double *gram) {
  SACD_TRY(check_mode(m, mode));
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  const int R = m->R, RP = m->RP;
  if ((mttkrp || selection) && !m->M[mode])
    return fail(SACD_ERR_BAD_STATE, "the column-at-a-time form records M and the selection only with diagnostics on");
  if (mttkrp) HIP_TRY(launch_copy_rows(m->M[mode], RP, mttkrp, R, I, R, R, m->s));
  if (selection) {
    HIP_TRY(hipMemcpy2DAsync(selection, (size_t)R, m->selmask[mode], (size_t)RP, (size_t)R, (size_t)I,
                             hipMemcpyDeviceToDevice, m->s));
  }
  if (gram) {
    std::vector<double> G((size_t)RP * RP);
    HIP_TRY(hipMemcpyAsync(G.data(), m->G64[mode], sizeof(double) * RP * RP, hipMemcpyDeviceToHost, m->s));
    HIP_TRY(hipStreamSynchronize(m->s));
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < R; ++j) gram[i * R + j] = G[(size_t)i * RP + j];
  }
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

sacd_status sacd_set_diagnostics(sacd_model *m, int32_t enable) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  const bool d = enable != 0;
  if (d != m->diag) {
    SACD_TRY(enter(m->t->dev));
    HIP_TRY(hipStreamSynchronize(m->s));
    drop_graph(m);
    if (d && m->cb > 0 && !m->M[0]) {
      // the column form keeps no whole M: the diagnostics get their own
      for (int n = 0; n < 3; ++n) {
        const size_t IR = (size_t)m->t->dims[n] * m->RP;
        SACD_TRY(m->mem.get_t(IR, &m->M[n]));
        SACD_TRY(m->mem.get_t(IR, &m->selmask[n]));
        HIP_TRY(hipMemsetAsync(m->M[n], 0, sizeof(float) * IR, m->s));
        HIP_TRY(hipMemsetAsync(m->selmask[n], 0, IR, m->s));
      }
      HIP_TRY(hipStreamSynchronize(m->s));
    }
    m->diag = d;
  }
  return SACD_OK;
}

sacd_status sacd_time_kernel(sacd_model *m, int32_t which, int32_t mode, int32_t reps, float *avg_ms) {
  SACD_TRY(check_mode(m, mode));
  if (which < 0 || which > 2 || reps < 1 || !avg_ms) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  if (m->cb > 0) return fail(SACD_ERR_BAD_STATE, "kernel timing applies to the row form only");
  SACD_TRY(enter(m->t->dev));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  // a save of the mode's selection state, so that timing does not advance it
  ModeState saved;
  SACD_TRY(read_state(m, mode, &saved));
  HIP_TRY(hipEventRecord(e0, m->s));
  for (int i = 0; i < reps; ++i) {
    if (which == 0)
      HIP_TRY(launch_mode_mttkrp(m, mode, m->s));
    else if (which == 1)
      HIP_TRY(launch_select_update(m->RP, (int)m->upd, m->diag, is_bf16(m), upd_args(m, mode), m->s));
    else
      HIP_TRY(launch_importance(m->RP, is_bf16(m), imp_args(m, mode), m->s));
  }
  HIP_TRY(hipEventRecord(e1, m->s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = ms / reps;
  if (which == 0) {
    // restore the complete MTTKRP (spanning slices) for later sweeps' diagnostics
    HIP_TRY(launch_mttkrp_fix(m->RP, fix_args(m, mode), m->s));
  }
  HIP_TRY(hipMemcpyAsync(m->st + mode, &saved, sizeof(ModeState), hipMemcpyHostToDevice, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

sacd_status sacd_kernel_bytes(const sacd_model *m, int32_t which, int32_t mode, double *bytes) {
  SACD_TRY(check_mode(m, mode));
  if (!bytes || which < 0 || which > 2) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  const sacd_tensor *t = m->t;
  int a, b;
  other_modes(mode, &a, &b);
  const double R = m->R, I = (double)t->dims[mode];
  if (which == 0) {
    // stream 12 B per entry (8 B key, 4 B value); each factor row of A_a, A_b
    // read once; M written once
    *bytes = 12.0 * (double)t->nnz + 4.0 * R * ((double)t->dims[a] + (double)t->dims[b]) + 4.0 * R * I;
  } else if (which == 1) {
    // read A, M, Z; write A, Z
    *bytes = 20.0 * R * I;
  } else {
    // read A, M
    *bytes = 8.0 * R * I;
  }
  return SACD_OK;
}

sacd_status sacd_model_bytes(const sacd_model *m, int64_t *bytes) {
  if (!m || !bytes) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  *bytes = m->mem.bytes;
  return SACD_OK;
}

void sacd_destroy_model(sacd_model *m) {
  if (!m) return;
  sacd_tensor *t = m->t;
  (void)hipSetDevice(t->dev);
  if (m->s) (void)hipStreamSynchronize(m->s);
  drop_graph(m);
  for (hipEvent_t e : m->tev) (void)hipEventDestroy(e);
  m->tev.clear();
  m->mem.release_all();
  pinned_put(m->h_pinned);
  const bool counted = m->counted;
  delete m;
  if (counted && t->nmodels > 0) t->nmodels--;
  if (t->destroy_pending && t->nmodels == 0) release_tensor(t);
}

}  // extern "C"

// ----------------------------------------------------------------- serving --
//
// Many independent factorization jobs resident on one GPU.  Each job is a
// tensor plus a model with its own buffers; an iteration of the server runs
// one outer iteration of every running job with job-batched launches: per
// mode and per padded rank, one launch of each of the five sweep kernels
// covers the blocks of all jobs of that rank (a block map gives each block
// its job and its block index within the job).  The blocks of a job are the
// ones its solo launches would run, so each job's arithmetic -- partials and
// their reduction order -- is the same as alone: results are bit-identical
// alone and in the mix.

namespace {

int64_t al256(int64_t b) { return ((b > 0 ? b : 16) + 255) & ~(int64_t)255; }

int pad_rank(int R) { return R <= 16 ? 16 : (R <= 32 ? 32 : (R <= 64 ? 64 : 128)); }

// Upper bounds of the device bytes of a job: resident (tensor + model) and
// the transient ingest buffers.
void job_bytes(const int64_t dims[3], int64_t nnz, int R, bool mixed, int64_t *resident, int64_t *transient) {
  const int RP = pad_rank(R);
  const int64_t slack = 64 * 1024;
  int64_t maxI = 0, maxunits = 0, ten = 0, mod = 0;
  for (int n = 0; n < 3; ++n) {
    const int64_t I = dims[n];
    maxI = std::max(maxI, I);
    const int64_t units = nnz / kSegment + I + 2;
    maxunits = std::max(maxunits, units);
    ten += al256(8 * (nnz + kKeySlack)) + al256(4 * (nnz + kKeySlack)) + al256(4 * (I + 1)) + al256(16 * units) +
           al256(16 * (I + 2)) + al256(4 * (units + 1)) + al256(16 * (I + 2));
    mod += 3 * al256(4 * I * RP) + al256(I * RP) + 2 * al256(4 * RP * RP) + al256(8 * RP * RP) +
           al256(sizeof(HInfo)) + al256(8 * RP);
  }
  const int64_t parts = (maxI + rows_per_block(RP) - 1) / rows_per_block(RP);
  const int64_t iparts = std::max(parts, (int64_t)importance_blocks(RP, (int)maxI));
  mod += al256(3 * sizeof(ModeState)) + al256(4 * maxunits * RP) + al256(4 * parts * RP * RP) +
         al256(8 * iparts) + al256(8 * parts) + al256(4 * parts * RP) + al256(8 * gram_model_parts(RP)) + al256(8 * 1024) +
         6 * 256;
  if (mixed) mod += al256(4 * parts * RP * RP) + 3 * al256(8 * RP * RP);  // the objective's Gram partials and Grams
  int64_t tb = (int64_t)radix_sort_temp_bytes(nnz);
  tb = std::max(tb, (int64_t)dedup_temp_bytes(nnz));
  for (int n = 0; n < 3; ++n) tb = std::max(tb, (int64_t)build_ptr_temp_bytes(nnz, (int)dims[n]));
  // tiled MTTKRP copies (modes in the tiled form): keys, values, units, slots
  // and block table resident; the sort buffers and (slice, tile) offsets
  // transient, while the model is set up (after the ingest buffers are gone)
  int64_t tiled_res = 0, tiled_tr = 0;
  for (int n = 0; n < 3; ++n) {
    if (!tiled_mode(dims, nnz, RP, 0, n)) continue;
    int a, b;
    other_modes(n, &a, &b);
    const int tbits = tile_bits(dims[b]);
    const int64_t runs = std::min<int64_t>(nnz, dims[n] << tbits);
    const int64_t units = nnz / kSegment + runs + 2;
    tiled_res += al256(8 * (nnz + kKeySlack)) + al256(4 * (nnz + kKeySlack)) + al256(16 * (units + 1)) +
                 al256(16 * (dims[n] + 2)) + al256(16 * (units + 1)) + al256(4 * units * RP);
    tiled_tr = std::max(tiled_tr, 2 * al256(8 * nnz) + 2 * al256(4 * nnz) + al256(4 * ((dims[n] << tbits) + 1)) +
                                      al256((int64_t)std::max(radix_sort_temp_bytes(nnz),
                                                              build_ptr_temp_bytes(nnz, (int)(dims[n] << tbits)))));
  }
  *resident = ten + mod + tiled_res + slack;
  *transient = std::max(2 * al256(8 * nnz) + 2 * al256(4 * nnz) + al256(tb) + al256(16 * maxunits), tiled_tr) + slack;
}

// Device memory of a server: one block of the budget's size, handed out in
// 256-byte aligned pieces (first fit, free neighbours merged on release), so
// that jobs come and go without a round trip to the system allocator.
struct Arena {
  char *base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length

  void init(void *b, size_t n) {
    base = (char *)b;
    size = n & ~(size_t)255;
    free_.clear();
    used_.clear();
    if (size) free_[0] = size;
  }
  void *alloc(size_t n) {
    n = (std::max<size_t>(n, 1) + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used_[off] = n;
      return base + off;
    }
    return nullptr;
  }
  void release(void *p) {
    auto u = used_.find((size_t)((char *)p - base));
    if (u == used_.end()) return;
    size_t off = u->first, len = u->second;
    used_.erase(u);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + len == nx->first) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += len;
        return;
      }
    }
    free_[off] = len;
  }
};

void *arena_alloc(size_t n, void *user) { return ((Arena *)user)->alloc(n); }
void arena_release(void *p, void *user) { ((Arena *)user)->release(p); }

struct ServerReq {
  int64_t ticket;
  int64_t dims[3];
  int64_t nnz;
  std::vector<int32_t> idx;
  std::vector<float> vals;
  int R;
  uint64_t seed;
  int64_t est_resident, est_transient;
};

struct ServerJob {
  int64_t ticket;
  sacd_tensor *t = nullptr;
  sacd_model *m = nullptr;
  int64_t bytes = 0;
  int iters = 0;
  double prev_fit = 0.0, fit = 0.0, f = 0.0;
};

struct ServerResult {
  int state = 0;  // SACD_JOB_*
  sacd_status err = SACD_OK;
  int iters = 0;
  double fit = 0.0, f = 0.0;
  int64_t dims[3] = {0, 0, 0};
  int R = 0;
  std::vector<float> A[3];
};

// Batched launch tables of the running jobs of one padded rank.
struct BatchGroup {
  int RP = 0;
  std::vector<int> jobs;  // indices into sacd_server::active
  MttkrpArgs *mt[3] = {};
  FixArgs *fx[3] = {};
  ImpArgs *im[3] = {};
  UpdArgs *up[3] = {};
  GramArgs *gf[3] = {};
  int4 *bm_mt[3] = {}, *bm_fx[3] = {}, *bm_im[3] = {}, *bm_up[3] = {}, *bm_gf[3] = {};
  int nb_mt[3] = {}, nb_fx[3] = {}, nb_im[3] = {}, nb_up[3] = {}, nb_gf[3] = {};
  bool big = false;  // element passes in 1024-thread blocks (few row blocks in all)
};

}  // namespace

struct sacd_server {
  sacd_server_config cfg{};
  DevAlloc block;          // the arena's one device block (caller's allocator or hipMalloc)
  Arena arena;
  sacd_allocator alloc{};  // hands out arena pieces to the jobs
  int dev = 0;
  hipStream_t s = nullptr;
  bool own_stream = false;
  // one stream per padded rank: the ranks' launch chains run concurrently,
  // forked from and joined back to s
  hipStream_t gs[4] = {};
  hipEvent_t ev_fork = nullptr, ev_join[4] = {};
  // uploads and ingests of admitted jobs, which run while the running jobs'
  // iteration is in flight on s
  hipStream_t s_admit = nullptr;
  std::deque<ServerReq> queue;
  std::vector<ServerJob> active;
  std::map<int64_t, ServerResult> results;
  std::vector<int64_t> finished;  // tickets finished in the last step
  int64_t next_ticket = 1;
  int64_t bytes_in_use = 0, peak_bytes = 0;
  int64_t budget_cap = 0;  // the budget at creation: the arena's size
  // launch tables
  DevAlloc tables;
  char *h_stage = nullptr;
  size_t h_stage_bytes = 0;
  std::vector<BatchGroup> groups;
  const ModeState **d_sts = nullptr;
  double *d_f = nullptr, *h_f = nullptr;
  size_t h_f_cap = 0;
  float *h_res = nullptr;  // pinned staging of a retiring job's factors
  size_t h_res_cap = 0;
  char *h_up = nullptr;  // pinned staging of an admitted job's coordinates and values
  size_t h_up_cap = 0;
  bool dirty = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int stable_steps = 0;
  int64_t steps = 0, graph_builds = 0, graph_launches = 0, eager_launches = 0;
  double sec_admit = 0.0, sec_tables = 0.0, sec_iterate = 0.0, sec_retire = 0.0;  // host wall time
};

namespace {
double now_sec() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

namespace {

void server_drop_graph(sacd_server *S) {
  if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
  if (S->graph) (void)hipGraphDestroy(S->graph);
  S->gexec = nullptr;
  S->graph = nullptr;
}

void destroy_job(ServerJob &j) {
  if (j.m) sacd_destroy_model(j.m);
  if (j.t) sacd_destroy_tensor(j.t);
  j.m = nullptr;
  j.t = nullptr;
}

// Admission of one queued request: upload, ingest, initial factors.
sacd_status admit(sacd_server *S, ServerReq &q, ServerJob *out) {
  ServerJob j;
  j.ticket = q.ticket;
  DevAlloc up;
  up.alloc = S->alloc;
  up.custom = true;
  int32_t *didx = nullptr;
  float *dvals = nullptr;
  sacd_status st = SACD_OK;
  if (q.nnz > 0) {
    st = up.get_t((size_t)q.nnz * 3, &didx);
    if (st == SACD_OK) st = up.get_t((size_t)q.nnz, &dvals);
    if (st == SACD_OK) {
      // through a pinned buffer, grown to powers of two (the previous
      // admission's copies are complete: every admission waits on s_admit
      // before it returns)
      const size_t bi = sizeof(int32_t) * 3 * (size_t)q.nnz, bv = sizeof(float) * (size_t)q.nnz;
      if (S->h_up_cap < bi + bv) {
        if (S->h_up) (void)hipHostFree(S->h_up);
        S->h_up = nullptr;
        S->h_up_cap = 0;
        size_t cap = 1 << 20;
        while (cap < bi + bv) cap *= 2;
        if (hipHostMalloc((void **)&S->h_up, cap, hipHostMallocDefault) == hipSuccess) S->h_up_cap = cap;
        else S->h_up = nullptr;
      }
      const void *src_i = q.idx.data(), *src_v = q.vals.data();
      if (S->h_up) {
        std::memcpy(S->h_up, q.idx.data(), bi);
        std::memcpy(S->h_up + bi, q.vals.data(), bv);
        src_i = S->h_up;
        src_v = S->h_up + bi;
      }
      hipError_t e = hipMemcpyAsync(didx, src_i, bi, hipMemcpyHostToDevice, S->s_admit);
      if (e == hipSuccess) e = hipMemcpyAsync(dvals, src_v, bv, hipMemcpyHostToDevice, S->s_admit);
      if (e != hipSuccess) st = fail(SACD_ERR_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }
  }
  if (st == SACD_OK)
    st = sacd_create_tensor(q.dims, q.nnz, didx, dvals, &S->alloc, S->s_admit, &j.t);
  (void)hipStreamSynchronize(S->s_admit);
  up.release_all();
  if (st == SACD_OK) st = sacd_init_factors(j.t, q.R, q.seed, S->cfg.precision, SACD_UPDATE_GS, &j.m);
  if (j.t) (void)hipStreamSynchronize(S->s_admit);
  if (st != SACD_OK) {
    destroy_job(j);
    return st;
  }
  // from here on the job's work is ordered on the server's stream
  j.t->stream = S->s;
  j.m->s = S->s;
  j.bytes = j.t->mem.bytes + j.m->mem.bytes;
  *out = j;
  return SACD_OK;
}

// Host table of one batched launch: per-job arguments, then the block map.
template <typename Args>
size_t table_bytes(size_t njobs, size_t nblocks) {
  return al256(sizeof(Args) * njobs) + al256(sizeof(int4) * nblocks);
}

sacd_status rebuild_tables(sacd_server *S) {
  server_drop_graph(S);
  S->tables.release_all();
  S->groups.clear();
  const int J = (int)S->active.size();
  for (int rp : {16, 32, 64, 128}) {
    BatchGroup g;
    g.RP = rp;
    for (int i = 0; i < J; ++i)
      if (S->active[i].m->RP == rp) g.jobs.push_back(i);
    if (!g.jobs.empty()) S->groups.push_back(g);
  }
  // sizes
  size_t total = al256(sizeof(ModeState *) * (J + 1)) + al256(sizeof(double) * (J + 1));
  for (BatchGroup &g : S->groups)
    for (int n = 0; n < 3; ++n) {
      g.nb_mt[n] = g.nb_fx[n] = g.nb_im[n] = g.nb_up[n] = g.nb_gf[n] = 0;
      for (int i : g.jobs) {
        const sacd_model *m = S->active[i].m;
        const int I = (int)m->t->dims[n];
        // a mode in the tiled form runs its own MTTKRP launch (below)
        if (!m->btab[n]) g.nb_mt[n] += mttkrp_blocks(g.RP, m->plan[n].nunits);
        g.nb_fx[n] += fix_blocks(g.RP, m->plan[n].nlong, m->plan[n].nbig);
        g.nb_im[n] += importance_blocks(g.RP, I);
        g.nb_up[n] += update_blocks(g.RP, I);
        g.nb_gf[n] += gram_final_blocks(g.RP);
      }
      const size_t nj = g.jobs.size();
      total += table_bytes<MttkrpArgs>(nj, g.nb_mt[n]) + table_bytes<FixArgs>(nj, g.nb_fx[n]) +
               table_bytes<ImpArgs>(nj, g.nb_im[n]) + table_bytes<UpdArgs>(nj, g.nb_up[n]) +
               table_bytes<GramArgs>(nj, g.nb_gf[n]);
    }
  // With few row blocks in all (at most one per compute unit), the element
  // passes run in 1024-thread blocks, which shorten each block's chain; with
  // many resident jobs, 256-thread blocks keep more of them in flight.
  for (BatchGroup &g : S->groups)
    g.big = g.RP <= 32 && std::max(g.nb_up[0], std::max(g.nb_up[1], g.nb_up[2])) <= 256;
  if (total > S->h_stage_bytes) {
    if (S->h_stage) (void)hipHostFree(S->h_stage);
    S->h_stage = nullptr;
    S->h_stage_bytes = 0;
    HIP_TRY(hipHostMalloc((void **)&S->h_stage, total, hipHostMallocDefault));
    S->h_stage_bytes = total;
  }
  char *dbase = nullptr;
  SACD_TRY(S->tables.get(total, (void **)&dbase));
  size_t off = 0;
  // carve host and device views at the same offsets
  auto carve = [&](size_t bytes, void **h, void **d) {
    *h = S->h_stage + off;
    *d = dbase + off;
    off += al256(bytes);
  };
  void *h, *d;
  carve(sizeof(ModeState *) * (J + 1), &h, &d);
  for (int i = 0; i < J; ++i) ((const ModeState **)h)[i] = S->active[i].m->st + 2;
  S->d_sts = (const ModeState **)d;
  carve(sizeof(double) * (J + 1), &h, &d);
  S->d_f = (double *)d;
  auto fill_map = [&](int4 *bm, const BatchGroup &g, int n, int which) {
    int b = 0;
    for (size_t k = 0; k < g.jobs.size(); ++k) {
      const sacd_model *m = S->active[g.jobs[k]].m;
      const int I = (int)m->t->dims[n];
      int nb = 0;
      if (which == 0) nb = m->btab[n] ? 0 : mttkrp_blocks(g.RP, m->plan[n].nunits);
      else if (which == 1) nb = fix_blocks(g.RP, m->plan[n].nlong, m->plan[n].nbig);
      else if (which == 2) nb = importance_blocks(g.RP, I);
      else if (which == 3) nb = gram_final_blocks(g.RP);
      else nb = update_blocks(g.RP, I);
      for (int q = 0; q < nb; ++q) bm[b++] = make_int4((int)k, q, nb, 0);
    }
  };
  for (BatchGroup &g : S->groups)
    for (int n = 0; n < 3; ++n) {
      const size_t nj = g.jobs.size();
      carve(sizeof(MttkrpArgs) * nj, &h, &d);
      for (size_t k = 0; k < nj; ++k) ((MttkrpArgs *)h)[k] = mttkrp_args(S->active[g.jobs[k]].m, n);
      g.mt[n] = (MttkrpArgs *)d;
      carve(sizeof(int4) * g.nb_mt[n], &h, &d);
      fill_map((int4 *)h, g, n, 0);
      g.bm_mt[n] = (int4 *)d;
      carve(sizeof(FixArgs) * nj, &h, &d);
      for (size_t k = 0; k < nj; ++k) ((FixArgs *)h)[k] = fix_args(S->active[g.jobs[k]].m, n);
      g.fx[n] = (FixArgs *)d;
      carve(sizeof(int4) * g.nb_fx[n], &h, &d);
      fill_map((int4 *)h, g, n, 1);
      g.bm_fx[n] = (int4 *)d;
      carve(sizeof(ImpArgs) * nj, &h, &d);
      for (size_t k = 0; k < nj; ++k) ((ImpArgs *)h)[k] = imp_args(S->active[g.jobs[k]].m, n);
      g.im[n] = (ImpArgs *)d;
      carve(sizeof(int4) * g.nb_im[n], &h, &d);
      fill_map((int4 *)h, g, n, 2);
      g.bm_im[n] = (int4 *)d;
      carve(sizeof(UpdArgs) * nj, &h, &d);
      for (size_t k = 0; k < nj; ++k) ((UpdArgs *)h)[k] = upd_args(S->active[g.jobs[k]].m, n);
      g.up[n] = (UpdArgs *)d;
      carve(sizeof(int4) * g.nb_up[n], &h, &d);
      fill_map((int4 *)h, g, n, 4);
      g.bm_up[n] = (int4 *)d;
      carve(sizeof(GramArgs) * nj, &h, &d);
      for (size_t k = 0; k < nj; ++k) ((GramArgs *)h)[k] = gram_args(S->active[g.jobs[k]].m, n, true);
      g.gf[n] = (GramArgs *)d;
      carve(sizeof(int4) * g.nb_gf[n], &h, &d);
      fill_map((int4 *)h, g, n, 3);
      g.bm_gf[n] = (int4 *)d;
    }
  HIP_TRY(hipMemcpyAsync(dbase, S->h_stage, off, hipMemcpyHostToDevice, S->s));
  HIP_TRY(hipStreamSynchronize(S->s));
  if ((size_t)J > S->h_f_cap) {
    if (S->h_f) (void)hipHostFree(S->h_f);
    S->h_f = nullptr;
    S->h_f_cap = 0;
    HIP_TRY(hipHostMalloc((void **)&S->h_f, sizeof(double) * J, hipHostMallocDefault));
    S->h_f_cap = J;
  }
  S->dirty = false;
  S->stable_steps = 0;
  return SACD_OK;
}

// One outer iteration of every running job, then the gather of their
// objectives.  Per mode, the ranks' launches follow each other on the stream.
sacd_status enqueue_batched_iteration(sacd_server *S) {
  const bool bf = S->cfg.precision == SACD_PREC_MIXED_BF16;
  HIP_TRY(hipEventRecord(S->ev_fork, S->s));
  for (size_t gi = 0; gi < S->groups.size(); ++gi) {
    BatchGroup &g = S->groups[gi];
    hipStream_t s = S->gs[gi];
    HIP_TRY(hipStreamWaitEvent(s, S->ev_fork, 0));
    for (int n = 0; n < 3; ++n) {
      HIP_TRY(launch_mttkrp_b(g.RP, g.mt[n], g.bm_mt[n], g.nb_mt[n], s));
      for (int i : g.jobs) {
        const sacd_model *m = S->active[i].m;
        if (m->btab[n]) HIP_TRY(launch_mode_mttkrp(m, n, s));  // the tiled form, as the job alone runs it
      }
      HIP_TRY(launch_mttkrp_fix_b(g.RP, g.fx[n], g.bm_fx[n], g.nb_fx[n], s));
      HIP_TRY(launch_importance_b(g.RP, bf, g.big, g.im[n], g.bm_im[n], g.nb_im[n], s));
      HIP_TRY(launch_select_update_b(g.RP, bf, g.big, g.up[n], g.bm_up[n], g.nb_up[n], s));
      HIP_TRY(launch_gram_final_b(g.RP, g.gf[n], g.bm_gf[n], g.nb_gf[n], s));
    }
    HIP_TRY(hipEventRecord(S->ev_join[gi], s));
    HIP_TRY(hipStreamWaitEvent(S->s, S->ev_join[gi], 0));
  }
  HIP_TRY(launch_gather_f(S->d_sts, (int)S->active.size(), S->d_f, S->s));
  return SACD_OK;
}

sacd_status run_iteration(sacd_server *S) {
  if (S->gexec) {
    HIP_TRY(hipGraphLaunch(S->gexec, S->s));
    S->graph_launches++;
    return SACD_OK;
  }
  if (S->cfg.use_graphs && S->stable_steps >= 1) {
    // the set of running jobs did not change last step: capture it
    HIP_TRY(hipStreamBeginCapture(S->s, hipStreamCaptureModeThreadLocal));
    sacd_status st = enqueue_batched_iteration(S);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(S->s, &g);
    if (st != SACD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(SACD_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&S->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      S->gexec = nullptr;
      return fail(SACD_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    S->graph = g;
    S->graph_builds++;
    HIP_TRY(hipGraphLaunch(S->gexec, S->s));
    S->graph_launches++;
    return SACD_OK;
  }
  SACD_TRY(enqueue_batched_iteration(S));
  S->eager_launches++;
  return SACD_OK;
}

sacd_status retire(sacd_server *S, ServerJob &j, int state) {
  ServerResult &r = S->results[j.ticket];
  r.state = state;
  r.iters = j.iters;
  r.fit = j.fit;
  r.f = j.f;
  r.R = j.m->R;
  size_t total = 0;
  for (int n = 0; n < 3; ++n) total += (size_t)j.t->dims[n] * j.m->R;
  if (total > S->h_res_cap) {
    if (S->h_res) (void)hipHostFree(S->h_res);
    S->h_res = nullptr;
    S->h_res_cap = 0;
    const size_t cap = std::max(total, (size_t)1 << 20);
    HIP_TRY(hipHostMalloc((void **)&S->h_res, sizeof(float) * cap, hipHostMallocDefault));
    S->h_res_cap = cap;
  }
  size_t off = 0;
  for (int n = 0; n < 3; ++n) {
    r.dims[n] = j.t->dims[n];
    HIP_TRY(hipMemcpy2DAsync(S->h_res + off, sizeof(float) * j.m->R, j.m->A[n], sizeof(float) * j.m->RP,
                             sizeof(float) * j.m->R, (size_t)j.t->dims[n], hipMemcpyDeviceToHost, S->s));
    off += (size_t)j.t->dims[n] * j.m->R;
  }
  HIP_TRY(hipStreamSynchronize(S->s));
  off = 0;
  for (int n = 0; n < 3; ++n) {
    const size_t len = (size_t)j.t->dims[n] * j.m->R;
    r.A[n].assign(S->h_res + off, S->h_res + off + len);
    off += len;
  }
  S->bytes_in_use -= j.bytes;
  destroy_job(j);
  S->finished.push_back(j.ticket);
  return SACD_OK;
}

// A running job that stops without a result (a non-finite objective, or a
// cancel): its state, its last iteration count, fit and objective; its device
// memory is freed.
void retire_without_result(sacd_server *S, ServerJob &j, int state, sacd_status err) {
  ServerResult &r = S->results[j.ticket];
  r.state = state;
  r.err = err;
  r.iters = j.iters;
  r.fit = j.fit;
  r.f = j.f;
  r.R = j.m ? j.m->R : 0;
  S->bytes_in_use -= j.bytes;
  destroy_job(j);
}

}  // namespace

extern "C" {

sacd_status sacd_job_bytes(const int64_t dims[3], int64_t nnz, int32_t R, sacd_precision prec, int64_t *resident,
                           int64_t *transient) {
  if (!dims || nnz < 0 || R < 1 || R > kMaxRP) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  if (prec != SACD_PREC_FP32 && prec != SACD_PREC_MIXED_BF16)
    return fail(SACD_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
  int64_t a = 0, b = 0;
  job_bytes(dims, nnz, R, prec == SACD_PREC_MIXED_BF16, &a, &b);
  if (resident) *resident = a;
  if (transient) *transient = b;
  return SACD_OK;
}

sacd_status sacd_server_create(const sacd_server_config *cfg, const sacd_allocator *alloc, void *stream,
                               sacd_server **out) {
  if (!out || !cfg) return fail(SACD_ERR_INVALID_ARG, "cfg / out is NULL");
  *out = nullptr;
  if (cfg->budget_bytes <= 0 || cfg->max_slots < 1 || cfg->max_iter < 1 || !(cfg->tol >= 0.0))
    return fail(SACD_ERR_INVALID_ARG, "budget, max_slots, max_iter must be positive and tol >= 0");
  if (cfg->precision != SACD_PREC_FP32 && cfg->precision != SACD_PREC_MIXED_BF16)
    return fail(SACD_ERR_INVALID_ARG, "unknown precision %d", (int)cfg->precision);
  if (alloc && (!alloc->alloc || !alloc->release)) return fail(SACD_ERR_INVALID_ARG, "allocator callbacks are NULL");
  (void)hipGetLastError();
  sacd_server *S = new (std::nothrow) sacd_server();
  if (!S) return fail(SACD_ERR_NO_MEMORY, "host allocation failed");
  S->cfg = *cfg;
  if (alloc) {
    S->block.alloc = *alloc;
    S->block.custom = true;
    S->tables.alloc = *alloc;
    S->tables.custom = true;
  }
  if (hipGetDevice(&S->dev) != hipSuccess) {
    delete S;
    return fail(SACD_ERR_DEVICE, "no HIP device");
  }
  void *base = nullptr;
  sacd_status st = S->block.get((size_t)cfg->budget_bytes, &base);
  if (st == SACD_OK) st = make_stream(stream, &S->s, &S->own_stream);
  for (int g = 0; g < 4 && st == SACD_OK; ++g) {
    if (hipStreamCreateWithFlags(&S->gs[g], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->ev_join[g], hipEventDisableTiming) != hipSuccess)
      st = fail(SACD_ERR_DEVICE, "stream / event creation failed");
  }
  if (st == SACD_OK && hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming) != hipSuccess)
    st = fail(SACD_ERR_DEVICE, "event creation failed");
  if (st == SACD_OK && hipStreamCreateWithFlags(&S->s_admit, hipStreamNonBlocking) != hipSuccess)
    st = fail(SACD_ERR_DEVICE, "stream creation failed");
  if (st != SACD_OK) {
    sacd_server_destroy(S);
    return st;
  }
  S->arena.init(base, (size_t)cfg->budget_bytes);
  S->budget_cap = cfg->budget_bytes;
  S->alloc.alloc = arena_alloc;
  S->alloc.release = arena_release;
  S->alloc.user = &S->arena;
  *out = S;
  return SACD_OK;
}

sacd_status sacd_server_submit(sacd_server *S, const int64_t dims[3], int64_t nnz, const int32_t *idx,
                               const float *vals, int32_t R, uint64_t seed, int64_t *ticket) {
  if (!S || !dims || !ticket) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  if (R < 1 || R > kMaxRP) return fail(SACD_ERR_INVALID_ARG, "rank %d not in [1, %d]", R, kMaxRP);
  if (nnz < 0 || (nnz > 0 && (!idx || !vals))) return fail(SACD_ERR_INVALID_ARG, "bad nnz / idx / vals");
  for (int n = 0; n < 3; ++n)
    if (dims[n] < 1 || dims[n] > 2147483647LL) return fail(SACD_ERR_INVALID_ARG, "dims[%d] out of range", n);
  ServerReq q;
  q.ticket = S->next_ticket;
  for (int n = 0; n < 3; ++n) q.dims[n] = dims[n];
  q.nnz = nnz;
  q.R = R;
  q.seed = seed;
  job_bytes(dims, nnz, R, S->cfg.precision == SACD_PREC_MIXED_BF16, &q.est_resident, &q.est_transient);
  if (q.est_resident + q.est_transient > S->cfg.budget_bytes)
    return fail(SACD_ERR_NO_MEMORY, "job needs up to %lld bytes, more than the whole budget",
                (long long)(q.est_resident + q.est_transient));
  q.idx.assign(idx, idx + 3 * nnz);
  q.vals.assign(vals, vals + nnz);
  S->queue.push_back(std::move(q));
  ServerResult &r = S->results[S->next_ticket];
  r.state = SACD_JOB_QUEUED;
  *ticket = S->next_ticket++;
  return SACD_OK;
}

namespace {
// Admission, first come first served, while the budget and the slots allow;
// the admitted jobs are appended to *out (not yet to the running set).
void admit_queue(sacd_server *S, std::vector<ServerJob> *out) {
  const double t0 = now_sec();
  while (!S->queue.empty() && (int)(S->active.size() + out->size()) < S->cfg.max_slots) {
    ServerReq &q = S->queue.front();
    if (S->bytes_in_use + q.est_resident + q.est_transient > S->cfg.budget_bytes) break;
    ServerJob j;
    sacd_status st = admit(S, q, &j);
    if (st == SACD_ERR_NO_MEMORY && !(S->active.empty() && out->empty())) break;  // fragmented: retry when jobs leave
    ServerResult &r = S->results[q.ticket];
    if (st != SACD_OK) {
      r.state = SACD_JOB_FAILED;
      r.err = st;
      S->finished.push_back(q.ticket);
    } else {
      r.state = SACD_JOB_RUNNING;
      out->push_back(j);
      S->bytes_in_use += j.bytes;
      S->peak_bytes = std::max(S->peak_bytes, S->bytes_in_use);
    }
    S->queue.pop_front();
  }
  S->sec_admit += now_sec() - t0;
}
}  // namespace

sacd_status sacd_server_step(sacd_server *S, int32_t *n_running, int32_t *n_queued) {
  if (!S) return fail(SACD_ERR_INVALID_ARG, "server is NULL");
  SACD_TRY(enter(S->dev));
  S->finished.clear();
  // With jobs running, their iteration is launched first and the queue is
  // admitted (upload and ingest on s_admit) while it runs; the admitted jobs
  // join the running set after it, for the next step.  With none running,
  // admission comes first and the admitted jobs iterate in this step.
  std::vector<ServerJob> admitted;
  if (S->active.empty()) {
    admit_queue(S, &admitted);
    for (ServerJob &j : admitted) S->active.push_back(j);
    if (!admitted.empty()) S->dirty = true;
    admitted.clear();
  }
  double t1 = now_sec();
  if (!S->active.empty()) {
    if (S->dirty) SACD_TRY(rebuild_tables(S));
    double t2 = now_sec();
    S->sec_tables += t2 - t1;
    SACD_TRY(run_iteration(S));
    const int J = (int)S->active.size();
    HIP_TRY(hipMemcpyAsync(S->h_f, S->d_f, sizeof(double) * J, hipMemcpyDeviceToHost, S->s));
    const double sa = S->sec_admit;
    admit_queue(S, &admitted);
    const hipError_t e = hipStreamSynchronize(S->s);
    if (e != hipSuccess) {
      // the admitted jobs stay with the server (freed with it)
      for (ServerJob &j : admitted) S->active.push_back(j);
      S->dirty = true;
      return fail(SACD_ERR_DEVICE, "server iteration failed: %s", hipGetErrorString(e));
    }
    t1 = now_sec();
    S->sec_iterate += t1 - t2 - (S->sec_admit - sa);
    S->steps++;
    S->stable_steps++;
    std::vector<ServerJob> keep;
    keep.reserve(J);
    for (int i = 0; i < J; ++i) {
      ServerJob &j = S->active[i];
      j.iters++;
      j.f = S->h_f[i];
      const double nx = std::sqrt(j.t->norm2);
      j.fit = nx > 0.0 ? 1.0 - std::sqrt(j.f > 0.0 ? j.f : 0.0) / nx : 0.0;
      if (!std::isfinite(j.f)) {  // a non-finite value arose: the job fails, the others run on
        retire_without_result(S, j, SACD_JOB_FAILED, SACD_ERR_NUMERIC);
        S->finished.push_back(j.ticket);
        S->dirty = true;
        continue;
      }
      // the stopping rule of sacd_run_until
      const bool conv = j.iters >= 2 && std::fabs(j.fit - j.prev_fit) < S->cfg.tol * std::fabs(j.prev_fit);
      j.prev_fit = j.fit;
      if (conv || j.iters >= S->cfg.max_iter || !(nx > 0.0)) {
        SACD_TRY(retire(S, j, SACD_JOB_DONE));
        S->dirty = true;
      } else {
        keep.push_back(j);
      }
    }
    S->active.swap(keep);
    for (ServerJob &j : admitted) S->active.push_back(j);
    if (!admitted.empty()) S->dirty = true;
    if (S->dirty) server_drop_graph(S);
    S->sec_retire += now_sec() - t1;
  }
  if (n_running) *n_running = (int32_t)S->active.size();
  if (n_queued) *n_queued = (int32_t)S->queue.size();
  return SACD_OK;
}

sacd_status sacd_server_finished(const sacd_server *S, int64_t *tickets, int32_t cap, int32_t *n) {
  if (!S || !n || cap < 0 || (cap > 0 && !tickets)) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  const int k = std::min<int>(cap, (int)S->finished.size());
  for (int i = 0; i < k; ++i) tickets[i] = S->finished[i];
  *n = (int32_t)S->finished.size();
  return SACD_OK;
}

sacd_status sacd_server_poll(const sacd_server *S, int64_t ticket, int32_t *state, int32_t *iters, double *fit,
                             double *objective) {
  if (!S) return fail(SACD_ERR_INVALID_ARG, "server is NULL");
  auto it = S->results.find(ticket);
  if (it == S->results.end()) return fail(SACD_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
  const ServerResult &r = it->second;
  if (state) *state = r.state;
  int it_now = r.iters;
  double fit_now = r.fit, f_now = r.f;
  if (r.state == SACD_JOB_RUNNING)
    for (const ServerJob &j : S->active)
      if (j.ticket == ticket) {
        it_now = j.iters;
        fit_now = j.fit;
        f_now = j.f;
      }
  if (iters) *iters = it_now;
  if (fit) *fit = fit_now;
  if (objective) *objective = f_now;
  return r.state == SACD_JOB_FAILED ? r.err : SACD_OK;
}

sacd_status sacd_server_result(const sacd_server *S, int64_t ticket, int32_t mode, float *dst) {
  if (!S || !dst || mode < 0 || mode > 2) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  auto it = S->results.find(ticket);
  if (it == S->results.end()) return fail(SACD_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
  if (it->second.state != SACD_JOB_DONE) return fail(SACD_ERR_BAD_STATE, "job %lld is not done", (long long)ticket);
  const std::vector<float> &A = it->second.A[mode];
  std::memcpy(dst, A.data(), sizeof(float) * A.size());
  return SACD_OK;
}

sacd_status sacd_server_release(sacd_server *S, int64_t ticket) {
  if (!S) return fail(SACD_ERR_INVALID_ARG, "server is NULL");
  auto it = S->results.find(ticket);
  if (it == S->results.end()) return fail(SACD_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
  const int st = it->second.state;
  if (st != SACD_JOB_DONE && st != SACD_JOB_FAILED && st != SACD_JOB_CANCELLED)
    return fail(SACD_ERR_BAD_STATE, "job %lld is still queued or running", (long long)ticket);
  S->results.erase(it);
  return SACD_OK;
}

sacd_status sacd_server_cancel(sacd_server *S, int64_t ticket) {
  if (!S) return fail(SACD_ERR_INVALID_ARG, "server is NULL");
  auto it = S->results.find(ticket);
  if (it == S->results.end()) return fail(SACD_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
  ServerResult &r = it->second;
  if (r.state == SACD_JOB_QUEUED) {
    for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
      if (q->ticket == ticket) {
        S->queue.erase(q);
        break;
      }
    r.state = SACD_JOB_CANCELLED;
    return SACD_OK;
  }
  if (r.state != SACD_JOB_RUNNING)
    return fail(SACD_ERR_BAD_STATE, "job %lld has already finished", (long long)ticket);
  SACD_TRY(enter(S->dev));
  // the server's work is synchronous: no launch of this job is in flight
  for (size_t i = 0; i < S->active.size(); ++i)
    if (S->active[i].ticket == ticket) {
      retire_without_result(S, S->active[i], SACD_JOB_CANCELLED, SACD_OK);
      S->active.erase(S->active.begin() + (long)i);
      S->dirty = true;
      server_drop_graph(S);
      break;
    }
  return SACD_OK;
}

sacd_status sacd_server_set_budget(sacd_server *S, int64_t budget_bytes) {
  if (!S) return fail(SACD_ERR_INVALID_ARG, "server is NULL");
  if (budget_bytes <= 0 || budget_bytes > S->budget_cap)
    return fail(SACD_ERR_INVALID_ARG, "budget %lld outside (0, %lld]", (long long)budget_bytes,
                (long long)S->budget_cap);
  S->cfg.budget_bytes = budget_bytes;
  // queued requests that can no longer fit at all fail now
  for (auto q = S->queue.begin(); q != S->queue.end();) {
    if (q->est_resident + q->est_transient > budget_bytes) {
      ServerResult &r = S->results[q->ticket];
      r.state = SACD_JOB_FAILED;
      r.err = SACD_ERR_NO_MEMORY;
      q = S->queue.erase(q);
    } else {
      ++q;
    }
  }
  return SACD_OK;
}

sacd_status sacd_server_stats(const sacd_server *S, sacd_server_stats_t *out) {
  if (!S || !out) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  out->running = (int32_t)S->active.size();
  out->queued = (int32_t)S->queue.size();
  out->bytes_in_use = S->bytes_in_use;
  out->peak_bytes = S->peak_bytes;
  out->steps = S->steps;
  out->graph_builds = S->graph_builds;
  out->graph_launches = S->graph_launches;
  out->eager_launches = S->eager_launches;
  out->sec_admit = S->sec_admit;
  out->sec_tables = S->sec_tables;
  out->sec_iterate = S->sec_iterate;
  out->sec_retire = S->sec_retire;
  return SACD_OK;
}

void sacd_server_destroy(sacd_server *S) {
  if (!S) return;
  (void)hipSetDevice(S->dev);
  if (S->s) (void)hipStreamSynchronize(S->s);
  server_drop_graph(S);
  for (ServerJob &j : S->active) destroy_job(j);
  S->active.clear();
  S->tables.release_all();
  S->block.release_all();
  if (S->h_stage) (void)hipHostFree(S->h_stage);
  if (S->h_f) (void)hipHostFree(S->h_f);
  if (S->h_res) (void)hipHostFree(S->h_res);
  if (S->h_up) (void)hipHostFree(S->h_up);
  for (int g = 0; g < 4; ++g) {
    if (S->gs[g]) (void)hipStreamDestroy(S->gs[g]);
    if (S->ev_join[g]) (void)hipEventDestroy(S->ev_join[g]);
  }
  if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
  if (S->s_admit) (void)hipStreamDestroy(S->s_admit);
  if (S->own_stream && S->s) (void)hipStreamDestroy(S->s);
  delete S;
}

}  // extern "C"

// ------------------------------------------------------------------ N-way --
//
// Tensors of N modes (Sec. 3 defines the factorization for any number of
// modes; the three-way sweep carries over with the Khatri-Rao product of the
// N - 1 other factors in the MTTKRP and the Hadamard product of their Gram
// matrices as H).  Keys pack mode n's index in the high field and the other
// indices below it in increasing mode order.  The sweep runs the N-way MTTKRP
// (nway.hip), then the three-way element kernels with H formed from P, the
// product of the other Grams, and a matrix of ones.

struct sacd_ntensor {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevAlloc mem;
  int N = 0;
  int64_t dims[kMaxModes] = {};
  long long nnz = 0;
  NLayout lay[kMaxModes] = {};
  unsigned long long *keys[kMaxModes] = {};
  float *vals[kMaxModes] = {};
  int *ptr[kMaxModes] = {};
  std::vector<int> hptr[kMaxModes];
  double norm2 = 0.0;
  int nmodels = 0;
  bool destroy_pending = false;
};

struct sacd_nmodel {
  sacd_ntensor *t = nullptr;
  hipStream_t s = nullptr;
  DevAlloc mem;
  int N = 0, R = 0, RP = 0;
  bool diag = false;
  float *A[kMaxModes] = {}, *Z[kMaxModes] = {}, *M[kMaxModes] = {}, *H[kMaxModes] = {};
  double *G64[kMaxModes] = {};
  HInfo *hinfo[kMaxModes] = {};
  long long *colcnt[kMaxModes] = {};
  uint8_t *selmask[kMaxModes] = {};
  ModeState *st = nullptr;  // N entries
  double *P = nullptr, *ones = nullptr;
  float *part = nullptr, *gpart = nullptr;
  double *mpart = nullptr;
  unsigned *gcounter = nullptr;
  double *ti_part = nullptr, *inner_part = nullptr;
  int *cnt_part = nullptr, *flag = nullptr;
  double *full_part = nullptr, *full_out = nullptr;
  unsigned *full_cnt = nullptr;
  int full_nparts = 0;
  int nparts[kMaxModes] = {};
  MttkrpPlan plan[kMaxModes];
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<hipEvent_t> tev;  // 3 per sweep: before and after the MTTKRP, end of the sweep
  double *h_pinned = nullptr;
  bool counted = false;
  int last_mode = -1;
  bool dirty = true;
};

namespace {

// Field layout of mode n: n first (highest bits), then the other modes in
// increasing order; field f sits above the fields after it.
NLayout nlayout(int N, const int64_t *dims, int n) {
  NLayout l{};
  l.nf = N;
  int order[kMaxModes];
  order[0] = n;
  for (int m = 0, f = 1; m < N; ++m)
    if (m != n) order[f++] = m;
  int sh = 0;
  for (int f = N - 1; f >= 0; --f) {
    const int b = bits_for(dims[order[f]]);
    l.sh[f] = sh;
    l.mask[f] = b == 0 ? 0ull : (b == 64 ? ~0ull : ((1ull << b) - 1ull));
    sh += b;
  }
  for (int f = 0; f < N; ++f) l.dims[f] = dims[order[f]];
  return l;
}

// Work plan of mode n of an N-way tensor: slices cut into segments of at most
// kSegment entries, longest first (stable, so the segments of a split slice
// stay together); the segments of a split slice that share a block of upb
// units form a run with one partial slot (number_runs).
sacd_status build_nplan(const sacd_ntensor *t, int n, int upb, DevAlloc &mem, MttkrpPlan *out) {
  const std::vector<int> &ptr = t->hptr[n];
  const int I = (int)t->dims[n];
  std::vector<int4> units;
  for (int r = 0; r < I; ++r) {
    const int len = ptr[r + 1] - ptr[r];
    if (len == 0) continue;
    if (len <= kSegment) {
      units.push_back(make_int4(r, ptr[r], len, -1));
      continue;
    }
    for (int b = ptr[r]; b < ptr[r + 1]; b += kSegment)
      units.push_back(make_int4(r, b, std::min(kSegment, ptr[r + 1] - b), -2));
  }
  std::stable_sort(units.begin(), units.end(), [](const int4 &x, const int4 &y) { return x.z > y.z; });
  std::vector<int4> longs;
  const int nslots = number_runs(units, upb, &longs);
  const int nbig = order_longs(&longs);
  MttkrpPlan p{};
  p.nnz = t->nnz;
  p.nunits = (int)units.size();
  p.nlong = (int)longs.size();
  p.nbig = nbig;
  p.nslots = nslots;
  int4 *du = nullptr, *dl = nullptr;
  SACD_TRY(mem.get_t(units.size() + 1, &du));
  SACD_TRY(mem.get_t(longs.size() + 1, &dl));
  if (!units.empty())
    HIP_TRY(hipMemcpyAsync(du, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice, t->stream));
  if (!longs.empty())
    HIP_TRY(hipMemcpyAsync(dl, longs.data(), sizeof(int4) * longs.size(), hipMemcpyHostToDevice, t->stream));
  HIP_TRY(hipStreamSynchronize(t->stream));
  p.units = du;
  p.longs = dl;
  *out = p;
  return SACD_OK;
}

sacd_status create_ntensor_impl(sacd_ntensor *t, const int32_t *idx, const float *vals, long long n) {
  const hipStream_t s = t->stream;
  const int N = t->N;
  for (int m = 0; m < N; ++m) t->lay[m] = nlayout(N, t->dims, m);
  int total_bits = 0;
  for (int m = 0; m < N; ++m) total_bits += bits_for(t->dims[m]);
  DevAlloc tmp;
  tmp.alloc = t->mem.alloc;
  tmp.custom = t->mem.custom;
  unsigned long long *k0 = nullptr, *k1 = nullptr;
  float *v0 = nullptr, *v1 = nullptr;
  int *err = nullptr, *cnt = nullptr;
  void *temp = nullptr;
  size_t tb = std::max(radix_sort_temp_bytes(n), dedup_temp_bytes(n));
  for (int m = 0; m < N; ++m) tb = std::max(tb, build_ptr_temp_bytes(n, (int)t->dims[m]));
  tb = std::max(tb, (size_t)8192);
  sacd_status rs = SACD_OK;
#define NT_TRY(expr)           \
  do {                         \
    rs = (expr);               \
    if (rs != SACD_OK) {       \
      tmp.release_all();       \
      return rs;               \
    }                          \
  } while (0)
#define NT_HIP(expr)                                                                \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      tmp.release_all();                                                            \
      return fail(SACD_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));  \
    }                                                                               \
  } while (0)
  NT_TRY(tmp.get_t(n > 0 ? n : 1, &k0));
  NT_TRY(tmp.get_t(n > 0 ? n : 1, &k1));
  NT_TRY(tmp.get_t(n > 0 ? n : 1, &v0));
  NT_TRY(tmp.get_t(n > 0 ? n : 1, &v1));
  NT_TRY(tmp.get_t(4, &err));
  NT_TRY(tmp.get_t(4, &cnt));
  NT_TRY(tmp.get(tb, &temp));
  NT_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
  NT_HIP(launch_make_keys_n(idx, vals, n, t->lay[0], k0, v0, err, s));
  int herr = 0;
  NT_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  NT_HIP(hipStreamSynchronize(s));
  if (herr & 1) {
    tmp.release_all();
    return fail(SACD_ERR_OUT_OF_RANGE, "a coordinate is outside dims");
  }
  if (herr & 2) {
    tmp.release_all();
    return fail(SACD_ERR_NUMERIC, "a value is NaN or Inf");
  }
  // mode 0: stable sort by the whole key, duplicates merged in input order
  bool in_alt = false;
  NT_HIP(radix_sort_pairs(k0, v0, k1, v1, n, 0, total_bits, temp, s, &in_alt));
  unsigned long long *ks = in_alt ? k1 : k0, *kd = in_alt ? k0 : k1;
  float *vs = in_alt ? v1 : v0, *vd = in_alt ? v0 : v1;
  NT_HIP(dedup_sorted(ks, vs, n, kd, vd, cnt, temp, s));
  int hcnt = 0;
  NT_HIP(hipMemcpyAsync(&hcnt, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
  NT_HIP(hipStreamSynchronize(s));
  const long long u = hcnt;
  t->nnz = u;
  for (int m = 0; m < N; ++m) {
    NT_TRY(t->mem.get_t((size_t)u + kKeySlack, &t->keys[m]));
    NT_TRY(t->mem.get_t((size_t)u + kKeySlack, &t->vals[m]));
    NT_TRY(t->mem.get_t((size_t)t->dims[m] + 1, &t->ptr[m]));
    NT_HIP(hipMemsetAsync(t->keys[m] + u, 0, sizeof(unsigned long long) * kKeySlack, s));
    NT_HIP(hipMemsetAsync(t->vals[m] + u, 0, sizeof(float) * kKeySlack, s));
  }
  if (u > 0) {
    NT_HIP(hipMemcpyAsync(t->keys[0], kd, sizeof(unsigned long long) * u, hipMemcpyDeviceToDevice, s));
    NT_HIP(hipMemcpyAsync(t->vals[0], vd, sizeof(float) * u, hipMemcpyDeviceToDevice, s));
  }
  // mode m > 0: the mode-0 order, re-keyed and sorted stably by i_m alone, is
  // (i_m, then the other indices in increasing mode order)
  for (int m = 1; m < N; ++m) {
    NShifts to{};
    // mode q sits in field 1 + q - (q > m) of mode m's layout (field 0: mode m)
    for (int q = 0; q < N; ++q) to.sh[q] = t->lay[m].sh[q == m ? 0 : (q < m ? q + 1 : q)];
    NT_HIP(launch_rekey_n(t->keys[0], u, t->lay[0], to, k0, s));
    if (u > 0) NT_HIP(hipMemcpyAsync(v0, t->vals[0], sizeof(float) * u, hipMemcpyDeviceToDevice, s));
    bool alt = false;
    const int lo = t->lay[m].sh[0];
    NT_HIP(radix_sort_pairs(k0, v0, k1, v1, u, lo, lo + bits_for(t->dims[m]), temp, s, &alt));
    if (u > 0) {
      NT_HIP(hipMemcpyAsync(t->keys[m], alt ? k1 : k0, sizeof(unsigned long long) * u, hipMemcpyDeviceToDevice, s));
      NT_HIP(hipMemcpyAsync(t->vals[m], alt ? v1 : v0, sizeof(float) * u, hipMemcpyDeviceToDevice, s));
    }
  }
  for (int m = 0; m < N; ++m) {
    NT_HIP(build_ptr(t->keys[m], u, t->lay[m].sh[0], (int)t->dims[m], t->ptr[m], temp, s));
    t->hptr[m].resize((size_t)t->dims[m] + 1);
    NT_HIP(hipMemcpyAsync(t->hptr[m].data(), t->ptr[m], sizeof(int) * ((size_t)t->dims[m] + 1),
                          hipMemcpyDeviceToHost, s));
  }
  NT_HIP(hipStreamSynchronize(s));
  {
    double *part = (double *)temp;
    NT_HIP(launch_norm2(t->vals[0], u, part, 512, part + 512, s));
    NT_HIP(hipMemcpyAsync(&t->norm2, part + 512, sizeof(double), hipMemcpyDeviceToHost, s));
    NT_HIP(hipStreamSynchronize(s));
  }
  tmp.release_all();
  return SACD_OK;
#undef NT_TRY
#undef NT_HIP
}

void release_ntensor(sacd_ntensor *t) {
  (void)hipSetDevice(t->dev);
  if (t->stream) (void)hipStreamSynchronize(t->stream);
  t->mem.release_all();
  if (t->own_stream && t->stream) (void)hipStreamDestroy(t->stream);
  delete t;
}

sacd_status check_nmode(const sacd_nmodel *m, int32_t mode) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  if (mode < 0 || mode >= m->N) return fail(SACD_ERR_INVALID_ARG, "mode %d not in [0, %d)", mode, m->N);
  return SACD_OK;
}

sacd_status nrecompute_gram(sacd_nmodel *m, int n) {
  HIP_TRY(launch_gram_partial(m->RP, false, (int)m->t->dims[n], m->A[n], m->gpart, nullptr, m->s));
  GramArgs g{};
  g.nparts = m->nparts[n];
  g.gpart = m->gpart;
  g.mpart = m->mpart;
  g.Gn = m->G64[n];
  g.with_f = 0;
  g.counter = m->gcounter;
  g.st = m->st + n;
  HIP_TRY(launch_gram_final(m->RP, g, m->s));
  return SACD_OK;
}

// One sweep of mode n: P = product of the other Grams; the N-way MTTKRP; H, L
// and the split slices; importance and total; selection and Gauss-Seidel
// update; Gram, counts and objective.  mark (optional): 3 events.
sacd_status enqueue_nsweep(sacd_nmodel *m, int n, const hipEvent_t *mark = nullptr) {
  const sacd_ntensor *t = m->t;
  hipStream_t s = m->s;
  const int RP = m->RP, N = m->N, I = (int)t->dims[n];
  NGrams ng{};
  ng.n = N;
  for (int q = 0; q < N; ++q) ng.G[q] = m->G64[q];
  HIP_TRY(launch_prod_grams(ng, n, RP, m->P, m->ones, s));
  NMttkrpArgs a{};
  a.keys = t->keys[n];
  a.vals = t->vals[n];
  a.units = m->plan[n].units;
  a.nunits = m->plan[n].nunits;
  a.nother = N - 1;
  for (int q = 0, f = 0; q < N; ++q) {
    if (q == n) continue;
    a.A[f] = m->A[q];
    a.sh[f] = t->lay[n].sh[f + 1];
    a.mask[f] = t->lay[n].mask[f + 1];
    ++f;
  }
  a.M = m->M[n];
  a.part = m->part;
  if (mark) HIP_TRY(hipEventRecord(mark[0], s));
  HIP_TRY(launch_mttkrp_n(RP, a, s));
  if (mark) HIP_TRY(hipEventRecord(mark[1], s));
  FixArgs fx{};
  fx.longs = m->plan[n].longs;
  fx.nlong = m->plan[n].nlong;
  fx.nbig = m->plan[n].nbig;
  fx.part = m->part;
  fx.M = m->M[n];
  fx.Ga = m->P;
  fx.Gb = m->ones;
  fx.H = m->H[n];
  fx.hinfo = m->hinfo[n];
  fx.st = m->st + n;
  HIP_TRY(launch_mttkrp_fix(RP, fx, s));
  ImpArgs ia{};
  ia.I = I;
  ia.A = m->A[n];
  ia.M = m->M[n];
  ia.H = m->H[n];
  ia.hi = m->hinfo[n];
  ia.ti_part = m->ti_part;
  ia.st = m->st + n;
  HIP_TRY(launch_importance(RP, false, ia, s));
  UpdArgs ua{};
  ua.I = I;
  ua.A = m->A[n];
  ua.M = m->M[n];
  ua.Z = m->Z[n];
  ua.H = m->H[n];
  ua.hi = m->hinfo[n];
  ua.st = m->st + n;
  ua.gpart = m->gpart;
  ua.gpart_obj = nullptr;
  ua.inner_part = m->inner_part;
  ua.cnt_part = m->cnt_part;
  ua.selmask = m->selmask[n];
  HIP_TRY(launch_select_update(RP, (int)SACD_UPDATE_GS, m->diag, false, ua, s));
  GramArgs g{};
  g.nparts = m->nparts[n];
  g.gpart = m->gpart;
  g.mpart = m->mpart;
  g.Gn = m->G64[n];
  g.Ga = m->P;  // sum over the Hadamard product of all Grams = sum(Gram_n * P * 1)
  g.Gb = m->ones;
  g.inner_part = m->inner_part;
  g.cnt_part = m->cnt_part;
  g.colcnt = m->colcnt[n];
  g.normX2 = t->norm2;
  g.with_f = 1;
  g.counter = m->gcounter;
  g.st = m->st + n;
  HIP_TRY(launch_gram_final(RP, g, s));
  if (mark) HIP_TRY(hipEventRecord(mark[2], s));
  return SACD_OK;
}

void drop_ngraph(sacd_nmodel *m) {
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->gexec = nullptr;
  m->graph = nullptr;
}

sacd_status ensure_ngraph(sacd_nmodel *m) {
  if (m->gexec) return SACD_OK;
  HIP_TRY(hipStreamBeginCapture(m->s, hipStreamCaptureModeThreadLocal));
  sacd_status st = SACD_OK;
  for (int n = 0; n < m->N && st == SACD_OK; ++n) st = enqueue_nsweep(m, n);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(m->s, &g);
  if (st != SACD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(SACD_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t ge = nullptr;
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(SACD_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  m->graph = g;
  m->gexec = ge;
  return SACD_OK;
}

sacd_status read_nstate(const sacd_nmodel *m, int n, ModeState *out) {
  HIP_TRY(hipMemcpyAsync(out, m->st + n, sizeof(ModeState), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

// Objective of the current factors from scratch: ||X||^2 - 2 <X, Xhat> + the
// sum over the Hadamard product of all Grams (FP64).
sacd_status nobjective_full(sacd_nmodel *m, double *f) {
  const sacd_ntensor *t = m->t;
  const int RP = m->RP, N = m->N;
  NFactors F{};
  for (int q = 0; q < N; ++q) F.A[q] = m->A[q];
  HIP_TRY(launch_inner_full_n(t->keys[0], t->vals[0], t->nnz, t->lay[0], F, RP, m->full_part, m->full_nparts,
                              m->full_out, m->full_cnt, m->s));
  std::vector<double> G((size_t)N * RP * RP);
  double inner = 0.0;
  for (int q = 0; q < N; ++q)
    HIP_TRY(hipMemcpyAsync(G.data() + (size_t)q * RP * RP, m->G64[q], sizeof(double) * RP * RP,
                           hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipMemcpyAsync(&inner, m->full_out, sizeof(double), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  double model = 0.0;
  for (int i = 0; i < RP * RP; ++i) {
    double p = 1.0;
    for (int q = 0; q < N; ++q) p *= G[(size_t)q * RP * RP + i];
    model += p;
  }
  *f = t->norm2 - 2.0 * inner + model;
  return SACD_OK;
}

sacd_status init_nmodel_impl(sacd_nmodel *m, uint64_t seed) {
  const sacd_ntensor *t = m->t;
  const int RP = m->RP, N = m->N;
  DevAlloc &A = m->mem;
  int maxI = 0, maxus = 1;
  for (int n = 0; n < N; ++n) {
    const int I = (int)t->dims[n];
    maxI = std::max(maxI, I);
    SACD_TRY(build_nplan(t, n, nway_units_per_block(RP), A, &m->plan[n]));
    maxus = std::max(maxus, m->plan[n].nslots);
    m->nparts[n] = (I + rows_per_block(RP) - 1) / rows_per_block(RP);
    const size_t IR = (size_t)I * RP;
    SACD_TRY(A.get_t(IR, &m->A[n]));
    SACD_TRY(A.get_t(IR, &m->Z[n]));
    SACD_TRY(A.get_t(IR, &m->M[n]));
    SACD_TRY(A.get_t(IR, &m->selmask[n]));
    SACD_TRY(A.get_t((size_t)RP * RP, &m->H[n]));
    SACD_TRY(A.get_t((size_t)RP * RP, &m->G64[n]));
    SACD_TRY(A.get_t(1, &m->hinfo[n]));
    SACD_TRY(A.get_t((size_t)RP, &m->colcnt[n]));
  }
  const int maxparts = (maxI + rows_per_block(RP) - 1) / rows_per_block(RP);
  SACD_TRY(A.get_t((size_t)N, &m->st));
  SACD_TRY(A.get_t((size_t)RP * RP, &m->P));
  SACD_TRY(A.get_t((size_t)RP * RP, &m->ones));
  SACD_TRY(A.get_t((size_t)maxus * RP, &m->part));
  SACD_TRY(A.get_t((size_t)maxparts * RP * RP, &m->gpart));
  SACD_TRY(A.get_t((size_t)std::max(maxparts, importance_blocks(RP, maxI)), &m->ti_part));
  SACD_TRY(A.get_t((size_t)maxparts, &m->inner_part));
  SACD_TRY(A.get_t((size_t)maxparts * RP, &m->cnt_part));
  SACD_TRY(A.get_t((size_t)gram_model_parts(RP), &m->mpart));
  SACD_TRY(A.get_t(1, &m->gcounter));
  SACD_TRY(A.get_t(4, &m->flag));
  m->full_nparts = 1024;
  SACD_TRY(A.get_t((size_t)m->full_nparts, &m->full_part));
  SACD_TRY(A.get_t(1, &m->full_out));
  SACD_TRY(A.get_t(4, &m->full_cnt));
  SACD_TRY(pinned_get(&m->h_pinned));
  hipStream_t s = m->s;
  HIP_TRY(hipMemsetAsync(m->st, 0, (size_t)N * sizeof(ModeState), s));
  HIP_TRY(hipMemsetAsync(m->full_cnt, 0, 16, s));
  HIP_TRY(hipMemsetAsync(m->gcounter, 0, sizeof(unsigned), s));
  unsigned long long off = 0;
  for (int n = 0; n < N; ++n) {
    const int I = (int)t->dims[n];
    HIP_TRY(launch_init_factor(m->A[n], I, m->R, RP, seed, off, s));
    off += (unsigned long long)I * m->R;
    HIP_TRY(hipMemsetAsync(m->Z[n], 0, sizeof(float) * I * RP, s));
    HIP_TRY(hipMemsetAsync(m->M[n], 0, sizeof(float) * I * RP, s));  // rows of empty slices stay zero
    HIP_TRY(hipMemsetAsync(m->selmask[n], 0, (size_t)I * RP, s));
    HIP_TRY(hipMemsetAsync(m->colcnt[n], 0, sizeof(long long) * RP, s));
  }
  for (int n = 0; n < N; ++n) SACD_TRY(nrecompute_gram(m, n));
  HIP_TRY(hipStreamSynchronize(s));
  return SACD_OK;
}

}  // namespace

extern "C" {

sacd_status sacd_create_ntensor(int32_t N, const int64_t *dims, int64_t nnz, const int32_t *idx, const float *vals,
                                const sacd_allocator *alloc, void *stream, sacd_ntensor **out) {
  if (!out) return fail(SACD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (N < 2 || N > kMaxModes) return fail(SACD_ERR_INVALID_ARG, "N = %d not in [2, %d]", (int)N, kMaxModes);
  if (!dims) return fail(SACD_ERR_INVALID_ARG, "dims is NULL");
  (void)hipGetLastError();
  int bits = 0;
  for (int n = 0; n < N; ++n) {
    if (dims[n] < 1 || dims[n] > 2147483647LL)
      return fail(SACD_ERR_INVALID_ARG, "dims[%d] = %lld not in [1, 2^31 - 1]", n, (long long)dims[n]);
    bits += bits_for(dims[n]);
  }
  if (bits > 64) return fail(SACD_ERR_INVALID_ARG, "mode lengths need %d > 64 key bits", bits);
  if (nnz < 0 || nnz > 2147483647LL) return fail(SACD_ERR_INVALID_ARG, "nnz = %lld not in [0, 2^31 - 1]", (long long)nnz);
  if (nnz > 0 && (!idx || !vals)) return fail(SACD_ERR_INVALID_ARG, "idx / vals is NULL");
  if (alloc && (!alloc->alloc || !alloc->release)) return fail(SACD_ERR_INVALID_ARG, "allocator callbacks are NULL");
  sacd_ntensor *t = new (std::nothrow) sacd_ntensor();
  if (!t) return fail(SACD_ERR_NO_MEMORY, "host allocation failed");
  if (hipGetDevice(&t->dev) != hipSuccess) {
    delete t;
    return fail(SACD_ERR_DEVICE, "no HIP device");
  }
  t->N = N;
  for (int n = 0; n < N; ++n) t->dims[n] = dims[n];
  if (alloc) {
    t->mem.alloc = *alloc;
    t->mem.custom = true;
  }
  sacd_status st = make_stream(stream, &t->stream, &t->own_stream);
  if (st == SACD_OK) st = create_ntensor_impl(t, idx, vals, nnz);
  if (st != SACD_OK) {
    release_ntensor(t);
    return st;
  }
  *out = t;
  return SACD_OK;
}

sacd_status sacd_ntensor_info(const sacd_ntensor *t, int32_t *N, int64_t *dims, int64_t *nnz, double *norm2,
                              int64_t *device_bytes) {
  if (!t) return fail(SACD_ERR_INVALID_ARG, "tensor is NULL");
  if (N) *N = t->N;
  if (dims)
    for (int n = 0; n < t->N; ++n) dims[n] = t->dims[n];
  if (nnz) *nnz = t->nnz;
  if (norm2) *norm2 = t->norm2;
  if (device_bytes) *device_bytes = t->mem.bytes;
  return SACD_OK;
}

sacd_status sacd_ntensor_mode_coo(const sacd_ntensor *t, int32_t mode, int32_t *coords, float *vals, int64_t *ptr) {
  if (!t) return fail(SACD_ERR_INVALID_ARG, "tensor is NULL");
  if (mode < 0 || mode >= t->N) return fail(SACD_ERR_INVALID_ARG, "mode %d not in [0, %d)", mode, t->N);
  SACD_TRY(enter(t->dev));
  HIP_TRY(launch_export_coo_n(t->keys[mode], t->vals[mode], t->nnz, t->lay[mode], coords, vals, t->ptr[mode],
                              (int)t->dims[mode], ptr, t->stream));
  HIP_TRY(hipStreamSynchronize(t->stream));
  return SACD_OK;
}

void sacd_destroy_ntensor(sacd_ntensor *t) {
  if (!t) return;
  if (t->nmodels > 0) {
    t->destroy_pending = true;
    return;
  }
  release_ntensor(t);
}

sacd_status sacd_init_nfactors(sacd_ntensor *t, int32_t R, uint64_t seed, sacd_nmodel **out) {
  if (!out) return fail(SACD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!t) return fail(SACD_ERR_INVALID_ARG, "tensor is NULL");
  if (R < 1 || R > kMaxRP) return fail(SACD_ERR_INVALID_ARG, "rank %d not in [1, %d]", R, kMaxRP);
  SACD_TRY(enter(t->dev));
  sacd_nmodel *m = new (std::nothrow) sacd_nmodel();
  if (!m) return fail(SACD_ERR_NO_MEMORY, "host allocation failed");
  m->t = t;
  m->s = t->stream;
  m->mem.alloc = t->mem.alloc;
  m->mem.custom = t->mem.custom;
  m->N = t->N;
  m->R = R;
  m->RP = pad_rank(R);
  sacd_status st = init_nmodel_impl(m, seed);
  if (st != SACD_OK) {
    sacd_destroy_nmodel(m);
    return st;
  }
  t->nmodels++;
  m->counted = true;
  *out = m;
  return SACD_OK;
}

sacd_status sacd_nsweep(sacd_nmodel *m, int32_t mode) {
  SACD_TRY(check_nmode(m, mode));
  SACD_TRY(enter(m->t->dev));
  SACD_TRY(enqueue_nsweep(m, mode));
  m->last_mode = mode;
  m->dirty = false;
  return SACD_OK;
}

sacd_status sacd_niterate(sacd_nmodel *m, int32_t n_iters) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  if (n_iters < 0) return fail(SACD_ERR_INVALID_ARG, "n_iters < 0");
  if (n_iters == 0) return SACD_OK;
  SACD_TRY(enter(m->t->dev));
  SACD_TRY(ensure_ngraph(m));
  for (int i = 0; i < n_iters; ++i) HIP_TRY(hipGraphLaunch(m->gexec, m->s));
  m->last_mode = m->N - 1;
  m->dirty = false;
  return SACD_OK;
}

sacd_status sacd_niterate_timed(sacd_nmodel *m, int32_t n_iters, float *mttkrp_ms, float *sweep_ms) {
  if (!m || !mttkrp_ms) return fail(SACD_ERR_INVALID_ARG, "model or output is NULL");
  if (n_iters < 1 || n_iters > 100000) return fail(SACD_ERR_INVALID_ARG, "n_iters out of [1, 100000]");
  SACD_TRY(enter(m->t->dev));
  const int N = m->N;
  while ((int)m->tev.size() < 3 * N * n_iters) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    m->tev.push_back(e);
  }
  for (int i = 0; i < n_iters; ++i)
    for (int n = 0; n < N; ++n) SACD_TRY(enqueue_nsweep(m, n, &m->tev[3 * (N * i + n)]));
  m->last_mode = N - 1;
  m->dirty = false;
  HIP_TRY(hipStreamSynchronize(m->s));
  for (int i = 0; i < n_iters; ++i)
    for (int n = 0; n < N; ++n) {
      const hipEvent_t *e = &m->tev[3 * (N * i + n)];
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, e[0], e[1]));
      mttkrp_ms[N * i + n] = ms;
      if (sweep_ms) {
        HIP_TRY(hipEventElapsedTime(&ms, e[0], e[2]));
        sweep_ms[N * i + n] = ms;
      }
    }
  return SACD_OK;
}

sacd_status sacd_nfit(sacd_nmodel *m, double *fit, double *objective) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  SACD_TRY(enter(m->t->dev));
  double f = 0.0;
  if (m->last_mode < 0 || m->dirty) {
    SACD_TRY(nobjective_full(m, &f));
  } else {
    ModeState s;
    SACD_TRY(read_nstate(m, m->last_mode, &s));
    f = s.f;
  }
  if (objective) *objective = f;
  if (!(m->t->norm2 > 0.0)) return fail(SACD_ERR_NUMERIC, "||X|| = 0: the fit is undefined");
  if (fit) *fit = 1.0 - std::sqrt(f > 0.0 ? f : 0.0) / std::sqrt(m->t->norm2);
  return SACD_OK;
}

sacd_status sacd_nrun_until(sacd_nmodel *m, double tol, int32_t max_iter, int32_t *iters_done, double *final_fit) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  if (max_iter < 1 || !(tol >= 0.0)) return fail(SACD_ERR_INVALID_ARG, "max_iter < 1 or tol < 0");
  if (!(m->t->norm2 > 0.0)) return fail(SACD_ERR_NUMERIC, "||X|| = 0: the fit is undefined");
  SACD_TRY(enter(m->t->dev));
  SACD_TRY(ensure_ngraph(m));
  const double nx = std::sqrt(m->t->norm2);
  double prev = 0.0, fit = 0.0;
  int it;
  for (it = 1; it <= max_iter; ++it) {
    HIP_TRY(hipGraphLaunch(m->gexec, m->s));
    HIP_TRY(hipMemcpyAsync(m->h_pinned, &m->st[m->N - 1].f, sizeof(double), hipMemcpyDeviceToHost, m->s));
    HIP_TRY(hipStreamSynchronize(m->s));
    m->last_mode = m->N - 1;
    m->dirty = false;
    const double f = m->h_pinned[0];
    fit = 1.0 - std::sqrt(f > 0.0 ? f : 0.0) / nx;
    if (it >= 2 && std::fabs(fit - prev) < tol * std::fabs(prev)) break;
    prev = fit;
  }
  if (it > max_iter) it = max_iter;
  if (iters_done) *iters_done = it;
  if (final_fit) *final_fit = fit;
  return SACD_OK;
}

sacd_status sacd_get_nfactor(const sacd_nmodel *m, int32_t mode, float *dst) {
  SACD_TRY(check_nmode(m, mode));
  if (!dst) return fail(SACD_ERR_INVALID_ARG, "dst is NULL");
  SACD_TRY(enter(m->t->dev));
  HIP_TRY(launch_copy_rows(m->A[mode], m->RP, dst, m->R, (int)m->t->dims[mode], m->R, m->R, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

sacd_status sacd_set_nfactor(sacd_nmodel *m, int32_t mode, const float *src) {
  SACD_TRY(check_nmode(m, mode));
  if (!src) return fail(SACD_ERR_INVALID_ARG, "src is NULL");
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  HIP_TRY(hipMemsetAsync(m->flag, 0, sizeof(int), m->s));
  HIP_TRY(launch_check_factor(src, (long long)I * m->R, m->flag, m->s));
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, m->flag, sizeof(int), hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  if (hflag) return fail(SACD_ERR_NUMERIC, "factor has negative or non-finite entries");
  HIP_TRY(launch_copy_rows(src, m->R, m->A[mode], m->RP, I, m->R, m->RP, m->s));
  SACD_TRY(nrecompute_gram(m, mode));
  HIP_TRY(hipStreamSynchronize(m->s));
  m->dirty = true;
  return SACD_OK;
}

sacd_status sacd_get_nstate(const sacd_nmodel *m, int32_t mode, float *zprev, double *ti_prev, int64_t *k) {
  SACD_TRY(check_nmode(m, mode));
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  if (zprev) HIP_TRY(launch_copy_rows(m->Z[mode], m->RP, zprev, m->R, I, m->R, m->R, m->s));
  ModeState s;
  SACD_TRY(read_nstate(m, mode, &s));
  if (ti_prev) *ti_prev = s.ti_prev;
  if (k) *k = s.k;
  return SACD_OK;
}

sacd_status sacd_set_nstate(sacd_nmodel *m, int32_t mode, const float *zprev, double ti_prev, int64_t k) {
  SACD_TRY(check_nmode(m, mode));
  if (k < 0) return fail(SACD_ERR_INVALID_ARG, "k < 0");
  if (k > 0 && !zprev) return fail(SACD_ERR_INVALID_ARG, "zprev is NULL with k > 0");
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode];
  if (zprev) HIP_TRY(launch_copy_rows(zprev, m->R, m->Z[mode], m->RP, I, m->R, m->RP, m->s));
  ModeState s;
  SACD_TRY(read_nstate(m, mode, &s));
  s.k = k;
  s.ti_prev = ti_prev;
  HIP_TRY(hipMemcpyAsync(m->st + mode, &s, sizeof(ModeState), hipMemcpyHostToDevice, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

sacd_status sacd_get_nstats(const sacd_nmodel *m, int32_t mode, sacd_sweep_stats *out) {
  SACD_TRY(check_nmode(m, mode));
  if (!out) return fail(SACD_ERR_INVALID_ARG, "out is NULL");
  SACD_TRY(enter(m->t->dev));
  ModeState s;
  SACD_TRY(read_nstate(m, mode, &s));
  out->k = s.k;
  out->lipschitz = s.L;
  out->ti = s.ti;
  out->flip = s.flip;
  out->n_selected = s.nsel;
  out->objective = s.f;
  return SACD_OK;
}

sacd_status sacd_get_ncolumn_counts(const sacd_nmodel *m, int32_t mode, int64_t *counts) {
  SACD_TRY(check_nmode(m, mode));
  if (!counts) return fail(SACD_ERR_INVALID_ARG, "counts is NULL");
  SACD_TRY(enter(m->t->dev));
  std::vector<long long> c((size_t)m->RP);
  HIP_TRY(hipMemcpyAsync(c.data(), m->colcnt[mode], sizeof(long long) * m->RP, hipMemcpyDeviceToHost, m->s));
  HIP_TRY(hipStreamSynchronize(m->s));
  for (int r = 0; r < m->R; ++r) counts[r] = (int64_t)c[(size_t)r];
  return SACD_OK;
}

sacd_status sacd_get_ndiagnostics(const sacd_nmodel *m, int32_t mode, float *mttkrp, uint8_t *selection,
                                  double *gram) {
  SACD_TRY(check_nmode(m, mode));
  SACD_TRY(enter(m->t->dev));
  const int I = (int)m->t->dims[mode], R = m->R, RP = m->RP;
  if (mttkrp) HIP_TRY(launch_copy_rows(m->M[mode], RP, mttkrp, R, I, R, R, m->s));
  if (selection)
    HIP_TRY(hipMemcpy2DAsync(selection, (size_t)R, m->selmask[mode], (size_t)RP, (size_t)R, (size_t)I,
                             hipMemcpyDeviceToDevice, m->s));
  if (gram) {
    std::vector<double> G((size_t)RP * RP);
    HIP_TRY(hipMemcpyAsync(G.data(), m->G64[mode], sizeof(double) * RP * RP, hipMemcpyDeviceToHost, m->s));
    HIP_TRY(hipStreamSynchronize(m->s));
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < R; ++j) gram[i * R + j] = G[(size_t)i * RP + j];
  }
  HIP_TRY(hipStreamSynchronize(m->s));
  return SACD_OK;
}

sacd_status sacd_set_ndiagnostics(sacd_nmodel *m, int32_t enable) {
  if (!m) return fail(SACD_ERR_INVALID_ARG, "model is NULL");
  const bool d = enable != 0;
  if (d != m->diag) {
    SACD_TRY(enter(m->t->dev));
    HIP_TRY(hipStreamSynchronize(m->s));
    drop_ngraph(m);
    m->diag = d;
  }
  return SACD_OK;
}

sacd_status sacd_nmodel_bytes(const sacd_nmodel *m, int64_t *bytes) {
  if (!m || !bytes) return fail(SACD_ERR_INVALID_ARG, "bad arguments");
  *bytes = m->mem.bytes;
  return SACD_OK;
}

void sacd_destroy_nmodel(sacd_nmodel *m) {
  if (!m) return;
  sacd_ntensor *t = m->t;
  (void)hipSetDevice(t->dev);
  if (m->s) (void)hipStreamSynchronize(m->s);
  drop_ngraph(m);
  for (hipEvent_t e : m->tev) (void)hipEventDestroy(e);
  m->tev.clear();
  m->mem.release_all();
  pinned_put(m->h_pinned);
  const bool counted = m->counted;
  delete m;
  if (counted && t->nmodels > 0) t->nmodels--;
  if (t->destroy_pending && t->nmodels == 0) release_ntensor(t);
}

}  // extern "C"
