// mttkrp.hip -- sparse MTTKRP of one mode (the first term of the gradient,
// eq. 9, in the slice form of Sec. 4.4):
//     M[i_n, :] = sum over Omega^n_{i_n} of x * (A_a[i_a, :] .* A_b[i_b, :])
//
// Work split: a static plan built once per tensor cuts every slice into
// segments of at most kSegment entries; each segment is one work unit, run by
// one lane group (LPN lanes, W columns each) from start to end, so the inner
// loop never meets a slice boundary.  Units are ordered longest first, so the
// groups of a wave run for about the same number of entries.  Entries are
// sorted by (i_n, i_a, i_b): a run sharing (i_n, i_a) -- a fibre -- gathers
// its A_a row once (A_b rows are gathered per entry).
// A slice held by one unit is written directly; the units of a longer slice
// write partial sums that the fix-up kernel adds in a fixed tree order, one
// block per such slice.  Empty slices are never written (M is zeroed when the
// model is set up).  No atomics: results are deterministic for a given tensor.
#include "common.hpp"

namespace sacd {

namespace {

// Four columns per lane (one float4 of a row), eight entries decoded per
// step (measured: 8 columns per lane and 10 or 12 entries per step were
// slower).
template <int RP>
struct MCfg {
  static constexpr int W = 4;          // columns per lane
  static constexpr int LPN = RP / W;   // lanes per unit
  static constexpr int NV = W / 4;     // float4 per lane
  static constexpr int U = 8;          // entries per step
};

__device__ __forceinline__ f32x4 ld4(const float *p) { return *(const f32x4 *)p; }
__device__ __forceinline__ void st4(float *p, f32x4 v) { *(f32x4 *)p = v; }

// One entry's contribution to four columns: acc + x (a .* b) -- the product
// a b rounded, then a fused multiply-add.  The plain kernel writes it as an
// expression, which the compiler contracts to exactly that (v_mul, v_fmac);
// the LDS-staged kernel spells the same two roundings with intrinsics (the
// expression there was scheduled into 25% slower code).  Both give the same
// sums bit for bit.
__device__ __forceinline__ f32x4 entry_fma(float x, f32x4 a, f32x4 b, f32x4 acc) { return x * (a * b) + acc; }
__device__ __forceinline__ f32x4 entry_fma_rn(float x, f32x4 a, f32x4 b, f32x4 acc) {
  f32x4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = __fmaf_rn(x, __fmul_rn(a[i], b[i]), acc[i]);
  return r;
}

// MTTKRP of one sweep.  Solo form (BATCHED false): block b is work item b
// of the job in `solo`.  Job-batched form: a persistent grid loops over the
// block map's entries (job in `jobs`, block of the job, blocks of the job).
// The body is written in the kernel itself rather than in a device function
// called by two kernels: the compiler then keeps the kernel-argument
// guarantees and schedules the row gathers without intermediate waits.
template <int RP, bool BATCHED>
__global__ __launch_bounds__(kThreads) void k_mttkrp(MttkrpArgs solo, const MttkrpArgs *__restrict__ jobs,
                                                     const int4 *__restrict__ bmap, int nb) {
 for (int item = blockIdx.x;; item += gridDim.x) {
  MttkrpArgs args;
  int blk;
  if constexpr (BATCHED) {
    if (item >= nb) break;
    const int4 m = bmap[item];
    args = jobs[m.x];
    blk = m.y;
  } else {
    args = solo;
    blk = blockIdx.x;
  }
  const unsigned long long *__restrict__ keys = args.keys;
  const float *__restrict__ vals = args.vals;
  const int4 *__restrict__ units = args.units;
  const int nunits = args.nunits;
  const KeyLayout lay = args.lay;
  const float *__restrict__ Aa = args.Aa;
  const float *__restrict__ Ab = args.Ab;
  float *__restrict__ M = args.M;
  float *__restrict__ part = args.part;
  using Cf = MCfg<RP>;
  constexpr int LPN = Cf::LPN, NV = Cf::NV, U = Cf::U;
  constexpr int UPB = kThreads / LPN;  // units per block
  __shared__ __align__(16) float s_acc[UPB * RP];
  __shared__ int s_slot[UPB];
  const int ub = threadIdx.x / LPN;  // unit within the block
  const int gid = blk * UPB + ub;
  const bool active = gid < nunits;
  // lane sub owns the float4 column chunks 4*sub + 4*LPN*j (j < NV): each
  // load instruction of a lane group covers contiguous bytes of a row
  const int sub = threadIdx.x % LPN;
  const int4 unit = active ? units[gid] : make_int4(0, 0, 0, -1);  // (slice, first, entries, slot)
  const long long p0 = unit.y;
  const int len = unit.z;

  f32x4 acc[NV], arow[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    arow[j] = acc[j];
  }
  // A unit lies in one slice, so its fibres are told apart by i_a alone.
  // Both row indices are decoded in 32 bits: i_b is the low field and i_a is
  // read across the word boundary by a funnel shift (sh_a < 32, and both
  // fields are narrower than 32 bits).
  const unsigned mb = (unsigned)lay.mask_b, ma = (unsigned)lay.mask_a, sha = (unsigned)lay.sh_a;
  const char *__restrict__ Ab_l = (const char *)(Ab + 4 * sub);
  const char *__restrict__ Aa_l = (const char *)(Aa + 4 * sub);
  constexpr int kRowShift = RP == 16 ? 6 : (RP == 32 ? 7 : (RP == 64 ? 8 : 9));  // log2 of a row's bytes
  static_assert((1 << kRowShift) == 4 * RP, "row size");
  unsigned fa = ~0u;  // i_a of the current fibre (never a valid index)
  // Each entry's key and value are loaded and decoded by one lane of the
  // group and handed to the group's other lanes through the LDS crossbar
  // (ds_bpermute), so the copies do not take vector-memory return cycles.
  // Lane sub owns entries sub, sub + LPN, ... of a batch.  Pipeline: the
  // raw entries of batch k + 1 are in flight while batch k's rows are
  // gathered and multiplied; then batch k + 1 is decoded and shared and the
  // raw entries of batch k + 2 are loaded.  The key and value arrays carry
  // kKeySlack zeroed entries past their end, so these loads need no bounds
  // test; entries past the unit are never used.
  constexpr int KPL = (U + LPN - 1) / LPN;  // entries loaded per lane and batch
  static_assert(2 * U <= kKeySlack, "raw loads run up to 2U - 1 entries past the unit");
  const int gb4 = (int)((threadIdx.x & 63u) & ~(unsigned)(LPN - 1)) * 4;  // group's first lane, bytes
  unsigned long long rk[KPL];
  float rx[KPL];
  unsigned ib[U], ia[U];
  float xv[U];
#define SACD_MT_LOAD_RAW(q)                                              \
  _Pragma("unroll") for (int k = 0; k < KPL; ++k) {                      \
    if (sub + LPN * k < U) {                                             \
      rk[k] = keys[p0 + (q) + sub + LPN * k];                            \
      rx[k] = vals[p0 + (q) + sub + LPN * k];                            \
    }                                                                    \
  }
#define SACD_MT_SHARE_RAW()                                                              \
  {                                                                                      \
    unsigned dib[KPL], dia[KPL];                                                         \
    _Pragma("unroll") for (int k = 0; k < KPL; ++k) {                                    \
      const unsigned lo = (unsigned)rk[k], hi = (unsigned)(rk[k] >> 32);                 \
      dib[k] = lo & mb;                                                                  \
      dia[k] = __builtin_amdgcn_alignbit(hi, lo, sha) & ma;                              \
    }                                                                                    \
    _Pragma("unroll") for (int u = 0; u < U; ++u) {                                      \
      const int src = gb4 + 4 * (u % LPN);                                               \
      ib[u] = (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)dib[u / LPN]);            \
      ia[u] = (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)dia[u / LPN]);            \
      xv[u] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(rx[u / LPN]))); \
    }                                                                                    \
  }
  SACD_MT_LOAD_RAW(0)
  SACD_MT_SHARE_RAW()
  SACD_MT_LOAD_RAW(U)
  int e = 0;
  // full batches: no per-entry predicate on the entry stream
  for (; e + U <= len; e += U) {
    bool nf[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      nf[u] = ia[u] != fa;
      fa = ia[u];
    }
    f32x4 bv[U][NV], av[U][NV];
    float xc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float *pb = (const float *)(Ab_l + ((size_t)ib[u] << kRowShift));
#pragma unroll
      for (int j = 0; j < NV; ++j) bv[u][j] = ld4(pb + 4 * LPN * j);
      if (nf[u]) {  // the A_a row is gathered once per fibre
        const float *pa = (const float *)(Aa_l + ((size_t)ia[u] << kRowShift));
#pragma unroll
        for (int j = 0; j < NV; ++j) av[u][j] = ld4(pa + 4 * LPN * j);
      }
      xc[u] = xv[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (nf[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) arow[j] = av[u][j];
      }
#pragma unroll
      for (int j = 0; j < NV; ++j) acc[j] = entry_fma(xc[u], arow[j], bv[u][j], acc[j]);
    }
    // batch k + 1 is shared after the products of batch k: sharing it
    // before them keeps its registers live across them and costs a wave
    SACD_MT_SHARE_RAW()
    SACD_MT_LOAD_RAW(e + 2 * U)
  }
#undef SACD_MT_LOAD_RAW
#undef SACD_MT_SHARE_RAW
  // the last, partial batch (fewer than U entries), predicated per entry
  if (e < len) {
    f32x4 bv[U][NV], av[U][NV];
    bool nf[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e + u < len;
      nf[u] = ok && ia[u] != fa;
      if (ok) fa = ia[u];
      if (ok) {
        const float *pb = (const float *)(Ab_l + ((size_t)ib[u] << kRowShift));
#pragma unroll
        for (int j = 0; j < NV; ++j) bv[u][j] = ld4(pb + 4 * LPN * j);
      }
      if (nf[u]) {
        const float *pa = (const float *)(Aa_l + ((size_t)ia[u] << kRowShift));
#pragma unroll
        for (int j = 0; j < NV; ++j) av[u][j] = ld4(pa + 4 * LPN * j);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (nf[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) arow[j] = av[u][j];
      }
      if (e + u < len) {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] = entry_fma(xv[u], arow[j], bv[u][j], acc[j]);
      }
    }
  }
  // A whole slice goes straight to M.  Segments of split slices are first
  // added up inside the block: consecutive units with the same partial slot
  // (the plan gives each such run of one slice its own slot) are summed in
  // unit order and the run's sum is written once.
  if (active && unit.w < 0) {
    float *dst = M + (long long)unit.x * RP + 4 * sub;
#pragma unroll
    for (int j = 0; j < NV; ++j) st4(dst + 4 * LPN * j, acc[j]);
  } else {
#pragma unroll
    for (int j = 0; j < NV; ++j) st4(&s_acc[ub * RP + 4 * sub + 4 * LPN * j], acc[j]);
  }
  if (threadIdx.x % LPN == 0) s_slot[ub] = active ? unit.w : -1;
  __syncthreads();
  for (int c = threadIdx.x; c < RP; c += kThreads) {
    int run = -1;
    float s = 0.0f;
    for (int q = 0; q < UPB; ++q) {
      const int w = s_slot[q];
      if (w != run) {
        if (run >= 0) part[(long long)run * RP + c] = s;
        run = w;
        s = 0.0f;
      }
      if (w >= 0) s += s_acc[q * RP + c];
    }
    if (run >= 0) part[(long long)run * RP + c] = s;
  }
  if constexpr (!BATCHED) break;
  __syncthreads();  // the block's LDS is reused by its next work item
 }
}

// MTTKRP with the per-entry table A_b staged in LDS, CS of its columns at a
// time (a column slab; S = RP / CS slabs), for modes whose A_b has few rows.
// Each entry then gathers only its A_a row chunk through the vector memory
// path; its A_b row chunk is read from LDS.  A block of kLdsThreads threads
// runs one slab of one block of kLdsUnits(CS) consecutive units of the plan,
// with CS / 4 lanes per unit: the lanes own the same four columns and add the
// same products in the same order as in k_mttkrp (entry_fma), and the split
// slices' runs -- which never span the plain kernel's blocks of units, and the
// block here covers a whole number of those -- are summed in the same unit
// order, so M is bit for bit that of k_mttkrp.  The S slab blocks of a unit
// block are numbered so that they go to one XCD one after the other, and the
// entry stream they all read is fetched from HBM about once.
//
// Tiled form (btab not null): for a mode whose A_b is too large for LDS, the
// model keeps its own copy of the mode's entries ordered by (i_n, i_b tile,
// i_a, i_b), tiles of kTileRows rows of A_b, and a block table: block q runs
// units [u0, u0 + nu) of the plan, all inside one tile, with rows
// [b0, b0 + rows) of A_b staged (btab[q] = (u0, nu, b0, rows)).  The entries
// a block reads then gather only their A_a rows through the vector memory
// path, and the A_b rows of a tile are read from HBM about once per slab.
constexpr int kLdsThreads = 1024;
constexpr int kLdsU = 6;  // entries per step: 1024 threads leave 128 VGPRs per lane (measured: 4, 6, 8 at 512 to 1024 threads)
constexpr long long kLdsTableBytes = 128 * 1024;  // the A_b slab; the run sums add 16 KB

template <int RP, int CS>
__global__ __launch_bounds__(kLdsThreads) void k_mttkrp_lds(MttkrpArgs args, int Ib, int nub,
                                                            const int4 *__restrict__ btab) {
  constexpr int S = RP / CS, LPN = CS / 4, UPB = kLdsThreads / LPN, U = kLdsU;
  extern __shared__ __align__(16) float smem[];  // A_b slab (Ib x CS), then UPB x CS run sums
  __shared__ int s_slot[UPB];
  // block -> (unit block, slab); blocks are dealt to the 8 XCDs round robin
  const int bx = blockIdx.x & 7, bk = blockIdx.x >> 3;
  const int ublk = 8 * (bk / S) + bx, slab = bk % S;
  if (ublk >= nub) return;  // the whole block, before any barrier
  const int c0 = slab * CS;
  const unsigned long long *__restrict__ keys = args.keys;
  const float *__restrict__ vals = args.vals;
  const float *__restrict__ Aa = args.Aa;
  const float *__restrict__ Ab = args.Ab;
  float *__restrict__ M = args.M;
  float *__restrict__ part = args.part;
  // units of this block and the rows of A_b it stages
  int u0 = ublk * UPB, nu = UPB, b0 = 0, rows = Ib;
  if (btab) {
    const int4 bt = btab[ublk];
    u0 = bt.x;
    nu = bt.y;
    b0 = bt.z;
    rows = bt.w;
  }
  float *sB = smem;
  float *s_acc = smem + (size_t)(btab ? kTileRows : Ib) * CS;
  for (int i = threadIdx.x; i < rows * (CS / 4); i += kLdsThreads) {
    const int r = i / (CS / 4), q = i % (CS / 4);
    st4(sB + (size_t)r * CS + 4 * q, ld4(Ab + (long long)(b0 + r) * RP + c0 + 4 * q));
  }
  __syncthreads();
  const int ub = threadIdx.x / LPN;
  const int gid = u0 + ub;
  const bool active = ub < nu && gid < args.nunits;
  const int sub = threadIdx.x % LPN;
  const int4 unit = active ? args.units[gid] : make_int4(0, 0, 0, -1);
  const long long p0 = unit.y;
  const int len = unit.z;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f}, arow = acc;
  const KeyLayout lay = args.lay;
  const unsigned mb = (unsigned)lay.mask_b, ma = (unsigned)lay.mask_a, sha = (unsigned)lay.sh_a;
  const char *__restrict__ Aa_l = (const char *)(Aa + c0 + 4 * sub);
  const float *sB_l = sB + 4 * sub;
  const unsigned ub0 = (unsigned)b0;  // row i_b sits at i_b - b0 of the staged rows
  constexpr int kRowShift = RP == 16 ? 6 : (RP == 32 ? 7 : (RP == 64 ? 8 : 9));
  static_assert((1 << kRowShift) == 4 * RP, "row size");
  unsigned fa = ~0u;
  constexpr int KPL = (U + LPN - 1) / LPN;
  static_assert(2 * U <= kKeySlack, "raw loads run up to 2U - 1 entries past the unit");
  const int gb4 = (int)((threadIdx.x & 63u) & ~(unsigned)(LPN - 1)) * 4;
  unsigned long long rk[KPL];
  float rx[KPL];
  unsigned ib[U], ia[U];
  float xv[U];
#define SACD_MT_LOAD_RAW(q)                                              \
  _Pragma("unroll") for (int k = 0; k < KPL; ++k) {                      \
    if (sub + LPN * k < U) {                                             \
      rk[k] = keys[p0 + (q) + sub + LPN * k];                            \
      rx[k] = vals[p0 + (q) + sub + LPN * k];                            \
    }                                                                    \
  }
#define SACD_MT_SHARE_RAW()                                                              \
  {                                                                                      \
    unsigned dib[KPL], dia[KPL];                                                         \
    _Pragma("unroll") for (int k = 0; k < KPL; ++k) {                                    \
      const unsigned lo = (unsigned)rk[k], hi = (unsigned)(rk[k] >> 32);                 \
      dib[k] = lo & mb;                                                                  \
      dia[k] = __builtin_amdgcn_alignbit(hi, lo, sha) & ma;                              \
    }                                                                                    \
    _Pragma("unroll") for (int u = 0; u < U; ++u) {                                      \
      const int src = gb4 + 4 * (u % LPN);                                               \
      ib[u] = (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)dib[u / LPN]);            \
      ia[u] = (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)dia[u / LPN]);            \
      xv[u] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(rx[u / LPN]))); \
    }                                                                                    \
  }
  SACD_MT_LOAD_RAW(0)
  SACD_MT_SHARE_RAW()
  SACD_MT_LOAD_RAW(U)
  int e = 0;
  for (; e + U <= len; e += U) {
    bool nf[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      nf[u] = ia[u] != fa;
      fa = ia[u];
    }
    f32x4 bv[U], av[U];
    float xc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (nf[u]) av[u] = ld4((const float *)(Aa_l + ((size_t)ia[u] << kRowShift)));
      bv[u] = *(const f32x4 *)(sB_l + (size_t)(ib[u] - ub0) * CS);
      xc[u] = xv[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (nf[u]) arow = av[u];
      acc = entry_fma_rn(xc[u], arow, bv[u], acc);
    }
    SACD_MT_SHARE_RAW()
    SACD_MT_LOAD_RAW(e + 2 * U)
  }
#undef SACD_MT_LOAD_RAW
#undef SACD_MT_SHARE_RAW
  if (e < len) {
    f32x4 bv[U], av[U];
    bool nf[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e + u < len;
      nf[u] = ok && ia[u] != fa;
      if (ok) fa = ia[u];
      if (ok) bv[u] = *(const f32x4 *)(sB_l + (size_t)(ib[u] - ub0) * CS);
      if (nf[u]) av[u] = ld4((const float *)(Aa_l + ((size_t)ia[u] << kRowShift)));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (nf[u]) arow = av[u];
      if (e + u < len) acc = entry_fma_rn(xv[u], arow, bv[u], acc);
    }
  }
  if (active && unit.w < 0) {
    st4(M + (long long)unit.x * RP + c0 + 4 * sub, acc);
  } else {
    st4(&s_acc[ub * CS + 4 * sub], acc);
  }
  if (sub == 0) s_slot[ub] = active ? unit.w : -1;
  __syncthreads();
  for (int c = threadIdx.x; c < CS; c += kLdsThreads) {
    int run = -1;
    float sum = 0.0f;
    for (int q = 0; q < UPB; ++q) {
      const int w = s_slot[q];
      if (w != run) {
        if (run >= 0) part[(long long)run * RP + c0 + c] = sum;
        run = w;
        sum = 0.0f;
      }
      if (w >= 0) sum += s_acc[q * CS + c];
    }
    if (run >= 0) part[(long long)run * RP + c0 + c] = sum;
  }
}

}  // namespace

int mttkrp_units_per_block(int RP) {
  switch (RP) {
    case 16: return kThreads / MCfg<16>::LPN;
    case 32: return kThreads / MCfg<32>::LPN;
    case 64: return kThreads / MCfg<64>::LPN;
    default: return kThreads / MCfg<128>::LPN;
  }
}

namespace {

// Fix-up: blocks [0, nbig) add the partial sums of one split slice with more
// than kFixSmall slots each, in a fixed tree order; the next blocks add those
// of the smaller split slices, one per row of lanes, in slot order; the last
// block forms H = Gram_a * Gram_b, L = ||H||_F
// and the diagonal of H for the element kernels of this sweep (eq. 10,
// eq. 15, Alg. 1).  Empty slices are never written: M is zeroed when the
// model is set up.  The slice sums need every MTTKRP block to have finished,
// which the kernel boundary provides; done inside the MTTKRP, each block
// would need a device-scope fence, which writes back and invalidates the L2
// that the row gathers rely on (measured 5-8x slower).
template <int RP, bool BATCHED>
__global__ __launch_bounds__(kThreads) void k_mttkrp_fix(FixArgs solo, const FixArgs *__restrict__ jobs,
                                                         const int4 *__restrict__ bmap, int nb) {
 for (int item = blockIdx.x;; item += gridDim.x) {
  FixArgs args;
  int blk;
  if constexpr (BATCHED) {
    if (item >= nb) break;
    const int4 m = bmap[item];
    args = jobs[m.x];
    blk = m.y;
  } else {
    args = solo;
    blk = blockIdx.x;
  }
  do {
  const int4 *__restrict__ longs = args.longs;
  const int nlong = args.nlong;
  const float *__restrict__ part = args.part;
  float *__restrict__ M = args.M;
  const double *__restrict__ Ga = args.Ga;
  const double *__restrict__ Gb = args.Gb;
  float *__restrict__ H = args.H;
  HInfo *hinfo = args.hinfo;
  ModeState *st = args.st;
  const int b = blk, tid = threadIdx.x;
  constexpr int Q = RP / 4;          // lanes per row (float4 each)
  constexpr int NS = kThreads / Q;   // rows of lanes per block
  const int nbig = args.nbig;
  const int nsb = (nlong - nbig + NS - 1) / NS;  // blocks of small split slices
  if (b < nbig) {
    // a split slice with many slots: NS lanes rows over its slots, then a tree
    const int4 L = longs[b];  // (slice, first slot, slots, -)
    __shared__ f32x4 red[NS][Q];
    const int slot = tid / Q, q = tid % Q;
    f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int j = slot; j < L.z; j += NS) s += ld4(part + (long long)(L.y + j) * RP + 4 * q);
    red[slot][q] = s;
    __syncthreads();
    for (int w = NS / 2; w > 0; w >>= 1) {
      if (slot < w) red[slot][q] += red[slot + w][q];
      __syncthreads();
    }
    if (slot == 0) st4(M + (long long)L.x * RP + 4 * q, red[0][q]);
    break;
  }
  if (b < nbig + nsb) {
    // small split slices, one per row of lanes: its (at most kFixSmall)
    // slots loaded together, then added in slot order
    const int g = nbig + (b - nbig) * NS + tid / Q, q = tid % Q;
    if (g < nlong) {
      const int4 L = longs[g];
      f32x4 v[kFixSmall];
#pragma unroll
      for (int j = 0; j < kFixSmall; ++j)
        v[j] = j < L.z ? ld4(part + (long long)(L.y + j) * RP + 4 * q) : f32x4{0.f, 0.f, 0.f, 0.f};
      f32x4 s = v[0];
#pragma unroll
      for (int j = 1; j < kFixSmall; ++j)
        if (j < L.z) s += v[j];
      st4(M + (long long)L.x * RP + 4 * q, s);
    }
    break;
  }
  // H, L, diagonal.  The loads of a chunk of CH entries per thread are
  // issued before any of them is used (one block does all RP x RP entries: a
  // load, multiply and store at a time would wait on every load).
  __shared__ double l2[kThreads];
  __shared__ float mx[kThreads];
  double s2 = 0.0;
  {
    constexpr int PER = (RP * RP + kThreads - 1) / kThreads;  // entries per thread
    constexpr int CH = PER < 16 ? PER : 16;
    static_assert(PER % CH == 0, "whole chunks");
#pragma unroll 1
    for (int c0 = 0; c0 < PER; c0 += CH) {
      double ga[CH], gb[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = tid + (c0 + k) * kThreads;
        ga[k] = i < RP * RP ? Ga[i] : 0.0;
        gb[k] = i < RP * RP ? Gb[i] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = tid + (c0 + k) * kThreads;
        const double h = ga[k] * gb[k];
        if (i < RP * RP) H[i] = (float)h;
        s2 += h * h;
      }
    }
  }
  float dmax = 0.0f;
  for (int r = tid; r < RP; r += kThreads) {
    const float d = (float)(Ga[r * RP + r] * Gb[r * RP + r]);
    hinfo->hdiag[r] = d;
    dmax = fmaxf(dmax, d);
  }
  l2[tid] = s2;
  mx[tid] = dmax;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      l2[tid] += l2[tid + w];
      mx[tid] = fmaxf(mx[tid], mx[tid + w]);
    }
    __syncthreads();
  }
  const double L = sqrt(l2[0]);
  const float hmax = mx[0];
  for (int r = tid; r < RP; r += kThreads) {
    const float d = (float)(Ga[r * RP + r] * Gb[r * RP + r]);
    hinfo->nearzero[r] = (d > 0.0f && d < 1e-6f * hmax) ? 1 : 0;
  }
  if (tid == 0) {
    hinfo->L64 = L;
    hinfo->L32 = (float)L;
    hinfo->halfL = 0.5f * (float)L;
    st->L = L;
  }
  } while (0);
  if constexpr (!BATCHED) break;
  __syncthreads();  // the block's LDS is reused by its next work item
 }
}

template <template <int> class F, typename... Args>
hipError_t rp_dispatch(int RP, Args &&...args) {
  switch (RP) {
    case 16: return F<16>::run(args...);
    case 32: return F<32>::run(args...);
    case 64: return F<64>::run(args...);
    case 128: return F<128>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <int RP>
struct MtL {
  static hipError_t run(const MttkrpArgs &a, hipStream_t s) {
    const int nb = mttkrp_blocks(RP, a.nunits);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_mttkrp<RP, false>), dim3(nb), dim3(kThreads), 0, s, a, nullptr, nullptr, 0);
    return hipGetLastError();
  }
};

template <int RP>
struct MtBL {
  static hipError_t run(const MttkrpArgs *jobs, const int4 *bmap, int nb, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_mttkrp<RP, true>), dim3(persistent_grid(nb)), dim3(kThreads), 0, s, MttkrpArgs{},
                       jobs, bmap, nb);
    return hipGetLastError();
  }
};

template <int RP>
struct FxL {
  static hipError_t run(const FixArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_mttkrp_fix<RP, false>), dim3(fix_blocks(RP, a.nlong, a.nbig)), dim3(kThreads), 0, s, a, nullptr,
                       nullptr, 0);
    return hipGetLastError();
  }
};

template <int RP>
struct FxBL {
  static hipError_t run(const FixArgs *jobs, const int4 *bmap, int nb, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_mttkrp_fix<RP, true>), dim3(persistent_grid(nb)), dim3(kThreads), 0, s, FixArgs{}, jobs,
                       bmap, nb);
    return hipGetLastError();
  }
};

}  // namespace

// Columns per slab of the LDS-staged form for a per-entry table of Ib rows,
// or 0 for the plain kernel.  The staged form pays where the row gathers
// dominate: at RP >= 64, with slabs of 64 columns (one pass at RP = 64, two at
// 128) whose Ib rows fit kLdsTableBytes.  At RP <= 32 every entry's key and
// value handling, repeated per slab, outweighs the 128-byte gather it saves
// (measured 1.7-1.9x slower on the 1e7-entry Zipf tensor at R = 32).
int mttkrp_lds_cols(int RP, long long Ib) {
  if (RP < 64) return 0;
  return Ib * 64 * 4 <= kLdsTableBytes ? 64 : 0;
}

template <int RP, int CS>
static hipError_t launch_lds(const MttkrpArgs &a, int Ib, const int4 *btab, int nbt, hipStream_t s) {
  constexpr int UPB = kLdsThreads / (CS / 4);
  static_assert(UPB % (kThreads / MCfg<RP>::LPN) == 0, "a block covers whole blocks of the plain kernel");
  const int nub = btab ? nbt : (a.nunits + UPB - 1) / UPB;
  if (nub == 0) return hipSuccess;
  const int S = RP / CS;
  const int nb = 8 * S * ((nub + 7) / 8);
  const long long rows = btab ? kTileRows : Ib;
  const size_t shm = ((size_t)rows * CS + (size_t)UPB * CS) * sizeof(float);
  if (rows * CS * 4 > kLdsTableBytes) return hipErrorInvalidValue;
  // more dynamic LDS than the default limit: allowed once per kernel
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(&k_mttkrp_lds<RP, CS>), hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(kLdsTableBytes + (long long)UPB * CS * sizeof(float)));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k_mttkrp_lds<RP, CS>), dim3(nb), dim3(kLdsThreads), shm, s, a, Ib, nub, btab);
  return hipGetLastError();
}

hipError_t launch_mttkrp_lds(int RP, int CS, const MttkrpArgs &a, int Ib, const int4 *btab, int nbt,
                             hipStream_t s) {
  if (CS != 64) return hipErrorInvalidValue;
  switch (RP) {
    case 64: return launch_lds<64, 64>(a, Ib, btab, nbt, s);
    case 128: return launch_lds<128, 64>(a, Ib, btab, nbt, s);
    default: return hipErrorInvalidValue;
  }
}

int mttkrp_lds_units_per_block(int CS) { return kLdsThreads / (CS / 4); }

int mttkrp_blocks(int RP, int nunits) {
  const int upb = mttkrp_units_per_block(RP);
  return (nunits + upb - 1) / upb;
}
int fix_blocks(int RP, int nlong, int nbig) {
  const int ns = kThreads / (RP / 4);
  return nbig + (nlong - nbig + ns - 1) / ns + 1;
}

hipError_t launch_mttkrp(int RP, const MttkrpArgs &a, hipStream_t s) { return rp_dispatch<MtL>(RP, a, s); }
hipError_t launch_mttkrp_b(int RP, const MttkrpArgs *jobs, const int4 *bmap, int nblocks, hipStream_t s) {
  return rp_dispatch<MtBL>(RP, jobs, bmap, nblocks, s);
}
hipError_t launch_mttkrp_fix(int RP, const FixArgs &a, hipStream_t s) { return rp_dispatch<FxL>(RP, a, s); }
hipError_t launch_mttkrp_fix_b(int RP, const FixArgs *jobs, const int4 *bmap, int nblocks, hipStream_t s) {
  return rp_dispatch<FxBL>(RP, jobs, bmap, nblocks, s);
}

}  // namespace sacd
