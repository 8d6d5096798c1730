// nway.hip -- kernels of the N-way form (Sec. 3: nonnegative tensor
// factorization of N modes).  Mode n's entries are a sorted stream of 64-bit
// keys packing i_n in the high bits and the other indices below it in
// increasing mode order (so a slice is a contiguous run), with slice
// pointers, as for three modes.  The MTTKRP multiplies the N - 1 other rows
// (eq. 9 with the Khatri-Rao product of all the other factors); H is the
// Hadamard product of the N - 1 other Gram matrices (eq. 10).  The element
// kernels of the three-way sweep (importance, selection and update, Gram
// reduction and objective) are mode-agnostic and are used as they are: they
// take H, and the objective's sum over the Hadamard product of all Grams comes
// out of k_gram_final given the product of the other Grams and a matrix of
// ones.
#include "common.hpp"

namespace sacd {

namespace {

__device__ __forceinline__ f32x4 ld4n(const float *p) { return *(const f32x4 *)p; }

// Mode-0 keys of the input entries: i_0 in the high field, i_{N-1} lowest;
// err bit 1: an index outside dims, bit 2: a NaN or Inf value.
__global__ __launch_bounds__(kThreads) void k_make_keys_n(const int32_t *__restrict__ idx,
                                                          const float *__restrict__ vals, long long nnz,
                                                          NLayout lay, unsigned long long *__restrict__ keys,
                                                          float *__restrict__ vout, int *err) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (long long)gridDim.x * blockDim.x) {
    unsigned long long k = 0;
    int bad = 0;
    for (int f = 0; f < lay.nf; ++f) {
      const int i = idx[p * lay.nf + f];  // field f of the mode-0 layout is mode f
      if (i < 0 || (long long)i >= lay.dims[f]) bad = 1;
      k |= ((unsigned long long)(unsigned)i & lay.mask[f]) << lay.sh[f];
    }
    const float v = vals[p];
    if (bad) atomicOr(err, 1);
    if (!isfinite(v)) atomicOr(err, 2);
    keys[p] = k;
    vout[p] = v;
  }
}

// Mode-0 keys re-encoded in mode n's layout: mode m's index moves from
// shift l0.sh[m] to to_sh[m], its shift in mode n's layout.
__global__ __launch_bounds__(kThreads) void k_rekey_n(const unsigned long long *__restrict__ k0, long long nnz,
                                                      NLayout l0, NShifts to_sh,
                                                      unsigned long long *__restrict__ kn) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (long long)gridDim.x * blockDim.x) {
    const unsigned long long k = k0[p];
    unsigned long long o = 0;
    for (int m = 0; m < l0.nf; ++m) o |= ((k >> l0.sh[m]) & l0.mask[m]) << to_sh.sh[m];
    kn[p] = o;
  }
}

// Mode n's sorted entries as coordinates (field order: i_n, then the other
// indices in increasing mode order), values, and 64-bit slice pointers.
__global__ __launch_bounds__(kThreads) void k_export_coo_n(const unsigned long long *__restrict__ keys,
                                                           const float *__restrict__ vals, long long nnz,
                                                           NLayout lay, int32_t *coords, float *vout,
                                                           const int *__restrict__ ptr, int I, int64_t *ptr64) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (long long)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[p];
    if (coords)
      for (int f = 0; f < lay.nf; ++f) coords[p * lay.nf + f] = (int32_t)((k >> lay.sh[f]) & lay.mask[f]);
    if (vout) vout[p] = vals[p];
  }
  if (ptr64)
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i <= I;
         i += (long long)gridDim.x * blockDim.x)
      ptr64[i] = ptr[i];
}

// Columns of the N-way MTTKRP: one lane group of RP / 4 lanes (four columns
// each) per work unit of the plan (a segment of one slice), entries in
// order, x times the product of the NO = N - 1 other rows added per column.
// The entries of a slice are sorted by the other indices in increasing mode
// order, so consecutive entries often share a prefix of them (a fibre and
// deeper): the running products of the rows of fields 0..f are kept, and an
// entry gathers and multiplies only the rows from its first field that
// differs from the previous entry's (the products are formed left to right
// either way, so the sums are the same).  Entries go in batches of U: each
// entry's key and value are loaded by one lane of the group and handed to
// the others through the LDS crossbar (ds_bpermute); the raw entries of
// batch k + 1 are in flight while batch k's rows are gathered and
// multiplied.  The gathers of a batch are all in flight together, so the
// entries in flight per SIMD are U times the waves that fit, and the U x NO
// rows held in registers set both (measured on a 4-way tensor at R = 32:
// U = 4 at four waves per SIMD beats U = 8 at two by 13%; staging the last
// field's small factor in LDS gained nothing).  The key and value arrays
// carry kKeySlack zeroed entries past their end, so these loads (at most
// 2U - 1 past a unit) need no bounds test.  A whole slice is written to M;
// the segments of a split slice that share a block are summed in LDS into
// one partial slot per run, which k_mttkrp_fix adds in a fixed order.
constexpr int kNU = 4;  // entries per batch

template <int RP, int NO>
__global__ __launch_bounds__(kThreads) void k_mttkrp_n(NMttkrpArgs a) {
  constexpr int LPN = RP / 4, UPB = kThreads / LPN, U = kNU;
  constexpr int KPL = (U + LPN - 1) / LPN;  // raw entries loaded per lane and batch
  constexpr int kRowShift = RP == 16 ? 6 : (RP == 32 ? 7 : (RP == 64 ? 8 : 9));
  static_assert((1 << kRowShift) == 4 * RP, "row size");
  static_assert(2 * U <= kKeySlack, "raw loads run up to 2U - 1 entries past the unit");
  const int ub = threadIdx.x / LPN, sub = threadIdx.x % LPN;
  const unsigned long long *__restrict__ keys = a.keys;
  const float *__restrict__ vals = a.vals;
  const char *Al[NO];
  int sh[NO];
  unsigned long long mk[NO];
#pragma unroll
  for (int f = 0; f < NO; ++f) {
    Al[f] = (const char *)(a.A[f] + 4 * sub);
    sh[f] = a.sh[f];
    mk[f] = a.mask[f];
  }
  const int gb4 = (int)((threadIdx.x & 63u) & ~(unsigned)(LPN - 1)) * 4;  // group's first lane, bytes
  const int gid = blockIdx.x * UPB + ub;
  const bool active = gid < a.nunits;
  const int4 unit = active ? a.units[gid] : make_int4(0, 0, 0, -1);  // (slice, first entry, entries, -)
  const long long p0 = unit.y;
  const int len = unit.z;
  unsigned long long rk[KPL];
  float rx[KPL];
  unsigned long long kv[U];
  float xv[U];
#define SACD_MN_LOAD_RAW(q)                                \
  _Pragma("unroll") for (int k = 0; k < KPL; ++k) {        \
    if (sub + LPN * k < U) {                               \
      rk[k] = keys[p0 + (q) + sub + LPN * k];              \
      rx[k] = vals[p0 + (q) + sub + LPN * k];              \
    }                                                      \
  }
#define SACD_MN_SHARE_RAW()                                                                              \
  _Pragma("unroll") for (int u = 0; u < U; ++u) {                                                        \
    const int src = gb4 + 4 * (u % LPN);                                                                 \
    const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)(unsigned)rk[u / LPN]);         \
    const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)(unsigned)(rk[u / LPN] >> 32)); \
    kv[u] = ((unsigned long long)hi << 32) | lo;                                                         \
    xv[u] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(rx[u / LPN])));              \
  }
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 pre[NO];  // pre[f]: product of the rows of fields 0..f of the previous entry
#pragma unroll
  for (int f = 0; f < NO; ++f) pre[f] = acc;
  unsigned long long pk = 0;  // previous entry's key
  bool have = false;          // pre holds a previous entry's products
  SACD_MN_LOAD_RAW(0)
  SACD_MN_SHARE_RAW()
  SACD_MN_LOAD_RAW(U)
  for (int e = 0; e < len; e += U) {
    const bool full = e + U <= len;
    int lv[U];  // first field whose row is read (NO: none)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int l = NO;
#pragma unroll
      for (int f = NO - 1; f >= 0; --f)
        if (((kv[u] ^ pk) >> sh[f]) & mk[f]) l = f;
      if (!have) l = 0;
      const bool ok = full || e + u < len;
      lv[u] = ok ? l : NO;
      if (ok) {
        pk = kv[u];
        have = true;
      }
    }
    f32x4 row[U][NO];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int f = 0; f < NO; ++f)
        if (f >= lv[u]) {
          const size_t off = (size_t)((kv[u] >> sh[f]) & mk[f]) << kRowShift;
          row[u][f] = ld4n((const float *)(Al[f] + off));
        }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int f = 0; f < NO; ++f)
        if (f >= lv[u]) pre[f] = f == 0 ? row[u][0] : pre[f - 1] * row[u][f];
      if (full || e + u < len) acc = xv[u] * pre[NO - 1] + acc;
    }
    SACD_MN_SHARE_RAW()
    // batch k + 2's raw entries, if it has any: the loads then end at most
    // U - 1 entries past the unit, inside the slack
    if (e + 2 * U < len) {
      SACD_MN_LOAD_RAW(e + 2 * U)
    }
  }
#undef SACD_MN_LOAD_RAW
#undef SACD_MN_SHARE_RAW
  // A whole slice goes straight to M.  Segments of split slices are first
  // added up inside the block: consecutive units with the same run slot are
  // summed in unit order and the run's sum is written once.
  __shared__ __align__(16) float s_acc[UPB * RP];
  __shared__ int s_slot[UPB];
  if (active && unit.w < 0) *(f32x4 *)(a.M + (long long)unit.x * RP + 4 * sub) = acc;
  else *(f32x4 *)(s_acc + ub * RP + 4 * sub) = acc;
  if (sub == 0) s_slot[ub] = active ? unit.w : -1;
  __syncthreads();
  for (int c = threadIdx.x; c < RP; c += kThreads) {
    int run = -1;
    float sum = 0.0f;
    for (int q = 0; q < UPB; ++q) {
      const int w = s_slot[q];
      if (w != run) {
        if (run >= 0) a.part[(long long)run * RP + c] = sum;
        run = w;
        sum = 0.0f;
      }
      if (w >= 0) sum += s_acc[q * RP + c];
    }
    if (run >= 0) a.part[(long long)run * RP + c] = sum;
  }
}

// P = Hadamard product of the Gram matrices of every mode but n (FP64, modes
// in increasing order), and a matrix of ones beside it.
__global__ __launch_bounds__(kThreads) void k_prod_grams(NGrams g, int n, int RP, double *__restrict__ P,
                                                         double *__restrict__ ones) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < RP * RP; i += gridDim.x * blockDim.x) {
    double v = 1.0;
    for (int m = 0; m < g.n; ++m)
      if (m != n) v *= g.G[m][i];
    P[i] = v;
    ones[i] = 1.0;
  }
}

// <X, Xhat> over the entries (mode-0 layout), FP64, per-block partials, the
// last block adds them in a fixed order.
__global__ __launch_bounds__(kThreads) void k_inner_full_n(const unsigned long long *__restrict__ keys,
                                                           const float *__restrict__ vals, long long nnz,
                                                           NLayout lay, NFactors F, int RP,
                                                           double *__restrict__ part, double *out,
                                                           unsigned *counter) {
  __shared__ double red[kThreads / 64];
  __shared__ int s_last;
  double s = 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (long long)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[p];
    double xh = 0.0;
    for (int r = 0; r < RP; ++r) {
      double prod = 1.0;
      for (int m = 0; m < lay.nf; ++m) {
        const unsigned long long i = (k >> lay.sh[m]) & lay.mask[m];
        prod *= (double)F.A[m][i * RP + r];
      }
      xh += prod;
    }
    s += (double)vals[p] * xh;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
    fence_release_device();
    s_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  fence_acquire_device();
  double t = 0.0;
  for (unsigned b = 0; b < gridDim.x; ++b) t += *(volatile double *)&part[b];
  *out = t;
  *counter = 0;
}

int grid_n(long long n) {
  long long g = (n + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

}  // namespace

hipError_t launch_make_keys_n(const int32_t *idx, const float *vals, long long nnz, const NLayout &lay,
                              unsigned long long *keys, float *vout, int *err, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_make_keys_n, dim3(grid_n(nnz)), dim3(kThreads), 0, s, idx, vals, nnz, lay, keys, vout, err);
  return hipGetLastError();
}

hipError_t launch_rekey_n(const unsigned long long *k0, long long nnz, const NLayout &l0, const NShifts &to_sh,
                          unsigned long long *kn, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rekey_n, dim3(grid_n(nnz)), dim3(kThreads), 0, s, k0, nnz, l0, to_sh, kn);
  return hipGetLastError();
}

hipError_t launch_export_coo_n(const unsigned long long *keys, const float *vals, long long nnz, const NLayout &lay,
                               int32_t *coords, float *vout, const int *ptr, int I, int64_t *ptr64, hipStream_t s) {
  const long long n = nnz > (long long)I + 1 ? nnz : (long long)I + 1;
  hipLaunchKernelGGL(k_export_coo_n, dim3(grid_n(n)), dim3(kThreads), 0, s, keys, vals, nnz, lay, coords, vout, ptr,
                     I, ptr64);
  return hipGetLastError();
}

namespace {

template <int RP>
hipError_t launch_mttkrp_n_rp(const NMttkrpArgs &a, dim3 g, hipStream_t s) {
  switch (a.nother) {
    case 1: hipLaunchKernelGGL((k_mttkrp_n<RP, 1>), g, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_mttkrp_n<RP, 2>), g, dim3(kThreads), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_mttkrp_n<RP, 3>), g, dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_mttkrp_n<RP, 4>), g, dim3(kThreads), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_mttkrp_n<RP, 5>), g, dim3(kThreads), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_mttkrp_n<RP, 6>), g, dim3(kThreads), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_mttkrp_n<RP, 7>), g, dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int nway_units_per_block(int RP) { return kThreads / (RP / 4); }

hipError_t launch_mttkrp_n(int RP, const NMttkrpArgs &a, hipStream_t s) {
  if (a.nunits == 0) return hipSuccess;
  const int upb = kThreads / (RP / 4);
  const dim3 g((a.nunits + upb - 1) / upb);
  switch (RP) {
    case 16: return launch_mttkrp_n_rp<16>(a, g, s);
    case 32: return launch_mttkrp_n_rp<32>(a, g, s);
    case 64: return launch_mttkrp_n_rp<64>(a, g, s);
    case 128: return launch_mttkrp_n_rp<128>(a, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prod_grams(const NGrams &g, int n, int RP, double *P, double *ones, hipStream_t s) {
  hipLaunchKernelGGL(k_prod_grams, dim3((RP * RP + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g, n, RP, P,
                     ones);
  return hipGetLastError();
}

hipError_t launch_inner_full_n(const unsigned long long *keys0, const float *vals0, long long nnz,
                               const NLayout &lay, const NFactors &F, int RP, double *part, int nparts, double *out,
                               unsigned *counter, hipStream_t s) {
  int g = grid_n(nnz);
  if (g > nparts) g = nparts;
  hipLaunchKernelGGL(k_inner_full_n, dim3(g), dim3(kThreads), 0, s, keys0, vals0, nnz, lay, F, RP, part, out,
                     counter);
  return hipGetLastError();
}

}  // namespace sacd
