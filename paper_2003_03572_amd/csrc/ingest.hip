// ingest.hip -- tensor ingest on the GPU: validation, bit-packed keys, stable
// LSD radix sort, merging of duplicate coordinates, slice pointers (the
// per-mode slices Omega^U_q, Omega^V_p, Omega^W_s of Sec. 3) and ||X||^2.
//
// Everything here is integer or order-preserving data movement, except the
// FP32 sums of duplicate entries (taken in input order, which the stable sort
// preserves) and the FP64 norm (fixed-order reduction).  Results are
// therefore deterministic and independent of launch timing.
#include "common.hpp"

namespace sacd {

namespace {

constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // elements per block in sort / scan

inline int grid_for(long long n, int per_block, int cap = 65535 * 8) {
  long long g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__global__ __launch_bounds__(kThreads) void k_make_keys0(const int32_t *__restrict__ idx,
                                                         const float *__restrict__ vals,
                                                         long long nnz, long long d0, long long d1,
                                                         long long d2, KeyLayout lay,
                                                         unsigned long long *__restrict__ keys,
                                                         float *__restrict__ vout, int *err) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  int bad = 0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
    const int i0 = idx[3 * p], i1 = idx[3 * p + 1], i2 = idx[3 * p + 2];
    const float v = vals[p];
    const bool in_range = i0 >= 0 && i0 < d0 && i1 >= 0 && i1 < d1 && i2 >= 0 && i2 < d2;
    if (!in_range) bad |= 1;
    if (!isfinite(v)) bad |= 2;
    const unsigned long long k = in_range ? (((unsigned long long)(unsigned)i0 << lay.sh_n) |
                                             ((unsigned long long)(unsigned)i1 << lay.sh_a) |
                                             (unsigned long long)(unsigned)i2)
                                          : 0ull;
    keys[p] = k;
    vout[p] = v;
  }
  if (bad) atomicOr(err, bad);
}

// ---------------------------------------------------------------- scan ----

// Sum of each tile of kTile ints.
__global__ __launch_bounds__(kThreads) void k_tile_sums(const int *__restrict__ in, long long n,
                                                        int *__restrict__ sums) {
  __shared__ int red[kThreads];
  const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
  int s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j)
    if (base + j < n) s += in[base + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Exclusive scan of each tile plus the tile's offset.
__global__ __launch_bounds__(kThreads) void k_tile_scan(const int *__restrict__ in, long long n,
                                                        const int *__restrict__ offs,
                                                        int *__restrict__ out) {
  __shared__ int sc[kThreads];
  const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
  int v[kItems];
  int s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    s += v[j];
  }
  sc[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int w = 1; w < kThreads; w <<= 1) {
    const int t = ((int)threadIdx.x >= w) ? sc[threadIdx.x - w] : 0;
    __syncthreads();
    sc[threadIdx.x] += t;
    __syncthreads();
  }
  int run = sc[threadIdx.x] - s + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
}

size_t scan_temp_ints(long long n) {
  size_t t = 0;
  long long m = n;
  while (m > kTile) {
    m = (m + kTile - 1) / kTile;
    t += 2 * (size_t)m;
  }
  return t + 16;
}

// Exclusive prefix sum of n ints (in and out may alias).
hipError_t scan_exclusive(const int *in, int *out, long long n, int *temp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = (n + kTile - 1) / kTile;
  if (nb == 1) {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kThreads), 0, s, in, n, (const int *)nullptr, out);
    return hipGetLastError();
  }
  int *sums = temp;
  int *sums_scanned = temp + nb;
  hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, sums);
  hipError_t e = scan_exclusive(sums, sums_scanned, nb, temp + 2 * nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n,
                     (const int *)sums_scanned, out);
  return hipGetLastError();
}

// ---------------------------------------------------------- radix sort ----

__global__ __launch_bounds__(kThreads) void k_radix_hist(const unsigned long long *__restrict__ keys,
                                                         long long n, int shift, int *__restrict__ hist,
                                                         int nblocks) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kTile;
  for (int j = 0; j < kItems; ++j) {
    const long long e = base + (long long)j * kThreads + threadIdx.x;
    if (e < n) atomicAdd(&h[(int)((keys[e] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  hist[(long long)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: elements are ranked in tile order (rounds of 256
// in order, lanes in order within a wave, waves in order within a round).
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const unsigned long long *__restrict__ keys,
                                                            const float *__restrict__ vals, long long n,
                                                            int shift, const int *__restrict__ offs,
                                                            int nblocks,
                                                            unsigned long long *__restrict__ kout,
                                                            float *__restrict__ vout) {
  __shared__ int s_base[256];
  __shared__ int s_wc[4][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  s_base[tid] = offs[(long long)tid * nblocks + blockIdx.x];
  for (int ww = 0; ww < 4; ++ww) s_wc[ww][tid] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kTile;
  const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int j = 0; j < kItems; ++j) {
    const long long e = base + (long long)j * kThreads + tid;
    const bool valid = e < n;
    const unsigned long long k = valid ? keys[e] : 0ull;
    const float v = valid ? vals[e] : 0.0f;
    const int d = (int)((k >> shift) & 255ull);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bit = (d >> b) & 1;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) s_wc[w][d] = __popcll(peers);
    __syncthreads();
    {
      int run = s_base[tid];
      for (int ww = 0; ww < 4; ++ww) {
        const int c = s_wc[ww][tid];
        s_wc[ww][tid] = run;
        run += c;
      }
      s_base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const int pos = s_wc[w][d] + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    for (int ww = 0; ww < 4; ++ww) s_wc[ww][tid] = 0;
    __syncthreads();
  }
}

// ------------------------------------------------------------- dedup ----

__global__ __launch_bounds__(kThreads) void k_flag_heads(const unsigned long long *__restrict__ keys,
                                                         long long n, int *__restrict__ flags) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    flags[p] = (p == 0 || keys[p] != keys[p - 1]) ? 1 : 0;
}

// One thread per run of equal keys adds the run's values in order (FP32).
__global__ __launch_bounds__(kThreads) void k_compact_sum(const unsigned long long *__restrict__ keys,
                                                          const float *__restrict__ vals, long long n,
                                                          const int *__restrict__ flags,
                                                          const int *__restrict__ pos,
                                                          unsigned long long *__restrict__ ukeys,
                                                          float *__restrict__ uvals, int *count) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    if (p == n - 1) *count = pos[p] + flags[p];
    if (!flags[p]) continue;
    const unsigned long long k = keys[p];
    float v = vals[p];
    for (long long q = p + 1; q < n && keys[q] == k; ++q) v = __fadd_rn(v, vals[q]);
    ukeys[pos[p]] = k;
    uvals[pos[p]] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_rekey(const unsigned long long *__restrict__ keys0,
                                                    long long n, KeyLayout l0, int mode,
                                                    KeyLayout ln,
                                                    unsigned long long *__restrict__ keysn) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const unsigned long long k = keys0[p];
    const unsigned long long c[3] = {k >> l0.sh_n, (k >> l0.sh_a) & l0.mask_a, k & l0.mask_b};
    const unsigned long long in = c[mode];
    const unsigned long long ia = (mode == 0) ? c[1] : c[0];
    const unsigned long long ib = (mode == 2) ? c[1] : c[2];
    keysn[p] = (in << ln.sh_n) | (ia << ln.sh_a) | ib;
  }
}

// Keys of mode n re-encoded for the tiled MTTKRP form: the tile i_b >> tsh
// inserted between i_n and i_a, (i_n, tile, i_a, i_b), tile field tb bits wide.
__global__ __launch_bounds__(kThreads) void k_tile_keys(const unsigned long long *__restrict__ keys, long long n,
                                                        KeyLayout lay, int tsh, int tb,
                                                        unsigned long long *__restrict__ out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const unsigned long long low = lay.sh_n >= 64 ? ~0ull : ((1ull << lay.sh_n) - 1ull);
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const unsigned long long k = keys[p];
    const unsigned long long in = k >> lay.sh_n, ib = k & lay.mask_b;
    out[p] = ((((in << tb) | (ib >> tsh)) << lay.sh_n)) | (k & low);
  }
}

// ---------------------------------------------------------------- ptr ----

// Slice pointers from sorted keys: position p is the start of every row in
// (row(p-1), row(p)], with row(-1) = -1 and row(n) = I.  Each pointer is
// written exactly once; no atomics.
__global__ __launch_bounds__(kThreads) void k_row_bounds(const unsigned long long *__restrict__ keys,
                                                         long long n, int sh_n, int I,
                                                         int *__restrict__ ptr) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p <= n; p += stride) {
    const int prev = (p == 0) ? -1 : (int)(keys[p - 1] >> sh_n);
    const int cur = (p == n) ? I : (int)(keys[p] >> sh_n);
    for (int r = prev + 1; r <= cur; ++r) ptr[r] = (int)p;
  }
}

// --------------------------------------------------------------- norm ----

__global__ __launch_bounds__(kThreads) void k_norm2_partial(const float *__restrict__ v, long long n,
                                                            double *__restrict__ part) {
  __shared__ double red[kThreads];
  const long long stride = (long long)gridDim.x * blockDim.x;
  double s = 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    s += (double)v[p] * (double)v[p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_norm2_final(const double *__restrict__ part, int nparts,
                                                          double *out) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ __launch_bounds__(kThreads) void k_export_coo(const unsigned long long *__restrict__ keys,
                                                         const float *__restrict__ vals, long long n,
                                                         KeyLayout lay, int32_t *coords, float *vout) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const unsigned long long k = keys[p];
    if (coords) {
      coords[3 * p] = (int32_t)(k >> lay.sh_n);
      coords[3 * p + 1] = (int32_t)((k >> lay.sh_a) & lay.mask_a);
      coords[3 * p + 2] = (int32_t)(k & lay.mask_b);
    }
    if (vout) vout[p] = vals[p];
  }
}

__global__ __launch_bounds__(kThreads) void k_ptr_widen(const int *__restrict__ ptr, int n,
                                                        int64_t *__restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = ptr[i];
}

}  // namespace

// ------------------------------------------------------------- launchers ----

hipError_t launch_make_keys0(const int32_t *idx, const float *vals, long long nnz, const int64_t *dims,
                             KeyLayout lay0, unsigned long long *keys, float *vout, int *err_flags,
                             hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_make_keys0, dim3(grid_for(nnz, kThreads * 4)), dim3(kThreads), 0, s, idx, vals,
                     nnz, (long long)dims[0], (long long)dims[1], (long long)dims[2], lay0, keys, vout,
                     err_flags);
  return hipGetLastError();
}

size_t radix_sort_temp_bytes(long long n) {
  const long long nb = (n + kTile - 1) / kTile;
  const long long h = 256 * (nb > 0 ? nb : 1);
  return (size_t)(2 * h + scan_temp_ints(h)) * sizeof(int) + 256;
}

hipError_t radix_sort_pairs(unsigned long long *keys, float *vals, unsigned long long *keys_alt,
                            float *vals_alt, long long n, int lo_bit, int hi_bit, void *temp,
                            hipStream_t s, bool *result_in_alt) {
  *result_in_alt = false;
  if (n <= 1 || hi_bit <= lo_bit) return hipSuccess;
  const int nb = (int)((n + kTile - 1) / kTile);
  const long long h = 256LL * nb;
  int *hist = (int *)temp;
  int *offs = hist + h;
  int *stemp = offs + h;
  unsigned long long *kin = keys, *kout = keys_alt;
  float *vin = vals, *vout = vals_alt;
  bool alt = false;
  for (int shift = lo_bit; shift < hi_bit; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kThreads), 0, s, kin, n, shift, hist, nb);
    hipError_t e = scan_exclusive(hist, offs, h, stemp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kThreads), 0, s, kin, vin, n, shift,
                       (const int *)offs, nb, kout, vout);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long *tk = kin; kin = kout; kout = tk;
    float *tv = vin; vin = vout; vout = tv;
    alt = !alt;
  }
  *result_in_alt = alt;
  return hipSuccess;
}

size_t dedup_temp_bytes(long long n) {
  return (size_t)(2 * (n > 0 ? n : 1) + scan_temp_ints(n > 0 ? n : 1)) * sizeof(int) + 256;
}

hipError_t dedup_sorted(const unsigned long long *keys, const float *vals, long long n,
                        unsigned long long *ukeys, float *uvals, int *d_count, void *temp,
                        hipStream_t s) {
  if (n <= 0) return hipMemsetAsync(d_count, 0, sizeof(int), s);
  int *flags = (int *)temp;
  int *pos = flags + n;
  int *stemp = pos + n;
  hipLaunchKernelGGL(k_flag_heads, dim3(grid_for(n, kThreads * 4)), dim3(kThreads), 0, s, keys, n, flags);
  hipError_t e = scan_exclusive(flags, pos, n, stemp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact_sum, dim3(grid_for(n, kThreads * 4)), dim3(kThreads), 0, s, keys, vals,
                     n, (const int *)flags, (const int *)pos, ukeys, uvals, d_count);
  return hipGetLastError();
}

hipError_t launch_rekey(const unsigned long long *keys0, long long n, KeyLayout lay0, int mode,
                        KeyLayout layn, unsigned long long *keysn, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rekey, dim3(grid_for(n, kThreads * 4)), dim3(kThreads), 0, s, keys0, n, lay0,
                     mode, layn, keysn);
  return hipGetLastError();
}

hipError_t launch_tile_keys(const unsigned long long *keys, long long n, KeyLayout lay, int tsh, int tb,
                            unsigned long long *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_keys, dim3(grid_for(n, kThreads * 4)), dim3(kThreads), 0, s, keys, n, lay, tsh, tb, out);
  return hipGetLastError();
}

size_t build_ptr_temp_bytes(long long n, int I) {
  (void)n;
  (void)I;
  return 16;
}

hipError_t build_ptr(const unsigned long long *keys, long long n, int sh_n, int I, int *ptr, void *temp,
                     hipStream_t s) {
  (void)temp;
  hipLaunchKernelGGL(k_row_bounds, dim3(grid_for(n + 1, kThreads * 4)), dim3(kThreads), 0, s, keys, n,
                     sh_n, I, ptr);
  return hipGetLastError();
}

hipError_t launch_norm2(const float *vals, long long n, double *partials, int nparts, double *out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_partial, dim3(nparts), dim3(kThreads), 0, s, vals, n, partials);
  hipLaunchKernelGGL(k_norm2_final, dim3(1), dim3(kThreads), 0, s, (const double *)partials, nparts, out);
  return hipGetLastError();
}

hipError_t launch_export_coo(const unsigned long long *keys, const float *vals, long long n,
                             KeyLayout lay, int32_t *coords, float *vout, const int *ptr, int I,
                             int64_t *ptr64, hipStream_t s) {
  if (n > 0 && (coords || vout))
    hipLaunchKernelGGL(k_export_coo, dim3(grid_for(n, kThreads * 4)), dim3(kThreads), 0, s, keys, vals,
                       n, lay, coords, vout);
  if (ptr64)
    hipLaunchKernelGGL(k_ptr_widen, dim3(grid_for((long long)I + 1, kThreads)), dim3(kThreads), 0, s,
                       ptr, I + 1, ptr64);
  return hipGetLastError();
}

}  // namespace sacd

namespace sacd {

namespace {
__global__ __launch_bounds__(kThreads) void k_gather_keys(const unsigned long long *__restrict__ keys,
                                                          const int *__restrict__ pos, int n,
                                                          unsigned long long *__restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = keys[pos[i]];
}
}  // namespace

hipError_t launch_gather_keys(const unsigned long long *keys, const int *pos, int n,
                              unsigned long long *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_keys, dim3((n + kThreads - 1) / kThreads < 4096 ? (n + kThreads - 1) / kThreads : 4096),
                     dim3(kThreads), 0, s, keys, pos, n, out);
  return hipGetLastError();
}

}  // namespace sacd
