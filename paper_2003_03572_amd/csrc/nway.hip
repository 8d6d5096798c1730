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
// each) per work unit of the plan (a segment of one slice), entries in order,
// x times the product of the N - 1 other rows added per column.  A whole
// slice is written to M; a segment of a split slice to its own unit slot,
// which k_mttkrp_fix adds in a fixed order.
template <int RP>
__global__ __launch_bounds__(kThreads) void k_mttkrp_n(NMttkrpArgs a) {
  constexpr int LPN = RP / 4, UPB = kThreads / LPN;
  const int ub = threadIdx.x / LPN, sub = threadIdx.x % LPN;
  const int u = blockIdx.x * UPB + ub;
  if (u >= a.nunits) return;
  const int4 unit = a.units[u];  // (slice, first entry, entries, -)
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  const int no = a.nother;
  for (long long p = unit.y; p < (long long)unit.y + unit.z; ++p) {
    const unsigned long long k = a.keys[p];
    const float x = a.vals[p];
    f32x4 prod;
    {
      const unsigned long long i = (k >> a.sh[0]) & a.mask[0];
      prod = ld4n(a.A[0] + i * RP + 4 * sub);
    }
    for (int f = 1; f < no; ++f) {
      const unsigned long long i = (k >> a.sh[f]) & a.mask[f];
      prod = prod * ld4n(a.A[f] + i * RP + 4 * sub);
    }
    acc = x * prod + acc;
  }
  const int us = a.uslot[u];
  float *dst = us < 0 ? a.M + (long long)unit.x * RP : a.part + (long long)us * RP;
  *(f32x4 *)(dst + 4 * sub) = acc;
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
    __threadfence();
    s_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  __threadfence();
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

hipError_t launch_mttkrp_n(int RP, const NMttkrpArgs &a, hipStream_t s) {
  if (a.nunits == 0) return hipSuccess;
  const int upb = kThreads / (RP / 4);
  const dim3 g((a.nunits + upb - 1) / upb);
  switch (RP) {
    case 16: hipLaunchKernelGGL(k_mttkrp_n<16>, g, dim3(kThreads), 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_mttkrp_n<32>, g, dim3(kThreads), 0, s, a); break;
    case 64: hipLaunchKernelGGL(k_mttkrp_n<64>, g, dim3(kThreads), 0, s, a); break;
    case 128: hipLaunchKernelGGL(k_mttkrp_n<128>, g, dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
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
