// lowmem.hip -- the column-at-a-time form of a sweep (Sec. 4.4, Alg. 2): the
// MTTKRP is formed CB columns at a time, as the paper's column form does one
// column at a time ("sparse tensor times vector"), so that no I_n x R buffer
// for M is held -- only I_n x CB.  The selection needs every importance of the
// mode before any update (ti, eq. 25), so a sweep makes two passes over the
// column blocks:
//
//   pass A, block by block:  M_b (k_sttvp, k_sttvp_fix), then per element the
//       gradient, step and importance (eq. 14, 11-12, 20); both possible
//       decisions (eq. 24, or z > 0 at k = 1; eq. 27) kept as two bits, z
//       stored as the next Z^{k-1}, per-block partial sums of z;
//   k_col_decide: ti, the eq. 27 branch, k;
//   pass B, block by block in ascending column order:  M_b again, then each
//       selected element of the block takes its one-variable step with the
//       gradient of its row's current values (Gauss-Seidel, as the row form),
//       and <M, A_n> is summed;
//   k_col_finish: <M, A_n>, the per-column counts |e_r|.
//
// The Gram matrix and the objective then follow as in the row form.  Every sum
// is formed in a fixed order: results are deterministic.
#include "common.hpp"

namespace sacd {

namespace {

// FP64 sum of v over the block (kColThreads threads) in a fixed order: a
// butterfly within each wave, then the waves in order.  Thread 0's value.
__device__ __forceinline__ double col_block_sum(double v, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kColThreads / 64; ++k) t += red[k];
  __syncthreads();
  return t;
}

// Columns [c0, c0 + CB) of the MTTKRP, one thread per work unit of the plan
// (a segment of at most kSegment entries of one slice): the unit's entries in
// order, x (a .* b) added per column.  A whole slice is written to M_b; a
// segment of a split slice to its own unit slot, which k_sttvp_fix adds.
template <int CB>
__global__ __launch_bounds__(256) void k_sttvp(MttkrpArgs a, int RP, int c0, const int *__restrict__ uslot,
                                               float *__restrict__ Mb, float *__restrict__ upart) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= a.nunits) return;
  const int4 unit = a.units[u];  // (slice, first entry, entries, -)
  const KeyLayout lay = a.lay;
  float acc[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) acc[j] = 0.0f;
  for (long long p = unit.y; p < (long long)unit.y + unit.z; ++p) {
    const unsigned long long k = a.keys[p];
    const float x = a.vals[p];
    const long long ia = (long long)((k >> lay.sh_a) & lay.mask_a), ib = (long long)(k & lay.mask_b);
    const float *ra = a.Aa + ia * RP + c0;
    const float *rb = a.Ab + ib * RP + c0;
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[j] = __fmaf_rn(x, __fmul_rn(ra[j], rb[j]), acc[j]);
  }
  const int us = uslot[u];
  float *dst = us < 0 ? Mb + (long long)unit.x * CB : upart + (long long)us * CB;
#pragma unroll
  for (int j = 0; j < CB; ++j) dst[j] = acc[j];
}

// Split slices: the unit slots of slice L.x (in entry order) added per column.
template <int CB>
__global__ __launch_bounds__(256) void k_sttvp_fix(const int4 *__restrict__ ulongs, int nulong,
                                                   const float *__restrict__ upart, float *__restrict__ Mb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nulong * CB) return;
  const int4 L = ulongs[t / CB];
  const int j = t % CB;
  float s = 0.0f;
  for (int k = 0; k < L.z; ++k) s += upart[(long long)(L.y + k) * CB + j];
  Mb[(long long)L.x * CB + j] = s;
}

// Pass A for the block's columns: one thread per row.
template <int CB>
__global__ __launch_bounds__(kColThreads) void k_col_importance(ColArgs a) {
  __shared__ double red[kColThreads / 64];
  const int q = blockIdx.x * kColThreads + threadIdx.x;
  const int RP = a.RP;
  const int first = a.st->k == 0;  // the sweep counter advances in k_col_decide
  const float halfL = a.hi->halfL;
  double zs = 0.0;
  if (q < a.I) {
    const float *arow = a.A + (long long)q * RP;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int r = a.c0 + j;
      float ah = 0.0f;
      for (int s = 0; s < RP; ++s) ah = __fmaf_rn(arow[s], a.H[s * RP + r], ah);
      const float m = a.Mb[(long long)q * CB + j];
      float d;
      const float z = element_importance(ah, m, arow[r], a.hi->hdiag[r], a.hi->nearzero[r], halfL, &d);
      const long long e = (long long)q * RP + r;
      const float zp = a.Z[e];
      const unsigned b24 = first ? (z > 0.0f) : (z > zp);  // eq. 24 (k = 1: z > 0)
      const unsigned b27 = z < zp;                           // eq. 27
      const unsigned w = (b24 | (b27 << 1)) << (2 * (e & 15));
      if (w) atomicOr(&a.bits[e >> 4], w);
      a.Z[e] = z;  // Z^{k-1} of the next sweep (Alg. 1): every element
      zs += (double)z;
    }
  }
  const double t = col_block_sum(zs, red);
  if (threadIdx.x == 0) a.part[a.part_off + blockIdx.x] = t;
}

// ti (eq. 25) from the pass-A partials in a fixed order, the eq. 27 branch
// and the sweep counter (one block).
__global__ __launch_bounds__(kColThreads) void k_col_decide(const double *__restrict__ part, int n, ModeState *st) {
  __shared__ double red[kColThreads / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kColThreads) s += part[i];
  const double ti = col_block_sum(s, red);
  if (threadIdx.x == 0) {
    const long long k = st->k + 1;
    const int first = (k == 1);
    st->flip = (!first && ti > st->ti_prev) ? 1 : 0;  // eq. 27 condition: "more than"
    st->first = first;
    st->k = k;
    st->ti = ti;
    st->ti_prev = ti;  // ti^{k-1} of the next sweep (eq. 26)
  }
}

// Pass B for the block's columns: one thread per row, the block's columns in
// ascending order; the gradient of a selected element uses the row's current
// values (earlier columns already updated in this sweep), as in the row form.
template <int CB>
__global__ __launch_bounds__(kColThreads) void k_col_update(ColArgs a) {
  __shared__ double red[kColThreads / 64];
  __shared__ int cnt[CB];
  if (threadIdx.x < CB) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int q = blockIdx.x * kColThreads + threadIdx.x;
  const int RP = a.RP;
  const int first = a.st->first, flip = a.st->flip;
  double inner = 0.0;
  if (q < a.I) {
    float *arow = const_cast<float *>(a.A) + (long long)q * RP;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int r = a.c0 + j;
      const long long e = (long long)q * RP + r;
      const unsigned w = a.bits[e >> 4] >> (2 * (e & 15));
      const bool sl = (first || !flip) ? (w & 1u) : ((w >> 1) & 1u);
      const float m = a.Mb[(long long)q * CB + j];
      const float h = a.hi->hdiag[r];
      if (sl && h > 0.0f) {
        float g = -m;
        for (int s = 0; s < RP; ++s) g = __fmaf_rn(arow[s], a.H[s * RP + r], g);
        const float qd = a.hi->nearzero[r] ? (float)((double)g / (double)h) : __fdiv_rn(g, h);
        arow[r] = fmaxf(__fsub_rn(arow[r], qd), 0.0f);  // eq. 11-13
      }
      if (sl) atomicAdd(&cnt[j], 1);
      if (a.selmask) a.selmask[e] = sl ? 1 : 0;
      if (a.Mdiag) a.Mdiag[e] = m;
      inner += (double)m * (double)arow[r];
    }
  }
  const double t = col_block_sum(inner, red);
  if (threadIdx.x == 0) a.part[a.part_off + blockIdx.x] = t;
  __syncthreads();
  if (threadIdx.x < CB) {
    // one writer per (row block, column) and sweep
    a.cnt_part[(long long)blockIdx.x * RP + a.c0 + threadIdx.x] = cnt[threadIdx.x];
  }
}

// <M, A_n> from the pass-B partials and the per-column counts (one block).
__global__ __launch_bounds__(kColThreads) void k_col_finish(const double *__restrict__ part, int n,
                                                            const int *__restrict__ cnt_part, int nrb, int RP,
                                                            int ncols, long long *__restrict__ colcnt,
                                                            ModeState *st) {
  __shared__ double red[kColThreads / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kColThreads) s += part[i];
  const double inner = col_block_sum(s, red);
  long long tot = 0;
  for (int c = threadIdx.x; c < RP; c += kColThreads) {
    long long v = 0;
    if (c < ncols)
      for (int b = 0; b < nrb; ++b) v += cnt_part[(long long)b * RP + c];
    colcnt[c] = v;
    tot += v;
  }
  const double all = col_block_sum((double)tot, red);
  if (threadIdx.x == 0) {
    st->inner = inner;
    st->nsel = (long long)all;
  }
}

template <int CB>
hipError_t sttvp_cb(const MttkrpArgs &a, int RP, int c0, const int *uslot, const int4 *ulongs, int nulong, float *Mb,
                    hipStream_t s) {
  if (a.nunits > 0)
    hipLaunchKernelGGL((k_sttvp<CB>), dim3((a.nunits + 255) / 256), dim3(256), 0, s, a, RP, c0, uslot, Mb, a.part);
  if (nulong > 0)
    hipLaunchKernelGGL((k_sttvp_fix<CB>), dim3((nulong * CB + 255) / 256), dim3(256), 0, s, ulongs, nulong,
                       (const float *)a.part, Mb);
  return hipGetLastError();
}

}  // namespace

int col_row_blocks(int I) { return (I + kColThreads - 1) / kColThreads; }

hipError_t launch_sttvp(int CB, const MttkrpArgs &a, int RP, int c0, const int *uslot, const int4 *ulongs, int nulong,
                        float *Mb, hipStream_t s) {
  switch (CB) {
    case 1: return sttvp_cb<1>(a, RP, c0, uslot, ulongs, nulong, Mb, s);
    case 2: return sttvp_cb<2>(a, RP, c0, uslot, ulongs, nulong, Mb, s);
    case 4: return sttvp_cb<4>(a, RP, c0, uslot, ulongs, nulong, Mb, s);
    case 8: return sttvp_cb<8>(a, RP, c0, uslot, ulongs, nulong, Mb, s);
    case 16: return sttvp_cb<16>(a, RP, c0, uslot, ulongs, nulong, Mb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col_importance(int CB, const ColArgs &a, hipStream_t s) {
  const dim3 g(col_row_blocks(a.I));
  if (a.I == 0) return hipSuccess;
  switch (CB) {
    case 1: hipLaunchKernelGGL(k_col_importance<1>, g, dim3(kColThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_col_importance<2>, g, dim3(kColThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_col_importance<4>, g, dim3(kColThreads), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_col_importance<8>, g, dim3(kColThreads), 0, s, a); break;
    case 16: hipLaunchKernelGGL(k_col_importance<16>, g, dim3(kColThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_decide(const double *part, int n, ModeState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_col_decide, dim3(1), dim3(kColThreads), 0, s, part, n, st);
  return hipGetLastError();
}

hipError_t launch_col_update(int CB, const ColArgs &a, hipStream_t s) {
  const dim3 g(col_row_blocks(a.I));
  if (a.I == 0) return hipSuccess;
  switch (CB) {
    case 1: hipLaunchKernelGGL(k_col_update<1>, g, dim3(kColThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_col_update<2>, g, dim3(kColThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_col_update<4>, g, dim3(kColThreads), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_col_update<8>, g, dim3(kColThreads), 0, s, a); break;
    case 16: hipLaunchKernelGGL(k_col_update<16>, g, dim3(kColThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_finish(const double *part, int n, const int *cnt_part, int nrb, int RP, int ncols,
                             long long *colcnt, ModeState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(kColThreads), 0, s, part, n, cnt_part, nrb, RP, ncols, colcnt, st);
  return hipGetLastError();
}

}  // namespace sacd
