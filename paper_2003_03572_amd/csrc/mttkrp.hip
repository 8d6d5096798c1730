// mttkrp.hip -- sparse MTTKRP of one mode (the first term of the gradient,
// eq. 9, in the slice form of Sec. 4.4):
//     M[i_n, :] = sum over Omega^n_{i_n} of x * (A_a[i_a, :] .* A_b[i_b, :])
//
// Work split: a static plan built once per tensor cuts every slice into
// segments of at most kSegment entries; each segment is one work unit, run by
// one lane group (LPN lanes, W columns each) from start to end, so the inner
// loop never meets a slice boundary.  Units are ordered longest first, so the
// groups of a wave run for about the same number of entries.  Entries are
// sorted by (i_n, i_a, i_b): a run sharing (i_n, i_a) -- a fibre -- multiplies
// its A_a row once, after the fibre sum  sum x * A_b[i_b, :]  is formed.
// A slice held by one unit is written directly; the units of a longer slice
// write partial sums that the fix-up kernel adds in a fixed tree order, one
// block per such slice.  The fix-up also zeroes empty slices.  No atomics:
// results are deterministic for a given tensor.
#include "common.hpp"

namespace sacd {

namespace {

// Columns per lane (compile-time tuning knob) and entries decoded per step.
#ifndef SACD_MT_W
#define SACD_MT_W 4
#endif
#ifndef SACD_MT_U
#define SACD_MT_U 8
#endif
// 1: per fibre, sum x * A_b rows and multiply by the A_a row once; 0: keep the
// fibre's A_a row and add x * (A_a .* A_b) per entry.
#ifndef SACD_MT_FIBRE
#define SACD_MT_FIBRE 0
#endif

template <int RP>
struct MCfg {
  static constexpr int W = SACD_MT_W < RP ? SACD_MT_W : RP;  // columns per lane
  static constexpr int LPN = RP / W;                           // lanes per unit
  static constexpr int NV = W / 4;                             // float4 per lane
  static constexpr int U = SACD_MT_U;
};

__device__ __forceinline__ f32x4 ld4(const float *p) { return *(const f32x4 *)p; }
__device__ __forceinline__ void st4(float *p, f32x4 v) { *(f32x4 *)p = v; }

template <int RP>
__global__ __launch_bounds__(kThreads) void k_mttkrp(const unsigned long long *__restrict__ keys,
                                                     const float *__restrict__ vals,
                                                     const int4 *__restrict__ units, int nunits,
                                                     KeyLayout lay, const float *__restrict__ Aa,
                                                     const float *__restrict__ Ab,
                                                     float *__restrict__ M,
                                                     float *__restrict__ part) {
  using Cf = MCfg<RP>;
  constexpr int LPN = Cf::LPN, NV = Cf::NV, U = Cf::U;
  constexpr int UPB = kThreads / LPN;  // units per block
  __shared__ __align__(16) float s_acc[UPB * RP];
  __shared__ int s_slot[UPB];
  const int ub = threadIdx.x / LPN;  // unit within the block
  const int gid = blockIdx.x * UPB + ub;
  const bool active = gid < nunits;
  // lane sub owns the float4 column chunks 4*sub + 4*LPN*j (j < NV): each
  // load instruction of a lane group covers contiguous bytes of a row
  const int sub = threadIdx.x % LPN;
  const int4 unit = active ? units[gid] : make_int4(0, 0, 0, -1);  // (slice, first, entries, slot)
  const long long p0 = unit.y;
  const int len = unit.z;

  f32x4 acc[NV], arow[NV];
#if SACD_MT_FIBRE
  f32x4 facc[NV];
#endif
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    arow[j] = acc[j];
#if SACD_MT_FIBRE
    facc[j] = acc[j];
#endif
  }
  unsigned long long fib = ~0ull;  // (i_n, i_a) of the current fibre
  for (int e = 0; e < len; e += U) {
    unsigned long long kk[U];
    float xv[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = e + u < len;
      kk[u] = ok[u] ? keys[p0 + e + u] : 0ull;
      xv[u] = ok[u] ? vals[p0 + e + u] : 0.0f;
    }
    f32x4 bv[U][NV], av[U][NV];
    bool nf[U];
    unsigned long long pf = fib;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned long long f = kk[u] >> lay.sh_a;
      nf[u] = ok[u] && f != pf;
      if (ok[u]) pf = f;
      const float *pb = Ab + (long long)(kk[u] & lay.mask_b) * RP + 4 * sub;
      if (ok[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) bv[u][j] = ld4(pb + 4 * LPN * j);
      }
      const float *pa = Aa + (long long)(f & lay.mask_a) * RP + 4 * sub;
      if (nf[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) av[u][j] = ld4(pa + 4 * LPN * j);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#if SACD_MT_FIBRE
      if (nf[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          acc[j] = arow[j] * facc[j] + acc[j];
          arow[j] = av[u][j];
          facc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
      if (ok[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) facc[j] = xv[u] * bv[u][j] + facc[j];
      }
#else
      if (nf[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) arow[j] = av[u][j];
      }
      if (ok[u]) {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] = xv[u] * (arow[j] * bv[u][j]) + acc[j];
      }
#endif
    }
    fib = pf;
  }
#if SACD_MT_FIBRE
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = arow[j] * facc[j] + acc[j];
#endif
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

// Fix-up: blocks [0, nlong) add the partial sums of one split slice in a
// fixed tree order; the next row_blocks blocks zero empty slices; the last
// block forms H = Gram_a * Gram_b, L = ||H||_F and the diagonal of H for the
// element kernels of this sweep (eq. 10, eq. 15, Alg. 1).
template <int RP>
__global__ __launch_bounds__(kThreads) void k_mttkrp_fix(const int4 *__restrict__ longs, int nlong,
                                                         const float *__restrict__ part,
                                                         const int *__restrict__ ptr, int I,
                                                         float *__restrict__ M, int row_blocks,
                                                         const double *__restrict__ Ga,
                                                         const double *__restrict__ Gb,
                                                         float *__restrict__ H, HInfo *hinfo,
                                                         ModeState *st) {
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b < nlong) {
    const int4 L = longs[b];  // (slice, first slot, slots, -)
    constexpr int Q = RP / 4;
    constexpr int NS = kThreads / Q;
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
    return;
  }
  if (b < nlong + row_blocks) {
    const int r = (b - nlong) * kThreads + tid;
    if (r < I && ptr[r] == ptr[r + 1]) {
      float *dst = M + (long long)r * RP;
#pragma unroll
      for (int c = 0; c < RP; c += 4) st4(dst + c, f32x4{0.f, 0.f, 0.f, 0.f});
    }
    return;
  }
  // H, L, diagonal
  __shared__ double l2[kThreads];
  __shared__ float mx[kThreads];
  double s2 = 0.0;
  for (int i = tid; i < RP * RP; i += kThreads) {
    const double h = Ga[i] * Gb[i];
    H[i] = (float)h;
    s2 += h * h;
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
}

template <int RP>
hipError_t launch_mttkrp_t(const MttkrpPlan &p, const unsigned long long *keys, const float *vals,
                           KeyLayout lay, const float *Aa, const float *Ab, float *M, float *part,
                           hipStream_t s) {
  if (p.nunits <= 0) return hipSuccess;
  const long long threads = (long long)p.nunits * MCfg<RP>::LPN;
  const int blocks = (int)((threads + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_mttkrp<RP>, dim3(blocks), dim3(kThreads), 0, s, keys, vals, p.units, p.nunits,
                     lay, Aa, Ab, M, part);
  return hipGetLastError();
}

template <int RP>
hipError_t launch_fix_t(const MttkrpPlan &p, const int *ptr, int I, const float *part, float *M,
                        const double *Ga, const double *Gb, float *H, HInfo *hinfo, ModeState *st,
                        hipStream_t s) {
  const int row_blocks = (I + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_mttkrp_fix<RP>, dim3(p.nlong + row_blocks + 1), dim3(kThreads), 0, s, p.longs,
                     p.nlong, part, ptr, I, M, row_blocks, Ga, Gb, H, hinfo, st);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mttkrp(int RP, const MttkrpPlan &p, const unsigned long long *keys, const float *vals,
                         KeyLayout lay, const float *Aa, const float *Ab, float *M, float *part,
                         hipStream_t s) {
  switch (RP) {
    case 16: return launch_mttkrp_t<16>(p, keys, vals, lay, Aa, Ab, M, part, s);
    case 32: return launch_mttkrp_t<32>(p, keys, vals, lay, Aa, Ab, M, part, s);
    case 64: return launch_mttkrp_t<64>(p, keys, vals, lay, Aa, Ab, M, part, s);
    case 128: return launch_mttkrp_t<128>(p, keys, vals, lay, Aa, Ab, M, part, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mttkrp_fix(int RP, const MttkrpPlan &p, const int *ptr, int I, const float *part,
                             float *M, const double *Ga, const double *Gb, float *H, HInfo *hinfo,
                             ModeState *st, hipStream_t s) {
  switch (RP) {
    case 16: return launch_fix_t<16>(p, ptr, I, part, M, Ga, Gb, H, hinfo, st, s);
    case 32: return launch_fix_t<32>(p, ptr, I, part, M, Ga, Gb, H, hinfo, st, s);
    case 64: return launch_fix_t<64>(p, ptr, I, part, M, Ga, Gb, H, hinfo, st, s);
    case 128: return launch_fix_t<128>(p, ptr, I, part, M, Ga, Gb, H, hinfo, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sacd
