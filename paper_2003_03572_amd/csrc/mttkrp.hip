// mttkrp.hip -- sparse MTTKRP of one mode (the first term of the gradient,
// eq. 9, in the slice form of Sec. 4.4):
//     M[i_n, :] = sum over Omega^n_{i_n} of x * (A_a[i_a, :] .* A_b[i_b, :])
//
// Work split (nnz-balanced, so skewed slices cost no imbalance):
//   * the mode-sorted entries are cut into wave chunks of C entries;
//   * inside a wave, lane groups of LPN lanes (W columns per lane) walk
//     contiguous runs of S entries.  Entries are sorted by (i_n, i_a, i_b), so
//     a run of entries sharing (i_n, i_a) -- a fibre -- reuses the A_a row kept
//     in registers: the fibre sum  sum x * A_b[i_b, :]  is formed first and
//     multiplied by A_a[i_a, :] once per fibre.
//   * slices entirely inside a group's run are stored directly; the first and
//     last slice pieces of every group go to LDS and are merged in entry order
//     by the wave; the wave chunk's pieces that continue into a neighbouring
//     chunk go to a carry buffer;
//   * the fix-up kernel sums, for every slice that spans chunks, its carry
//     pieces in chunk order (one block per such slice, fixed reduction tree),
//     and writes zeros for empty slices.
// No floating-point atomics: results are deterministic for a given shape.
#include "common.hpp"

namespace sacd {

namespace {

template <int RP>
struct MCfg {
  static constexpr int W = 8;          // columns per lane
  static constexpr int LPN = RP / W;   // lanes per entry
  static constexpr int GW = 64 / LPN;  // lane groups per wave
  static constexpr int NV = W / 4;     // float4 per lane
  static constexpr int U = 4;          // entries in flight per group
};

__device__ __forceinline__ f32x4 ld4(const float *p) { return *(const f32x4 *)p; }
__device__ __forceinline__ void st4(float *p, f32x4 v) { *(f32x4 *)p = v; }

template <int RP>
__global__ __launch_bounds__(kThreads) void k_mttkrp(const unsigned long long *__restrict__ keys,
                                                     const float *__restrict__ vals, long long nnz,
                                                     int S, long long C, KeyLayout lay,
                                                     const float *__restrict__ Aa,
                                                     const float *__restrict__ Ab,
                                                     float *__restrict__ M,
                                                     float *__restrict__ carry) {
  using Cf = MCfg<RP>;
  constexpr int W = Cf::W, LPN = Cf::LPN, GW = Cf::GW, NV = Cf::NV, U = Cf::U;
  __shared__ __align__(16) float s_part[4][2 * GW][RP];
  __shared__ int s_row[4][2 * GW];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = lane / LPN, sub = lane % LPN, col0 = sub * W;
  const long long wave_id = (long long)blockIdx.x * 4 + wv;
  const long long P0 = wave_id * C;
  const bool wave_active = P0 < nnz;
  const long long P1 = wave_active ? (P0 + C < nnz ? P0 + C : nnz) : P0;
  long long p = P0 + (long long)g * S;
  const long long pe = (p + S < P1) ? p + S : P1;

  f32x4 acc[NV], facc[NV], arow[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    facc[j] = acc[j];
    arow[j] = acc[j];
  }
  int row = -1, fib = -1, nseg = 0, head_row = -1, tail_row = -1;

  for (; p < pe; p += U) {
    unsigned long long kk[U];
    float xv[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = p + u < pe;
      kk[u] = ok[u] ? keys[p + u] : 0ull;
      xv[u] = ok[u] ? vals[p + u] : 0.0f;
    }
    int in[U], ia[U], ib[U];
    bool nrow[U], nfib[U];
    int pin = row, pia = fib;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      in[u] = (int)(kk[u] >> lay.sh_n);
      ia[u] = (int)((kk[u] >> lay.sh_a) & lay.mask_a);
      ib[u] = (int)(kk[u] & lay.mask_b);
      nrow[u] = in[u] != pin;
      nfib[u] = nrow[u] || ia[u] != pia;
      pin = in[u];
      pia = ia[u];
    }
    f32x4 bv[U][NV], av[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok[u]) {
        const float *pb = Ab + (long long)ib[u] * RP + col0;
#pragma unroll
        for (int j = 0; j < NV; ++j) bv[u][j] = ld4(pb + 4 * j);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok[u] && nfib[u]) {
        const float *pa = Aa + (long long)ia[u] * RP + col0;
#pragma unroll
        for (int j = 0; j < NV; ++j) av[u][j] = ld4(pa + 4 * j);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      if (nfib[u]) {
        if (row >= 0) {
#pragma unroll
          for (int j = 0; j < NV; ++j) acc[j] = arow[j] * facc[j] + acc[j];
        }
        if (nrow[u]) {
          if (row >= 0) {
            if (nseg == 0) {
              head_row = row;
#pragma unroll
              for (int j = 0; j < NV; ++j) st4(&s_part[wv][2 * g][col0 + 4 * j], acc[j]);
            } else {
              float *dst = M + (long long)row * RP + col0;
#pragma unroll
              for (int j = 0; j < NV; ++j) st4(dst + 4 * j, acc[j]);
            }
            ++nseg;
          }
          row = in[u];
#pragma unroll
          for (int j = 0; j < NV; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        fib = ia[u];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          arow[j] = av[u][j];
          facc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
#pragma unroll
      for (int j = 0; j < NV; ++j) facc[j] = xv[u] * bv[u][j] + facc[j];
    }
  }
  if (row >= 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = arow[j] * facc[j] + acc[j];
    const int slot = (nseg == 0) ? 2 * g : 2 * g + 1;
    if (nseg == 0) head_row = row; else tail_row = row;
#pragma unroll
    for (int j = 0; j < NV; ++j) st4(&s_part[wv][slot][col0 + 4 * j], acc[j]);
  }
  if (sub == 0) {
    s_row[wv][2 * g] = head_row;
    s_row[wv][2 * g + 1] = tail_row;
  }
  __syncthreads();
  if (!wave_active) return;

  // Merge the groups' first / last slice pieces in entry order.
  constexpr int NCL = (RP + 63) / 64;
  const int rowP0 = key_row(keys[P0], lay.sh_n);
  const int rowPL = key_row(keys[P1 - 1], lay.sh_n);
  const bool lo_open = P0 > 0 && key_row(keys[P0 - 1], lay.sh_n) == rowP0;
  const bool ro_open = P1 < nnz && key_row(keys[P1], lay.sh_n) == rowPL;
  float cur[NCL];
#pragma unroll
  for (int i = 0; i < NCL; ++i) cur[i] = 0.0f;
  int cur_row = -1;
  bool first = true;
  auto finalize = [&](int r, bool lo, bool ro) {
    float *dst = (!lo && !ro) ? M + (long long)r * RP
                              : carry + (wave_id * 2 + (lo ? 0 : 1)) * (long long)RP;
#pragma unroll
    for (int i = 0; i < NCL; ++i) {
      const int c = lane + 64 * i;
      if (c < RP) dst[c] = cur[i];
    }
  };
  for (int e = 0; e < 2 * GW; ++e) {
    const int r = s_row[wv][e];
    if (r < 0) continue;
    if (r == cur_row) {
#pragma unroll
      for (int i = 0; i < NCL; ++i) {
        const int c = lane + 64 * i;
        if (c < RP) cur[i] += s_part[wv][e][c];
      }
    } else {
      if (cur_row >= 0) {
        finalize(cur_row, first && lo_open, false);
        first = false;
      }
      cur_row = r;
#pragma unroll
      for (int i = 0; i < NCL; ++i) {
        const int c = lane + 64 * i;
        cur[i] = (c < RP) ? s_part[wv][e][c] : 0.0f;
      }
    }
  }
  if (cur_row >= 0) finalize(cur_row, first && lo_open, ro_open);
}

// Fix-up: blocks [0, nchunks) own the slices that start in their chunk and
// continue past it; the next row_blocks blocks zero empty slices; the last
// block forms H = Gram_a * Gram_b, L = ||H||_F and the diagonal of H for the
// element kernels of this sweep (eq. 10, eq. 15, Alg. 1).
template <int RP>
__global__ __launch_bounds__(kThreads) void k_mttkrp_fix(const unsigned long long *__restrict__ keys,
                                                         long long nnz, long long C, int nchunks,
                                                         int sh_n, const int *__restrict__ ptr, int I,
                                                         const float *__restrict__ carry,
                                                         float *__restrict__ M, int row_blocks,
                                                         const double *__restrict__ Ga,
                                                         const double *__restrict__ Gb,
                                                         float *__restrict__ H, HInfo *hinfo,
                                                         ModeState *st) {
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b < nchunks) {
    const long long P0 = (long long)b * C;
    const long long P1 = (P0 + C < nnz) ? P0 + C : nnz;
    if (P1 >= nnz) return;
    const int r = key_row(keys[P1 - 1], sh_n);
    const long long e = ptr[r + 1];
    if (e <= P1) return;
    if ((long long)ptr[r] < P0) return;
    const long long jend = (e - 1) / C;
    constexpr int Q = RP / 4;
    constexpr int NS = kThreads / Q;
    __shared__ f32x4 red[NS][Q];
    const int slot = tid / Q, q = tid % Q;
    f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
    if (slot == 0) s = ld4(carry + ((long long)b * 2 + 1) * RP + 4 * q);
    for (long long j = b + 1 + slot; j <= jend; j += NS) s += ld4(carry + (j * 2) * RP + 4 * q);
    red[slot][q] = s;
    __syncthreads();
    for (int w = NS / 2; w > 0; w >>= 1) {
      if (slot < w) red[slot][q] += red[slot + w][q];
      __syncthreads();
    }
    if (slot == 0) st4(M + (long long)r * RP + 4 * q, red[0][q]);
    return;
  }
  if (b < nchunks + row_blocks) {
    const int r = (b - nchunks) * kThreads + tid;
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

}  // namespace

MttkrpPlan mttkrp_plan(int RP, long long nnz) {
  const int GW = 64 / (RP / 8);
  MttkrpPlan p;
  p.nnz = nnz;
  // about 8192 waves for large tensors, wave chunks of at most 4096 entries
  long long C = (nnz + 8191) / 8192;
  const long long q = (long long)GW * 8;
  C = (C + q - 1) / q * q;
  if (C < q) C = q;
  if (C > 4096) C = 4096 / q * q;
  p.C = C;
  p.S = (int)(C / GW);
  p.nchunks = (int)((nnz + C - 1) / C);
  p.blocks = (p.nchunks + 3) / 4;
  return p;
}

template <int RP>
static hipError_t launch_mttkrp_t(const MttkrpPlan &p, const unsigned long long *keys, const float *vals,
                                  KeyLayout lay, const float *Aa, const float *Ab, float *M, float *carry,
                                  hipStream_t s) {
  if (p.nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mttkrp<RP>, dim3(p.blocks), dim3(kThreads), 0, s, keys, vals, p.nnz, p.S, p.C,
                     lay, Aa, Ab, M, carry);
  return hipGetLastError();
}

hipError_t launch_mttkrp(int RP, const MttkrpPlan &p, const unsigned long long *keys, const float *vals,
                         KeyLayout lay, const float *Aa, const float *Ab, float *M, float *carry,
                         hipStream_t s) {
  switch (RP) {
    case 16: return launch_mttkrp_t<16>(p, keys, vals, lay, Aa, Ab, M, carry, s);
    case 32: return launch_mttkrp_t<32>(p, keys, vals, lay, Aa, Ab, M, carry, s);
    case 64: return launch_mttkrp_t<64>(p, keys, vals, lay, Aa, Ab, M, carry, s);
    case 128: return launch_mttkrp_t<128>(p, keys, vals, lay, Aa, Ab, M, carry, s);
    default: return hipErrorInvalidValue;
  }
}

template <int RP>
static hipError_t launch_fix_t(const MttkrpPlan &p, const unsigned long long *keys, int sh_n,
                               const int *ptr, int I, const float *carry, float *M, const double *Ga,
                               const double *Gb, float *H, HInfo *hinfo, ModeState *st, hipStream_t s) {
  const int nchunks = p.nnz > 0 ? p.nchunks : 0;
  const int row_blocks = (I + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_mttkrp_fix<RP>, dim3(nchunks + row_blocks + 1), dim3(kThreads), 0, s, keys,
                     p.nnz, p.C, nchunks, sh_n, ptr, I, carry, M, row_blocks, Ga, Gb, H, hinfo, st);
  return hipGetLastError();
}

hipError_t launch_mttkrp_fix(int RP, const MttkrpPlan &p, const unsigned long long *keys, int sh_n,
                             const int *ptr, int I, const float *carry, float *M, const double *Ga,
                             const double *Gb, float *H, HInfo *hinfo, ModeState *st, hipStream_t s) {
  switch (RP) {
    case 16: return launch_fix_t<16>(p, keys, sh_n, ptr, I, carry, M, Ga, Gb, H, hinfo, st, s);
    case 32: return launch_fix_t<32>(p, keys, sh_n, ptr, I, carry, M, Ga, Gb, H, hinfo, st, s);
    case 64: return launch_fix_t<64>(p, keys, sh_n, ptr, I, carry, M, Ga, Gb, H, hinfo, st, s);
    case 128: return launch_fix_t<128>(p, keys, sh_n, ptr, I, carry, M, Ga, Gb, H, hinfo, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sacd
