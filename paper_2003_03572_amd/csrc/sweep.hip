// sweep.hip -- the dense part of one SaCD sweep of mode n (Alg. 1):
//
//   k_importance     A_n H on MFMA (16x16x4 FP32), gradient G0 = -M + A_n H
//                    (eq. 9, eq. 14), projected step (eq. 11-12), Lipschitz
//                    importance z (eq. 20); per-block partial sums of z in
//                    FP64; the last block to finish forms the total importance
//                    (eq. 25) in a fixed order and decides the eq. 27 branch.
//   k_select_update  recomputes z bit for bit, selects (Alg. 1, eq. 24 / 27),
//                    stores z as the next Z^{k-1}, updates the selected
//                    elements of each row (eq. 13; Gauss-Seidel refresh of the
//                    row's gradient, or Jacobi), and emits per-block partials
//                    of the new Gram matrix (MFMA), of <M, A_n> (FP64) and of
//                    the per-column selection counts.
//   k_gram_final     reduces the Gram partials in FP64 in a fixed order; its
//                    last block, or k_gram_finish (RP >= 64 and the
//                    job-batched form), forms the objective eq. 6 in FP64.
//
// Rows are split into blocks of RB rows (256 at RP <= 32, fewer above); a
// block keeps its rows of A_n and H in LDS (row stride RP + 1 floats:
// conflict-free for the row-wise update).  The row blocks fix every partial
// sum; the number of threads working on a block (256 to 1024) changes no
// result.
#include "common.hpp"

#include <utility>

namespace sacd {

namespace {

// Rows per block: the importance pass uses RB = 256 / 128 / 64 at
// RP <= 32 / 64 / 128; the update pass uses 256 rows at RP <= 32 and 64 rows
// above.  With the thread counts below, 4 (RP <= 32) or 8 lanes share each
// row's Gauss-Seidel chain.  Smaller row blocks at RP <= 32 were measured
// slower: the Gram reduction over more partial blocks costs more than they
// save.
template <int RP>
constexpr int imp_rows() {
  return RP <= 32 ? 256 : (RP == 64 ? 128 : 64);
}
template <int RP>
constexpr int upd_rows() {
  return RP <= 32 ? 256 : 64;
}
// Threads per block of the importance and update passes.  The row blocks
// above fix which rows' partial sums are added together; the thread count
// only sets how many waves work on a block's chain of dependent steps, and
// no result depends on it (tiles are summed per wave in a fixed order, see
// tile_sums_total).  A job alone takes 1024 threads at RP <= 32 and 512
// above, except the update pass at RP = 128 (below) (measured fastest: the
// chain, not bandwidth, bounds these passes);
// the job-batched forms take 256, which suits many small jobs resident at
// once, or, at RP <= 32, 1024 when the jobs of a launch have few row blocks
// in all (the caller's choice, `big`).
template <int RP>
constexpr int elem_threads() {
  return RP <= 32 ? 1024 : 512;
}
// The update pass of a job alone at RP = 128 takes 1024 threads (16 lanes
// per row): measured 94 against 115 us per mode at I = 20000 (one 132 KB
// block per compute unit either way); at RP = 64, 512 stays faster.
template <int RP>
constexpr int upd_threads() {
  return RP == 128 ? 1024 : elem_threads<RP>();
}

template <int RP, int RB_, int NTH_ = kThreads>
struct UCfg {
  static constexpr int RB = RB_;        // rows per block
  static constexpr int NTH = NTH_;      // threads per block
  static constexpr int W = NTH / 64;    // waves per block
  static constexpr int STR = RP + 1;    // LDS row stride (floats)
  static constexpr int TC = RP / 16;    // 16-column tiles
  static constexpr int NT = (RB / 16) * TC;  // 16x16 tiles per block
  static constexpr int NTW = NT / W;    // tiles per wave
  static_assert(NT % W == 0, "tiles must divide evenly over the waves");
};

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 operands (mixed-precision form): FP32 -> BF16 with round to nearest
// even (inputs are finite), 16x16x16 MFMA with FP32 accumulation.  Lane l
// supplies A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16], j < 4.
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Load of data stored by other blocks of the same grid.  Every block stores,
// then issues the release half of a device-scope fence before it increments
// the arrival counter; the last block issues the acquire half after reading
// the counter, which invalidates its caches, so plain loads that follow
// observe the other blocks' stores (fence_release_device /
// fence_acquire_device).  Plain loads can be pipelined, unlike atomic ones.
template <typename T>
__device__ __forceinline__ T ld_coherent(const T *p) {
  return *p;
}

// A block's rows of A_n and H are staged in LDS in two halves: fetch issues
// the global loads into registers, commit stores them to LDS.  A kernel
// fetches everything it reads before the first commit, so that the block
// waits on memory once instead of once per array.
template <int RP, int RB, int NTH = kThreads>
struct RowStage {
  static_assert((RB * RP / 4) % NTH == 0, "whole float4 per thread");
  static constexpr int N4 = RB * RP / 4 / NTH;  // float4 per thread
  f32x4 v[N4];
  // Rows past I read row I - 1 and keep zeros: a load whose value is used
  // on every path is not sunk past the first wait, as a branch around it
  // would allow.  A block exists only for row0 < I.
  __device__ __forceinline__ void fetch(const float *__restrict__ A, int row0, int I) {
#pragma unroll
    for (int k = 0; k < N4; ++k) {
      const int i = (threadIdx.x + k * NTH) * 4;
      const int r = row0 + i / RP;
      const f32x4 x = *(const f32x4 *)(A + (long long)(r < I ? r : I - 1) * RP + i % RP);
      v[k] = (r < I) ? x : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
  __device__ __forceinline__ void commit(float *sA) const {
#pragma unroll
    for (int k = 0; k < N4; ++k) {
      const int i = (threadIdx.x + k * NTH) * 4;
      float *d = sA + (i / RP) * (RP + 1) + i % RP;
      d[0] = v[k][0];
      d[1] = v[k][1];
      d[2] = v[k][2];
      d[3] = v[k][3];
    }
  }
};

// H (RP x RP) into LDS with row stride RP + 1, VEC consecutive words per
// load.  Where the block's threads divide H evenly (every RP >= 32 with the
// thread counts used here) every thread loads and stores unconditionally,
// so that the load stays where it is issued.
template <int RP, int NTH = kThreads>
struct HStage {
  static constexpr int TOT = RP * RP;
  static constexpr int VEC = (TOT % (4 * NTH) == 0 || TOT < NTH) ? 4 : 1;
  static constexpr bool EXACT = TOT % (VEC * NTH) == 0;
  static constexpr int N = (TOT / VEC + NTH - 1) / NTH;  // loads per thread
  static_assert(VEC == 4 || EXACT, "single words only where every thread has one");
  f32x4 v[N];
  __device__ __forceinline__ void fetch(const float *__restrict__ H) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int i = (threadIdx.x + k * NTH) * VEC;
      if constexpr (VEC == 4) {
        v[k] = *(const f32x4 *)(H + (i < TOT ? i : 0));
      } else {
        v[k][0] = H[i];
      }
    }
  }
  __device__ __forceinline__ void commit(float *sH) const {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int i = (threadIdx.x + k * NTH) * VEC;
      if (EXACT || i < TOT) {
        float *d = sH + (i / RP) * (RP + 1) + i % RP;
#pragma unroll
        for (int e = 0; e < VEC; ++e) d[e] = v[k][e];
      }
    }
  }
};

// With 512 or more threads a block fetches its rows and H together; the
// 256-thread blocks of the job-batched forms hold 4-8 times as many words per
// thread and fetch H after committing the rows, which keeps them from spilling.
template <int NTH>
constexpr bool stage_together() {
  return NTH >= 512;
}

template <int RP, int RB, int NTH = kThreads>
__device__ __forceinline__ void load_rows(float *sA, const float *__restrict__ A, int row0, int I) {
  RowStage<RP, RB, NTH> rs;
  rs.fetch(A, row0, I);
  rs.commit(sA);
}

// C tile (16 x 16) of the block's rows times H: rows tr*16.., columns tc*16..
// BF: operands rounded to BF16, FP32 accumulation.
template <int RP, int RB, bool BF>
__device__ __forceinline__ f32x4 tile_AH(const float *sA, const float *sH, int tr, int tc, int lane) {
  using Cf = UCfg<RP, RB>;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  if constexpr (BF) {
#pragma unroll
    for (int kk = 0; kk < RP / 16; ++kk) {
      bf16x4 a, b;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kk * 16 + 4 * (lane >> 4) + j;
        a[j] = to_bf16(sA[(tr * 16 + (lane & 15)) * Cf::STR + k]);
        b[j] = to_bf16(sH[k * (RP + 1) + tc * 16 + (lane & 15)]);
      }
      acc = mfma_bf16(a, b, acc);
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < RP / 4; ++kk) {
      const float a = sA[(tr * 16 + (lane & 15)) * Cf::STR + kk * 4 + (lane >> 4)];
      const float b = sH[(kk * 4 + (lane >> 4)) * (RP + 1) + tc * 16 + (lane & 15)];
      acc = mfma4(a, b, acc);
    }
  }
  return acc;
}

// Partial Gram matrix of the block's rows (the upper 16x16 tiles of
// sA^T sA), written to gp.  Each tile is split into P = RB / 64 row quarters
// of 64 rows; a quarter is four independent MFMA accumulation chains over
// interleaved row groups, added as (c0 + c1) + (c2 + c3), and a tile's
// quarters are added in order, ((q0 + q1) + (q2 + q3)).  The (tile, quarter)
// items are spread over the W waves, so with many waves the quarters run in
// parallel; the arithmetic of every item, and so the result, does not depend
// on W.  scratch: P x (upper tiles) x 256 floats of LDS, used when P > 1.
// BF: operands rounded to BF16, FP32 accumulation.
template <int RP, int RB, bool BF, int W = 4>
__device__ __forceinline__ void gram_tiles(const float *sA, float *gp, float *scratch, int wv, int lane) {
  using Cf = UCfg<RP, RB>;
  constexpr int n16 = RP / 16, NUT = n16 * (n16 + 1) / 2, P = RB / 64;
  static_assert(RB % 64 == 0 && (P == 1 || P == 2 || P == 4), "row quarters of 64 rows");
  for (int it = wv; it < NUT * P; it += W) {
    const int u = it / P, p = it % P;
    int ti_ = 0, rem = u;
    while (rem >= n16 - ti_) {
      rem -= n16 - ti_;
      ++ti_;
    }
    const int tj = ti_ + rem;
    f32x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r0 = p * 64;
    if constexpr (BF) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        bf16x4 a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = r0 + 16 * c + 4 * (lane >> 4) + j;
          a[j] = to_bf16(sA[row * Cf::STR + ti_ * 16 + (lane & 15)]);
          b[j] = to_bf16(sA[row * Cf::STR + tj * 16 + (lane & 15)]);
        }
        acc[c] = mfma_bf16(a, b, acc[c]);
      }
    } else {
#pragma unroll
      for (int k0 = r0; k0 < r0 + 64; k0 += 16) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int row = k0 + 4 * c + (lane >> 4);
          const float a = sA[row * Cf::STR + ti_ * 16 + (lane & 15)];
          const float b = sA[row * Cf::STR + tj * 16 + (lane & 15)];
          acc[c] = mfma4(a, b, acc[c]);
        }
      }
    }
    const f32x4 q = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if constexpr (P == 1) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        gp[(ti_ * 16 + 4 * (lane >> 4) + v) * RP + tj * 16 + (lane & 15)] = q[v];
    } else {
      *(f32x4 *)(scratch + (size_t)it * 256 + 4 * lane) = q;
    }
  }
  if constexpr (P > 1) {
    __syncthreads();
    for (int u = wv; u < NUT; u += W) {
      int ti_ = 0, rem = u;
      while (rem >= n16 - ti_) {
        rem -= n16 - ti_;
        ++ti_;
      }
      const int tj = ti_ + rem;
      f32x4 q[P];
#pragma unroll
      for (int p = 0; p < P; ++p) q[p] = *(const f32x4 *)(scratch + (size_t)(u * P + p) * 256 + 4 * lane);
      f32x4 tot;
      if constexpr (P == 4) tot = (q[0] + q[1]) + (q[2] + q[3]);
      else tot = q[0] + q[1];
#pragma unroll
      for (int v = 0; v < 4; ++v)
        gp[(ti_ * 16 + 4 * (lane >> 4) + v) * RP + tj * 16 + (lane & 15)] = tot[v];
    }
  }
}

// FP64 sum over the 64 lanes of a wave by a butterfly of lane exchanges;
// lane 0's value is the one used (its order of additions is fixed).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NTH = kThreads>
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < NTH / 64; ++k) r += red[k];
  __syncthreads();  // red may be written again right after
  return r;
}

// Total of the per-tile sums sT[0..NT) in tile order (thread 0 calls it after
// a barrier).  Each tile's sum is formed by the wave that holds the tile --
// its lanes' values in row order, then wave_sum -- so the total does not
// depend on how many waves share the block's tiles.
template <int NT>
__device__ __forceinline__ double tile_sums_total(const double *sT) {
  double t = 0.0;
  for (int k = 0; k < NT; ++k) t += sT[k];
  return t;
}

// Block blk (of nblk) of the importance pass of one sweep.
// Importance pass of one sweep.  Solo form: block b of the job in `solo`.
// Job-batched form: a persistent grid loops over the block map's entries
// (job in `jobs`, block of the job, blocks of the job).  The body sits in the
// kernel itself (see k_mttkrp).
template <int RP, bool BF, bool BATCHED, int NTH>
__global__ __launch_bounds__(NTH) void k_importance(ImpArgs solo, const ImpArgs *__restrict__ jobs,
                                                         const int4 *__restrict__ bmap, int nb) {
 for (int item = blockIdx.x;; item += gridDim.x) {
  ImpArgs args;
  int blk, nblk;
  if constexpr (BATCHED) {
    if (item >= nb) break;
    const int4 m = bmap[item];
    args = jobs[m.x];
    blk = m.y;
    nblk = m.z;
  } else {
    args = solo;
    blk = blockIdx.x;
    nblk = gridDim.x;
  }
  do {
  const int I = args.I;
  const float *__restrict__ A = args.A;
  const float *__restrict__ M = args.M;
  const float *__restrict__ H = args.H;
  const HInfo *__restrict__ hi = args.hi;
  double *__restrict__ ti_part = args.ti_part;
  ModeState *st = args.st;
  using Cf = UCfg<RP, imp_rows<RP>(), NTH>;
  __shared__ float sA[Cf::RB * Cf::STR];
  __shared__ float sH[RP * (RP + 1)];
  __shared__ double red[Cf::W];
  __shared__ double sT[Cf::NT];  // per-tile sums
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blk * Cf::RB;
  // everything the block reads is requested before the first wait: L, h_rr
  // and its near-zero flag for this thread's columns, the MTTKRP entries of
  // its tiles, the block's rows and H (the 256-thread blocks read h_rr per
  // tile and H after the rows, with fewer registers)
  const float halfL = hi->halfL;
  float mv[Cf::NTW][4], hv[Cf::NTW];
  int nzv[Cf::NTW];
#pragma unroll
  for (int ti = 0; ti < Cf::NTW; ++ti) {
    const int t = wv + Cf::W * ti;
    const int tr = t / Cf::TC, tc = t % Cf::TC;
    const int cc = tc * 16 + (lane & 15);
    if constexpr (stage_together<Cf::NTH>()) {
      hv[ti] = hi->hdiag[cc];
      nzv[ti] = hi->nearzero[cc];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long long q = row0 + tr * 16 + 4 * (lane >> 4) + v;
      mv[ti][v] = (q < I) ? M[q * RP + cc] : 0.0f;
    }
  }
  RowStage<RP, Cf::RB, Cf::NTH> rows;
  HStage<RP, Cf::NTH> hst;
  rows.fetch(A, row0, I);
  if constexpr (stage_together<Cf::NTH>()) hst.fetch(H);
  rows.commit(sA);
  if constexpr (!stage_together<Cf::NTH>()) hst.fetch(H);
  hst.commit(sH);
  __syncthreads();
#pragma unroll
  for (int ti = 0; ti < Cf::NTW; ++ti) {
    const int t = wv + Cf::W * ti;
    const int tr = t / Cf::TC, tc = t % Cf::TC;
    const f32x4 ah = tile_AH<RP, Cf::RB, BF>(sA, sH, tr, tc, lane);
    const int cc = tc * 16 + (lane & 15);
    float h;
    int nz;
    if constexpr (stage_together<Cf::NTH>()) {
      h = hv[ti];
      nz = nzv[ti];
    } else {
      h = hi->hdiag[cc];
      nz = hi->nearzero[cc];
    }
    double zs = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = tr * 16 + 4 * (lane >> 4) + v;
      if (row0 + rr < I) {
        float d;
        const float z = element_importance(ah[v], mv[ti][v], sA[rr * Cf::STR + cc], h, nz, halfL, &d);
        zs += (double)z;
      }
    }
    zs = wave_sum(zs);
    if (lane == 0) sT[t] = zs;
  }
  __syncthreads();
  if (tid == 0) {
    ti_part[blk] = tile_sums_total<Cf::NT>(sT);
    fence_release_device();
    const unsigned prev = atomicAdd(&st->cnt_imp, 1u);
    s_last = (prev == (unsigned)nblk - 1);
  }
  __syncthreads();
  if (!s_last) break;
  fence_acquire_device();
  // the sweep count and ti^{k-1}, read while the partials are summed
  const long long kprev = st->k;
  const double tprev = st->ti_prev;
  // the block partials in a fixed 256-lane pattern whatever the block size
  // (extra waves add exact zeros at the end)
  double s = 0.0;
  if (tid < kThreads)
    for (int i = tid; i < nblk; i += kThreads) s += ld_coherent(&ti_part[i]);
  const double ti = block_sum<Cf::NTH>(s, red);
  if (tid == 0) {
    const long long k = kprev + 1;
    const int first = (k == 1);
    st->flip = (!first && ti > tprev) ? 1 : 0;  // eq. 27 condition: "more than"
    st->first = first;
    st->k = k;
    st->ti = ti;
    st->ti_prev = ti;  // becomes ti^{k-1} of the next sweep (eq. 26)
    st->cnt_imp = 0;
  }
  } while (0);
  if constexpr (!BATCHED) break;
  __syncthreads();  // the block's LDS is reused by its next work item
 }
}

// A lane with at most this many of a row's columns holds their h_rr and
// near-zero flags in registers through the chain; one with more reads them
// from their LDS copy at each step (registers would spill).
constexpr int kPreCols = 16;

// Value of lane OWNER of the caller's row group of LPR lanes, to every lane
// of the group, by a DPP lane move (row groups are aligned to LPR lanes):
// quad_perm within quads of 4 lanes, row_newbcast within rows of 16 (the
// row groups the element passes use: 4, 8 or 16 lanes).
template <int LPR, int OWNER>
__device__ __forceinline__ float row_bcast(float d) {
  static_assert(LPR == 4 || LPR == 8 || LPR == 16, "row groups of 4, 8 or 16 lanes");
  const int x = __float_as_int(d);
  if constexpr (LPR == 4) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, x, OWNER * 0x55, 0xF, 0xF, false));
  } else if constexpr (LPR == 8) {
    const int lo = __builtin_amdgcn_update_dpp(0, x, 0x150 + OWNER, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, x, 0x158 + OWNER, 0xF, 0xF, false);
    return __int_as_float((threadIdx.x & 8u) ? hi : lo);
  } else {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x150 + OWNER, 0xF, 0xF, false));
  }
}

// Step r of a row's chain (r a constant): skipped unless column r is
// selected (with h_rr > 0).
template <int RP, int UPD, int LPR, int NW, int R>
__device__ __forceinline__ void chain_step(float *a, float *g, const float *hl, const bool *nzl,
                                           const unsigned long long *sel, const float *sH, const float *sHd,
                                           const int *sNz, int part) {
  constexpr int CPL = RP / LPR, OWNER = R % LPR, J = R / LPR;
  constexpr bool PRE = CPL <= kPreCols;
  if (!((sel[R >> 6] >> (R & 63)) & 1ull)) return;
  float d = 0.0f;
  if (LPR == 1 || part == OWNER) {
    const float h = PRE ? hl[J] : sHd[R];
    const bool nz = PRE ? nzl[J] : (sNz[R] != 0);
    const float q = nz ? (float)((double)g[J] / (double)h) : __fdiv_rn(g[J], h);
    const float an = fmaxf(__fsub_rn(a[J], q), 0.0f);  // eq. 11-13
    d = __fsub_rn(an, a[J]);
    a[J] = an;
  }
  if (UPD == 0) {
    if constexpr (LPR > 1) d = row_bcast<LPR, OWNER>(d);
    if (d != 0.0f) {
      if constexpr (LPR == 1) {
#pragma unroll
        for (int s = R + 1; s < RP; ++s) g[s] = __fmaf_rn(d, sH[R * (RP + 1) + s], g[s]);
      } else if (part + LPR * (CPL - 1) > R) {
        // the row group reads consecutive words of H's row R for each jj
#pragma unroll
        for (int jj = 0; jj < CPL; ++jj) g[jj] = __fmaf_rn(d, sH[R * (RP + 1) + part + LPR * jj], g[jj]);
      }
    }
  }
}

template <int RP, int UPD, int LPR, int NW, int... Rs>
__device__ __forceinline__ void chain_steps(float *a, float *g, const float *hl, const bool *nzl,
                                            const unsigned long long *sel, const float *sH, const float *sHd,
                                            const int *sNz, int part, std::integer_sequence<int, Rs...>) {
  (chain_step<RP, UPD, LPR, NW, Rs>(a, g, hl, nzl, sel, sH, sHd, sNz, part), ...);
}

// One row's Gauss-Seidel (UPD 0) or Jacobi (UPD 1) steps over its selected
// columns in increasing order (Alg. 1, eq. 11-13).  The row's LPR lanes
// share it: lane `part` keeps the row's columns part, part + LPR, ... of a
// and g in registers.  For each selected column r in order, the lane owning
// r takes the one-variable step; under Gauss-Seidel the step d is passed to
// the row's other lanes, which refresh their columns' gradient,
// g_s += d H_rs.  Only columns s > r are read again, so the refresh of the
// others (done to keep the loop free of per-lane bounds) changes nothing.
template <int RP, int UPD, int LPR>
__device__ __forceinline__ void update_row(float *a_l, const float *g_l, const unsigned short *s_l,
                                           const float *sH, const float *sHd, const int *sNz,
                                           const unsigned long long *hpos, int part) {
  constexpr int CPL = RP / LPR;  // columns per lane
  constexpr bool PRE = CPL <= kPreCols;
  constexpr int NPRE = PRE ? CPL : 1;
  float a[CPL], g[CPL], hl[NPRE];
  bool nzl[NPRE];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    a[j] = a_l[part + LPR * j];
    g[j] = g_l[part + LPR * j];
  }
  // h_rr and its near-zero flag of the lane's columns (from their LDS copy)
  // are held in registers through the chain when the lane has few columns
  if constexpr (PRE) {
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      hl[j] = sHd[part + LPR * j];
      nzl[j] = sNz[part + LPR * j] != 0;
    }
  }
  // selection bits of the whole row, less the columns with h_rr <= 0 (no
  // step there): the row's lanes walk the same steps
  constexpr int NW = (RP + 63) / 64;
  unsigned long long sel[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    sel[w] = 0;
#pragma unroll
    for (int k = 0; k < 4 && 4 * w + k < RP / 16; ++k)
      sel[w] |= (unsigned long long)s_l[4 * w + k] << (16 * k);
    sel[w] &= hpos[w];
  }
  chain_steps<RP, UPD, LPR, NW>(a, g, hl, nzl, sel, sH, sHd, sNz, part, std::make_integer_sequence<int, RP>{});
#pragma unroll
  for (int j = 0; j < CPL; ++j) a_l[part + LPR * j] = a[j];
}

// Block blk of the selection / update pass of one sweep.
// Selection / update pass of one sweep (solo or job-batched, as k_importance).
template <int RP, int UPD, bool DIAG, bool BF, bool BATCHED, int NTH>
__global__ __launch_bounds__(NTH) void k_select_update(UpdArgs solo, const UpdArgs *__restrict__ jobs,
                                                            const int4 *__restrict__ bmap, int nb) {
 for (int item = blockIdx.x;; item += gridDim.x) {
  UpdArgs args;
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
  const int I = args.I;
  float *__restrict__ A = args.A;
  const float *__restrict__ M = args.M;
  float *__restrict__ Z = args.Z;
  const float *__restrict__ H = args.H;
  const HInfo *__restrict__ hi = args.hi;
  const ModeState *__restrict__ st = args.st;
  float *__restrict__ gpart = args.gpart;
  double *__restrict__ inner_part = args.inner_part;
  int *__restrict__ cnt_part = args.cnt_part;
  uint8_t *__restrict__ selmask = args.selmask;
  using Cf = UCfg<RP, upd_rows<RP>(), NTH>;
  __shared__ float sA[Cf::RB * Cf::STR];
  __shared__ __align__(16) float sG[Cf::RB * Cf::STR];  // gradients, then the Gram tiles' scratch
  static_assert((Cf::RB / 64 > 1 ? (Cf::RB / 64) * (RP / 16) * (RP / 16 + 1) / 2 * 256 : 0) <= Cf::RB * Cf::STR,
                "Gram scratch fits in sG");
  __shared__ float sH[RP * (RP + 1)];
  __shared__ unsigned short sSel[Cf::RB * (RP / 16)];  // selection bits, 16 columns a word
  __shared__ double sT[Cf::NT];  // per-tile sums
  __shared__ int sCnt[RP];
  __shared__ unsigned long long sHpos[(RP + 63) / 64];  // bit r: h_rr > 0
  __shared__ float sHd[RP];  // h_rr
  __shared__ int sNz[RP];    // h_rr near zero: divide in FP64
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blk * Cf::RB;
  // everything the block reads is requested before the first wait: the
  // sweep's selection state, L, h_rr and its near-zero flag (thread c holds
  // column c), the MTTKRP and previous-importance entries of this thread's
  // tiles, the block's rows and H
  static_assert(RP <= Cf::NTH, "a thread per column of H");
  const int first = st->first, flip = st->flip;
  const float halfL = hi->halfL;
  const int cown = tid < RP ? tid : 0;
  const float hd_own = hi->hdiag[cown];
  const int nz_own = hi->nearzero[cown];
  float mreg[Cf::NTW][4], zpreg[Cf::NTW][4];
#pragma unroll
  for (int ti = 0; ti < Cf::NTW; ++ti) {
    const int t = wv + Cf::W * ti;
    const int tr = t / Cf::TC, tc = t % Cf::TC;
    const int cc = tc * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long long q = row0 + tr * 16 + 4 * (lane >> 4) + v;
      mreg[ti][v] = (q < I) ? M[q * RP + cc] : 0.0f;
      zpreg[ti][v] = (q < I) ? Z[q * RP + cc] : 0.0f;
    }
  }
  RowStage<RP, Cf::RB, Cf::NTH> rows;
  HStage<RP, Cf::NTH> hst;
  rows.fetch(A, row0, I);
  if constexpr (stage_together<Cf::NTH>()) hst.fetch(H);
  if (tid < RP) {
    sHd[tid] = hd_own;
    sNz[tid] = nz_own;
  }
  if (wv < (RP + 63) / 64) {
    const unsigned long long b = __ballot(tid < RP && hd_own > 0.0f);  // lane l: column 64 wv + l
    if (lane == 0) sHpos[wv] = b;
  }
  rows.commit(sA);
  if constexpr (!stage_together<Cf::NTH>()) hst.fetch(H);
  hst.commit(sH);
  for (int c = tid; c < RP; c += Cf::NTH) sCnt[c] = 0;
  __syncthreads();
#pragma unroll
  for (int ti = 0; ti < Cf::NTW; ++ti) {
    const int t = wv + Cf::W * ti;
    const int tr = t / Cf::TC, tc = t % Cf::TC;
    const f32x4 ah = tile_AH<RP, Cf::RB, BF>(sA, sH, tr, tc, lane);
    const int cc = tc * 16 + (lane & 15);
    const float h = sHd[cc];
    const int nz = sNz[cc];
    int cnt = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = tr * 16 + 4 * (lane >> 4) + v;
      const long long q = row0 + rr;
      bool sl = false;
      float gv = 0.0f;
      if (q < I) {
        const float m = mreg[ti][v];
        float d;
        const float z = element_importance(ah[v], m, sA[rr * Cf::STR + cc], h, nz, halfL, &d);
        const float zp = zpreg[ti][v];
        // Alg. 1: first sweep z > 0; later sp = z - zprev (eq. 24) or zprev - z (eq. 27) > 0
        sl = first ? (z > 0.0f) : (flip ? (z < zp) : (z > zp));
        Z[q * RP + cc] = z;
        gv = __fsub_rn(ah[v], m);
        if (DIAG) selmask[q * RP + cc] = sl ? 1 : 0;
      }
      sG[rr * Cf::STR + cc] = gv;
      // lane l holds row 4 (l / 16) + v, column l % 16 of the tile
      const unsigned long long bal = __ballot(sl);
      if ((lane & 15) == 0) sSel[rr * (RP / 16) + tc] = (unsigned short)(bal >> (lane & 48));
      cnt += __popcll(bal & (0x0001000100010001ull << (lane & 15)));
    }
    if (lane < 16 && cnt) atomicAdd(&sCnt[cc], cnt);
  }
  __syncthreads();
  {
    constexpr int LPR = Cf::NTH / Cf::RB;  // lanes per row
    const int row = tid / LPR;
    if (row0 + row < I)  // the same for all lanes of a row
      update_row<RP, UPD, LPR>(sA + row * Cf::STR, sG + row * Cf::STR, sSel + row * (RP / 16), sH, sHd, sNz,
                               sHpos, tid % LPR);
  }
  __syncthreads();
  for (int i = tid; i < Cf::RB * RP; i += Cf::NTH) {
    const int r = i / RP, c = i % RP;
    if (row0 + r < I) A[(long long)(row0 + r) * RP + c] = sA[r * Cf::STR + c];
  }
  // <M, A_n> over the block, FP64, tile by tile
#pragma unroll
  for (int ti = 0; ti < Cf::NTW; ++ti) {
    const int t = wv + Cf::W * ti;
    const int tr = t / Cf::TC, tc = t % Cf::TC;
    const int cc = tc * 16 + (lane & 15);
    double inner = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = tr * 16 + 4 * (lane >> 4) + v;
      inner += (double)mreg[ti][v] * (double)sA[rr * Cf::STR + cc];
    }
    inner = wave_sum(inner);
    if (lane == 0) sT[t] = inner;
  }
  __syncthreads();
  if (tid == 0) inner_part[blk] = tile_sums_total<Cf::NT>(sT);
  for (int c = tid; c < RP; c += Cf::NTH) cnt_part[(long long)blk * RP + c] = sCnt[c];
  // partial Gram matrix of the block's new rows (upper triangle of 16x16 tiles)
  // (sG is free again: it serves as the tiles' LDS scratch)
  gram_tiles<RP, Cf::RB, BF, Cf::W>(sA, gpart + (long long)blk * RP * RP, sG, wv, lane);
  if constexpr (BF) {
    // the objective's Gram from FP32 operands (eq. 6 in FP64 of the factors
    // as they are, not of their BF16 roundings)
    if (args.gpart_obj) {
      __syncthreads();  // the scratch of the first pass is read until here
      gram_tiles<RP, Cf::RB, false, Cf::W>(sA, args.gpart_obj + (long long)blk * RP * RP, sG, wv, lane);
    }
  }
  } while (0);
  if constexpr (!BATCHED) break;
  __syncthreads();  // the block's LDS is reused by its next work item
 }
}

// Gram partials of an arbitrary factor (initialisation, set_factor).
template <int RP, bool BF>
__global__ __launch_bounds__(kThreads) void k_gram_partial(int I, const float *__restrict__ A,
                                                           float *__restrict__ gpart,
                                                           float *__restrict__ gpart_obj) {
  using Cf = UCfg<RP, upd_rows<RP>()>;
  constexpr int NUT = (RP / 16) * (RP / 16 + 1) / 2, P = Cf::RB / 64;
  __shared__ float sA[Cf::RB * Cf::STR];
  __shared__ __align__(16) float scratch[P > 1 ? P * NUT * 256 : 4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  load_rows<RP, Cf::RB>(sA, A, blockIdx.x * Cf::RB, I);
  __syncthreads();
  gram_tiles<RP, Cf::RB, BF>(sA, gpart + (long long)blockIdx.x * RP * RP, scratch, wv, lane);
  if constexpr (BF) {
    if (gpart_obj) {
      __syncthreads();
      gram_tiles<RP, Cf::RB, false>(sA, gpart_obj + (long long)blockIdx.x * RP * RP, scratch, wv, lane);
    }
  }
}

// Threads per block of the Gram reduction: 16 entries x kGramStripes.  One
// block size serves a job alone and the job-batched form (the stripes fix
// the order of additions); 256 suits the many small jobs of the batched form,
// 512 would save about 1 us per launch on a 1e7-entry tensor.
constexpr int kGramThreads = 256;
constexpr int kGramStripes = kGramThreads / 16;

// Sum of the values base[p * stride], p = s, s + S, s + 2S, ... < n (S =
// kGramStripes), in index order, sixteen loads in flight at a time.
template <typename Acc, typename T>
__device__ __forceinline__ Acc stripe_sum(const T *base, long long stride, int s, int n) {
  constexpr int S = kGramStripes;
  Acc acc = 0;
  for (int p0 = s; p0 < n; p0 += 16 * S) {
    T v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int p = p0 + S * k;
      v[k] = (p < n) ? base[(long long)p * stride] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += (Acc)v[k];
  }
  return acc;
}

// Sum of v over the kGramStripes stripes s = tid / 16 of entry e = tid % 16,
// in a fixed order: the four stripes of a wave by lane exchanges, then the
// waves in order.  Threads 0..15 get their entry's sum.  red holds
// kGramThreads / 4 values.
template <typename T>
__device__ __forceinline__ T stripe_tree(T v, T *red) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane < 16) red[wv * 16 + lane] = v;
  __syncthreads();
  T t = 0;
  if (threadIdx.x < 16) {
#pragma unroll
    for (int k = 0; k < kGramThreads / 64; ++k) t += red[k * 16 + threadIdx.x];
  }
  __syncthreads();
  return t;
}

// Number of 16-entry strips of the upper 16x16 tiles of an RP x RP matrix.
template <int RP>
constexpr int gram_strips() {
  return 16 * (RP / 16) * (RP / 16 + 1) / 2;
}

// The sweep's objective (eq. 6) and total selection count from the shares
// k_gram_final wrote, by one block in a fixed order:
//   f = ||X||^2 - 2 <M_n, A_n> + sum_rs (Gram_0 * Gram_1 * Gram_2)_rs.
// The shares must be visible to the block: written by an earlier kernel, or
// by blocks that issued a device-scope fence before the caller's arrival
// counter showed them done.  red holds kGramThreads / 64 values.
template <int RP>
__device__ __forceinline__ void gram_finish_body(const GramArgs &args, double *red) {
  constexpr int NS = gram_strips<RP>();
  const int tid = threadIdx.x;
  ModeState *st = args.st;
  double mv = 0.0;
  long long cv = 0;
  if (args.with_f)
    for (int k = tid; k < NS; k += kGramThreads) mv += ld_coherent(&args.mpart[k]);
  if (args.cnt_part && tid < RP) cv = ld_coherent(&args.colcnt[tid]);
  if (args.with_f) {
    const double inner = ld_coherent(&st->inner);
    const double model = block_sum<kGramThreads>(mv, red);
    if (tid == 0) st->f = args.normX2 - 2.0 * inner + model;
  }
  if (args.cnt_part) {
    const double all = block_sum<kGramThreads>((double)cv, red);
    if (tid == 0) st->nsel = (long long)all;
  }
}

// Where the objective is formed: at RP >= 64 (hundreds of strip blocks) and
// in the job-batched form by k_gram_finish after k_gram_final; for a job alone
// at smaller ranks by the last block of k_gram_final to arrive.  An arrival
// counter needs a device-scope fence and an atomic round trip in every block
// (measured 10 us per launch at R = 128, 585 blocks), a kernel of its own
// about 4 us per launch (more than the fences of the 51 blocks at R = 32).  A
// persistent block of the batched form works through the strips of many
// jobs, one fence and round trip per strip.  The result is the same either
// way.
template <int RP, bool BATCHED>
constexpr bool gram_split() {
  return BATCHED || RP >= 64;
}

// Gram reduction in FP64 and the sweep's scalars, one level, fixed order.
// Blocks [0, NS): one 16-entry strip (row i, columns 16 tj .. 16 tj + 15,
// tile tj >= tile of i) of Gram_n each; thread (e, s) = (tid % 16, tid / 16)
// adds the block partials s, s + 16, ... of entry e in order, the 16 stripes
// are then added in a fixed tree order.  The strip is written to Gram_n and
// mirrored, and with with_f the block also writes its share of
//   sum_rs (Gram_n * Gram_a * Gram_b)_rs
// (entries of off-diagonal tiles count twice).  Blocks [NS, NS + RP/16):
// selection counts of 16 columns.  Block NS + RP/16: <M, A_n>.  Then
// gram_finish_body forms the objective and the total selection count (see
// gram_split).
template <int RP, bool BATCHED>
__global__ __launch_bounds__(kGramThreads) void k_gram_final(GramArgs solo, const GramArgs *__restrict__ jobs,
                                                         const int4 *__restrict__ bmap, int nb) {
 for (int item = blockIdx.x;; item += gridDim.x) {
  GramArgs args;
  int blk, nblk;
  if constexpr (BATCHED) {
    if (item >= nb) break;
    const int4 m = bmap[item];
    args = jobs[m.x];
    blk = m.y;
    nblk = m.z;
  } else {
    args = solo;
    blk = blockIdx.x;
    nblk = gridDim.x;
  }
  do {
  const int nparts = args.nparts;
  const float *__restrict__ gpart = args.gpart;
  double *__restrict__ mpart = args.mpart;
  double *Gn = args.Gn;
  const double *__restrict__ Ga = args.Ga;
  const double *__restrict__ Gb = args.Gb;
  const float *__restrict__ gpart_obj = args.gpart_obj;
  double *Gn_obj = args.Gn_obj;
  const double *__restrict__ Ga_obj = args.Ga_obj;
  const double *__restrict__ Gb_obj = args.Gb_obj;
  const double *__restrict__ inner_part = args.inner_part;
  const int *__restrict__ cnt_part = args.cnt_part;
  long long *__restrict__ colcnt = args.colcnt;
  const int with_f = args.with_f;
  ModeState *st = args.st;
  constexpr int RR = RP * RP, n16 = RP / 16, NS = gram_strips<RP>();
  __shared__ double red[kGramThreads / 4];
  __shared__ long long redl[kGramThreads / 4];
  __shared__ int s_last;
  const int tid = threadIdx.x, e = tid & 15, s = tid >> 4;
  const int b = blk;
  if (b < NS) {
    int rem = b, ti = 0;
    while (rem >= 16 * (n16 - ti)) {
      rem -= 16 * (n16 - ti);
      ++ti;
    }
    const int i = ti * 16 + rem / (n16 - ti), tj = ti + rem % (n16 - ti);
    const int j = tj * 16 + e;
    const int x = i * RP + j;
    double wab = 0.0;
    if (with_f && s == 0)  // issued early
      wab = (ti == tj ? 1.0 : 2.0) * (gpart_obj ? Ga_obj[x] * Gb_obj[x] : Ga[x] * Gb[x]);
    const double tot = stripe_tree(stripe_sum<double>(gpart + x, RR, s, nparts), red);
    if (s == 0) {
      Gn[x] = tot;
      Gn[j * RP + i] = tot;
    }
    double vobj = tot;
    if (gpart_obj) {  // mixed form: the objective's Gram from the FP32 partials
      vobj = stripe_tree(stripe_sum<double>(gpart_obj + x, RR, s, nparts), red);
      if (s == 0) {
        Gn_obj[x] = vobj;
        Gn_obj[j * RP + i] = vobj;
      }
    }
    if (with_f && s == 0) red[tid] = vobj * wab;
    if (with_f) {
      __syncthreads();
      if (tid == 0) {
        double m = 0.0;
        for (int k = 0; k < 16; ++k) m += red[k];
        mpart[b] = m;
      }
    }
  } else if (b < NS + n16) {
    if (cnt_part) {
      const int c = (b - NS) * 16 + e;
      const long long tot = stripe_tree(stripe_sum<long long>(cnt_part + c, RP, s, nparts), redl);
      if (s == 0) colcnt[c] = tot;
    }
  } else {
    if (inner_part) {
      double v = 0.0;
      for (int p0 = tid; p0 < nparts; p0 += 4 * kGramThreads) {
        double w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = (p0 + k * kGramThreads < nparts) ? inner_part[p0 + k * kGramThreads] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) v += w[k];
      }
      const double in = block_sum<kGramThreads>(v, red);
      if (tid == 0) st->inner = in;
    }
  }
  if constexpr (!gram_split<RP, BATCHED>()) {
    __syncthreads();
    if (tid == 0) {
      fence_release_device();
      const unsigned prev = atomicAdd(args.counter, 1u);
      s_last = (prev == (unsigned)nblk - 1);
    }
    __syncthreads();
    if (!s_last) break;
    fence_acquire_device();
    gram_finish_body<RP>(args, red);
    if (tid == 0) *args.counter = 0;
  }
  } while (0);
  if constexpr (!BATCHED) break;
  __syncthreads();  // the block's LDS is reused by its next work item
 }
}

// The objective and total selection count as a kernel of its own, one block
// per job (batched form: the block map's first block of each job), where
// gram_split holds.
template <int RP, bool BATCHED>
__global__ __launch_bounds__(kGramThreads) void k_gram_finish(GramArgs solo, const GramArgs *__restrict__ jobs,
                                                          const int4 *__restrict__ bmap, int nb) {
 for (int item = blockIdx.x;; item += gridDim.x) {
  GramArgs args;
  if constexpr (BATCHED) {
    if (item >= nb) break;
    const int4 m = bmap[item];
    if (m.y != 0) continue;  // uniform over the block
    args = jobs[m.x];
  } else {
    args = solo;
  }
  __shared__ double red[kGramThreads / 64];
  gram_finish_body<RP>(args, red);
  if constexpr (!BATCHED) break;
 }
}

__global__ __launch_bounds__(kThreads) void k_init_factor(float *__restrict__ A, int I, int R, int RP,
                                                          unsigned long long seed,
                                                          unsigned long long offset) {
  const long long n = (long long)I * RP;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (long long)gridDim.x * blockDim.x) {
    const long long q = x / RP;
    const int c = (int)(x % RP);
    float v = 0.0f;
    if (c < R) {
      // output number e of SplitMix64(seed): mix(seed + (e + 1) * golden gamma)
      const unsigned long long e = offset + (unsigned long long)q * R + c;
      unsigned long long z = seed + (e + 1ull) * 0x9E3779B97F4A7C15ull;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      v = (float)(z >> 40) * (1.0f / 16777216.0f);
    }
    A[x] = v;
  }
}

// <X, Xhat> = sum over Omega of x * sum_r A0[i0,r] A1[i1,r] A2[i2,r] (eq. 8),
// FP64; the last block reduces the block partials in a fixed order.
__global__ __launch_bounds__(kThreads) void k_inner_full(const unsigned long long *__restrict__ keys,
                                                         const float *__restrict__ vals, long long nnz,
                                                         KeyLayout lay, int RP,
                                                         const float *__restrict__ A0,
                                                         const float *__restrict__ A1,
                                                         const float *__restrict__ A2,
                                                         double *__restrict__ part, double *out,
                                                         unsigned *counter) {
  __shared__ double red[kThreads];
  __shared__ int s_last;
  double s = 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (long long)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[p];
    const long long i0 = (long long)(k >> lay.sh_n), i1 = (long long)((k >> lay.sh_a) & lay.mask_a),
                    i2 = (long long)(k & lay.mask_b);
    double xh = 0.0;
    for (int r = 0; r < RP; ++r)
      xh += (double)A0[i0 * RP + r] * (double)A1[i1 * RP + r] * (double)A2[i2 * RP + r];
    s += (double)vals[p] * xh;
  }
  const double bs = block_sum(s, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bs;
    fence_release_device();
    const unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return;
  fence_acquire_device();
  double t = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kThreads) t += ld_coherent(&part[i]);
  const double tot = block_sum(t, red);
  if (threadIdx.x == 0) {
    *out = tot;
    *counter = 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_copy_rows(const float *__restrict__ src, int ss,
                                                        float *__restrict__ dst, int ds, int I,
                                                        int ncols, int zero_to) {
  const long long n = (long long)I * zero_to;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (long long)gridDim.x * blockDim.x) {
    const long long q = x / zero_to;
    const int c = (int)(x % zero_to);
    dst[q * ds + c] = (c < ncols) ? src[q * ss + c] : 0.0f;
  }
}

// Sum of squared errors of the model on n entries (the numerator of eq. 30):
// x_hat = sum_r A0[i0, r] A1[i1, r] A2[i2, r] from the FP32 factors, in FP64.
// Block partials are reduced by the last block in a fixed order.  A
// coordinate outside dims sets *bad and adds nothing.
__global__ __launch_bounds__(kThreads) void k_sq_error(const int32_t *__restrict__ idx,
                                                       const float *__restrict__ vals, long long n,
                                                       int d0, int d1, int d2, int RP,
                                                       const float *__restrict__ A0,
                                                       const float *__restrict__ A1,
                                                       const float *__restrict__ A2,
                                                       double *__restrict__ part, double *out,
                                                       unsigned *counter, int *bad) {
  __shared__ double red[kThreads];
  __shared__ int s_last;
  double s = 0.0;
  int oob = 0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int i0 = idx[3 * p], i1 = idx[3 * p + 1], i2 = idx[3 * p + 2];
    if (i0 < 0 || i0 >= d0 || i1 < 0 || i1 >= d1 || i2 < 0 || i2 >= d2) {
      oob = 1;
      continue;
    }
    double xh = 0.0;
    for (int r = 0; r < RP; ++r)
      xh += (double)A0[(long long)i0 * RP + r] * (double)A1[(long long)i1 * RP + r] *
            (double)A2[(long long)i2 * RP + r];
    const double e = (double)vals[p] - xh;
    s += e * e;
  }
  if (oob) atomicOr(bad, 1);
  const double bs = block_sum(s, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bs;
    fence_release_device();
    const unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return;
  fence_acquire_device();
  double t = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kThreads) t += ld_coherent(&part[i]);
  const double tot = block_sum(t, red);
  if (threadIdx.x == 0) {
    *out = tot;
    *counter = 0;
  }
}

// Zero n 32-bit words: a fill kernel, so that code a caller captures into a
// graph records no memset node.
__global__ __launch_bounds__(kThreads) void k_zero_words(unsigned *__restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// eq. 30 from the sum of squared errors of n entries: out[0] = sqrt(sum / n)
// (0 for n = 0), or NaN when a coordinate was outside dims; out[1] = 1 in
// that case, else 0.  Correctly rounded division and square root.
__global__ void k_rmse_finish(const double *__restrict__ sum, const int *__restrict__ bad, long long n,
                              double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int b = *bad;
  out[0] = b ? __longlong_as_double(0x7ff8000000000000ll)
             : (n > 0 ? __dsqrt_rn(__ddiv_rn(*sum, (double)n)) : 0.0);
  out[1] = b ? 1.0 : 0.0;
}

// Objective of the last sweep of each of n jobs, gathered into one array.
__global__ __launch_bounds__(kThreads) void k_gather_f(const ModeState *const *__restrict__ sts, int n,
                                                       double *__restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = sts[i]->f;
}

__global__ __launch_bounds__(kThreads) void k_check_factor(const float *__restrict__ a, long long n,
                                                           int *flag) {
  int bad = 0;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (long long)gridDim.x * blockDim.x) {
    const float v = a[x];
    if (!isfinite(v)) bad |= 2;
    else if (v < 0.0f) bad |= 1;
  }
  if (bad) atomicOr(flag, bad);
}

inline int grid_for(long long n, int per_block = kThreads * 4, int cap = 65535 * 4) {
  long long g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

int rows_per_block(int RP) {
  switch (RP) {
    case 16: return upd_rows<16>();
    case 32: return upd_rows<32>();
    case 64: return upd_rows<64>();
    case 128: return upd_rows<128>();
    default: return 0;
  }
}

hipError_t launch_init_factor(float *A, int I, int R, int RP, unsigned long long seed,
                              unsigned long long offset, hipStream_t s) {
  hipLaunchKernelGGL(k_init_factor, dim3(grid_for((long long)I * RP)), dim3(kThreads), 0, s, A, I, R,
                     RP, seed, offset);
  return hipGetLastError();
}

int importance_blocks(int RP, int I) {
  const int rb = RP <= 16 ? imp_rows<16>() : RP <= 32 ? imp_rows<32>() : RP <= 64 ? imp_rows<64>() : imp_rows<128>();
  return (I + rb - 1) / rb;
}
int update_blocks(int RP, int I) { return (I + rows_per_block(RP) - 1) / rows_per_block(RP); }
int gram_final_blocks(int RP) { return 16 * (RP / 16) * (RP / 16 + 1) / 2 + RP / 16 + 1; }
int gram_model_parts(int RP) { return 16 * (RP / 16) * (RP / 16 + 1) / 2; }

namespace {

// Dispatch of a launcher template over the padded rank.
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
struct ImpL {
  static hipError_t run(bool bf, const ImpArgs &a, hipStream_t s) {
    const int nb = importance_blocks(RP, a.I);
    if (nb == 0) return hipSuccess;
    if (bf) hipLaunchKernelGGL((k_importance<RP, true, false, elem_threads<RP>()>), dim3(nb), dim3(elem_threads<RP>()), 0, s, a, nullptr, nullptr, 0);
    else hipLaunchKernelGGL((k_importance<RP, false, false, elem_threads<RP>()>), dim3(nb), dim3(elem_threads<RP>()), 0, s, a, nullptr, nullptr, 0);
    return hipGetLastError();
  }
};

template <int RP>
struct ImpBL {
  static hipError_t run(bool bf, bool big, const ImpArgs *jobs, const int4 *bmap, int nb, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    if constexpr (RP <= 32) {
      if (big) {
        constexpr int T = elem_threads<RP>();
        if (bf)
          hipLaunchKernelGGL((k_importance<RP, true, true, T>), dim3(persistent_grid(nb)), dim3(T), 0, s, ImpArgs{},
                             jobs, bmap, nb);
        else
          hipLaunchKernelGGL((k_importance<RP, false, true, T>), dim3(persistent_grid(nb)), dim3(T), 0, s, ImpArgs{},
                             jobs, bmap, nb);
        return hipGetLastError();
      }
    }
    if (bf)
      hipLaunchKernelGGL((k_importance<RP, true, true, kThreads>), dim3(persistent_grid(nb)), dim3(kThreads), 0, s, ImpArgs{},
                         jobs, bmap, nb);
    else
      hipLaunchKernelGGL((k_importance<RP, false, true, kThreads>), dim3(persistent_grid(nb)), dim3(kThreads), 0, s, ImpArgs{},
                         jobs, bmap, nb);
    return hipGetLastError();
  }
};

template <int RP, int UPD, bool DIAG>
hipError_t upd_launch(bool bf, const UpdArgs &a, int nb, hipStream_t s) {
  constexpr int T = upd_threads<RP>();
  if (bf)
    hipLaunchKernelGGL((k_select_update<RP, UPD, DIAG, true, false, T>), dim3(nb), dim3(T), 0, s, a, nullptr, nullptr, 0);
  else
    hipLaunchKernelGGL((k_select_update<RP, UPD, DIAG, false, false, T>), dim3(nb), dim3(T), 0, s, a, nullptr, nullptr, 0);
  return hipGetLastError();
}

template <int RP>
struct UpdL {
  static hipError_t run(int update, bool diag, bool bf, const UpdArgs &a, hipStream_t s) {
    const int nb = update_blocks(RP, a.I);
    if (nb == 0) return hipSuccess;
    if (update == 0)
      return diag ? upd_launch<RP, 0, true>(bf, a, nb, s) : upd_launch<RP, 0, false>(bf, a, nb, s);
    return diag ? upd_launch<RP, 1, true>(bf, a, nb, s) : upd_launch<RP, 1, false>(bf, a, nb, s);
  }
};

template <int RP>
struct UpdBL {
  static hipError_t run(bool bf, bool big, const UpdArgs *jobs, const int4 *bmap, int nb, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    if constexpr (RP <= 32) {
      if (big) {
        constexpr int T = elem_threads<RP>();
        if (bf)
          hipLaunchKernelGGL((k_select_update<RP, 0, false, true, true, T>), dim3(persistent_grid(nb)), dim3(T), 0,
                             s, UpdArgs{}, jobs, bmap, nb);
        else
          hipLaunchKernelGGL((k_select_update<RP, 0, false, false, true, T>), dim3(persistent_grid(nb)), dim3(T), 0,
                             s, UpdArgs{}, jobs, bmap, nb);
        return hipGetLastError();
      }
    }
    if (bf)
      hipLaunchKernelGGL((k_select_update<RP, 0, false, true, true, kThreads>), dim3(persistent_grid(nb)), dim3(kThreads), 0, s,
                         UpdArgs{}, jobs, bmap, nb);
    else
      hipLaunchKernelGGL((k_select_update<RP, 0, false, false, true, kThreads>), dim3(persistent_grid(nb)), dim3(kThreads), 0, s,
                         UpdArgs{}, jobs, bmap, nb);
    return hipGetLastError();
  }
};

template <int RP>
struct GpL {
  static hipError_t run(bool bf, int I, const float *A, float *gpart, float *gpart_obj, hipStream_t s) {
    const int nb = update_blocks(RP, I);
    if (nb == 0) return hipSuccess;
    if (bf) hipLaunchKernelGGL((k_gram_partial<RP, true>), dim3(nb), dim3(kThreads), 0, s, I, A, gpart, gpart_obj);
    else hipLaunchKernelGGL((k_gram_partial<RP, false>), dim3(nb), dim3(kThreads), 0, s, I, A, gpart, nullptr);
    return hipGetLastError();
  }
};

template <int RP>
struct GfL {
  static hipError_t run(const GramArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_gram_final<RP, false>), dim3(gram_final_blocks(RP)), dim3(kGramThreads), 0, s, a, nullptr,
                       nullptr, 0);
    if constexpr (gram_split<RP, false>())
      hipLaunchKernelGGL((k_gram_finish<RP, false>), dim3(1), dim3(kGramThreads), 0, s, a, nullptr, nullptr, 0);
    return hipGetLastError();
  }
};

template <int RP>
struct GfBL {
  static hipError_t run(const GramArgs *jobs, const int4 *bmap, int nb, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_gram_final<RP, true>), dim3(persistent_grid(nb)), dim3(kGramThreads), 0, s, GramArgs{}, jobs,
                       bmap, nb);
    if constexpr (gram_split<RP, true>())
      hipLaunchKernelGGL((k_gram_finish<RP, true>), dim3(persistent_grid(nb)), dim3(kGramThreads), 0, s, GramArgs{},
                         jobs, bmap, nb);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_importance(int RP, bool bf, const ImpArgs &a, hipStream_t s) {
  return rp_dispatch<ImpL>(RP, bf, a, s);
}
hipError_t launch_importance_b(int RP, bool bf, bool big, const ImpArgs *jobs, const int4 *bmap, int nblocks,
                               hipStream_t s) {
  return rp_dispatch<ImpBL>(RP, bf, big, jobs, bmap, nblocks, s);
}
hipError_t launch_select_update(int RP, int update, bool diag, bool bf, const UpdArgs &a, hipStream_t s) {
  return rp_dispatch<UpdL>(RP, update, diag, bf, a, s);
}
hipError_t launch_select_update_b(int RP, bool bf, bool big, const UpdArgs *jobs, const int4 *bmap, int nblocks,
                                  hipStream_t s) {
  return rp_dispatch<UpdBL>(RP, bf, big, jobs, bmap, nblocks, s);
}
hipError_t launch_gram_partial(int RP, bool bf, int I, const float *A, float *gpart, float *gpart_obj,
                               hipStream_t s) {
  return rp_dispatch<GpL>(RP, bf, I, A, gpart, gpart_obj, s);
}
hipError_t launch_gram_final(int RP, const GramArgs &a, hipStream_t s) { return rp_dispatch<GfL>(RP, a, s); }
hipError_t launch_gram_final_b(int RP, const GramArgs *jobs, const int4 *bmap, int nblocks, hipStream_t s) {
  return rp_dispatch<GfBL>(RP, jobs, bmap, nblocks, s);
}

hipError_t launch_inner_full(const unsigned long long *keys0, const float *vals0, long long nnz,
                             KeyLayout lay0, int RP, const float *A0, const float *A1, const float *A2,
                             double *partials, int nparts, double *out, unsigned *counter,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_inner_full, dim3(nparts), dim3(kThreads), 0, s, keys0, vals0, nnz, lay0, RP, A0,
                     A1, A2, partials, out, counter);
  return hipGetLastError();
}

hipError_t launch_copy_rows(const float *src, int src_stride, float *dst, int dst_stride, int I,
                            int ncols, int zero_cols_to, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_rows, dim3(grid_for((long long)I * zero_cols_to)), dim3(kThreads), 0, s, src,
                     src_stride, dst, dst_stride, I, ncols, zero_cols_to);
  return hipGetLastError();
}

hipError_t launch_sq_error(const int32_t *idx, const float *vals, long long n, const int64_t *dims, int RP,
                           const float *A0, const float *A1, const float *A2, double *partials, int nparts,
                           double *out, unsigned *counter, int *bad, hipStream_t s) {
  long long g = (n + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  if (g > nparts) g = nparts;
  hipLaunchKernelGGL(k_sq_error, dim3((int)g), dim3(kThreads), 0, s, idx, vals, n, (int)dims[0], (int)dims[1],
                     (int)dims[2], RP, A0, A1, A2, partials, out, counter, bad);
  return hipGetLastError();
}

hipError_t launch_zero_words(unsigned *p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_rmse_finish(const double *sum, const int *bad, long long n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_rmse_finish, dim3(1), dim3(64), 0, s, sum, bad, n, out);
  return hipGetLastError();
}

hipError_t launch_gather_f(const ModeState *const *sts, int n, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_f, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, sts, n, out);
  return hipGetLastError();
}

hipError_t launch_check_factor(const float *src, long long n, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_factor, dim3(grid_for(n)), dim3(kThreads), 0, s, src, n, flag);
  return hipGetLastError();
}

}  // namespace sacd
