// common.hpp -- internal declarations shared by the HIP sources of libsacd.
//
// Device data layout (one tensor, one model):
//   tensor, per mode n:  keys[n]  nnz x uint64  bit-packed (i_n, i_a, i_b), i_n in
//                                 the high bits, sorted ascending (so entries of a
//                                 slice are contiguous, fibres (i_n, i_a) too)
//                        vals[n]  nnz x f32
//                        ptr[n]   (I_n + 1) x int32 slice offsets
//   model, per mode n:   A[n]     I_n x RP f32 factor, row stride RP (R padded to
//                                 16/32/64/128 with zero columns)
//                        Z[n]     I_n x RP f32 importance of the last sweep
//                        M[n]     I_n x RP f32 MTTKRP of the last sweep
//                        G64[n]   RP x RP f64 Gram matrix A_n^T A_n
//   Padded columns are exactly zero in A, so their Gram rows/columns, H rows/
//   columns and MTTKRP columns are zero: h_rr = 0 columns take no step and add
//   nothing to any sum, which leaves every result of the real columns unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sacd {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kMaxRP = 128;

// Grid of a job-batched (persistent) launch: at most kPersistentBlocks
// blocks, each looping over the launch's work items (block-map entries).
constexpr int kPersistentBlocks = 2048;
inline int persistent_grid(int nb) { return nb < kPersistentBlocks ? nb : kPersistentBlocks; }

// Per-mode selection / sweep state, resident in device memory so that a whole
// iteration can be replayed as a HIP graph without host decisions.
struct ModeState {
  long long k;          // sweeps of this mode done
  double ti_prev;       // total importance of the previous sweep (eq. 26)
  double ti;            // total importance of the current sweep (eq. 25)
  double f;             // objective after the last sweep of this mode (eq. 6)
  double L;             // Lipschitz constant ||H||_F of the last sweep
  double inner;         // <M_n, A_n> after the last sweep
  long long nsel;       // elements selected in the last sweep
  int flip;             // eq. 27 branch taken in the current sweep
  int first;            // current sweep is the first of this mode (k == 1)
  unsigned cnt_imp;     // arrival counters of the "last block" reductions
  unsigned cnt_gram;
  unsigned cnt_inner;
  unsigned pad;
};

// H = Gram_a * Gram_b of the current sweep and what the element kernels need.
struct HInfo {
  float halfL;            // L / 2 in FP32
  float L32;
  double L64;
  float hdiag[kMaxRP];    // h_rr
  int nearzero[kMaxRP];   // h_rr < 1e-6 max_s h_ss: divide in FP64
};

// Key layout of one mode.
struct KeyLayout {
  int sh_n;       // shift of i_n
  int sh_a;       // shift of i_a (= bits of i_b)
  unsigned long long mask_a;
  unsigned long long mask_b;
};

__device__ __forceinline__ int key_row(unsigned long long k, int sh_n) { return (int)(k >> sh_n); }

// The two halves of a device-scope fence for an arrival counter: a block
// stores its partial results, issues the release half, then increments the
// counter (a relaxed atomic); the block that sees the count complete issues
// the acquire half before it reads the others' results.  The release half
// writes back the L2; only the last block needs the acquire half, which
// invalidates the caches that later reads would otherwise hit.
__device__ __forceinline__ void fence_release_device() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire_device() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Importance of one element (eq. 20) from the MTTKRP entry m, the entry ah of
// A_n H, the current value a, h = h_rr and L / 2.  Explicitly rounded FP32
// operations: the importance and the update kernels recompute the same z
// bit for bit.  Returns z; *step receives the projected step (eq. 11-12).
__device__ __forceinline__ float element_importance(float ah, float m, float a, float h,
                                                    int nearzero, float halfL, float *step) {
  const float g = __fsub_rn(ah, m);  // eq. 14: g = -M + (A H)
  float d = 0.0f;
  if (h > 0.0f) {
    const float q = nearzero ? (float)((double)g / (double)h) : __fdiv_rn(g, h);  // eq. 11
    const float u = __fsub_rn(a, q);
    d = __fsub_rn(fmaxf(u, 0.0f), a);  // eq. 12
  }
  *step = d;
  return __fsub_rn(-__fmul_rn(g, d), __fmul_rn(__fmul_rn(halfL, d), d));  // eq. 20
}

// --------------------------------------------------------------------------
// Launchers (host functions defined in the .hip files)
// --------------------------------------------------------------------------

// ingest.hip
hipError_t launch_make_keys0(const int32_t *idx, const float *vals, long long nnz, const int64_t *dims,
                             KeyLayout lay0, unsigned long long *keys, float *vout, int *err_flags,
                             hipStream_t s);
size_t radix_sort_temp_bytes(long long n);
hipError_t radix_sort_pairs(unsigned long long *keys, float *vals, unsigned long long *keys_alt,
                            float *vals_alt, long long n, int lo_bit, int hi_bit, void *temp,
                            hipStream_t s, bool *result_in_alt);
size_t dedup_temp_bytes(long long n);
hipError_t dedup_sorted(const unsigned long long *keys, const float *vals, long long n,
                        unsigned long long *ukeys, float *uvals, int *d_count, void *temp,
                        hipStream_t s);
hipError_t launch_rekey(const unsigned long long *keys0, long long n, KeyLayout lay0, int mode,
                        KeyLayout layn, unsigned long long *keysn, hipStream_t s);
hipError_t build_ptr(const unsigned long long *keys, long long n, int sh_n, int I, int *ptr,
                     void *temp, hipStream_t s);
// Tiled order of mode n's keys (the MTTKRP's tiled form): (i_n, i_b >> tsh,
// i_a, i_b) with a tile field of tb bits; sorting on bits [sh_n, sh_n + tb +
// bits(i_n)) of the stable mode-n order gives that order.
hipError_t launch_tile_keys(const unsigned long long *keys, long long n, KeyLayout lay, int tsh, int tb,
                            unsigned long long *out, hipStream_t s);
size_t build_ptr_temp_bytes(long long n, int I);
hipError_t launch_gather_keys(const unsigned long long *keys, const int *pos, int n,
                              unsigned long long *out, hipStream_t s);
hipError_t launch_norm2(const float *vals, long long n, double *partials, int nparts, double *out,
                        hipStream_t s);
hipError_t launch_export_coo(const unsigned long long *keys, const float *vals, long long n,
                             KeyLayout lay, int32_t *coords, float *vout, const int *ptr, int I,
                             int64_t *ptr64, hipStream_t s);

// mttkrp.hip
// Static work plan of one mode (built once per tensor from the slice
// pointers): every slice cut into segments of at most kSegment entries.
constexpr int kSegment = 256;
// Zeroed entries kept after the end of every mode's key and value arrays, so
// that the MTTKRP can load the keys of a next batch without a bounds test.
constexpr int kKeySlack = 16;
constexpr int kGatherBuckets = 64;  // i_a ranges that order the full-length segments
struct MttkrpPlan {
  long long nnz;
  int nunits;         // work units, longest first
  const int4 *units;  // device: (slice, first entry, entries, partial slot or -1)
  int nlong;          // slices split over several units
  int nbig;           // of them, those with more than kFixSmall slots (first in longs)
  const int4 *longs;  // device: (slice, first partial slot, slots, 0)
  int nslots;         // partial slots
  // one partial slot per unit of a split slice (the column-at-a-time form):
  const int *uslot;   // device, per unit: its slot, or -1 for a whole slice
  int nuslots;
  int nulong;
  const int4 *ulongs; // device: (slice, first unit slot, unit slots, 0), slots in entry order
};
int mttkrp_units_per_block(int RP);
int mttkrp_blocks(int RP, int nunits);
// Split slices of at most kFixSmall slots are added by one lane group each,
// kThreads / (RP / 4) of them per block; larger ones by a block each.
constexpr int kFixSmall = 8;
int fix_blocks(int RP, int nlong, int nbig);
struct MttkrpArgs {
  const unsigned long long *keys;
  const float *vals;
  const int4 *units;
  int nunits;
  KeyLayout lay;
  const float *Aa, *Ab;
  float *M, *part;
};
struct FixArgs {
  const int4 *longs;  // big split slices first (nbig of them), then the small ones
  int nlong;
  int nbig;
  const float *part;
  float *M;
  const double *Ga, *Gb;
  float *H;
  HInfo *hinfo;
  ModeState *st;
};
hipError_t launch_mttkrp(int RP, const MttkrpArgs &a, hipStream_t s);
// LDS-staged form (same M, bit for bit): CS columns of A_b (Ib rows) per slab;
// mttkrp_lds_cols gives CS for a table of Ib rows, or 0 when it does not apply.
// Tiled form (btab not null, nbt blocks): each block stages kTileRows rows of
// A_b, btab[q] = (first unit, units, first row, rows) over a plan whose
// entries are ordered by (i_n, i_b / kTileRows, i_a, i_b).
constexpr int kTileRows = 512;  // 64 columns x 512 rows x 4 B = the 128 KB LDS table
int mttkrp_lds_cols(int RP, long long Ib);
int mttkrp_lds_units_per_block(int CS);
hipError_t launch_mttkrp_lds(int RP, int CS, const MttkrpArgs &a, int Ib, const int4 *btab, int nbt,
                             hipStream_t s);
hipError_t launch_mttkrp_b(int RP, const MttkrpArgs *jobs, const int4 *bmap, int nblocks, hipStream_t s);
hipError_t launch_mttkrp_fix(int RP, const FixArgs &a, hipStream_t s);
hipError_t launch_mttkrp_fix_b(int RP, const FixArgs *jobs, const int4 *bmap, int nblocks, hipStream_t s);

// lowmem.hip: the column-at-a-time form (the MTTKRP a block of CB columns at
// a time, Sec. 4.4; no I_n x R buffer for M).  Mb: I_n x CB block of M.
struct ColArgs {
  int I, RP, c0, CB;
  const float *A;       // I x RP, the factor being swept
  const float *Mb;      // I x CB
  const float *H;       // RP x RP
  const HInfo *hi;
  ModeState *st;
  float *Z;             // I x RP
  unsigned *bits;       // 2 bits per element of I x RP: eq. 24 (k = 1: z > 0) and eq. 27 outcomes
  double *part;         // per (column block, row block) partial sums (ti, then <M, A_n>)
  int part_off;         // first partial of this column block
  int *cnt_part;        // per row block x RP selected counts
  uint8_t *selmask;     // diagnostics (or nullptr)
  float *Mdiag;         // diagnostics: the whole M (or nullptr)
};
constexpr int kColThreads = 256;  // rows per block of the column-form element kernels
int col_row_blocks(int I);
hipError_t launch_sttvp(int CB, const MttkrpArgs &a, int RP, int c0, const int *uslot, const int4 *ulongs, int nulong,
                        float *Mb, hipStream_t s);
hipError_t launch_col_importance(int CB, const ColArgs &a, hipStream_t s);
hipError_t launch_col_decide(const double *part, int n, ModeState *st, hipStream_t s);
hipError_t launch_col_update(int CB, const ColArgs &a, hipStream_t s);
hipError_t launch_col_finish(const double *part, int n, const int *cnt_part, int nrb, int RP, int ncols,
                             long long *colcnt, ModeState *st, hipStream_t s);

// nway.hip: the N-way form (N in [2, kMaxModes]).
constexpr int kMaxModes = 8;
// Key layout of one mode of an N-way tensor: field f holds the index of the
// f-th mode of the layout's order (mode n first, then the others in
// increasing mode order), at shift sh[f] with mask[f].
struct NLayout {
  int nf;                        // number of fields (modes)
  long long dims[kMaxModes];     // mode lengths, in field order of the mode-0 layout
  int sh[kMaxModes];
  unsigned long long mask[kMaxModes];
};
struct NShifts {
  int sh[kMaxModes];
};
struct NMttkrpArgs {
  const unsigned long long *keys;
  const float *vals;
  const int4 *units;  // (slice, first entry, entries, run slot or -1)
  int nunits;
  int nother;                          // N - 1
  const float *A[kMaxModes - 1];       // the other modes' factors, in increasing mode order
  int sh[kMaxModes - 1];               // their fields in mode n's layout
  unsigned long long mask[kMaxModes - 1];
  float *M, *part;
};
struct NGrams {
  int n;
  const double *G[kMaxModes];
};
struct NFactors {
  const float *A[kMaxModes];
};
hipError_t launch_make_keys_n(const int32_t *idx, const float *vals, long long nnz, const NLayout &lay,
                              unsigned long long *keys, float *vout, int *err, hipStream_t s);
hipError_t launch_rekey_n(const unsigned long long *k0, long long nnz, const NLayout &l0, const NShifts &to_sh,
                          unsigned long long *kn, hipStream_t s);
hipError_t launch_export_coo_n(const unsigned long long *keys, const float *vals, long long nnz, const NLayout &lay,
                               int32_t *coords, float *vout, const int *ptr, int I, int64_t *ptr64, hipStream_t s);
hipError_t launch_mttkrp_n(int RP, const NMttkrpArgs &a, hipStream_t s);
int nway_units_per_block(int RP);
hipError_t launch_prod_grams(const NGrams &g, int n, int RP, double *P, double *ones, hipStream_t s);
hipError_t launch_inner_full_n(const unsigned long long *keys0, const float *vals0, long long nnz,
                               const NLayout &lay, const NFactors &F, int RP, double *part, int nparts, double *out,
                               unsigned *counter, hipStream_t s);

// sweep.hip
// Arguments of one job's element kernels.  The solo launchers pass them by
// value; the job-batched launchers take device arrays of them plus a block
// map with one int4 (job, block of the job, blocks of the job, 0) per work
// item; their blocks loop over the work items (persistent grid).
struct ImpArgs {
  int I;
  const float *A, *M, *H;
  const HInfo *hi;
  double *ti_part;
  ModeState *st;
};
struct UpdArgs {
  int I;
  float *A;
  const float *M;
  float *Z;
  const float *H;
  const HInfo *hi;
  const ModeState *st;
  float *gpart;
  float *gpart_obj;  // mixed form: FP32 Gram partials for the objective (else nullptr)
  double *inner_part;
  int *cnt_part;
  uint8_t *selmask;
};
struct GramArgs {
  int nparts;           // per-block partials written by the update / Gram kernel
  const float *gpart;   // nparts x RP x RP
  double *mpart;        // gram_model_parts(RP) model-norm partials
  double *Gn;           // result Gram_n (RP x RP, FP64)
  const double *Ga, *Gb;  // the other modes' Grams (objective only)
  const double *inner_part;
  const int *cnt_part;
  long long *colcnt;
  // mixed form: the objective's Grams, reduced from FP32 partials (gpart_obj)
  // into Gn_obj; the other modes' objective Grams Ga_obj, Gb_obj.  nullptr in
  // the FP32 form, where Gn, Ga, Gb serve both.
  const float *gpart_obj;
  double *Gn_obj;
  const double *Ga_obj, *Gb_obj;
  double normX2;
  int with_f;
  unsigned *counter;    // arrival counter (zero between launches)
  ModeState *st;
};
int rows_per_block(int RP);  // rows per block of the update pass (Gram partials per block)
int importance_blocks(int RP, int I);
int update_blocks(int RP, int I);
int gram_final_blocks(int RP);
int gram_model_parts(int RP);
hipError_t launch_init_factor(float *A, int I, int R, int RP, unsigned long long seed,
                              unsigned long long offset, hipStream_t s);
hipError_t launch_importance(int RP, bool bf, const ImpArgs &a, hipStream_t s);
// big: at RP <= 32, blocks of 1024 threads instead of 256 (no result depends
// on the block size); for launches whose jobs have few row blocks in all.
hipError_t launch_importance_b(int RP, bool bf, bool big, const ImpArgs *jobs, const int4 *bmap, int nblocks,
                               hipStream_t s);
hipError_t launch_select_update(int RP, int update, bool diag, bool bf, const UpdArgs &a, hipStream_t s);
hipError_t launch_select_update_b(int RP, bool bf, bool big, const UpdArgs *jobs, const int4 *bmap, int nblocks,
                                  hipStream_t s);
// bf: BF16 operands into gpart, and FP32 ones into gpart_obj when it is not
// nullptr (mixed form); otherwise FP32 into gpart.
hipError_t launch_gram_partial(int RP, bool bf, int I, const float *A, float *gpart, float *gpart_obj,
                               hipStream_t s);
hipError_t launch_gram_final(int RP, const GramArgs &a, hipStream_t s);
hipError_t launch_gram_final_b(int RP, const GramArgs *jobs, const int4 *bmap, int nblocks, hipStream_t s);
hipError_t launch_inner_full(const unsigned long long *keys0, const float *vals0, long long nnz,
                             KeyLayout lay0, int RP, const float *A0, const float *A1,
                             const float *A2, double *partials, int nparts, double *out,
                             unsigned *counter, hipStream_t s);
hipError_t launch_copy_rows(const float *src, int src_stride, float *dst, int dst_stride, int I,
                            int ncols, int zero_cols_to, hipStream_t s);
hipError_t launch_sq_error(const int32_t *idx, const float *vals, long long n, const int64_t *dims, int RP,
                           const float *A0, const float *A1, const float *A2, double *partials, int nparts,
                           double *out, unsigned *counter, int *bad, hipStream_t s);
hipError_t launch_gather_f(const ModeState *const *sts, int n, double *out, hipStream_t s);
hipError_t launch_zero_words(unsigned *p, int n, hipStream_t s);
hipError_t launch_rmse_finish(const double *sum, const int *bad, long long n, double *out, hipStream_t s);
hipError_t launch_check_factor(const float *src, long long n, int *flag, hipStream_t s);

}  // namespace sacd
