// Internal declarations of the lcemd library (host side + kernel launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lcemd.h"

namespace lcemd {

// ---------------------------------------------------------------------------
// constants shared by kernels and host planning
// ---------------------------------------------------------------------------
constexpr int kRows = 64;        // phase-1 rows per workgroup
constexpr int kKChunk = 32;      // phase-1 K (embedding dim) chunk staged in LDS
constexpr int kColChunk = 64;    // phase-1 columns per MFMA pass
constexpr int kThreads = 256;    // threads per workgroup for every kernel
constexpr int kSelectBuf = 2048; // LDS slots of the selection sort
// Segments (the histogram whose words are a phase-1 workgroup's columns) of
// up to kSegShort words keep their per-column arrays in LDS in every
// phase-1 kernel variant; longer ones (up to LCEMD_MAX_HIST) run on float32
// variants sized for them.
constexpr int kSegShort = 512;
// ICT's phase-1 lists stop here (its tables hold more); the few rows whose
// capacities do not yet cover the word's largest weight are redone exactly.
constexpr int kIctList = 16;
// bfloat16 phase-1 rows: the real dims plus six folded-in terms, rounded up
// to 64 dims; the bf16 kernel holds rows of up to this many dims in
// registers (wider embeddings select with float32 keys).
constexpr int kBf16MaxDims = 384;
__host__ __device__ inline int bf16_row_dims(int m) { return (m + 6 + 63) / 64 * 64; }
// The keys kernel for segments longer than kSegShort keeps its rows of keys
// in device memory: one region of kRows x (LCEMD_MAX_HIST + 4) floats per
// workgroup of a launch, launches of at most kDeepSlots workgroups.
constexpr int kDeepSlots = 2048;
constexpr int64_t kDeepSlotFloats = (int64_t)kRows * (LCEMD_MAX_HIST + 4);

// How a phase-1 workgroup finds its rows and its column segment, and what
// it emits.
enum P1Mode : int {
  P1_TABLE = 0,       // rows = used vocabulary block, segment = one query;
                      // emits depth-limited (z, w) rows for phase 2
  P1_TABLE_FULL = 1,  // same rows/segment; emits S, Z, W at full depth k_eff
  P1_PAIR = 2,        // rows = one query's words, segment = one database row;
                      // emits the summed per-row transfer cost (Q2D)
};

enum P1Prec : int { PREC_F32 = 0, PREC_BF16 = 1, PREC_FP8 = 2 };

struct P1Args {
  // embeddings
  const float* V;         // [v][m_pad] float32, zero padded
  const float* vnorm;     // [v] |v|^2 (float64 accumulation, stored float32)
  const uint16_t* Vb;     // [v][mb] bfloat16 rows: -2 v, then 1, 1, 1 and a three-piece
                          // split of |v|^2 in the six dims after the m real ones
  const uint16_t* Vbq;    // [v][mb] the same words as query operands: v, the split, 1, 1, 1
  const float* vres;      // [v] |v - bf16(v)|, rounded up (bf16 error bound)
  float4* rinfo;          // bf16 kernel scratch: [v_used] row records
  float4* qinfo;          // bf16 kernel scratch: [qnnz] query-word records
  float2* qmx;            // bf16 kernel scratch: [nq] per query (max |q|^2, max |q - bf16(q)|)
  int64_t qnnz;           // query non-zeros (qptr[B]) the records cover
  int mb;                 // dims per bfloat16 row (bf16_row_dims(m))
  int m;                  // real dims
  const uint8_t* V8;      // [v][m8] fp8 (OCP e4m3) codes of V / vscale (PREC_FP8)
  const float* vscale;    // [v] fp8 row scales
  int m8;                 // bytes per fp8 row: m_pad rounded up to 128
  int m_pad;
  int m4;                 // float4 groups holding the m real dims, ceil(m / 4) (the rest are zero)
  // measure
  int method;             // LCEMD_RWMD / OMR / ACT / ICT
  int k;                  // ACT k
  int KT;                 // table stride (entries per table row)
  int KT_margin;          // extra candidates kept for the exact re-sort (bf16/fp8 keys)
  // database
  int64_t n;
  const int64_t* xptr;    // [n+1]
  const int2* xcv;        // [nnz] (compact word id, weight bits)
  const int32_t* xcol;    // [nnz] original word ids
  int64_t v_used;
  const int32_t* used;    // [v_used] original id of each used word
  const float* xmax;      // [v_used] largest database weight per used word
  // queries
  const int64_t* qptr;    // [B+1]
  const int32_t* qcol;
  const float* qval;
  int64_t q0;             // first query of this launch (table modes)
  int64_t nq;             // queries in this launch (table modes)
  // pair mode
  int64_t npairs;
  const int64_t* pair_q;  // [npairs] query index, or NULL: full grid
  const int64_t* pair_u;  // [npairs] database row, or NULL: full grid
  const uint64_t* cand;   // candidate list (packed key | index), or NULL
  int64_t cand_ld;        // candidates per query in `cand`
  int64_t cand_use;       // candidates evaluated per query
  const int32_t* qlist;   // query ids for candidate mode (NULL: identity)
  int rb_max;             // row blocks per pair (grid y)
  // outputs
  float2* ZW;             // P1_TABLE: see zw_at
  int64_t zw_nq;          // P1_TABLE: queries per table (the tile's or batch's slot count)
  int32_t* S;             // P1_TABLE_FULL: [nq][v_used][k]
  float* Z;
  float* W;
  float* partial;         // P1_PAIR: [npairs][rb_max]
  int* overflow;          // set to 1 when a row needed more than KT entries
  int* fix_count;         // bf16 table modes: rows whose exactness certificate failed ...
  int64_t* fix_list;      // ... are appended here (flat table row index) for k_fix_rows
  int fix_cap;
  unsigned long long* fix_total;  // optional: k_fix_rows adds the rows it redoes
  // persistent kernels: eight work counters (one per XCD), zeroed by the
  // launcher on its stream before the kernel
  unsigned long long* work_ctr;
  // keys kernel on segments longer than kSegShort: kDeepSlots regions of
  // kDeepSlotFloats floats, and the first workgroup of the current launch
  float* deep_keys;
  int64_t blk0;
};

// Table layout of P1_TABLE: entry l of query qi's row for used word r.
// Entries go in pairs (2p, 2p + 1) of 16 bytes, and pair p of one word lies
// next to pair p of the same word for every query of the table, so that
// phase 2 reads a word's first pair for a group of queries as one
// contiguous run: float2 index ((r * KP + p) * zw_nq + qi) * 2 + (l & 1),
// KP = ceil(KT / 2), zw_nq = zw_pitch(queries of the table).  Tables hold
// zw_nq * v_used * KP float4.
__host__ __device__ inline int64_t zw_pairs(int KT) { return (KT + 1) >> 1; }
// Queries per table run, padded so that consecutive words' runs are not a
// multiple of a large power of two apart (which would send a word-strided
// gather to few memory channels).
__host__ __device__ inline int64_t zw_pitch(int64_t nq) { return (nq + 15) / 16 * 16 + 16; }
__device__ __forceinline__ float4* zw_pair(float2* ZW, int64_t zw_nq, int KT, int64_t qi, int64_t r,
                                           int p) {
  return (float4*)ZW + (r * zw_pairs(KT) + p) * zw_nq + qi;
}
// Write the D entries (z_l, w_l) of one table row (pairs; an odd tail pair
// gets zeros in its second half).
template <typename ZF, typename WF>
__device__ __forceinline__ void zw_write_row(float2* ZW, int64_t zw_nq, int KT, int64_t qi,
                                             int64_t r, int D, ZF zf, WF wf) {
  for (int l = 0; l < D && l < KT; l += 2) {
    const bool two = l + 1 < D && l + 1 < KT;
    *zw_pair(ZW, zw_nq, KT, qi, r, l >> 1) =
        make_float4(zf(l), wf(l), two ? zf(l + 1) : 0.f, two ? wf(l + 1) : 0.f);
  }
}

// kernel launchers (each in the translation unit of its kernel)
hipError_t launch_phase1_deep(const P1Args& a, int mode, int hmax, int prec, hipStream_t s);
hipError_t launch_phase1_fast(const P1Args& a, int mode, int KT, int prec, hipStream_t s);
hipError_t launch_phase1_wide(const P1Args& a, int mode, int KL, int prec, int seg_hmax, hipStream_t s);
// bfloat16 table modes (lists of depth + 8 <= 32, segments <= kSegShort words,
// rows of at most kBf16MaxDims dims)
bool phase1_bf16_fits(int mb, int seg_hmax, int depth);
hipError_t launch_phase1_bf16(const P1Args& a, int mode, int depth, hipStream_t s);
int phase1_wide_rows();
hipError_t launch_fix_rows(const P1Args& a, int mode, int count, hipStream_t s);
hipError_t launch_pair_reduce(const float* partial, int64_t npairs, int rb_max, float* out,
                              int64_t out_ld, int64_t per_row, hipStream_t s);
hipError_t launch_prep_embeddings(const float* Vin, int64_t v, int m, int m_pad, int l2norm,
                                  float* Vpad, float* vnorm, hipStream_t s);
hipError_t launch_make_bf16_rows(const float* V, const float* vnorm, int64_t v, int m, int m_pad, int mb,
                                 uint16_t* out_row, uint16_t* out_query, float* vres, hipStream_t s);
hipError_t launch_make_fp8(const float* V, int64_t v, int m_pad, int m8, uint8_t* out, float* scale,
                           hipStream_t s);
hipError_t launch_validate_csr(const int64_t* ptr, const int32_t* col, const float* val,
                               int64_t rows, int64_t v, int normalized, int* err,
                               hipStream_t s);
// L smallest (distance, index) keys of each row; rows longer than one
// workgroup's part go through a first pass per part into `tmp`
// (select_tmp_elems entries; may be null when that is 0).
int64_t select_parts(int64_t n);
int64_t select_tmp_elems(int64_t rows, int64_t n, int L);
hipError_t launch_select(const float* keys, int64_t ld, int64_t n, int64_t rows, int L,
                         const int32_t* row_list, int64_t exclude_base, uint64_t* out,
                         uint64_t* tmp, hipStream_t s);
hipError_t launch_finalize_sym(const uint64_t* cand, int64_t cand_ld, int64_t cand_use,
                               const float* q2d, int64_t rows, const int32_t* row_list,
                               int64_t n, int L, int64_t* idx, float* dist, int* flags,
                               hipStream_t s);
hipError_t launch_unpack_topl(const uint64_t* cand, int64_t cand_ld, int64_t rows,
                              const int32_t* row_list, int L, int64_t* idx, float* dist,
                              hipStream_t s);
hipError_t launch_max_inplace(float* a, const float* b, int64_t count, hipStream_t s);
hipError_t launch_record_weights(const int2* xcv, int64_t nnz, float* val, hipStream_t s);
// Records of a query batch as the set phase 2 walks (reverse.hip): scratch
// holds reverse_scratch_ints(v) ints; used / xmax hold up to min(H, v)
// entries, cv H, perm B; *nu (device) gets the used word count.
int64_t reverse_scratch_ints(int64_t v);
hipError_t launch_reverse_records(const int64_t* ptr, const int32_t* col, const float* val, int64_t B, int64_t H,
                                  int64_t v, int* scratch, int2* cv, int32_t* used, float* xmax, int32_t* perm,
                                  int* nu, hipStream_t s);
// in-place n x n: mode 0 transpose, 1 symmetric maximum
hipError_t launch_square_pair(float* D, int64_t n, int mode, hipStream_t s);
// out[c * ld_out + r] = in[r * cols + c] for a rows x cols row-major `in`
hipError_t launch_transpose(const float* in, int64_t rows, int64_t cols, float* out, int64_t ld_out,
                            hipStream_t s);
hipError_t launch_zero_ints(int* p, int count, hipStream_t s);
// Resident workgroups per CU for a kernel (cached) and the CU count.
int persistent_grid(const void* kernel, int threads, size_t shmem, int64_t items);
// Phase 2 on a persistent grid: the query count is nq_dev[0] when nq_dev is
// not null (fixed-shape batches; nq is then its largest value), else nq.
// perm: the documents in order of length (used for batches of up to 32
// queries).  counters: 8 u64, zeroed here.
// Word-major phase 2 (phase2.hip) for one group of 64 queries: wptr[v_used
// + 1] / wwt = the database's weights grouped by compact word id (CSR
// order within a word, every word with at least one), winv[i] = the
// by-word index of CSR non-zero i; cost: nnz x 64 floats of scratch; ZW
// and out start at the group's first query; KT <= 16; counters: 16 u64.
hipError_t launch_phase2_wordmajor(const int64_t* xptr, int64_t n, const int64_t* wptr, const float* wwt,
                                   const uint32_t* winv, int64_t nnz, int64_t v_used, const float2* ZW,
                                   int64_t zw_nq, int KT, float* cost, float* out, int64_t ld,
                                   unsigned long long* counters, hipStream_t s);
hipError_t launch_phase2_persistent(const int64_t* xptr, const int2* xcv, int64_t n, const int32_t* perm,
                                    const float2* ZW, int64_t zw_nq, int KT, int64_t nq,
                                    const int* nq_dev, float* out, int64_t ld,
                                    unsigned long long* counters, hipStream_t s);

}  // namespace lcemd
