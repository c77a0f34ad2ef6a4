// Phase 1 of LC-ACT (Sec. 4, Phase 1; App. B): distances between a block of
// vocabulary words and one query's words as a dense contraction on MFMA,
// followed by a per-row selection of the nearest query words and the
// gather of their weights (the matrices Z, S, W of Sec. 4).
//
// One workgroup owns 64 "rows" (embedding ids) and one "segment" of columns
// (embedding ids with weights):
//   P1_TABLE / P1_TABLE_FULL : rows = a block of the used vocabulary,
//                              segment = one query histogram (D2Q tables);
//   P1_PAIR                  : rows = one query's words (64 at a time),
//                              segment = one database histogram (Q2D of Alg.
//                              1-3 evaluated directly for that pair).
//
// Step 1 (MFMA): key[r][c] = |c|^2 - 2 <v_r, c> for all rows and columns,
//   written to LDS.  |v_r|^2 is constant per row, so the key ranks the
//   columns of a row exactly as the squared distance does.
// Step 2 (VALU): four lanes per row extract columns in ascending
//   (key, position) order -- position breaks ties -- and recompute each
//   extracted column's squared distance exactly in float32 by direct
//   differences (identical words give exactly 0).  Extraction stops at the
//   row's effective depth: k_eff = min(k, h) for ACT (Alg. 3), 1 for RWMD,
//   2 after an exact-zero nearest distance for OMR (Alg. 1), h for ICT
//   (Alg. 2) -- or earlier, once the extracted capacities cover the largest
//   mass the row can ever have to move (Lemma 1/2: a transfer never uses a
//   destination past that point).  The last entry of a row is a sink with
//   infinite capacity, which is Alg. 3's final "move the rest" step.
#include <algorithm>

#include "internal.h"

namespace lcemd {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint32_t order_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint64_t pack_key(float f, uint32_t pos) {
  return ((uint64_t)order_bits(f) << 32) | (uint64_t)pos;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// Rows of keys live in LDS for segments of up to kSegShort words; longer
// segments (GKEYS) keep them in a device-memory region of the workgroup's
// own (kDeepSlotFloats floats per workgroup of the launch).
template <int MODE, int HMAX>
struct P1Smem {
  static constexpr bool GKEYS = HMAX > kSegShort;
  static constexpr int KS = HMAX + 4;        // key row stride (floats); KS % 64 == 4
  static constexpr int SS = kKChunk + 4;     // staging row stride (floats)
  float keys[GKEYS ? 1 : kRows * KS];
  float Vs[kRows * SS];
  float Qs[kColChunk * SS];
  int cid[HMAX];
  float cap[HMAX];
  float qn[HMAX];
  int rid[kRows];
  float rbound[kRows];
  float rcost[kRows];
};

template <int MODE, int HMAX>
__global__ __launch_bounds__(kThreads) void k_phase1_f32(P1Args a) {
  using Sm = P1Smem<MODE, HMAX>;
  constexpr int KS = Sm::KS, SS = Sm::SS;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Sm& sm = *reinterpret_cast<Sm*>(smem_raw);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  static_assert(!Sm::GKEYS || Sm::KS * (int64_t)kRows <= kDeepSlotFloats, "key region too small");

  // ---------------- task decode ----------------
  // (bx, by): (pair, row block) or (row block, query).  The device-memory
  // key variant runs on a 1-D grid of at most kDeepSlots workgroups per
  // launch, starting at workgroup a.blk0 of the whole task.
  int64_t bx, by;
  if constexpr (Sm::GKEYS) {
    const int64_t t = a.blk0 + blockIdx.x;
    if constexpr (MODE == P1_PAIR) {
      bx = t / a.rb_max;
      by = t % a.rb_max;
    } else {
      const int64_t nbx = (a.v_used + kRows - 1) / kRows;
      bx = t % nbx;
      by = t / nbx;
    }
  } else {
    bx = blockIdx.x;
    by = blockIdx.y;
  }
  float* const keys = Sm::GKEYS ? a.deep_keys + (int64_t)blockIdx.x * kRows * KS : sm.keys;
  int nrows = 0, h = 0;
  int64_t out_row0 = 0;  // first output table row (table modes)
  int64_t pidx = 0;
  int rb = 0;
  if constexpr (MODE == P1_PAIR) {
    pidx = bx;
    rb = (int)by;
    int64_t b, u;
    if (a.cand) {
      const int64_t qi = pidx / a.cand_use, c = pidx % a.cand_use;
      b = a.qlist ? (int64_t)a.qlist[qi] : qi;
      u = (int64_t)(uint32_t)a.cand[qi * a.cand_ld + c];
    } else if (a.pair_q) {
      b = a.pair_q[pidx];
      u = a.pair_u[pidx];
    } else {
      b = a.q0 + pidx / a.n;
      u = pidx % a.n;
    }
    const int64_t qs = a.qptr[b];
    const int hq = (int)(a.qptr[b + 1] - qs);
    nrows = min(kRows, hq - rb * kRows);
    if (nrows <= 0 || u < 0 || u >= a.n) {
      if (tid == 0) a.partial[pidx * a.rb_max + rb] = 0.f;
      return;
    }
    if (tid < kRows) {
      const bool ok = tid < nrows;
      sm.rid[tid] = ok ? a.qcol[qs + rb * kRows + tid] : 0;
      sm.rbound[tid] = ok ? a.qval[qs + rb * kRows + tid] : 0.f;
    }
    const int64_t s0 = a.xptr[u];
    h = (int)(a.xptr[u + 1] - s0);
    for (int c = tid; c < h; c += kThreads) {
      const int w = a.xcol[s0 + c];
      sm.cid[c] = w;
      sm.cap[c] = __int_as_float(a.xcv[s0 + c].y);
      sm.qn[c] = a.vnorm[w];
    }
  } else {
    const int64_t r0 = bx * kRows;
    const int64_t qi = by;
    const int64_t b = a.q0 + qi;
    nrows = (int)min((int64_t)kRows, a.v_used - r0);
    out_row0 = qi * a.v_used + r0;
    if (tid < kRows) {
      const bool ok = tid < nrows;
      sm.rid[tid] = ok ? a.used[r0 + tid] : 0;
      sm.rbound[tid] = ok ? (MODE == P1_TABLE ? a.xmax[r0 + tid] : INFINITY) : 0.f;
    }
    const int64_t s0 = a.qptr[b];
    h = (int)(a.qptr[b + 1] - s0);
    if (h <= 0) return;  // padding slot of a fixed-size batch
    for (int c = tid; c < h; c += kThreads) {
      const int w = a.qcol[s0 + c];
      sm.cid[c] = w;
      sm.cap[c] = a.qval[s0 + c];
      sm.qn[c] = a.vnorm[w];
    }
  }
  __syncthreads();

  // ---------------- step 1: keys on MFMA (32x32x2 f32) ----------------
  // Wave w computes the 32x32 sub-tile (rows wr.., columns wc..) of each
  // 64x64 pass.  Inside a K chunk of 32, lane half lh supplies the 16
  // consecutive dims [16*lh, 16*lh+16) over 16 MFMA steps (the same K
  // permutation on both operands, so the contraction is unchanged).
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 31, lh = lane >> 5;
  const int m_pad = a.m_pad;
  for (int c0 = 0; c0 < h; c0 += kColChunk) {
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int kc = 0; kc < 4 * a.m4; kc += kKChunk) {  // chunks past 4*m4 are zero padding
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int f = tid + it * kThreads;  // 0..511 float4 slots per tile
        const int r = f >> 3, q4 = (f & 7) * 4;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < nrows) x = *(const float4*)(a.V + (size_t)sm.rid[r] * m_pad + kc + q4);
        *(float4*)(&sm.Vs[r * SS + q4]) = x;
        const int c = c0 + r;
        float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c < h) y = *(const float4*)(a.V + (size_t)sm.cid[c] * m_pad + kc + q4);
        *(float4*)(&sm.Qs[r * SS + q4]) = y;
      }
      __syncthreads();
      const float* ap = &sm.Vs[(wr + li) * SS + 16 * lh];
      const float* bp = &sm.Qs[(wc + li) * SS + 16 * lh];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 av = *(const float4*)(ap + 4 * j);
        const float4 bv = *(const float4*)(bp + 4 * j);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, bv.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, bv.w, acc, 0, 0, 0);
      }
      __syncthreads();
    }
    // accumulator element r of lane (li, lh) is row 8*(r/4) + 4*lh + r%4,
    // column li of the wave's sub-tile
    const int c = c0 + wc + li;
    if (c < h) {
      const float qc = sm.qn[c];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = wr + 8 * (r >> 2) + 4 * lh + (r & 3);
        keys[i * KS + c] = qc - 2.f * acc[r];
      }
    }
  }
  __syncthreads();

  // ---------------- step 2: ordered extraction, exact distances ----------
  const int row = tid >> 2, sub = tid & 3;
  bool done = row >= nrows;
  const float bound = done ? 0.f : sm.rbound[row];
  int kef;
  if constexpr (MODE == P1_TABLE_FULL) {
    kef = min(a.k, h);
  } else {
    if (a.method == LCEMD_ICT) kef = h;
    else if (a.method == LCEMD_OMR) kef = min(2, h);
    else if (a.method == LCEMD_RWMD) kef = 1;
    else kef = min(a.k, h);
  }
  const float* vrow = a.V + (size_t)(done ? 0 : sm.rid[row]) * m_pad;
  const float* krow = &keys[row * KS];
  int depth = 0;
  float P = 0.f, rem = bound, cost = 0.f;
  uint64_t last = 0;
  while (__any(!done)) {
    uint64_t best = ~0ull;
    if (!done) {
      for (int c = sub; c < h; c += 4) {
        const uint64_t kk = pack_key(krow[c], (uint32_t)c);
        if (kk > last && kk < best) best = kk;
      }
    }
    uint64_t o = shfl_xor_u64(best, 1);
    best = o < best ? o : best;
    o = shfl_xor_u64(best, 2);
    best = o < best ? o : best;
    if (best == ~0ull) done = true;  // row exhausted (cannot happen when kef <= h)
    const int pos = (int)(uint32_t)best;
    float d2 = 0.f;
    if (!done) {
      const float* crow = a.V + (size_t)sm.cid[pos] * m_pad;
      for (int d = sub * 4; d < 4 * a.m4; d += 16) {  // past 4*m4 only zero padding
        const float4 x = *(const float4*)(vrow + d);
        const float4 y = *(const float4*)(crow + d);
        const float e0 = x.x - y.x, e1 = x.y - y.y, e2 = x.z - y.z, e3 = x.w - y.w;
        d2 = fmaf(e0, e0, d2);
        d2 = fmaf(e1, e1, d2);
        d2 = fmaf(e2, e2, d2);
        d2 = fmaf(e3, e3, d2);
      }
    }
    d2 += __shfl_xor(d2, 1);
    d2 += __shfl_xor(d2, 2);
    if (!done) {
      const float w = sm.cap[pos];
      const float Pn = P + w;
      ++depth;
      const float z = sqrtf(d2);
      bool stop = depth >= kef;
      if constexpr (MODE != P1_TABLE_FULL) {
        stop = stop || Pn >= bound || (a.method == LCEMD_OMR && depth == 1 && d2 != 0.f);
      }
      if constexpr (MODE == P1_TABLE) {
        const bool ovf = !stop && depth >= a.KT;
        if (sub == 0) {
          const int64_t flat = out_row0 + row;
          float2* pr = (float2*)zw_pair(a.ZW, a.zw_nq, a.KT, flat / a.v_used, flat % a.v_used, (depth - 1) >> 1);
          pr[(depth - 1) & 1] = make_float2(z, (stop || ovf) ? INFINITY : w);
          // a row's last pair is written whole (phase 2 steps the second
          // entry of the first pair without testing the remaining mass)
          if ((stop || ovf) && ((depth - 1) & 1) == 0) pr[1] = make_float2(0.f, 0.f);
          if (ovf) a.overflow[0] = 1;
        }
        stop = stop || ovf;
      } else if constexpr (MODE == P1_TABLE_FULL) {
        if (sub == 0) {
          const int64_t o2 = (out_row0 + row) * a.k + depth - 1;
          a.S[o2] = pos;
          a.Z[o2] = z;
          a.W[o2] = w;
        }
      } else {
        const float r = stop ? rem : fminf(rem, w);
        rem -= r;
        cost = fmaf(r, z, cost);
      }
      P = Pn;
      last = best;
      if (stop) done = true;
    }
  }

  if constexpr (MODE == P1_TABLE_FULL) {
    if (sub == 0 && row < nrows) {
      for (int l = depth; l < a.k; ++l) {
        const int64_t o2 = (out_row0 + row) * a.k + l;
        a.S[o2] = -1;
        a.Z[o2] = 0.f;
        a.W[o2] = 0.f;
      }
    }
  }
  if constexpr (MODE == P1_PAIR) {
    if (sub == 0) sm.rcost[row] = cost;
    __syncthreads();
    if (tid == 0) {
      float tot = 0.f;
      for (int r = 0; r < nrows; ++r) tot += sm.rcost[r];
      a.partial[pidx * a.rb_max + rb] = tot;
    }
  }
}

template <int MODE, int HMAX>
static hipError_t launch_one(const P1Args& a, hipStream_t s) {
  const size_t shmem = sizeof(P1Smem<MODE, HMAX>);
  hipError_t e = hipFuncSetAttribute((const void*)k_phase1_f32<MODE, HMAX>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  if constexpr (P1Smem<MODE, HMAX>::GKEYS) {
    // launches of at most kDeepSlots workgroups, one key region each; the
    // launches of a stream run one after another, so regions are reused
    if (!a.deep_keys) return hipErrorInvalidValue;
    const int64_t total = MODE == P1_PAIR ? a.npairs * (int64_t)a.rb_max
                                          : (a.v_used + kRows - 1) / kRows * a.nq;
    for (int64_t b0 = 0; b0 < total; b0 += kDeepSlots) {
      P1Args c = a;
      c.blk0 = b0;
      const unsigned g = (unsigned)std::min<int64_t>(kDeepSlots, total - b0);
      hipLaunchKernelGGL((k_phase1_f32<MODE, HMAX>), dim3(g), dim3(kThreads), shmem, s, c);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  dim3 grid;
  if (MODE == P1_PAIR) {
    grid = dim3((unsigned)a.npairs, (unsigned)a.rb_max, 1);
  } else {
    grid = dim3((unsigned)((a.v_used + kRows - 1) / kRows), (unsigned)a.nq, 1);
  }
  hipLaunchKernelGGL((k_phase1_f32<MODE, HMAX>), grid, dim3(kThreads), shmem, s, a);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(const P1Args& a, int hmax, hipStream_t s) {
  if (hmax <= 128) return launch_one<MODE, 128>(a, s);
  if (hmax <= 256) return launch_one<MODE, 256>(a, s);
  if (hmax <= 512) return launch_one<MODE, 512>(a, s);
  if (hmax <= LCEMD_MAX_HIST) return launch_one<MODE, LCEMD_MAX_HIST>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_phase1_deep(const P1Args& a, int mode, int hmax, int prec, hipStream_t s) {
  if (prec != PREC_F32) return hipErrorInvalidValue;
  switch (mode) {
    case P1_TABLE: return launch_mode<P1_TABLE>(a, hmax, s);
    case P1_TABLE_FULL: return launch_mode<P1_TABLE_FULL>(a, hmax, s);
    case P1_PAIR: return launch_mode<P1_PAIR>(a, hmax, s);
  }
  return hipErrorInvalidValue;
}

// Sum of the per-row-block partial Q2D costs of each pair, in row-block
// order (deterministic).  out[(p / per_row) * out_ld + p % per_row].
__global__ __launch_bounds__(kThreads) void k_pair_reduce(const float* partial, int64_t npairs,
                                                          int rb_max, float* out, int64_t out_ld,
                                                          int64_t per_row) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= npairs) return;
  float t = 0.f;
  for (int r = 0; r < rb_max; ++r) t += partial[p * rb_max + r];
  out[(p / per_row) * out_ld + (p % per_row)] = t;
}

hipError_t launch_pair_reduce(const float* partial, int64_t npairs, int rb_max, float* out,
                              int64_t out_ld, int64_t per_row, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const unsigned g = (unsigned)((npairs + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_pair_reduce, dim3(g), dim3(kThreads), 0, s, partial, npairs, rb_max, out,
                     out_ld, per_row);
  return hipGetLastError();
}

}  // namespace lcemd
