// Phase 1 of LC-ACT (Sec. 4, Phase 1), wide variant: 128 rows per
// workgroup and up to 128 columns per MFMA pass.
//
// Contraction: wave w owns rows [32w, 32w+32).  Its row operand (32 rows x
// one 128-byte slice of dims) is read straight from global memory into
// registers -- no other wave needs it -- while the column slice (128
// columns) is staged once in LDS for all four waves.  Each wave keeps four
// 32x32 accumulators (one per 32-column tile) and issues them interleaved.
// The next slice is prefetched into registers during the MFMAs, so a slice
// costs one LDS store and two barriers.
//
// Selection: after a pass the keys |c|^2 - 2 <v, c> go to LDS 64 columns at
// a time and two lanes per row merge them into the row's sorted candidate
// list (packed (key, position); position breaks ties; for lists of 8 or more
// entries each lane first sorts its 32 keys in registers and the merge takes
// from their heads, else it scans them for the next), cut at k_eff = min(k,
// h) (Alg. 3; 1 for RWMD, 2 for OMR) or as soon as the listed capacities
// reach the row's bound (Lemma 1/2: no transfer of at most that much mass
// passes this point).
//
// Exact distances: float32 keys -- the list distance is |v|^2 + key unless
// cancellation could bite (below a quarter of |v|^2 + |c|^2), where it is
// recomputed by direct differences.  bfloat16 keys -- every bf16-rounded
// product is within 2^-8 of the exact one, so a key is off by at most
// 2^-7 * 1.0625 * |v||c| (float32 accumulation included for m <= 4096);
// the list therefore keeps, past the cut, every candidate whose key is
// within 2^-6 * 1.07 * |v| * max|c| of the cut key: in exact order nothing
// outside that band can precede the cut.  All listed candidates then get
// float32 distances -- |v|^2 + |c|^2 - 2<v, c> with the dot product
// accumulated in float32 over the original vectors (staged through LDS a
// chunk of dims at a time), or by direct differences where cancellation
// could bite, as for float32 keys -- and are re-sorted and cut again.
#include <algorithm>

#include "internal.h"

namespace lcemd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kWR = 128;        // rows per workgroup
constexpr int kWC = 128;        // columns per MFMA pass
constexpr int kStride = 144;    // bytes per staged column slice (128 + 16 pad)
constexpr int kCK = 66;         // floats per key row (64 columns + 2 pad)
constexpr int kQSCap = kWR * kCK;  // floats of the staging area (the key buffer's size)
constexpr int kSeg = kSegShort;            // segment words held in LDS (short variant)
constexpr int kSegLong = LCEMD_MAX_HIST;   // long variant (float32 keys)
// queries per tile group (table modes): 8, or 32 with float32 keys over
// vocabularies of at least 2^18 used words, where a row block's vectors are
// reused by more items before they leave L2 (1M words: phase 1 -2 %; with
// fp8 keys 32 was 3 % slower; 70,000 words: 8 keeps a group's query vectors
// within an XCD's L2)
__host__ __device__ inline int wide_group_log2(int64_t v_used, int prec) {
  return prec == PREC_F32 && v_used >= (int64_t(1) << 18) ? 5 : 3;
}
constexpr float kGuardW = 0.25f;
constexpr float kBandBF16 = 0.015625f * 1.07f;  // 2^-6 * 1.07
// fp8 (e4m3, 3 mantissa bits): a statistical band, not a worst-case one --
// about six standard deviations of the key error of a few-hundred-term dot
// product with independent relative rounding errors of at most 2^-4
constexpr float kBandFP8 = 0.04f;
template <int PREC>
__device__ __forceinline__ float band_coef() {
  return PREC == PREC_F32 ? 0.f : (PREC == PREC_BF16 ? kBandBF16 : kBandFP8);
}

__device__ __forceinline__ uint32_t w_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint64_t w_pack(float f, uint32_t pos) {
  return ((uint64_t)w_bits(f) << 32) | (uint64_t)pos;
}
__device__ __forceinline__ float w_unpack(uint64_t k) {
  const uint32_t o = (uint32_t)(k >> 32);
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}
__device__ __forceinline__ uint64_t w_shfl1(uint64_t v) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  lo = __shfl_xor(lo, 1);
  hi = __shfl_xor(hi, 1);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// Selection keys.  Exact keys: (order-preserving key bits, position) in 64
// bits (float32 pair mode).  Quantised keys (the table modes): the key's PB
// low bits give way to the position (9 bits for segments of up to 512
// words, 10 up to 1024), one 32-bit word, rounded down in value by at most
// 2^(PB-23) of the key's magnitude; lists keep every entry within twice
// that band past their cut and are re-sorted afterwards by the exact keys
// (float32: the contraction's key, kept beside the list; bf16/fp8: the
// recomputed distances).
template <bool QK, int PB = 9>
struct KeyOps {
  using T = uint32_t;
  static constexpr T kNone = 0xffffffffu;
  static constexpr uint32_t kPos = (1u << PB) - 1u;
  // twice the largest relative rounding of a key, 2 * 2^(PB-23)
  static constexpr float kRound = (float)(1u << PB) / (float)(1u << 22);
  __device__ static T pack(float f, uint32_t pos) { return (w_bits(f) & ~kPos) | pos; }
  __device__ static float key(T k) {
    const uint32_t o = k & ~kPos;
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
  }
  __device__ static uint32_t pos(T k) { return k & kPos; }
  __device__ static T shfl1(T v) { return (T)__shfl_xor((int)v, 1); }
};
template <int PB>
struct KeyOps<false, PB> {
  using T = uint64_t;
  static constexpr T kNone = ~0ull;
  static constexpr float kRound = 0.f;  // exact keys
  __device__ static T pack(float f, uint32_t pos) { return w_pack(f, pos); }
  __device__ static float key(T k) { return w_unpack(k); }
  __device__ static uint32_t pos(T k) { return (uint32_t)k; }
  __device__ static T shfl1(T v) { return w_shfl1(v); }
};

// Squared distance by direct differences over the m4 float4 groups that
// hold the real dims (the zero padding would add exact zeros).
__device__ __forceinline__ float w_exact_d2(const float* __restrict__ V, int m_pad, int m4, int a, int b) {
  const float4* x = (const float4*)(V + (size_t)a * m_pad);
  const float4* y = (const float4*)(V + (size_t)b * m_pad);
  float s = 0.f;
  const int n4 = m4;
  for (int d = 0; d < n4; ++d) {
    const float4 p = x[d], q = y[d];
    const float e0 = p.x - q.x, e1 = p.y - q.y, e2 = p.z - q.z, e3 = p.w - q.w;
    s = fmaf(e0, e0, s);
    s = fmaf(e1, e1, s);
    s = fmaf(e2, e2, s);
    s = fmaf(e3, e3, s);
  }
  return s;
}

// One staged slice on NT 32-column tiles (NT fixed at compile time so the
// MFMAs issue back to back without branches).
template <int NT>
__device__ __forceinline__ void slice_f32(floatx16 (&acc)[4], const uint4 (&a_cur)[4],
                                          const unsigned char* st, int li, int lh) {
  // lane half lh supplies dims [16 lh, 16 lh + 16) of the 32-dim slice
  const float* af = (const float*)a_cur;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float4 bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
      bv[t] = *(const float4*)(st + (32 * t + li) * kStride + lh * 64 + j * 16);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[4 * j + 0], bv[t].x, acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[4 * j + 1], bv[t].y, acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[4 * j + 2], bv[t].z, acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[4 * j + 3], bv[t].w, acc[t], 0, 0, 0);
  }
}

template <int NT>
__device__ __forceinline__ void slice_bf16(floatx16 (&acc)[4], const uint4 (&a_cur)[4],
                                           const unsigned char* st, int li, int lh) {
  // lane half lh supplies dims [32 lh + 8 s, +8) of the 64-dim slice
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(&a_cur[s]);
    bf16x8 bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bv[t] = *(const bf16x8*)(st + (32 * t + li) * kStride + lh * 64 + s * 16);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[t], acc[t], 0, 0, 0);
  }
}

template <int NT>
__device__ __forceinline__ void slice_fp8(floatx16 (&acc)[4], const uint4 (&a_cur)[4],
                                          const unsigned char* st, int li, int lh) {
  // lane half lh supplies dims [64 lh + 8 s, +8) of the 128-dim slice
  const long* ap = reinterpret_cast<const long*>(a_cur);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    long bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bv[t] = *(const long*)(st + (32 * t + li) * kStride + lh * 64 + s * 8);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(ap[s], bv[t], acc[t], 0, 0, 0);
  }
}

template <int PREC>
__device__ __forceinline__ void slice_mfma(int ntile, floatx16 (&acc)[4], const uint4 (&a_cur)[4],
                                           const unsigned char* st, int li, int lh) {
  if constexpr (PREC == PREC_F32) {
    switch (ntile) {
      case 1: slice_f32<1>(acc, a_cur, st, li, lh); break;
      case 2: slice_f32<2>(acc, a_cur, st, li, lh); break;
      case 3: slice_f32<3>(acc, a_cur, st, li, lh); break;
      default: slice_f32<4>(acc, a_cur, st, li, lh); break;
    }
  } else if constexpr (PREC == PREC_BF16) {
    switch (ntile) {
      case 1: slice_bf16<1>(acc, a_cur, st, li, lh); break;
      case 2: slice_bf16<2>(acc, a_cur, st, li, lh); break;
      case 3: slice_bf16<3>(acc, a_cur, st, li, lh); break;
      default: slice_bf16<4>(acc, a_cur, st, li, lh); break;
    }
  } else {
    switch (ntile) {
      case 1: slice_fp8<1>(acc, a_cur, st, li, lh); break;
      case 2: slice_fp8<2>(acc, a_cur, st, li, lh); break;
      case 3: slice_fp8<3>(acc, a_cur, st, li, lh); break;
      default: slice_fp8<4>(acc, a_cur, st, li, lh); break;
    }
  }
}

template <int KL, int PREC, bool QK, bool EX, int SEG = kSeg>
struct WideSmem {
  static constexpr int KLS = KL + 1 + (EX ? 1 : 0);  // list row stride (odd or +1: spreads rows over banks)
  union {
    unsigned char st[kWC * kStride];  // staged column slice
    float ck[kWR * kCK];              // keys of 64 columns of a pass
    float qs[PREC == PREC_F32 ? 1 : kQSCap];  // segment vectors, a chunk of dims (exact recompute)
    float zb[kWR * KLS];              // exact squared distances of the lists
  } u;
  typename KeyOps<QK>::T lst[2][kWR * KLS];
  float lkx[EX ? 2 : 1][EX ? kWR * KLS : 1];  // float32 quantised keys: the exact keys beside the list
  int cid[SEG];
  float cap[SEG];
  float qn[SEG];
  int rid[kWR];
  float rbound[kWR];
  float rvn[kWR];
  int rlen[kWR];
  float rcost[kWR];
  float rdrop[kWR];  // smallest key dropped because the list was full
  int rcut[kWR];     // the last merge reached k_eff or the row's bound
  float qmax;
  float rsc[PREC == PREC_FP8 ? kWR : 1];   // fp8 row scales
  float csc[PREC == PREC_FP8 ? SEG : 1];  // fp8 column scales
};

// Float32 dot products <v_row, c_pos> of a thread's listed candidates
// (ex[e] for list entry sub + 2e), D dims at a time: the row's D dims are
// loaded into registers before the barrier, the segment's vectors are
// staged in LDS (row stride D + 4 floats).  Dims are accumulated in order.
template <int D, int KH>
__device__ __forceinline__ void wide_dots(float (&ex)[KH], const int (&ps)[KH], int len, int sub,
                                          bool row_ok, const float* __restrict__ vr,
                                          const P1Args& a, float* qs, const int* cid, int h,
                                          int tid) {
  constexpr int D4 = D / 4, QS = D + 4;
  for (int d0 = 0; d0 < a.m_pad; d0 += D) {
    float4 v[D4];
#pragma unroll
    for (int q = 0; q < D4; ++q) v[q] = row_ok ? *(const float4*)(vr + d0 + 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    for (int f = tid; f < h * D4; f += kThreads) {
      const int c = f / D4, q = f % D4;
      *(float4*)(&qs[c * QS + q * 4]) = *(const float4*)(a.V + (size_t)cid[c] * a.m_pad + d0 + q * 4);
    }
    __syncthreads();
    if (row_ok) {
#pragma unroll
      for (int e = 0; e < KH; ++e) {
        if (sub + 2 * e < len) {
          const float* cp = &qs[ps[e] * QS];
          float s = ex[e];
#pragma unroll
          for (int q = 0; q < D4; ++q) {
            const float4 c = *(const float4*)(cp + 4 * q);
            s = fmaf(v[q].x, c.x, s);
            s = fmaf(v[q].y, c.y, s);
            s = fmaf(v[q].z, c.z, s);
            s = fmaf(v[q].w, c.w, s);
          }
          ex[e] = s;
        }
      }
    }
  }
}

}  // namespace

// One work item: (query, 128-row block) in the table modes, (pair, row
// block) in pair mode.  Returns early (uniformly) for empty items.
template <int MODE, int KL, int PREC, bool LONG>
__device__ __forceinline__ void wide_task(const P1Args& a, unsigned char* smem_raw, int64_t item) {
  // quantised keys everywhere but in the float32 pair mode; EX: float32
  // with quantised keys keeps the exact keys and one more list slot.
  // LONG: segments of up to kSegLong words (float32 only, 10 position bits)
  static_assert(!LONG || PREC == PREC_F32, "long segments run with float32 keys");
  constexpr bool QK = PREC != PREC_F32 || MODE != P1_PAIR;
  constexpr bool EX = PREC == PREC_F32 && QK;
  constexpr int KLC = KL + (EX ? 1 : 0);  // list capacity
  constexpr int PB = LONG ? 10 : 9;
  using Sm = WideSmem<KL, PREC, QK, EX, LONG ? kSegLong : kSeg>;
  constexpr int KLS = Sm::KLS;
  Sm& sm = *reinterpret_cast<Sm*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // ---------------- task decode ----------------
  int nrows = 0, h = 0;
  int64_t out_row0 = 0, pidx = 0;
  int rb = 0;
  if constexpr (MODE == P1_PAIR) {
    pidx = item / a.rb_max;
    rb = (int)(item % a.rb_max);
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
    const int64_t qs0 = a.qptr[b];
    const int hq = (int)(a.qptr[b + 1] - qs0);
    nrows = min(kWR, hq - rb * kWR);
    if (nrows <= 0 || u < 0 || u >= a.n) {
      if (tid == 0) a.partial[pidx * a.rb_max + rb] = 0.f;
      return;
    }
    if (tid < kWR) {
      const bool ok = tid < nrows;
      const int w = ok ? a.qcol[qs0 + rb * kWR + tid] : 0;
      sm.rid[tid] = w;
      sm.rbound[tid] = ok ? a.qval[qs0 + rb * kWR + tid] : 0.f;
      sm.rvn[tid] = a.vnorm[w];
      if constexpr (PREC == PREC_FP8) sm.rsc[tid] = a.vscale[w];
      sm.rlen[tid] = 0;
      sm.rdrop[tid] = INFINITY;
    }
    const int64_t s0 = a.xptr[u];
    h = (int)(a.xptr[u + 1] - s0);
    for (int c = tid; c < h; c += kThreads) {
      const int w = a.xcol[s0 + c];
      sm.cid[c] = w;
      sm.cap[c] = __int_as_float(a.xcv[s0 + c].y);
      sm.qn[c] = a.vnorm[w];
      if constexpr (PREC == PREC_FP8) sm.csc[c] = a.vscale[w];
    }
  } else {
    // items run query-fastest within a group of queries, then row
    // block, then group: an XCD's contiguous range of items keeps a group's
    // query vectors and a row block's vectors in its L2
    const int64_t nrb = (a.v_used + kWR - 1) / kWR;
    const int64_t work = item;
    const int lg = wide_group_log2(a.v_used, PREC);
    const int64_t qin = work & ((int64_t(1) << lg) - 1), t = work >> lg;
    const int64_t rblk = t % nrb, g = t / nrb;
    const int64_t qi = (g << lg) + qin;
    if (qi >= a.nq) return;
    const int64_t r0 = rblk * kWR;
    const int64_t b = a.q0 + qi;
    nrows = (int)min((int64_t)kWR, a.v_used - r0);
    out_row0 = qi * a.v_used + r0;
    if (tid < kWR) {
      const bool ok = tid < nrows;
      const int w = ok ? a.used[r0 + tid] : 0;
      sm.rid[tid] = w;
      sm.rbound[tid] = ok ? (MODE == P1_TABLE ? a.xmax[r0 + tid] : INFINITY) : 0.f;
      sm.rvn[tid] = a.vnorm[w];
      if constexpr (PREC == PREC_FP8) sm.rsc[tid] = a.vscale[w];
      sm.rlen[tid] = 0;
      sm.rdrop[tid] = INFINITY;
    }
    const int64_t s0 = a.qptr[b];
    h = (int)(a.qptr[b + 1] - s0);
    if (h <= 0) return;  // padding slot of a fixed-size batch
    for (int c = tid; c < h; c += kThreads) {
      const int w = a.qcol[s0 + c];
      sm.cid[c] = w;
      sm.cap[c] = a.qval[s0 + c];
      sm.qn[c] = a.vnorm[w];
      if constexpr (PREC == PREC_FP8) sm.csc[c] = a.vscale[w];
    }
  }
  if (tid == 0) sm.qmax = 0.f;
  __syncthreads();
  if (QK && tid < 64) {
    float mx = 0.f;
    for (int c = tid; c < h; c += 64) mx = fmaxf(mx, sm.qn[c]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (tid == 0) sm.qmax = sqrtf(mx);
  }

  int kef;
  if constexpr (MODE == P1_TABLE_FULL) {
    kef = min(a.k, h);
  } else {
    if (a.method == LCEMD_ICT) kef = h;
    else if (a.method == LCEMD_OMR) kef = min(2, h);
    else if (a.method == LCEMD_RWMD) kef = 1;
    else kef = min(a.k, h);
  }
  constexpr bool kCapStop = MODE != P1_TABLE_FULL;

  // ---------------- contraction ----------------
  const unsigned char* base = PREC == PREC_F32    ? (const unsigned char*)a.V
                              : PREC == PREC_BF16 ? (const unsigned char*)a.Vb
                                                  : (const unsigned char*)a.V8;
  const size_t rowbytes = PREC == PREC_FP8 ? (size_t)a.m8 : (size_t)a.m_pad * (PREC == PREC_F32 ? 4 : 2);
  // 128-byte slices that hold real dims (the zero padding past them would
  // add exact zeros): 4 * m4 dims of 4, 2 or 1 bytes
  const int realbytes = 4 * a.m4 * (PREC == PREC_F32 ? 4 : PREC == PREC_BF16 ? 2 : 1);
  const int nsl = min((int)(rowbytes / 128), (realbytes + 127) / 128);
  const int li = lane & 31, lh = lane >> 5;
  const int arow = 32 * wave + li;
  const bool arow_ok = arow < nrows;
  const unsigned char* aptr = base + (size_t)sm.rid[arow] * rowbytes + lh * 64;

  uint4 a_cur[4], a_nxt[4], b_nxt[4];
  auto load_a = [&](int sl) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a_nxt[i] = arow_ok ? *(const uint4*)(aptr + sl * 128 + i * 16) : make_uint4(0, 0, 0, 0);
  };
  // column operand: the 4 (column, 16-byte piece) addresses this thread
  // stages are fixed for a pass; only the slice offset moves
  const unsigned char* bptr[4];
  auto set_b = [&](int c0) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int f = tid + it * kThreads;
      const int cc = c0 + (f >> 3);
      bptr[it] = cc < h ? base + (size_t)sm.cid[cc] * rowbytes + (f & 7) * 16 : nullptr;
    }
  };
  auto load_b = [&](int sl) {
#pragma unroll
    for (int it = 0; it < 4; ++it)
      b_nxt[it] = bptr[it] ? *(const uint4*)(bptr[it] + sl * 128) : make_uint4(0, 0, 0, 0);
  };

  const int row = tid >> 1, sub = tid & 1;
  const bool row_ok = row < nrows;
  const float bound = row_ok ? sm.rbound[row] : 0.f;
  int par = 0;

  load_a(0);
  set_b(0);
  load_b(0);
  for (int c0 = 0; c0 < h; c0 += kWC) {
    const int ntile = min(4, (h - c0 + 31) >> 5);
    floatx16 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
    for (int sl = 0; sl < nsl; ++sl) {
      __syncthreads();
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int f = tid + it * kThreads;
        *(uint4*)(sm.u.st + (f >> 3) * kStride + (f & 7) * 16) = b_nxt[it];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) a_cur[i] = a_nxt[i];
      __syncthreads();
      if (sl + 1 < nsl) {
        load_a(sl + 1);
        load_b(sl + 1);
      } else if (c0 + kWC < h) {
        load_a(0);
        set_b(c0 + kWC);
        load_b(0);
      }
      slice_mfma<PREC>(ntile, acc, a_cur, sm.u.st, li, lh);
    }

    // ---- selection: 64 columns at a time ----
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int cb = c0 + 64 * half;
      if (cb >= h) break;
      __syncthreads();
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        const int t = 2 * half + tt;
        const int c = cb + 32 * tt + li;
        const float qc = c < h ? sm.qn[c] : 0.f;
        const float csc = PREC == PREC_FP8 && c < h ? sm.csc[PREC == PREC_FP8 ? c : 0] : 1.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
          if constexpr (PREC == PREC_FP8)
            sm.u.ck[i * kCK + 32 * tt + li] = qc - 2.f * (sm.rsc[i] * csc) * acc[t][r];
          else
            sm.u.ck[i * kCK + 32 * tt + li] = qc - 2.f * acc[t][r];
        }
      }
      __syncthreads();
      // this thread's 32 contiguous columns, read without branches (the
      // buffer is fully allocated; columns past h are masked afterwards)
      using KO = KeyOps<QK, PB>;
      using KT_ = typename KO::T;
      KT_ kk[32];
      const float2* krow = (const float2*)&sm.u.ck[row * kCK + 32 * sub];
#pragma unroll
      for (int j2 = 0; j2 < 16; ++j2) {
        const float2 kv = krow[j2];
        const int c = cb + 32 * sub + 2 * j2;
        const KT_ m0 = (row_ok && c < h) ? (KT_)0 : KO::kNone;
        const KT_ m1 = (row_ok && c + 1 < h) ? (KT_)0 : KO::kNone;
        kk[2 * j2] = KO::pack(kv.x, (uint32_t)c) | m0;
        kk[2 * j2 + 1] = KO::pack(kv.y, (uint32_t)(c + 1)) | m1;
      }
      // lists of 8 or more entries: the thread's 32 keys are sorted once
      // (bitonic network in registers) and the merge takes from their head;
      // shorter lists scan the keys for the next one instead
      constexpr bool kSorted = QK && KL >= 8;
      if constexpr (kSorted) {
#pragma unroll
        for (int kb = 2; kb <= 32; kb <<= 1) {
#pragma unroll
          for (int jb = kb >> 1; jb > 0; jb >>= 1) {
#pragma unroll
            for (int i = 0; i < 32; ++i) {
              const int l2 = i ^ jb;
              if (l2 > i) {
                const KT_ x = kk[i], y = kk[l2];
                const KT_ lo = x < y ? x : y, hi = x < y ? y : x;
                const bool up = (i & kb) == 0;
                kk[i] = up ? lo : hi;
                kk[l2] = up ? hi : lo;
              }
            }
          }
        }
      }
      const KT_* cur = &sm.lst[par][row * KLS];
      KT_* nxt = &sm.lst[par ^ 1][row * KLS];
      const float* curx = &sm.lkx[EX ? par : 0][EX ? row * KLS : 0];
      float* nxtx = &sm.lkx[EX ? (par ^ 1) : 0][EX ? row * KLS : 0];
      const int len = row_ok ? sm.rlen[row] : 0;
      // approximate keys: the error band plus the rounding of 32-bit keys
      const float band = !QK ? 0.f
                             : band_coef<PREC>() * sqrtf(sm.rvn[row]) * sm.qmax +
                                   KO::kRound * (sm.qmax * sm.qmax + 2.f * sqrtf(sm.rvn[row]) * sm.qmax);
      int ptr = 0, w = 0;
      float P = 0.f, K0 = 0.f;
      bool cut = false;
      KT_ last = 0;
      bool act = row_ok;
      while (__any(act)) {
        KT_ best = KO::kNone;
        if (act) {
          if constexpr (kSorted) {
            best = kk[0];
          } else {
#pragma unroll
            for (int j = 0; j < 32; ++j) {
              const KT_ cand = kk[j] > last ? kk[j] : KO::kNone;
              best = cand < best ? cand : best;
            }
          }
        }
        const KT_ mine = best;
        const KT_ o = KO::shfl1(best);
        best = o < best ? o : best;
        if (act) {
          const KT_ lc = ptr < len ? cur[ptr] : KO::kNone;
          const KT_ take = lc < best ? lc : best;
          if (take == KO::kNone) {
            act = false;
          } else if (cut && (!QK || KO::key(take) > K0 + band)) {
            act = false;
          } else if (w >= KLC) {
            // the list is full: remember the smallest key left out; the
            // final lists are certified against it after the exact re-sort
            act = false;
            if (sub == 0) sm.rdrop[row] = fminf(sm.rdrop[row], KO::key(take));
          } else {
            if constexpr (EX) {
              if (sub == 0) nxtx[w] = lc < best ? curx[ptr] : sm.u.ck[row * kCK + (int)(KO::pos(take)) - cb];
            }
            if (lc < best) {
              ++ptr;
            } else {
              last = best;
              if constexpr (kSorted) {
                if (mine == best) {  // this thread's head was taken
#pragma unroll
                  for (int j = 0; j < 31; ++j) kk[j] = kk[j + 1];
                  kk[31] = KO::kNone;
                }
              }
            }
            if (sub == 0) nxt[w] = take;
            ++w;
            if (!cut) {
              P += sm.cap[KO::pos(take)];
              if (w >= kef || (kCapStop && P >= bound)) {
                cut = true;
                K0 = KO::key(take);
              }
            }
          }
        }
      }
      __syncthreads();
      if (sub == 0 && row_ok) {
        sm.rlen[row] = w;
        sm.rcut[row] = cut ? 1 : 0;
      }
      par ^= 1;
    }
  }
  __syncthreads();

  // ---------------- exact distances of the final lists ----------------
  const int len = row_ok ? sm.rlen[row] : 0;
  const auto* L = &sm.lst[par][row * KLS];
  if constexpr (PREC == PREC_F32) {
    for (int l = sub; l < len; l += 2) {
      const auto e = L[l];
      const int pos = (int)KeyOps<QK, PB>::pos(e);
      float d2 = sm.rvn[row] + (EX ? sm.lkx[EX ? par : 0][EX ? row * KLS + l : 0] : KeyOps<QK, PB>::key(e));
      bool need = !(d2 >= kGuardW * (sm.rvn[row] + sm.qn[pos]));
      if (MODE != P1_TABLE_FULL && a.method == LCEMD_OMR && l == 0) need = true;
      if (need) d2 = w_exact_d2(a.V, a.m_pad, a.m4, sm.rid[row], sm.cid[pos]);
      sm.u.zb[row * KLS + l] = d2;
    }
  } else {
    constexpr int KH = (KL + 1) / 2;
    float ex[KH];
    int ps[KH];
#pragma unroll
    for (int e = 0; e < KH; ++e) {
      ex[e] = 0.f;
      const int l = sub + 2 * e;
      ps[e] = l < len ? (int)KeyOps<QK, PB>::pos(L[l]) : 0;
    }
    const float* vr = a.V + (size_t)sm.rid[row] * a.m_pad;
    // chunks of D dims of all h segment vectors per LDS pass, as wide as
    // the staging area allows (fewer passes and barriers)
    if (h * 68 <= kQSCap && a.m_pad % 64 == 0)
      wide_dots<64, KH>(ex, ps, len, sub, row_ok, vr, a, sm.u.qs, sm.cid, h, tid);
    else if (h * 36 <= kQSCap && a.m_pad % 32 == 0)
      wide_dots<32, KH>(ex, ps, len, sub, row_ok, vr, a, sm.u.qs, sm.cid, h, tid);
    else if (h * 20 <= kQSCap && a.m_pad % 16 == 0)
      wide_dots<16, KH>(ex, ps, len, sub, row_ok, vr, a, sm.u.qs, sm.cid, h, tid);
    else
      wide_dots<8, KH>(ex, ps, len, sub, row_ok, vr, a, sm.u.qs, sm.cid, h, tid);
    // squared distances from the float32 dot products; where cancellation
    // could bite, by direct differences (as for float32 keys)
#pragma unroll
    for (int e = 0; e < KH; ++e) {
      if (row_ok && sub + 2 * e < len) {
        const float qn = sm.qn[ps[e]];
        float d2 = (sm.rvn[row] + qn) - 2.f * ex[e];
        if (!(d2 >= kGuardW * (sm.rvn[row] + qn))) d2 = w_exact_d2(a.V, a.m_pad, a.m4, sm.rid[row], sm.cid[ps[e]]);
        ex[e] = d2;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < KH; ++e) {
      const int l = sub + 2 * e;
      if (l < len) sm.u.zb[row * KLS + l] = ex[e];
    }
  }
  __syncthreads();

  if (sub == 0 && row_ok) {
    auto* Lw = &sm.lst[par][row * KLS];
    float* Z2 = &sm.u.zb[row * KLS];
    float* Lx = &sm.lkx[EX ? par : 0][EX ? row * KLS : 0];
    if constexpr (EX) {
      // exact re-sort by (contraction key, position), distances moving
      // along; the list then holds positions
      for (int i = 0; i < len; ++i) Lw[i] = KeyOps<QK, PB>::pos(Lw[i]);
      for (int i = 1; i < len; ++i) {
        const uint64_t e = w_pack(Lx[i], (uint32_t)Lw[i]);
        const float z = Z2[i];
        int j = i - 1;
        while (j >= 0 && w_pack(Lx[j], (uint32_t)Lw[j]) > e) {
          Lw[j + 1] = Lw[j];
          Lx[j + 1] = Lx[j];
          Z2[j + 1] = Z2[j];
          --j;
        }
        Lw[j + 1] = (uint32_t)e;
        Lx[j + 1] = w_unpack(e);
        Z2[j + 1] = z;
      }
    } else if constexpr (PREC != PREC_F32) {
      // exact re-sort by (squared distance, position); the list then holds
      // positions
      for (int i = 0; i < len; ++i) Lw[i] = KeyOps<QK, PB>::pos(Lw[i]);
      for (int i = 1; i < len; ++i) {
        const uint64_t e = w_pack(Z2[i], (uint32_t)Lw[i]);
        int j = i - 1;
        while (j >= 0 && w_pack(Z2[j], (uint32_t)Lw[j]) > e) {
          Lw[j + 1] = Lw[j];
          Z2[j + 1] = Z2[j];
          --j;
        }
        Lw[j + 1] = (uint32_t)e;
        Z2[j + 1] = w_unpack(e);
      }
    }
    int D = 0;
    bool covered = false;
    {
      float Pc = 0.f;
      for (int l = 0; l < len; ++l) {
        ++D;
        Pc += sm.cap[(uint32_t)Lw[l]];
        if (D >= kef) { covered = true; break; }
        if (kCapStop) {
          if (Pc >= bound) { covered = true; break; }
          if (a.method == LCEMD_OMR && l == 0 && Z2[0] != 0.f) { covered = true; break; }
        }
      }
    }
    // the merge cut this list (k_eff or capacity reached in key order); a
    // shortfall after the exact re-sort is a rounding residue of the
    // capacity sum, which the last entry absorbs
    if (!covered && sm.rcut[row]) covered = true;
    // rows redone exactly by k_fix_rows (table modes, while their list has
    // room; otherwise the launch reports overflow): a list that ran out
    // before the row's bound was covered (an ICT row deeper than the list;
    // the table may hold up to KT entries), or a cut that is not certified
    const bool can_redo = MODE != P1_PAIR && a.fix_list != nullptr;
    bool redo = false;
    if (!covered && D < h) {
      if (can_redo) redo = true;
      else if (a.overflow) a.overflow[0] = 1;
    }
    // a candidate left out of a full list has a key >= rdrop - half a band
    // (bf16; exact keys for float32): the used entries must all be nearer
    if (QK && D > 0 && sm.rdrop[row] < INFINITY && a.overflow) {
      bool certified;
      if constexpr (EX) {
        // exact keys left out are at least their quantised value
        certified = Lx[D - 1] < sm.rdrop[row];
      } else {
        const float half_band = 0.5f * band_coef<PREC>() * sqrtf(sm.rvn[row]) * sm.qmax;
        const float last_key = Z2[D - 1] - sm.rvn[row];
        certified = last_key < sm.rdrop[row] - half_band - 1e-6f * (sm.rvn[row] + sm.qmax * sm.qmax);
      }
      if (!certified) {
        if (can_redo) redo = true;
        else a.overflow[0] = 1;
      }
    }
    if (redo) {
      const int slot = atomicAdd(a.fix_count, 1);
      if (slot < a.fix_cap) a.fix_list[slot] = out_row0 + row;
      else if (a.overflow) a.overflow[0] = 1;
    }
    if constexpr (MODE == P1_TABLE) {
      const int64_t flat = out_row0 + row;
      zw_write_row(a.ZW, a.zw_nq, a.KT, flat / a.v_used, flat % a.v_used, D,
                   [&](int l) { return sqrtf(fmaxf(Z2[l], 0.f)); },
                   [&](int l) { return l == D - 1 ? INFINITY : sm.cap[(uint32_t)Lw[l]]; });
      if (D > a.KT && a.overflow) a.overflow[0] = 1;
    } else if constexpr (MODE == P1_TABLE_FULL) {
      const int64_t o0 = (out_row0 + row) * (int64_t)a.k;
      for (int l = 0; l < a.k; ++l) {
        if (l < D) {
          const int pos = (int)(uint32_t)Lw[l];
          a.S[o0 + l] = pos;
          a.Z[o0 + l] = sqrtf(fmaxf(Z2[l], 0.f));
          a.W[o0 + l] = sm.cap[pos];
        } else {
          a.S[o0 + l] = -1;
          a.Z[o0 + l] = 0.f;
          a.W[o0 + l] = 0.f;
        }
      }
    } else {
      float rem = bound, cost = 0.f;
      for (int l = 0; l < D; ++l) {
        const float w = sm.cap[(uint32_t)Lw[l]];
        const float r = l == D - 1 ? rem : fminf(rem, w);
        rem -= r;
        cost = fmaf(r, sqrtf(fmaxf(Z2[l], 0.f)), cost);
      }
      sm.rcost[row] = cost;
    }
  }
  if constexpr (MODE == P1_PAIR) {
    __syncthreads();
    if (tid == 0) {
      float tot = 0.f;
      for (int r = 0; r < nrows; ++r) tot += sm.rcost[r];
      a.partial[pidx * a.rb_max + rb] = tot;
    }
  }
}

// Persistent grid: as many workgroups as stay resident, each pulling items
// from the counter of its XCD (workgroup i runs on XCD i % 8), which walks a
// contiguous eighth of the items.  No workgroup waits on another; each
// exits once its counter passes the end of its range.
template <int MODE, int KL, int PREC, bool LONG>
__global__ __launch_bounds__(kThreads, 2) void k_phase1_wide(P1Args a, int64_t total) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int64_t s_item;
  const int xcd = blockIdx.x & 7;
  const int64_t lo = total * xcd / 8, hi = total * (xcd + 1) / 8;
  while (true) {
    __syncthreads();  // the previous item is done with LDS and s_item
    if (threadIdx.x == 0) s_item = lo + (int64_t)atomicAdd(&a.work_ctr[xcd], 1ull);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= hi) break;
    wide_task<MODE, KL, PREC, LONG>(a, smem_raw, item);
  }
}

template <int MODE, int KL, int PREC, bool LONG>
static hipError_t launch_wide_one(const P1Args& a, hipStream_t s) {
  constexpr bool QK = PREC != PREC_F32 || MODE != P1_PAIR;
  const size_t shmem = sizeof(WideSmem<KL, PREC, QK, PREC == PREC_F32 && QK, LONG ? kSegLong : kSeg>);
  const void* fn = (const void*)k_phase1_wide<MODE, KL, PREC, LONG>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  int64_t total;
  if (MODE == P1_PAIR) {
    total = a.npairs * (int64_t)a.rb_max;
  } else {
    const int64_t nrb = (a.v_used + kWR - 1) / kWR;
    const int64_t gw = int64_t(1) << wide_group_log2(a.v_used, PREC);
    total = (a.nq + gw - 1) / gw * nrb * gw;
  }
  if (total <= 0) return hipSuccess;
  if (!a.work_ctr) return hipErrorInvalidValue;
  e = launch_zero_ints((int*)a.work_ctr, 16, s);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid(fn, kThreads, shmem, total);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_phase1_wide<MODE, KL, PREC, LONG>), dim3(grid), dim3(kThreads), shmem, s, a, total);
  return hipGetLastError();
}

template <int MODE, int PREC, bool LONG>
static hipError_t launch_wide_mode(const P1Args& a, int KL, hipStream_t s) {
  if (KL <= 2) return launch_wide_one<MODE, 2, PREC, LONG>(a, s);
  if (KL <= 4) return launch_wide_one<MODE, 4, PREC, LONG>(a, s);
  if (KL <= 8) return launch_wide_one<MODE, 8, PREC, LONG>(a, s);
  if (KL <= 16) return launch_wide_one<MODE, 16, PREC, LONG>(a, s);
  if (KL <= 32) return launch_wide_one<MODE, 32, PREC, LONG>(a, s);
  return hipErrorInvalidValue;
}

template <int PREC, bool LONG = false>
static hipError_t launch_wide_prec(const P1Args& a, int mode, int KL, hipStream_t s) {
  switch (mode) {
    case P1_TABLE: return launch_wide_mode<P1_TABLE, PREC, LONG>(a, KL, s);
    case P1_TABLE_FULL: return launch_wide_mode<P1_TABLE_FULL, PREC, LONG>(a, KL, s);
    case P1_PAIR: return launch_wide_mode<P1_PAIR, PREC, LONG>(a, KL, s);
  }
  return hipErrorInvalidValue;
}

// Exact redo of single table rows (rows whose selection certificate
// failed): one wave per row computes float32 squared distances to all of the
// query's words by direct differences (16 columns per lane in registers),
// then takes them in ascending (distance, position) order by repeated wave
// minimum -- at most KT + 1 of them -- with the same cut and outputs as the
// table modes.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_fix_rows(P1Args a, const int64_t* __restrict__ list) {
  constexpr int kCols = kSegLong / 64;  // columns per lane
  constexpr int kTake = 64;             // entries a row can take; deeper rows are flagged as overflow
  __shared__ uint64_t taken[kThreads / 64][kTake];
  const int count = min(*a.fix_count, a.fix_cap);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (a.fix_total && blockIdx.x == 0 && threadIdx.x == 0 && count > 0) atomicAdd(a.fix_total, (unsigned long long)count);
  const int nw = gridDim.x * (kThreads / 64);
  uint64_t* tk = taken[wv];
  for (int item = blockIdx.x * (kThreads / 64) + wv; item < count; item += nw) {
    const int64_t flat = list[item];
    const int64_t qi = flat / a.v_used, r = flat % a.v_used;
    const int64_t b = a.q0 + qi;
    const int64_t s0 = a.qptr[b];
    const int h = (int)(a.qptr[b + 1] - s0);
    const float* vrow = a.V + (size_t)a.used[r] * a.m_pad;
    uint64_t key[kCols];
#pragma unroll
    for (int j = 0; j < kCols; ++j) {
      const int c = lane + 64 * j;
      key[j] = ~0ull;
      if (c < h) {
        const float4* q = (const float4*)(a.V + (size_t)a.qcol[s0 + c] * a.m_pad);
        float d2 = 0.f;
        // eight float4 of each vector (one 128-byte line) are loaded together
        // and then added in the same order as one at a time (indices past
        // the end are clamped and their values unused); the zero padding
        // adds exact zeros
        for (int d0 = 0; d0 < a.m4; d0 += 8) {
          float4 y[8], x[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int d = min(d0 + i, a.m4 - 1);
            y[i] = q[d];
            x[i] = *(const float4*)(vrow + 4 * d);
          }
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            if (d0 + i < a.m4) {
              float e;
              e = x[i].x - y[i].x; d2 = fmaf(e, e, d2);
              e = x[i].y - y[i].y; d2 = fmaf(e, e, d2);
              e = x[i].z - y[i].z; d2 = fmaf(e, e, d2);
              e = x[i].w - y[i].w; d2 = fmaf(e, e, d2);
            }
          }
        }
        key[j] = w_pack(d2, (uint32_t)c);
      }
    }
    int kef;
    const float bound = MODE == P1_TABLE ? a.xmax[r] : INFINITY;
    if (MODE == P1_TABLE_FULL) kef = min(a.k, h);
    else if (a.method == LCEMD_ICT) kef = h;
    else if (a.method == LCEMD_OMR) kef = min(2, h);
    else if (a.method == LCEMD_RWMD) kef = 1;
    else kef = min(a.k, h);
    const int limit = min(MODE == P1_TABLE ? min(h, a.KT + 1) : min(h, a.k), kTake);
    int D = 0;
    float Pc = 0.f;
    bool done = false;  // a cut was reached
    for (int l = 0; l < limit; ++l) {
      uint64_t m = ~0ull;
#pragma unroll
      for (int j = 0; j < kCols; ++j) m = key[j] < m ? key[j] : m;
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) {
        int lo = (int)(uint32_t)m, hi = (int)(uint32_t)(m >> 32);
        lo = __shfl_xor(lo, sh);
        hi = __shfl_xor(hi, sh);
        const uint64_t o = ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
        m = o < m ? o : m;
      }
#pragma unroll
      for (int j = 0; j < kCols; ++j)
        if (key[j] == m) key[j] = ~0ull;  // keys are distinct (position bits)
      if (lane == 0) tk[l] = m;
      ++D;
      Pc += a.qval[s0 + (uint32_t)m];
      done = D >= kef || D == h;
      if (MODE == P1_TABLE)
        done = done || Pc >= bound || (a.method == LCEMD_OMR && l == 0 && w_unpack(m) != 0.f);
      if (done) break;
    }
    if (lane == 0) {  // the lane that recorded the taken entries
      if (MODE == P1_TABLE) {
        if (D > a.KT || !done) {  // deeper than the table, or than kTake entries
          a.overflow[0] = 1;
        } else {
          zw_write_row(a.ZW, a.zw_nq, a.KT, qi, r, D,
                       [&](int l) { return sqrtf(fmaxf(w_unpack(tk[l]), 0.f)); },
                       [&](int l) { return l == D - 1 ? INFINITY : a.qval[s0 + (uint32_t)tk[l]]; });
        }
      } else {
        const int64_t o0 = flat * (int64_t)a.k;
        for (int l = 0; l < a.k; ++l) {
          if (l < D) {
            const int pos = (int)(uint32_t)tk[l];
            a.S[o0 + l] = pos;
            a.Z[o0 + l] = sqrtf(fmaxf(w_unpack(tk[l]), 0.f));
            a.W[o0 + l] = a.qval[s0 + pos];
          } else {
            a.S[o0 + l] = -1;
            a.Z[o0 + l] = 0.f;
            a.W[o0 + l] = 0.f;
          }
        }
      }
    }
  }
}

hipError_t launch_fix_rows(const P1Args& a, int mode, int count, hipStream_t s) {
  // `count` bounds the grid; the kernel reads the live count from a.fix_count
  if (count <= 0) return hipSuccess;
  if (mode == P1_TABLE_FULL && a.k > 64) return hipErrorInvalidValue;
  const int per = kThreads / 64;
  const unsigned grid = (unsigned)std::min<int64_t>((count + per - 1) / per, 65536);
  if (mode == P1_TABLE)
    hipLaunchKernelGGL(k_fix_rows<P1_TABLE>, dim3(grid), dim3(kThreads), 0, s, a, a.fix_list);
  else if (mode == P1_TABLE_FULL)
    hipLaunchKernelGGL(k_fix_rows<P1_TABLE_FULL>, dim3(grid), dim3(kThreads), 0, s, a, a.fix_list);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int phase1_wide_rows() { return kWR; }

hipError_t launch_phase1_wide(const P1Args& a, int mode, int KL, int prec, int seg_hmax, hipStream_t s) {
  if (seg_hmax > kSegLong) return hipErrorInvalidValue;
  if (seg_hmax > kSeg) return prec == PREC_F32 ? launch_wide_prec<PREC_F32, true>(a, mode, KL, s) : hipErrorInvalidValue;
  if (prec == PREC_F32) return launch_wide_prec<PREC_F32>(a, mode, KL, s);
  if (prec == PREC_BF16) return hipErrorInvalidValue;  // bf16 keys: launch_phase1_bf16
  if (prec == PREC_FP8) {
    if (!a.V8 || !a.vscale || a.m8 % 128 != 0) return hipErrorInvalidValue;
    return launch_wide_prec<PREC_FP8>(a, mode, KL, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lcemd
