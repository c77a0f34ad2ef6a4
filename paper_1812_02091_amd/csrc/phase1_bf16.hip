// Phase 1 of LC-ACT (Sec. 4, Phase 1) with bfloat16 keys, table modes:
// per (vocabulary row, query) the nearest query words of Alg. 3 (and their
// capacities), selected on bfloat16 contractions and finished with float32
// distances recomputed from the float32 embeddings.
//
// Work item: one query against a block of 256 used vocabulary rows; a
// workgroup of 8 waves, wave w owning rows 32w..32w+31.  The contraction
// runs on the 32x32x16 bf16 MFMA with the vocabulary rows as its N operand
// -- each lane holds all K steps of its row in registers for the whole item
// -- and the query's words as its M operand, staged in LDS 128 words at a
// time and read by every wave.  After a 32-word tile, lane l therefore
// holds 16 keys of its own row l % 32: words 8(r/4) + 4(l/32) + (r%4) of the
// tile, r = 0..15.
//
// Keys are approximate squared distances.  The bf16 rows (built at load)
// hold -2 v in their first m dims, 1 in the next three and a three-piece
// bf16 split of |v|^2 in the three after (three bf16 significands hold a
// float32 one exactly); the query form of a word holds v, the split of its
// |q|^2 and three ones.  One contraction then gives |v|^2 + |q|^2 -
// 2 <v_b, q_b> with float32 accumulation.
//
// Error band.  With e_v = v - v_b: <v,q> - <v_b,q_b> = <e_v, q> + <v_b, e_q>,
// so by Cauchy-Schwarz the key is off the exact squared distance by at
// most eps = 2 (|e_v| |q| + |v_b| |e_q|) plus the float32 accumulation of
// K + 6 terms (|e_v| is stored per row at load, rounded up).  A row keeps
// every candidate whose key is within band = 2 eps (plus the rounding of
// the packed keys) of its cut key: a word outside that band is farther,
// exactly, than every word up to the cut, so it can never be needed.
//
// Selection.  Each lane keeps the smallest keys it has seen for its row in
// a sorted register list (packed key | word position; a bitonic sort makes
// the list from the first tile, later tiles insert their candidates by a
// min/max network).  A key above the row's threshold (cut key + band,
// from the lanes' own lists, which bound the row's) is no candidate.
// After the last tile the two lanes of a row merge their lists; keys pushed
// out of a full list are remembered (the smallest of them) and the row is
// redone exactly unless every used entry is provably nearer.
//
// Exact distances.  Every listed candidate gets a float32 dot product with
// the float32 row: the query's float32 vectors are staged through LDS a
// chunk of dims at a time, each of a row's two lanes takes half of every
// chunk's dims for all the row's entries, and the halves are added in a
// fixed order.  Where cancellation could bite the distance is taken by
// direct differences (identical words: exactly 0).  The list is re-sorted
// by (distance, position) and cut as Alg. 3 / the capacity bound say.
#include <algorithm>

#include "internal.h"

namespace lcemd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kBT = 512;              // threads per workgroup (one workgroup per CU)
constexpr int kBR = 256;              // rows per item (8 waves x 32)
constexpr int kBW = 128;              // query words per staged chunk
constexpr int kBMaxMb = kBf16MaxDims; // bf16 row width held in registers
constexpr int kBKS = kBMaxMb / 16;    // K steps held in registers
constexpr int kBQa = 2 * kBMaxMb + 16; // bytes per staged word (16 bytes of padding)
constexpr int kBSeg = kSegShort;      // query words per item
constexpr int kBStg = 34;             // u32 per row: candidate staging [2][17] / final list
constexpr int kBGroup = 32;           // queries per item group (query-fastest): a row block stays in L2 for 32 items
constexpr uint32_t kNone = 0xffffffffu;
constexpr uint32_t kPosMask = 511u;   // 9 position bits (words < 512)
// twice the largest relative rounding of a packed key: 2 * 2^(9 - 23)
constexpr float kQuant = 1.f / 8192.f;
constexpr float kGuard = 0.25f;       // cancellation guard of the float32 form

struct BfSmem {
  union {
    unsigned char qa[kBW * kBQa];   // bf16 query words (M operand), one chunk
    float qf[kBSeg * 36];           // float32 query vectors, a chunk of dims (h (RD + 4) floats)
    float zb[kBR * 32];             // exact squared distances of the lists
  } u;
  uint32_t lst[kBR * kBStg];        // candidate staging, then the final lists
  int cid[kBSeg];
  float cap[kBSeg];
  float qn[kBSeg];
  int rid[kBR];
  float rbound[kBR];
  float rvn[kBR];
  float reps[kBR];
  float rband[kBR];
  int rlen[kBR];
  uint32_t rdrop[kBR];
  int rflag[kBR];  // 2: the merged list has its cut; 1: full without a cut; 0: neither
  int rorder[kBR];  // rows by list length (the recompute's row of each lane pair)
  int lhist[34];    // rows per list length, then the next free rank of each length
  float qmax;
  float eqmax;
};

__device__ __forceinline__ uint32_t pk(float d2, int j) {
  // d2 >= 0: its bits order like the values; the 9 low bits give way to j
  return (__float_as_uint(d2) & ~kPosMask) | (uint32_t)j;
}
__device__ __forceinline__ float pk_key(uint32_t k) { return __uint_as_float(k & ~kPosMask); }
__device__ __forceinline__ int pk_pos(uint32_t k) { return (int)(k & kPosMask); }
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a < b ? b : a; }

// ascending bitonic sort of 16 packed keys
__device__ __forceinline__ void sort16(uint32_t (&k)[16]) {
#pragma unroll
  for (int kb = 2; kb <= 16; kb <<= 1) {
#pragma unroll
    for (int jb = kb >> 1; jb > 0; jb >>= 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int l = i ^ jb;
        if (l > i) {
          const uint32_t x = k[i], y = k[l];
          const bool up = (i & kb) == 0;
          k[i] = up ? umin(x, y) : umax(x, y);
          k[l] = up ? umax(x, y) : umin(x, y);
        }
      }
    }
  }
}

// insert c into the ascending list a; returns what fell off the end
template <int LK>
__device__ __forceinline__ uint32_t insert(uint32_t (&a)[LK], uint32_t c) {
  const uint32_t out = umax(a[LK - 1], c);
#pragma unroll
  for (int i = LK - 1; i > 0; --i) a[i] = umax(a[i - 1], umin(a[i], c));
  a[0] = umin(a[0], c);
  return out;
}

// Cut of an ascending list (Alg. 3 / Lemma 1-2): the first entry where
// k_eff entries are listed or the listed capacities reach the row's bound.
// Returns the cut entry (kNone if none).
template <int LK, bool CAPSTOP>
__device__ __forceinline__ uint32_t list_cut(const uint32_t (&a)[LK], const float* cap, int kef, float bound) {
  // the capacities of the first entries are read together (one LDS round
  // trip instead of one per entry); lists are cut within a few entries
  constexpr int kPre = LK < 8 ? LK : 8;
  float c[kPre];
#pragma unroll
  for (int i = 0; i < kPre; ++i) c[i] = (CAPSTOP && a[i] != kNone) ? cap[pk_pos(a[i])] : 0.f;
  float P = 0.f;
  uint32_t K0 = kNone;
#pragma unroll
  for (int i = 0; i < LK; ++i) {
    const bool live = K0 == kNone && a[i] != kNone;
    if (!__any(live)) break;
    if (live) {
      if (CAPSTOP) P += i < kPre ? c[i] : cap[pk_pos(a[i])];
      if (i + 1 >= kef || (CAPSTOP && P >= bound)) K0 = a[i];
    }
  }
  return K0;
}

__device__ __forceinline__ float exact_d2(const float* __restrict__ V, int m_pad, int m4, int a, int b) {
  const float4* x = (const float4*)(V + (size_t)a * m_pad);
  const float4* y = (const float4*)(V + (size_t)b * m_pad);
  float s = 0.f;
  for (int d = 0; d < m4; ++d) {
    const float4 p = x[d], q = y[d];
    const float e0 = p.x - q.x, e1 = p.y - q.y, e2 = p.z - q.z, e3 = p.w - q.w;
    s = fmaf(e0, e0, s);
    s = fmaf(e1, e1, s);
    s = fmaf(e2, e2, s);
    s = fmaf(e3, e3, s);
  }
  return s;
}

// Stage words [c0, c0 + cw) of the query in LDS as the M operand (their
// query-form bf16 rows).  Wave w takes words c0 + w, c0 + w + 8, ...; a
// lane copies one 16-byte piece (mb <= 512: at most 64 pieces).
__device__ __forceinline__ void stage_words(const P1Args& a, BfSmem& sm, int c0, int cw, int mb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int npc = mb / 8;
  for (int c = wave; c < cw; c += kBT / 64)
    if (lane < npc)
      *(uint4*)(sm.u.qa + c * kBQa + 16 * lane) = *(const uint4*)(a.Vbq + (size_t)sm.cid[c0 + c] * mb + 8 * lane);
}

// Float32 squared distances of row xr's listed words (lane pair xr, sub):
// the query's float32 vectors are staged RD dims at a time; lane sub takes
// dims [sub RD/2, (sub+1) RD/2) of every chunk for all the row's entries,
// its row dims loaded one chunk ahead, and the halves are added in a fixed
// order.  Results (by direct differences where cancellation could bite) go
// to zb.  m4dims: the real dims rounded up to 4.
template <int RD, int LK>
__device__ __forceinline__ void recompute(const P1Args& a, BfSmem& sm, int h, int m4dims, int xr, int sub) {
  constexpr int RS = RD + 4;      // floats per staged word
  constexpr int HALF = RD / 2;
  constexpr int Q = HALF / 4;     // float4 of a lane's half chunk
  constexpr int N4 = RD / 4;      // float4 per staged word and chunk
  const int tid = threadIdx.x;
  const int xlen = sm.rlen[xr];
  const int xw = sm.rid[xr];
  int pos[LK];
  float dot[LK];
#pragma unroll
  for (int e = 0; e < LK; ++e) {
    pos[e] = e < xlen ? pk_pos(sm.lst[xr * kBStg + e]) : 0;
    dot[e] = 0.f;
  }
  // the longest list of the wave bounds its (uniform) entry loop; shorter
  // lists compute on word 0 and drop the result
  int wlen = xlen;
  for (int o = 32; o > 0; o >>= 1) wlen = max(wlen, __shfl_xor(wlen, o));
  const int per = (h * N4 + kBT - 1) / kBT;  // float4 a thread stages per chunk (<= 8)
  const int nch = (m4dims + RD - 1) / RD;
  float4 nx[8];
  auto fetch = [&](int d0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int f = tid + i * kBT;
      const int c = f / N4, q4 = f % N4, d = d0 + 4 * q4;
      nx[i] = (i < per && c < h && d < a.m_pad) ? *(const float4*)(a.V + (size_t)sm.cid[c] * a.m_pad + d)
                                              : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  const float* vrow = a.V + (size_t)xw * a.m_pad + sub * HALF;
  float4 vc[Q];
  fetch(0);
  for (int ch = 0; ch < nch; ++ch) {
    const int d0 = ch * RD;
#pragma unroll
    for (int q = 0; q < Q; ++q)  // the row's chunk, in flight through the staging
      vc[q] = d0 + 4 * q + sub * HALF < a.m_pad ? *(const float4*)(vrow + d0 + 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();  // the previous chunk is consumed
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int f = tid + i * kBT;
      const int c = f / N4, q4 = f % N4;
      if (i < per && c < h) *(float4*)(&sm.u.qf[c * RS + 4 * q4]) = nx[i];
    }
    __syncthreads();
    if (ch + 1 < nch) fetch(d0 + RD);  // in flight during this chunk's products
    float4 qv[Q];
    // fully unrolled (entries skipped by a wave-uniform test, not a loop
    // exit), so pos[] and dot[] stay in fixed registers
#pragma unroll
    for (int e = 0; e < LK; ++e) {
      if (e < wlen) {
        const float* qp = &sm.u.qf[pos[e] * RS + sub * HALF];
#pragma unroll
        for (int q = 0; q < Q; ++q) qv[q] = *(const float4*)(qp + 4 * q);
        float t = dot[e];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          t = fmaf(vc[q].x, qv[q].x, t);
          t = fmaf(vc[q].y, qv[q].y, t);
          t = fmaf(vc[q].z, qv[q].z, t);
          t = fmaf(vc[q].w, qv[q].w, t);
        }
        dot[e] = t;
      }
    }
  }
  __syncthreads();  // the staged vectors are dead: zb may reuse their LDS
  const float vn = sm.rvn[xr];
#pragma unroll
  for (int e = 0; e < LK; ++e) {
    const float o = __shfl_xor(dot[e], 1);
    if (e < xlen && (e & 1) == sub) {
      const float full = sub == 0 ? dot[e] + o : o + dot[e];  // fixed order: even half first
      const float qn = sm.qn[pos[e]];
      float d2 = (vn + qn) - 2.f * full;
      if (!(d2 >= kGuard * (vn + qn))) d2 = exact_d2(a.V, a.m_pad, a.m4, xw, sm.cid[pos[e]]);
      sm.u.zb[xr * 32 + e] = d2;
    }
  }
}

template <int MODE, int LK, int NKS>
__device__ __forceinline__ void bf16_task(const P1Args& a, BfSmem& sm, int64_t item) {
  static_assert(LK == 16 || LK == 32, "list sizes 16 or 32");
  static_assert(NKS >= 1 && NKS <= kBKS, "K steps held in registers");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lh = lane >> 5, li = lane & 31;
  constexpr bool kCapStop = MODE != P1_TABLE_FULL;

  // ---------------- item decode ----------------
  const int64_t nsb = (a.v_used + kBR - 1) / kBR;
  const int64_t qin = item % kBGroup, t0 = item / kBGroup;
  const int64_t sb = t0 % nsb, g = t0 / nsb;
  const int64_t qi = g * kBGroup + qin;
  if (qi >= a.nq) return;
  const int64_t r0 = sb * kBR;
  const int64_t b = a.q0 + qi;
  const int nrows = (int)min((int64_t)kBR, a.v_used - r0);
  const int64_t out_row0 = qi * a.v_used + r0;
  const int64_t s0 = a.qptr[b];
  const int h = (int)(a.qptr[b + 1] - s0);
  if (h <= 0) return;  // padding slot of a fixed-size batch
  const int m = 4 * a.m4 <= a.m_pad ? a.m4 * 4 : a.m_pad;  // real dims rounded up to 4
  const int mb = a.mb;  // == 16 * NKS (checked by the launcher)

  // one 16-byte record per row and per query word (built per call by
  // k_bf16_info): word id, bound / weight, |v|^2, |v - bf16(v)|
  if (tid < kBR) {
    const bool ok = tid < nrows;
    const float4 ri = ok ? a.rinfo[r0 + tid] : make_float4(0.f, 0.f, 0.f, 0.f);
    sm.rid[tid] = __float_as_int(ri.x);
    sm.rbound[tid] = ok ? (MODE == P1_TABLE ? ri.y : INFINITY) : 0.f;
    sm.rvn[tid] = ri.z;
    sm.reps[tid] = ri.w;  // |e_v|, replaced by the row's eps below
    sm.rflag[tid] = 0;
  }
  for (int c = tid; c < h; c += kBT) {
    const float4 qi = a.qinfo[s0 + c];
    sm.cid[c] = __float_as_int(qi.x);
    sm.cap[c] = qi.y;
    sm.qn[c] = qi.z;
  }
  if (tid == 0) {  // the query's largest |q|^2 and |q - bf16(q)| (k_bf16_qmax)
    const float2 mx = a.qmx[qi];
    sm.qmax = sqrtf(mx.x) * 1.0001f;
    sm.eqmax = mx.y;
  }
  __syncthreads();
  if (tid < kBR) {
    const float nv = sqrtf(sm.rvn[tid]) * 1.0001f, qm = sm.qmax;
    const float ev = sm.reps[tid];
    // |v_b| <= |v| (1 + 2^-8); K + 6 float32 accumulation steps
    const float eps = 2.02f * (ev * qm + nv * sm.eqmax) +
                      (float)(mb + 8) * 6.0e-8f * (sm.rvn[tid] + qm * qm + 2.f * nv * qm) * 1.1f + 1e-30f;
    sm.reps[tid] = eps;
    sm.rband[tid] = 2.f * eps + kQuant * (sm.rvn[tid] + qm * qm + 2.f * nv * qm);
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

  // ---------------- row operand: all K steps in registers ----------------
  const int row = 32 * wave + li;
  const bool row_ok = row < nrows;
  uint4 bfr[NKS];
  {
    const uint16_t* bp = a.Vb + (size_t)sm.rid[row] * mb + 8 * lh;
#pragma unroll
    for (int s = 0; s < NKS; ++s) bfr[s] = *(const uint4*)(bp + 16 * s);
  }
  __syncthreads();  // row bands ready
  const float band = sm.rband[row];
  const float bound = sm.rbound[row];

  uint32_t lst[LK];
#pragma unroll
  for (int i = 0; i < LK; ++i) lst[i] = kNone;
  uint32_t drop = kNone;  // smallest key pushed out of a full list
  float theta = INFINITY;
  bool first = true;
  uint32_t* stg = &sm.lst[row * kBStg + lh * 17];

  for (int c0 = 0; c0 < h; c0 += kBW) {
    const int cw = min(kBW, h - c0);
    if (c0 > 0) __syncthreads();  // every wave is done with the previous chunk
    stage_words(a, sm, c0, cw, mb);
    __syncthreads();
    const int nt = (cw + 31) >> 5;
    for (int t = 0; t < nt; ++t) {
      floatx16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
      const unsigned char* ap = sm.u.qa + (32 * t + li) * kBQa + 16 * lh;
      // A fragments read three steps ahead of their MFMA (LDS latency)
      constexpr int kAhead = 3;
      bf16x8 av[kAhead];
#pragma unroll
      for (int s = 0; s < kAhead && s < NKS; ++s) av[s] = *(const bf16x8*)(ap + 32 * s);
#pragma unroll
      for (int s = 0; s < NKS; ++s) {
        const bf16x8 cur = av[s % kAhead];
        if (s + kAhead < NKS) av[s % kAhead] = *(const bf16x8*)(ap + 32 * (s + kAhead));
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&bfr[s]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur, bv, acc, 0, 0, 0);
      }
      const int jb = c0 + 32 * t + 4 * lh;
      if (first) {
        uint32_t kk[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int j = jb + 8 * (r >> 2) + (r & 3);
          kk[r] = (row_ok && j < h) ? pk(fmaxf(acc[r], 0.f), j) : kNone;
        }
        sort16(kk);
#pragma unroll
        for (int i = 0; i < LK; ++i) lst[i] = i < 16 ? kk[i] : kNone;
        first = false;
      } else {
        int cnt = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int j = jb + 8 * (r >> 2) + (r & 3);
          const float d2 = fmaxf(acc[r], 0.f);
          const bool cand = row_ok && j < h && d2 < theta;
          stg[cnt] = pk(d2, j);  // slot cnt is overwritten unless this key counts
          cnt += cand ? 1 : 0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if (!__any(i < cnt)) break;
          const uint32_t cnd = i < cnt ? stg[i] : kNone;
          drop = umin(drop, insert<LK>(lst, cnd));
        }
      }
      // threshold from this lane's list; the row's cut key is at most it
      const uint32_t K0 = list_cut<LK, kCapStop>(lst, sm.cap, kef, bound);
      // (no cut yet: no threshold -- keys pushed out of a full list are
      // remembered by insert(), never dropped silently)
      float th = K0 != kNone ? pk_key(K0) * (1.f + kQuant) + band : INFINITY;
      th = fminf(th, __shfl_xor(th, 32));
      theta = fminf(theta, th);
    }
  }

  // ---------------- the row's list: merge of its two lanes ----------------
  {
    uint32_t other[LK];
#pragma unroll
    for (int i = 0; i < LK; ++i) other[i] = (uint32_t)__shfl_xor((int)lst[i], 32);
    uint32_t lost = kNone;
#pragma unroll
    for (int i = 0; i < LK; ++i) {
      const uint32_t x = lst[i], y = other[LK - 1 - i];
      lst[i] = umin(x, y);
      lost = umin(lost, umax(x, y));
    }
    // lst is now bitonic and holds the LK smallest: clean it
#pragma unroll
    for (int jb = LK >> 1; jb > 0; jb >>= 1) {
#pragma unroll
      for (int i = 0; i < LK; ++i) {
        const int l = i ^ jb;
        if (l > i) {
          const uint32_t x = lst[i], y = lst[l];
          lst[i] = umin(x, y);
          lst[l] = umax(x, y);
        }
      }
    }
    drop = umin(umin(drop, lost), (uint32_t)__shfl_xor((int)drop, 32));
    const uint32_t K0 = list_cut<LK, kCapStop>(lst, sm.cap, kef, bound);
    int len = 0;
    const float lim = K0 != kNone ? pk_key(K0) * (1.f + kQuant) + band : INFINITY;
#pragma unroll
    for (int i = 0; i < LK; ++i)
      if (lst[i] != kNone && pk_key(lst[i]) <= lim) len = i + 1;
    // both lanes hold the same list: each writes half of it
    uint32_t* L = &sm.lst[row * kBStg];
#pragma unroll
    for (int i = 0; i < LK; ++i)
      if ((i >= LK / 2) == (lh == 1)) L[i] = lst[i];
    if (lh == 0 && row_ok) {
      sm.rlen[row] = len;
      sm.rdrop[row] = drop;
      // a full list without a cut is an ICT row deeper than the list
      sm.rflag[row] = K0 != kNone ? 2 : (lst[LK - 1] != kNone ? 1 : 0);
    }
    if (lh == 0 && !row_ok) sm.rlen[row] = 0;
  }
  __syncthreads();

  // ---------------- exact float32 distances of the listed words ----------------
  // rows by list length (counting sort): the lanes of a wave then take rows
  // of similar lengths, so a wave's entry loop is not set by one long list
  // among short ones (which row a lane pair takes does not change results)
  if (tid < 34) sm.lhist[tid] = 0;
  __syncthreads();
  if (tid < kBR) atomicAdd(&sm.lhist[sm.rlen[tid]], 1);
  __syncthreads();
  if (tid == 0) {
    int acc0 = 0;
    for (int L = 33; L >= 0; --L) {  // longest lists first
      const int c = sm.lhist[L];
      sm.lhist[L] = acc0;
      acc0 += c;
    }
  }
  __syncthreads();
  if (tid < kBR) sm.rorder[atomicAdd(&sm.lhist[sm.rlen[tid]], 1)] = tid;
  __syncthreads();
  const int xr = sm.rorder[tid >> 1], sub = tid & 1;
  if (h <= 256) recompute<64, LK>(a, sm, h, m, xr, sub);
  else recompute<32, LK>(a, sm, h, m, xr, sub);
  __syncthreads();

  // ---------------- re-sort, cut, certificate, outputs ----------------
  if (sub == 0 && xr < nrows) {
    uint32_t* Lw = &sm.lst[xr * kBStg];
    float* Z2 = &sm.u.zb[xr * 32];
    const int len = sm.rlen[xr];
    for (int i = 0; i < len; ++i) Lw[i] = (uint32_t)pk_pos(Lw[i]);
    for (int i = 1; i < len; ++i) {
      const float z = Z2[i];
      const uint32_t p = Lw[i];
      int j = i - 1;
      while (j >= 0 && (Z2[j] > z || (Z2[j] == z && Lw[j] > p))) {
        Lw[j + 1] = Lw[j];
        Z2[j + 1] = Z2[j];
        --j;
      }
      Lw[j + 1] = p;
      Z2[j + 1] = z;
    }
    const float xb = sm.rbound[xr];
    int D = 0;
    bool covered = false;
    {
      float Pc = 0.f;
      for (int l = 0; l < len; ++l) {
        ++D;
        Pc += sm.cap[Lw[l]];
        if (D >= kef) { covered = true; break; }
        if (kCapStop) {
          if (Pc >= xb) { covered = true; break; }
          if (a.method == LCEMD_OMR && l == 0 && Z2[0] != 0.f) { covered = true; break; }
        }
      }
    }
    // the merge cut this list (k_eff or capacity reached in key order); a
    // shortfall after the exact re-sort is a rounding residue of the
    // capacity sum, which the last entry absorbs
    if (!covered && sm.rflag[xr] == 2) covered = true;
    const bool can_redo = a.fix_list != nullptr;
    bool redo = false;
    if (!covered && D < h) {
      if (can_redo) redo = true;
      else if (a.overflow) a.overflow[0] = 1;
    }
    // a word pushed out of a full list has an exact squared distance of at
    // least its key minus eps: every used entry must be nearer
    const uint32_t dr = sm.rdrop[xr];
    if (dr != kNone && D > 0 && !(Z2[D - 1] < pk_key(dr) - sm.reps[xr])) {
      if (can_redo) redo = true;
      else if (a.overflow) a.overflow[0] = 1;
    }
    if (redo) {
      const int slot = atomicAdd(a.fix_count, 1);
      if (slot < a.fix_cap) a.fix_list[slot] = out_row0 + xr;
      else if (a.overflow) a.overflow[0] = 1;
    }
    if constexpr (MODE == P1_TABLE) {
      const int64_t flat = out_row0 + xr;
      zw_write_row(a.ZW, a.zw_nq, a.KT, flat / a.v_used, flat % a.v_used, D,
                   [&](int l) { return sqrtf(fmaxf(Z2[l], 0.f)); },
                   [&](int l) { return l == D - 1 ? INFINITY : sm.cap[Lw[l]]; });
      if (D > a.KT && a.overflow) a.overflow[0] = 1;
    } else {
      const int64_t o0 = (out_row0 + xr) * (int64_t)a.k;
      for (int l = 0; l < a.k; ++l) {
        if (l < D) {
          const int p = (int)Lw[l];
          a.S[o0 + l] = p;
          a.Z[o0 + l] = sqrtf(fmaxf(Z2[l], 0.f));
          a.W[o0 + l] = sm.cap[p];
        } else {
          a.S[o0 + l] = -1;
          a.Z[o0 + l] = 0.f;
          a.W[o0 + l] = 0.f;
        }
      }
    }
  }
}

// Persistent grid: one workgroup per CU pulls items from the counter of its
// XCD (workgroup i runs on XCD i % 8), which walks a contiguous eighth of the
// items; every workgroup exits once its counter passes its range.
template <int MODE, int LK, int NKS>
__global__ __launch_bounds__(kBT, 1) void k_phase1_bf16(P1Args a, int64_t total) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int64_t s_item;
  BfSmem& sm = *reinterpret_cast<BfSmem*>(smem_raw);
  const int xcd = blockIdx.x & 7;
  const int64_t lo = total * xcd / 8, hi = total * (xcd + 1) / 8;
  // the counter is read one item ahead: its round trip overlaps an item
  unsigned long long nxt = 0;
  if (threadIdx.x == 0) nxt = atomicAdd(&a.work_ctr[xcd], 1ull);
  while (true) {
    __syncthreads();  // the previous item is done with LDS and s_item
    if (threadIdx.x == 0) {
      s_item = lo + (int64_t)nxt;
      if (lo + (int64_t)nxt < hi) nxt = atomicAdd(&a.work_ctr[xcd], 1ull);
    }
    __syncthreads();
    const int64_t item = s_item;
    if (item >= hi) break;
    bf16_task<MODE, LK, NKS>(a, sm, item);
  }
}

template <int MODE, int LK, int NKS>
hipError_t launch_bf16_one(const P1Args& a, hipStream_t s) {
  const size_t shmem = sizeof(BfSmem);
  const void* fn = (const void*)k_phase1_bf16<MODE, LK, NKS>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  const int64_t nsb = (a.v_used + kBR - 1) / kBR;
  const int64_t total = (a.nq + kBGroup - 1) / kBGroup * nsb * kBGroup;
  if (total <= 0) return hipSuccess;
  if (!a.work_ctr) return hipErrorInvalidValue;
  e = launch_zero_ints((int*)a.work_ctr, 16, s);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid(fn, kBT, shmem, total);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_phase1_bf16<MODE, LK, NKS>), dim3(grid), dim3(kBT), shmem, s, a, total);
  return hipGetLastError();
}

// Row and query-word records for the bf16 kernel: rinfo[r] = (word id bits,
// largest database weight, |v|^2, |v - bf16(v)|) for the used words of the
// rows, qinfo[i] = (word id bits, weight, |v|^2, |v - bf16(v)|) for the
// non-zeros i of the launch's queries (qptr[q0] <= i < qptr[q0 + nq]).
__global__ __launch_bounds__(kThreads) void k_bf16_info(P1Args a) {
  const int64_t qlo = a.qptr[a.q0], qhi = a.qptr[a.q0 + a.nq];
  const int64_t n = max(a.v_used, qhi - qlo);
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    if (i < a.v_used) {
      const int w = a.used[i];
      a.rinfo[i] = make_float4(__int_as_float(w), a.xmax ? a.xmax[i] : INFINITY, a.vnorm[w], a.vres[w]);
    }
    if (i < qhi - qlo) {
      const int64_t j = qlo + i;
      const int w = a.qcol[j];
      a.qinfo[j] = make_float4(__int_as_float(w), a.qval[j], a.vnorm[w], a.vres[w]);
    }
  }
}

// Per query of the launch, the largest |q|^2 and |q - bf16(q)| over its
// words (from qinfo): one wave per query.
__global__ __launch_bounds__(kThreads) void k_bf16_qmax(P1Args a) {
  const int64_t qi = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (qi >= a.nq) return;
  const int64_t s0 = a.qptr[a.q0 + qi], s1 = a.qptr[a.q0 + qi + 1];
  float mq = 0.f, me = 0.f;
  for (int64_t j = s0 + lane; j < s1; j += 64) {
    const float4 q = a.qinfo[j];
    mq = fmaxf(mq, q.z);
    me = fmaxf(me, q.w);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mq = fmaxf(mq, __shfl_xor(mq, o));
    me = fmaxf(me, __shfl_xor(me, o));
  }
  if (lane == 0) a.qmx[qi] = make_float2(mq, me);
}

}  // namespace

bool phase1_bf16_fits(int mb, int seg_hmax, int depth) {
  return mb <= kBMaxMb && mb % 64 == 0 && seg_hmax <= kBSeg && depth + 8 <= 32;
}

template <int MODE, int LK>
hipError_t launch_bf16_width(const P1Args& a, hipStream_t s) {
  switch (a.mb / 16) {  // K steps of the rows: one instantiation per width
    case 4: return launch_bf16_one<MODE, LK, 4>(a, s);
    case 8: return launch_bf16_one<MODE, LK, 8>(a, s);
    case 12: return launch_bf16_one<MODE, LK, 12>(a, s);
    case 16: return launch_bf16_one<MODE, LK, 16>(a, s);
    case 20: return launch_bf16_one<MODE, LK, 20>(a, s);
    case 24: return launch_bf16_one<MODE, LK, 24>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_phase1_bf16(const P1Args& a, int mode, int depth, hipStream_t s) {
  if (!a.Vb || !a.Vbq || !a.vres || !a.rinfo || !a.qinfo || !a.qmx || a.mb % 64 != 0 || a.mb > kBMaxMb ||
      a.mb < a.m + 6)
    return hipErrorInvalidValue;
  {
    // grid-stride over the rows and the launch's query words (at most qnnz)
    const int64_t n = std::max<int64_t>(a.v_used, a.qnnz);
    const unsigned g = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(k_bf16_info, dim3(g), dim3(kThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nq > 0) {
      hipLaunchKernelGGL(k_bf16_qmax, dim3((unsigned)((a.nq + kThreads / 64 - 1) / (kThreads / 64))), dim3(kThreads),
                         0, s, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  const bool small = depth + 8 <= 16;
  if (mode == P1_TABLE) return small ? launch_bf16_width<P1_TABLE, 16>(a, s) : launch_bf16_width<P1_TABLE, 32>(a, s);
  if (mode == P1_TABLE_FULL)
    return small ? launch_bf16_width<P1_TABLE_FULL, 16>(a, s) : launch_bf16_width<P1_TABLE_FULL, 32>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace lcemd
