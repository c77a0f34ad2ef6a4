// Phase 1 of LC-ACT (Sec. 4, Phase 1), streaming variant: the distance
// contraction between 64 rows and one column segment runs on MFMA in
// 64-column passes, and after each pass every row merges the pass's columns
// into a short sorted candidate list held in LDS.  The list never holds more
// than the row can use: k_eff = min(k, h) entries (Alg. 3), 1 for RWMD, 2 for
// OMR (Alg. 1), or -- for every measure -- fewer once the listed capacities
// cover the largest mass the row can have to move (Lemma 1/2: no transfer
// reaches past that point).  Only the final list entries get their distance
// from float32 direct differences; the candidate keys come from the
// contraction.
//
// Rows, segments and outputs are those of the table/pair modes of phase 1
// (see internal.h).  Keys: |c|^2 - 2 <v_r, c>, ranking a row's columns like
// the squared distance; ties go to the lower column position.
//
// Precision of the contraction:
//   float32  (32x32x2 f32 MFMA): list distances use the contraction value
//            |v|^2 + key unless that value is below a quarter of
//            |v|^2 + |c|^2 (cancellation), where they are recomputed exactly;
//   bfloat16 (32x32x16 bf16 MFMA, float32 accumulation): the list is
//            over-selected by the host-given margin, every entry is
//            recomputed exactly in float32, re-sorted by the exact value,
//            and only then cut to k_eff / capacity.
//
// Work order: table-mode workgroups are mapped so that each of the eight
// XCDs walks a contiguous range of (query group, row block, query) tiles,
// query fastest: a row block's embeddings and a query group's embeddings
// stay in that XCD's L2 while they are reused.
#include "internal.h"

namespace lcemd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ uint32_t f_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint64_t f_pack(float f, uint32_t pos) {
  return ((uint64_t)f_bits(f) << 32) | (uint64_t)pos;
}
__device__ __forceinline__ float f_unpack(uint64_t k) {
  const uint32_t o = (uint32_t)(k >> 32);
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

constexpr int kStageStride = 144;  // bytes per staged row (128 data + 16 pad)
constexpr int kCKS = 68;           // floats per row of a pass's keys; 68 % 64 == 4
constexpr int kSeg = LCEMD_MAX_HIST;
constexpr int kGroup = 8;          // queries per tile group (table modes)
constexpr float kGuard = 0.25f;    // float32 path: recompute below this cancellation ratio

template <int KL>
struct FastSmem {
  union {
    unsigned char st[2 * kRows * kStageStride];  // staged row / column slices
    float ck[kRows * kCKS];                      // keys of one 64-column pass
    float zb[kRows * KL];                        // squared distances of the lists
  } u;
  uint64_t lst[2][kRows * KL];  // per-row candidate lists (packed key | position)
  int cid[kSeg];
  float cap[kSeg];
  float qn[kSeg];
  int rid[kRows];
  float rbound[kRows];
  float rvn[kRows];
  int rlen[kRows];
  float rcost[kRows];
};

// Squared distance by direct differences; the float4 groups past the m4
// that hold the real dims are zero padding and would add exact zeros.
__device__ __forceinline__ float exact_d2(const float* __restrict__ V, int m_pad, int m4, int a, int b) {
  const float4* x = (const float4*)(V + (size_t)a * m_pad);
  const float4* y = (const float4*)(V + (size_t)b * m_pad);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  const int n4 = (m4 + 1) & ~1;  // pairs of groups; m_pad / 4 is even
  for (int d = 0; d < n4; d += 2) {
    const float4 p = x[d], q = y[d], p2 = x[d + 1], q2 = y[d + 1];
    const float e0 = p.x - q.x, e1 = p.y - q.y, e2 = p.z - q.z, e3 = p.w - q.w;
    const float f0 = p2.x - q2.x, f1 = p2.y - q2.y, f2 = p2.z - q2.z, f3 = p2.w - q2.w;
    s0 = fmaf(e0, e0, s0);
    s1 = fmaf(e1, e1, s1);
    s2 = fmaf(e2, e2, s2);
    s3 = fmaf(e3, e3, s3);
    s0 = fmaf(f0, f0, s0);
    s1 = fmaf(f1, f1, s1);
    s2 = fmaf(f2, f2, s2);
    s3 = fmaf(f3, f3, s3);
  }
  return (s0 + s1) + (s2 + s3);
}

}  // namespace

// One work item: (query, 64-row block) in the table modes, (pair, row
// block) in pair mode.  Returns early (uniformly) for empty items.
template <int MODE, int KL, int PREC>
__device__ __forceinline__ void fast_task(const P1Args& a, unsigned char* smem_raw, int64_t item) {
  using Sm = FastSmem<KL>;
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
    const int64_t qs = a.qptr[b];
    const int hq = (int)(a.qptr[b + 1] - qs);
    nrows = min(kRows, hq - rb * kRows);
    if (nrows <= 0 || u < 0 || u >= a.n) {
      if (tid == 0) a.partial[pidx * a.rb_max + rb] = 0.f;
      return;
    }
    if (tid < kRows) {
      const bool ok = tid < nrows;
      const int w = ok ? a.qcol[qs + rb * kRows + tid] : 0;
      sm.rid[tid] = w;
      sm.rbound[tid] = ok ? a.qval[qs + rb * kRows + tid] : 0.f;
      sm.rvn[tid] = a.vnorm[w];
      sm.rlen[tid] = 0;
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
    const int64_t nrb = (a.v_used + kRows - 1) / kRows;
    const int64_t work = item;
    const int64_t qin = work % kGroup, t = work / kGroup;
    const int64_t rblk = t % nrb, g = t / nrb;
    const int64_t qi = g * kGroup + qin;
    if (qi >= a.nq) return;
    const int64_t r0 = rblk * kRows;
    const int64_t b = a.q0 + qi;
    nrows = (int)min((int64_t)kRows, a.v_used - r0);
    out_row0 = qi * a.v_used + r0;
    if (tid < kRows) {
      const bool ok = tid < nrows;
      const int w = ok ? a.used[r0 + tid] : 0;
      sm.rid[tid] = w;
      sm.rbound[tid] = ok ? (MODE == P1_TABLE ? a.xmax[r0 + tid] : INFINITY) : 0.f;
      sm.rvn[tid] = a.vnorm[w];
      sm.rlen[tid] = 0;
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

  int kef;
  if constexpr (MODE == P1_TABLE_FULL) {
    kef = min(a.k, h);
  } else {
    if (a.method == LCEMD_ICT) kef = h;
    else if (a.method == LCEMD_OMR) kef = min(2, h);
    else if (a.method == LCEMD_RWMD) kef = 1;
    else kef = min(a.k, h);
  }
  // list length during selection: exact path keeps k_eff, approximate keys
  // keep a margin of extra candidates for the exact re-sort
  const int sel_limit = PREC == PREC_F32 ? min(KL, kef) : min(KL, min(h, kef + a.KT_margin));
  constexpr bool kCapStop = PREC == PREC_F32 && MODE != P1_TABLE_FULL;

  // ---------------- contraction, pass by pass ----------------
  const unsigned char* base = PREC == PREC_F32 ? (const unsigned char*)a.V : (const unsigned char*)a.Vb;
  const size_t rowbytes = (size_t)a.m_pad * (PREC == PREC_F32 ? 4 : 2);
  // 128-byte slices that hold real dims (the zero padding past them would
  // add exact zeros)
  const int realbytes = 4 * a.m4 * (PREC == PREC_F32 ? 4 : 2);
  const int nsl = min((int)(rowbytes / 128), (realbytes + 127) / 128);
  unsigned char* stV = sm.u.st;
  unsigned char* stQ = sm.u.st + kRows * kStageStride;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 31, lh = lane >> 5;
  const int row = tid >> 2, sub = tid & 3;
  const bool row_ok = row < nrows;
  const float bound = row_ok ? sm.rbound[row] : 0.f;

  uint4 pv[2], pq[2];
  auto gload = [&](int c0, int sl) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int f = tid + it * kThreads;
      const int r = f >> 3, q = f & 7;
      pv[it] = make_uint4(0, 0, 0, 0);
      pq[it] = make_uint4(0, 0, 0, 0);
      if (r < nrows) pv[it] = *(const uint4*)(base + (size_t)sm.rid[r] * rowbytes + sl * 128 + q * 16);
      const int c = c0 + r;
      if (c < h) pq[it] = *(const uint4*)(base + (size_t)sm.cid[c] * rowbytes + sl * 128 + q * 16);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int f = tid + it * kThreads;
      const int r = f >> 3, q = f & 7;
      *(uint4*)(stV + r * kStageStride + q * 16) = pv[it];
      *(uint4*)(stQ + r * kStageStride + q * 16) = pq[it];
    }
  };

  int par = 0;
  gload(0, 0);
  for (int c0 = 0; c0 < h; c0 += kColChunk) {
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int sl = 0; sl < nsl; ++sl) {
      __syncthreads();
      lstore();
      __syncthreads();
      if (sl + 1 < nsl) gload(c0, sl + 1);
      else if (c0 + kColChunk < h) gload(c0 + kColChunk, 0);
      if constexpr (PREC == PREC_F32) {
        // lane half lh supplies dims [16*lh, 16*lh+16) of the 32-dim slice
        const float* ap = (const float*)(stV + (wr + li) * kStageStride) + 16 * lh;
        const float* bp = (const float*)(stQ + (wc + li) * kStageStride) + 16 * lh;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float4 av = *(const float4*)(ap + 4 * j);
          const float4 bv = *(const float4*)(bp + 4 * j);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.x, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv.y, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, bv.z, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, bv.w, acc, 0, 0, 0);
        }
      } else {
        // 64-dim slice: step s, lane half lh supplies dims [16s + 8lh, +8)
        const __bf16* ap = (const __bf16*)(stV + (wr + li) * kStageStride) + 8 * lh;
        const __bf16* bp = (const __bf16*)(stQ + (wc + li) * kStageStride) + 8 * lh;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const bf16x8 av = *(const bf16x8*)(ap + 16 * s);
          const bf16x8 bv = *(const bf16x8*)(bp + 16 * s);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
      }
    }
    __syncthreads();
    // keys of this pass: accumulator element r of lane (li, lh) is row
    // 8*(r/4) + 4*lh + r%4, column li of the wave's sub-tile
    {
      const int c = c0 + wc + li;
      const float qc = c < h ? sm.qn[c] : 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = wr + 8 * (r >> 2) + 4 * lh + (r & 3);
        sm.u.ck[i * kCKS + wc + li] = qc - 2.f * acc[r];
      }
    }
    __syncthreads();

    // ---- merge this pass into the per-row lists (4 lanes per row) ----
    uint64_t kk[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int c = c0 + sub + 4 * j;
      kk[j] = (row_ok && c < h) ? f_pack(sm.u.ck[row * kCKS + sub + 4 * j], (uint32_t)c) : ~0ull;
    }
    const uint64_t* cur = &sm.lst[par][row * KL];
    uint64_t* nxt = &sm.lst[par ^ 1][row * KL];
    const int len = row_ok ? sm.rlen[row] : 0;
    int ptr = 0, w = 0;
    float P = 0.f;
    uint64_t last = 0;
    bool act = row_ok;
    while (__any(act)) {
      uint64_t best = ~0ull;
      if (act) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (kk[j] > last && kk[j] < best) best = kk[j];
      }
      uint64_t o = shfl_xor64(best, 1);
      best = o < best ? o : best;
      o = shfl_xor64(best, 2);
      best = o < best ? o : best;
      if (act) {
        const uint64_t lc = ptr < len ? cur[ptr] : ~0ull;
        const uint64_t take = lc < best ? lc : best;
        if (take == ~0ull) {
          act = false;
        } else {
          if (lc < best) ++ptr;
          else last = best;
          if (sub == 0) nxt[w] = take;
          ++w;
          P += sm.cap[(uint32_t)take];
          bool stop = w >= sel_limit;
          if (kCapStop) stop = stop || P >= bound;
          if (stop) act = false;
        }
      }
    }
    __syncthreads();
    if (sub == 0 && row_ok) sm.rlen[row] = w;
    par ^= 1;
  }
  __syncthreads();

  // ---------------- final lists: exact distances where needed ----------
  const int len = row_ok ? sm.rlen[row] : 0;
  const uint64_t* lst = &sm.lst[par][row * KL];
  for (int l = sub; l < len; l += 4) {
    const uint64_t e = lst[l];
    const int pos = (int)(uint32_t)e;
    float d2 = sm.rvn[row] + f_unpack(e);
    bool need = PREC != PREC_F32 || !(d2 >= kGuard * (sm.rvn[row] + sm.qn[pos]));
    if (MODE != P1_TABLE_FULL && a.method == LCEMD_OMR && l == 0) need = true;
    if (need) d2 = exact_d2(a.V, a.m_pad, a.m4, sm.rid[row], sm.cid[pos]);
    sm.u.zb[row * KL + l] = d2;
  }
  __syncthreads();

  if (sub == 0 && row_ok) {
    uint64_t* L = &sm.lst[par][row * KL];
    float* Z2 = &sm.u.zb[row * KL];
    if constexpr (PREC != PREC_F32) {
      // re-sort by the exact squared distance (position breaks ties)
      for (int i = 1; i < len; ++i) {
        const uint64_t e = f_pack(Z2[i], (uint32_t)L[i]);
        int j = i - 1;
        while (j >= 0 && f_pack(Z2[j], (uint32_t)L[j]) > e) {
          L[j + 1] = L[j];
          Z2[j + 1] = Z2[j];
          --j;
        }
        L[j + 1] = e;
        Z2[j + 1] = f_unpack(e);
      }
    }
    // depth actually used by the row
    int D = 0;
    bool covered = false;
    {
      float Pc = 0.f;
      for (int l = 0; l < len; ++l) {
        ++D;
        Pc += sm.cap[(uint32_t)L[l]];
        if (D >= kef) { covered = true; break; }
        if (MODE != P1_TABLE_FULL) {
          if (Pc >= bound) { covered = true; break; }
          if (a.method == LCEMD_OMR && l == 0 && Z2[0] != 0.f) { covered = true; break; }
        }
      }
    }
    if (!covered && D < h && a.overflow) a.overflow[0] = 1;  // list too short (ICT only)
    if constexpr (MODE == P1_TABLE) {
      const int64_t flat = out_row0 + row;
      zw_write_row(a.ZW, a.zw_nq, a.KT, flat / a.v_used, flat % a.v_used, D,
                   [&](int l) { return sqrtf(fmaxf(Z2[l], 0.f)); },
                   [&](int l) { return l == D - 1 ? INFINITY : sm.cap[(uint32_t)L[l]]; });
      if (D > a.KT && a.overflow) a.overflow[0] = 1;
    } else if constexpr (MODE == P1_TABLE_FULL) {
      const int64_t o0 = (out_row0 + row) * (int64_t)a.k;
      for (int l = 0; l < a.k; ++l) {
        if (l < D) {
          const int pos = (int)(uint32_t)L[l];
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
        const float w = sm.cap[(uint32_t)L[l]];
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

// Persistent grid fed by per-XCD counters (as the 128-row kernel).
template <int MODE, int KL, int PREC>
__global__ __launch_bounds__(kThreads, 2) void k_phase1_fast(P1Args a, int64_t total) {
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
    fast_task<MODE, KL, PREC>(a, smem_raw, item);
  }
}

template <int MODE, int KL, int PREC>
static hipError_t launch_fast_one(const P1Args& a, hipStream_t s) {
  const size_t shmem = sizeof(FastSmem<KL>);
  const void* fn = (const void*)k_phase1_fast<MODE, KL, PREC>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  int64_t total;
  if (MODE == P1_PAIR) {
    total = a.npairs * (int64_t)a.rb_max;
  } else {
    const int64_t nrb = (a.v_used + kRows - 1) / kRows;
    total = (a.nq + kGroup - 1) / kGroup * nrb * kGroup;
  }
  if (total <= 0) return hipSuccess;
  if (!a.work_ctr) return hipErrorInvalidValue;
  e = launch_zero_ints((int*)a.work_ctr, 16, s);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid(fn, kThreads, shmem, total);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_phase1_fast<MODE, KL, PREC>), dim3(grid), dim3(kThreads), shmem, s, a, total);
  return hipGetLastError();
}

template <int MODE, int PREC>
static hipError_t launch_fast_mode(const P1Args& a, int KL, hipStream_t s) {
  if (KL <= 2) return launch_fast_one<MODE, 2, PREC>(a, s);
  if (KL <= 4) return launch_fast_one<MODE, 4, PREC>(a, s);
  if (KL <= 8) return launch_fast_one<MODE, 8, PREC>(a, s);
  if (KL <= 16) return launch_fast_one<MODE, 16, PREC>(a, s);
  if (KL <= 32) return launch_fast_one<MODE, 32, PREC>(a, s);
  if (KL <= 64) return launch_fast_one<MODE, 64, PREC>(a, s);
  return hipErrorInvalidValue;
}

template <int PREC>
static hipError_t launch_fast_prec(const P1Args& a, int mode, int KL, hipStream_t s) {
  switch (mode) {
    case P1_TABLE: return launch_fast_mode<P1_TABLE, PREC>(a, KL, s);
    case P1_TABLE_FULL: return launch_fast_mode<P1_TABLE_FULL, PREC>(a, KL, s);
    case P1_PAIR: return launch_fast_mode<P1_PAIR, PREC>(a, KL, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_phase1_fast(const P1Args& a, int mode, int KL, int prec, hipStream_t s) {
  if (prec == PREC_F32) return launch_fast_prec<PREC_F32>(a, mode, KL, s);
  if (prec == PREC_BF16) return hipErrorInvalidValue;  // bf16 keys: launch_phase1_bf16
  return hipErrorInvalidValue;
}

}  // namespace lcemd
