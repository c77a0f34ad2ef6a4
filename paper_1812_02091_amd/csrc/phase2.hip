// Phase 2/3 of LC-ACT (Sec. 4, Eq. 6-9): for every non-zero X_ui of the
// database, the capacity-limited transfers of its mass against the query's
// table row for word i, summed per database row (document).
//
// Each table row holds (z, w) pairs in ascending distance order; its last
// valid entry carries w = +inf, so the walk below is Eq. (6)-(8) followed by
// Eq. (9) (the rest of the mass at the last distance) and always ends.
//
// Layout and mapping: a wave's 64 lanes are QL consecutive queries times
// 64/QL documents.  A lane walks its document's non-zeros in order, so the
// QL lanes of a document read one contiguous run of the table (QL entries of
// 16 bytes per non-zero, the interleaved layout) and every (query, document)
// sum has one fixed order: groups of eight consecutive non-zeros summed as a
// binary tree, the groups accumulated in order with Kahan compensation (the
// error stays a few ulps for rows of any length) -- the same bits whatever
// QL, the batch or the launch.  QL = 64 for batches of more
// than 32 queries (then a wave works on one document at a time); smaller
// batches put several documents in a wave, taken in order of length within
// windows of 128 documents (a permutation made when the database is loaded)
// so that the lanes of a wave finish together while its outputs stay close.
#include <algorithm>
#include <climits>
#include <mutex>
#include <vector>

#include "internal.h"

namespace lcemd {

constexpr int kUnroll = 8;       // non-zeros whose table loads are in flight together
constexpr int kItemSlots = 16;   // document slots per lane and work item
static_assert(kItemSlots % 4 == 0, "results are stored four at a time");

// One transfer step of Eq. (6)-(8) against table entry (z, w).  rem >= +0
// (never -0: rem - rem is +0) and w > 0 (or +inf), so the smaller float is
// the smaller bit pattern: one integer minimum (fminf would first
// canonicalise both operands).  A step with rem = +0 changes nothing
// (r = +0, acc + 0 z = acc for finite z >= 0): so the second entry of a
// table row's first 16-byte pair, which is always written (as (0, 0) when
// the row has one entry), is stepped without testing rem; later pairs are
// read only while some mass remains (their entries past the row's sink are
// never written).
__device__ __forceinline__ void step(float& rem, float& acc, float z, float w) {
  const float r = __uint_as_float(min(__float_as_uint(rem), __float_as_uint(w)));
  rem -= r;
  acc = fmaf(r, z, acc);
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Cost of document u against query q (one lane): the non-zeros in order,
// kUnroll at a time with their first table pairs loaded together; further
// pairs are loaded together for every non-zero that still has mass.
// Entries past a row's sink are never used: the sink leaves no mass.
// kUni: every lane of the wave is on this document, so its records and the
// table row offsets are wave-uniform (scalar loads and arithmetic).
// kGroup: the QL >= 8 lanes from `glane` on share the document: its first
// lanes load one record each and the group reads them by lane shuffle
// (every lane of the group runs this with the same e0, e1).  kSolo (QL < 8):
// every lane loads its document's records itself.
enum { kUni = 0, kGroup = 1, kSolo = 2 };
template <int RM>
__device__ __forceinline__ float doc_cost(int64_t e0, int64_t e1, const int2* __restrict__ xcv,
                                          const float4* __restrict__ Zq, int64_t zw_nq, int KP,
                                          int lane, int glane) {
  static_assert(kUnroll == 8, "the group sum below is a tree over 8 terms");
  constexpr bool UNI = RM == kUni;
  if constexpr (UNI) {
    e0 = uniform64(e0);
    e1 = uniform64(e1);
  }
  const int64_t rstride = (int64_t)KP * zw_nq;  // float4s from one word's run to the next
  float t = 0.f, comp = 0.f;
  for (int64_t e = e0; e < e1; e += kUnroll) {
    const int cnt = (int)min((int64_t)kUnroll, e1 - e);
    int2 cv[kUnroll];
    if constexpr (UNI) {
      if (cnt == kUnroll) {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) cv[k] = xcv[e + k];
      } else {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) cv[k] = k < cnt ? xcv[e + k] : make_int2(0, 0);
      }
    } else if constexpr (RM == kGroup) {
      const int j = lane - glane;
      const int2 rec = j < cnt ? xcv[e + j] : make_int2(0, 0);
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        cv[k].x = __shfl(rec.x, glane + k);
        cv[k].y = __shfl(rec.y, glane + k);
      }
    } else {
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) cv[k] = k < cnt ? xcv[e + k] : make_int2(0, 0);
    }
    const float4* base[kUnroll];
    float4 f[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int w = UNI ? __builtin_amdgcn_readfirstlane(cv[k].x) : cv[k].x;
      base[k] = Zq + (int64_t)w * rstride;
      f[k] = k < cnt ? base[k][0] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float rem[kUnroll], acc[kUnroll];
    bool any = false;
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      rem[k] = __int_as_float(cv[k].y);  // 0 for the padding slots
      acc[k] = 0.f;
      step(rem[k], acc[k], f[k].x, f[k].y);
      step(rem[k], acc[k], f[k].z, f[k].w);
      any = any || rem[k] > 0.f;
    }
    for (int p = 1; any && p < KP; ++p) {
#pragma unroll
      for (int k = 0; k < kUnroll; ++k)
        if (rem[k] > 0.f) f[k] = base[k][p * zw_nq];
      any = false;
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        if (rem[k] > 0.f) {
          step(rem[k], acc[k], f[k].x, f[k].y);
          if (rem[k] > 0.f) step(rem[k], acc[k], f[k].z, f[k].w);
          any = any || rem[k] > 0.f;
        }
      }
    }
    // padding slots hold exact zeros
    const float g = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    const float y = g - comp;
    const float tt = t + y;
    comp = (tt - t) - y;
    t = tt;
  }
  return t;
}

// Persistent grid: waves pull (query group of QL, 64/QL x kItemSlots
// documents) items from eight work counters, one per XCD, each walking a
// contiguous eighth of the items, query group major (an XCD keeps one
// group's slice of the tables hot in its L2).  For fixed-shape batches the
// live query count is read from device memory, and the launcher issues one
// kernel per lane width: the one whose band (QL/2, QL] holds the live count
// works, the others return at once (so a batch with few live queries does
// not pay for the lanes of its empty slots).  Every wave exits once its
// counter passes the end of its range.
template <int QL>
__global__ __launch_bounds__(kThreads) void k_phase2_persistent(
    const int64_t* __restrict__ xptr, const int2* __restrict__ xcv, int64_t n,
    const int32_t* __restrict__ perm, const float4* __restrict__ ZP, int64_t zw_nq, int KP,
    int64_t nq_arg, const int* __restrict__ nq_dev, float* __restrict__ out, int64_t ld,
    unsigned long long* __restrict__ counters) {
  constexpr int S = 64 / QL;  // documents side by side
  constexpr int64_t kDocs = (int64_t)S * kItemSlots;
  const int lane = threadIdx.x & 63, qs = lane % QL, ds = lane / QL;
  const int xcd = blockIdx.x & 7;
  const int64_t nq = nq_dev ? (int64_t)*nq_dev : nq_arg;
  if (nq_dev && (nq > nq_arg || (QL > 1 && 2 * nq <= QL))) return;  // another width's band
  const int64_t nd = (n + kDocs - 1) / kDocs;
  const int64_t total = (nq + QL - 1) / QL * nd;
  const int64_t lo = total * xcd / 8, hi = total * (xcd + 1) / 8;
  while (true) {
    unsigned long long it = 0;
    if (lane == 0) it = atomicAdd(&counters[xcd], 1ull);
    const int64_t item = uniform64(lo + (int64_t)__shfl((long long)it, 0));
    if (item >= hi) break;
    // lanes past the batch walk the last query's table (so every lane of a
    // document group takes part in its record shuffles) and write nothing
    const int64_t q = (item / nd) * QL + qs;
    const bool qok = q < nq;
    const float4* Zq = ZP + (qok ? q : nq - 1);
    const int64_t d0 = (item % nd) * kDocs + ds;
    if constexpr (S == 1) {
      // one document at a time for all 64 lanes: each lane's kItemSlots
      // results are consecutive in its query's row, so they are staged in
      // the wave's own LDS rows (lane-private slots: no barrier) and written
      // together, 16-byte stores where aligned
      __shared__ float st[kThreads / 64][kItemSlots][64];
      float(*sw)[64] = st[threadIdx.x >> 6];
      int cnt = 0;
      for (int j = 0; j < kItemSlots; ++j) {
        const int64_t i = d0 + j;
        if (i >= n) break;
        sw[j][lane] = doc_cost<kUni>(xptr[i], xptr[i + 1], xcv, Zq, zw_nq, KP, lane, 0);
        ++cnt;
      }
      if (qok && cnt > 0) {
        float* o = out + q * ld + d0;
        if (cnt == kItemSlots && (reinterpret_cast<uintptr_t>(o) & 15) == 0) {
#pragma unroll
          for (int t = 0; t < kItemSlots; t += 4)
            *reinterpret_cast<float4*>(o + t) = make_float4(sw[t][lane], sw[t + 1][lane], sw[t + 2][lane], sw[t + 3][lane]);
        } else {
          for (int t = 0; t < cnt; ++t) o[t] = sw[t][lane];
        }
      }
    } else {
      for (int j = 0; j < kItemSlots; ++j) {
        const int64_t i = d0 + (int64_t)j * S;
        if (i >= n) break;
        const int64_t u = (int64_t)perm[i];
        const float c = doc_cost<(QL >= kUnroll ? kGroup : kSolo)>(xptr[u], xptr[u + 1], xcv, Zq, zw_nq, KP,
                                                                   lane, ds * QL);
        if (qok) out[q * ld + u] = c;
      }
    }
  }
}

__global__ void k_zero_ints(int* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ints, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
  return hipGetLastError();
}

namespace {
struct OccEntry {
  const void* fn;
  size_t shmem;
  int device;
  int per_cu;
};
// a fixed table (no allocation at launch time); once full, further
// kernels are queried at every launch
constexpr int kOccCap = 512;
std::mutex g_occ_mu;
OccEntry g_occ[kOccCap];
int g_nocc = 0;
int g_cus[64] = {0};
}  // namespace

int persistent_grid(const void* fn, int threads, size_t shmem, int64_t items) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  int per_cu = -1;
  {
    std::lock_guard<std::mutex> g(g_occ_mu);
    for (int i = 0; i < g_nocc; ++i)
      if (g_occ[i].fn == fn && g_occ[i].shmem == shmem && g_occ[i].device == dev) per_cu = g_occ[i].per_cu;
    if (!g_cus[dev] && hipDeviceGetAttribute(&g_cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -1;
    if (per_cu < 0) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, shmem) != hipSuccess) return -1;
      if (g_nocc < kOccCap) g_occ[g_nocc++] = OccEntry{fn, shmem, dev, per_cu};
    }
  }
  if (per_cu < 1) return -1;
  int64_t grid = (int64_t)per_cu * g_cus[dev];
  grid = std::min<int64_t>(grid, (items + 7) / 8 * 8);
  grid = std::max<int64_t>(8, (grid + 7) / 8 * 8);
  return (int)grid;
}

template <int QL>
static hipError_t launch_p2(const int64_t* xptr, const int2* xcv, int64_t n, const int32_t* perm,
                            const float2* ZW, int64_t zw_nq, int KT, int64_t nq, const int* nq_dev,
                            float* out, int64_t ld, unsigned long long* counters, hipStream_t s) {
  // waves needed at most (bounds the grid)
  const int64_t items = (nq + QL - 1) / QL * ((n + (64 / QL) * kItemSlots - 1) / ((64 / QL) * kItemSlots));
  const int grid = persistent_grid((const void*)k_phase2_persistent<QL>, kThreads, 0, (items + 3) / 4);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_phase2_persistent<QL>, dim3(grid), dim3(kThreads), 0, s, xptr, xcv, n, perm,
                     (const float4*)ZW, zw_nq, (int)zw_pairs(KT), nq, nq_dev, out, ld, counters);
  return hipGetLastError();
}

hipError_t launch_phase2_persistent(const int64_t* xptr, const int2* xcv, int64_t n, const int32_t* perm,
                                    const float2* ZW, int64_t zw_nq, int KT, int64_t nq,
                                    const int* nq_dev, float* out, int64_t ld,
                                    unsigned long long* counters, hipStream_t s) {
  // nq: the batch size, or with nq_dev the largest live count
  if (n <= 0 || nq <= 0) return hipSuccess;
  hipError_t e = launch_zero_ints((int*)counters, 16, s);
  if (e != hipSuccess) return e;
  if (nq <= 32 && !perm) return hipErrorInvalidValue;
  // lane width: the smallest power of two >= the queries (at most 64); with
  // a device-side live count, every width up to that one (each works only
  // for live counts in its band)
  int top = 1;
  while (top < 64 && top < nq) top *= 2;
  for (int ql = top; ql >= (nq_dev ? 1 : top); ql /= 2) {
    const int64_t qmax = ql == top ? nq : std::min<int64_t>(nq, ql);  // the most queries this width takes
    switch (ql) {
      case 64: e = launch_p2<64>(xptr, xcv, n, perm, ZW, zw_nq, KT, qmax, nq_dev, out, ld, counters, s); break;
      case 32: e = launch_p2<32>(xptr, xcv, n, perm, ZW, zw_nq, KT, qmax, nq_dev, out, ld, counters, s); break;
      case 16: e = launch_p2<16>(xptr, xcv, n, perm, ZW, zw_nq, KT, qmax, nq_dev, out, ld, counters, s); break;
      case 8: e = launch_p2<8>(xptr, xcv, n, perm, ZW, zw_nq, KT, qmax, nq_dev, out, ld, counters, s); break;
      case 4: e = launch_p2<4>(xptr, xcv, n, perm, ZW, zw_nq, KT, qmax, nq_dev, out, ld, counters, s); break;
      case 2: e = launch_p2<2>(xptr, xcv, n, perm, ZW, zw_nq, KT, qmax, nq_dev, out, ld, counters, s); break;
      default: e = launch_p2<1>(xptr, xcv, n, perm, ZW, zw_nq, KT, qmax, nq_dev, out, ld, counters, s); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Word-major phase 2 for large vocabularies.  When a query group's tables
// are far larger than the caches, the per-document walk above re-reads a
// word's table run from HBM for every document that holds the word.  Here
// the same transfers run in two passes over one group of 64 queries:
//  A. the database's non-zeros word by word (their weights grouped by word,
//     made at load): a wave keeps the 64 queries' table run of the current
//     word in registers (pairs loaded as some lane's walk first needs them)
//     and writes each non-zero's 64 costs as one 256-byte row, in the same
//     by-word order (a sequential stream);
//  B. the documents in order: every (query, document) sum takes the costs
//     of its non-zeros in CSR order (each non-zero's by-word index from a
//     map made at load) with the grouping and compensation of doc_cost
//     (eight-term trees, Kahan across groups).
// The walk in A is the same sequence of step() calls as in doc_cost, so
// the results are the same bits whichever phase 2 ran.
constexpr int kWmSpan = 2048;  // non-zeros per pass-A wave (a fixed range: no work counter)

// Pass A.  Wave w takes the by-word records [w kWmSpan, (w + 1) kWmSpan),
// which may span many words; a lane per query.  The next two words' first
// table pairs and end offsets are in flight while the current word runs,
// and the next 64 weights while the current 64 are walked.
template <int KPM>
__global__ __launch_bounds__(kThreads) void k_p2_word_costs(
    const int64_t* __restrict__ wptr, const float* __restrict__ wwt, int64_t nnz, int64_t v_used,
    const float4* __restrict__ ZP, int64_t zw_nq, int KP, float* __restrict__ cost) {
  const int lane = threadIdx.x & 63;
  // the wave's index, made visibly wave-uniform (its range, offsets and
  // counts then live in scalar registers)
  const int64_t gw = (int64_t)blockIdx.x * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t e0 = gw * kWmSpan, e1 = min(nnz, e0 + kWmSpan);
  if (e0 >= e1) return;
  // the word of e0: the last p with wptr[p] <= e0 (wave-uniform search)
  int64_t lo = 0, hi = v_used;  // wptr[lo] <= e0 < wptr[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (uniform64(wptr[mid]) <= e0) lo = mid;
    else hi = mid;
  }
  int64_t word = lo;
  int64_t wend = uniform64(wptr[word + 1]);
  // indices past the last word are clamped to it: those loads are never used
  // (no record lies past the last word), and plain loads of valid rows keep
  // the compiler from selecting between pointers
  const int64_t lastw = v_used - 1;
  int64_t nend = uniform64(wptr[min(word + 2, v_used)]);
  int64_t nend2 = uniform64(wptr[min(word + 3, v_used)]);
  const int64_t rs = (int64_t)KP * zw_nq;  // float4s from one word's run to the next
  const float4* run = ZP + word * rs + lane;
  float4 f[KPM];
  f[0] = run[0];
  float4 fn = ZP[min(word + 1, lastw) * rs + lane];
  float4 fn2 = ZP[min(word + 2, lastw) * rs + lane];
  int loaded = 1;
  // weights come 64 at a time, one per lane (the next 64 in flight while
  // these are walked), and are read out to every lane by readlane
  float wcur = e0 + lane < e1 ? wwt[e0 + lane] : 0.f, wnext = 0.f;
  for (int64_t e = e0; e < e1; e += kUnroll) {
    const int cnt = (int)min((int64_t)kUnroll, e1 - e);
    const int off = (int)((e - e0) & 63);
    if (off == 0 && e + 64 < e1) wnext = e + 64 + lane < e1 ? wwt[e + 64 + lane] : 0.f;
    const float wcur0 = wcur;  // this batch's block of weights
    float rec[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k)
      rec[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wcur), off + k));
    if (off + kUnroll == 64) wcur = wnext;
    float* cb = cost + e * 64 + lane;  // this batch's cost rows (offsets k * 256 bytes)
    if (e + cnt <= wend) {
      // the whole batch on the current word: the eight walks side by side,
      // pair by pair (the same steps per walk as one at a time)
      float rem[kUnroll], acc[kUnroll];
      bool any = false;
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        rem[k] = rec[k];  // 0 past the range: the weight blocks hold 0 there
        acc[k] = 0.f;
        step(rem[k], acc[k], f[0].x, f[0].y);
        step(rem[k], acc[k], f[0].z, f[0].w);
        any = any || rem[k] > 0.f;
      }
#pragma unroll
      for (int p = 1; p < KPM; ++p) {
        if (p >= KP || !__any(any)) break;
        if (p >= loaded) {
          f[p] = run[p * zw_nq];
          loaded = p + 1;
        }
        any = false;
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          if (rem[k] > 0.f) {
            step(rem[k], acc[k], f[p].x, f[p].y);
            if (rem[k] > 0.f) step(rem[k], acc[k], f[p].z, f[p].w);
            any = any || rem[k] > 0.f;
          }
        }
      }
      if (cnt == kUnroll) {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) cb[k * 64] = acc[k];
      } else {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k)
          if (k < cnt) cb[k * 64] = acc[k];
      }
      continue;
    }
    // the batch crosses into later words: one walk at a time
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      if (k >= cnt) break;
      const int64_t ee = e + k;
      if (ee >= wend) {  // the next word (wave-uniform)
        ++word;
        if (ee < nend) {
          f[0] = fn;
          fn = fn2;
          wend = nend;
          nend = nend2;
        } else {  // words without records (none in a loaded database): search on
          while (uniform64(wptr[word + 1]) <= ee) ++word;
          wend = uniform64(wptr[word + 1]);
          f[0] = ZP[word * rs + lane];
          fn = ZP[min(word + 1, lastw) * rs + lane];
          nend = uniform64(wptr[min(word + 2, v_used)]);
        }
        run = ZP + word * rs + lane;
        loaded = 1;
        nend2 = uniform64(wptr[min(word + 3, v_used)]);
        fn2 = ZP[min(word + 2, lastw) * rs + lane];
      }
      float rem = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wcur0), off + k)), acc = 0.f;
      step(rem, acc, f[0].x, f[0].y);
      step(rem, acc, f[0].z, f[0].w);
#pragma unroll
      for (int p = 1; p < KPM; ++p) {
        if (p >= KP || !__any(rem > 0.f)) break;
        if (p >= loaded) {  // the first walk to reach this pair loads it for the wave
          f[p] = run[p * zw_nq];
          loaded = p + 1;
        }
        if (rem > 0.f) {
          step(rem, acc, f[p].x, f[p].y);
          if (rem > 0.f) step(rem, acc, f[p].z, f[p].w);
        }
      }
      cb[k * 64] = acc;
    }
  }
}

// Pass B: one wave per kItemSlots consecutive documents, a lane per query.
__global__ __launch_bounds__(kThreads) void k_p2_doc_sums(const int64_t* __restrict__ xptr, int64_t n,
                                                          const uint32_t* __restrict__ winv,
                                                          const float* __restrict__ cost, float* __restrict__ out,
                                                          int64_t ld, unsigned long long* __restrict__ counters) {
  __shared__ float st[kThreads / 64][kItemSlots][64];
  float(*sw)[64] = st[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;
  const int xcd = blockIdx.x & 7;
  const int64_t total = (n + kItemSlots - 1) / kItemSlots;
  const int64_t lo = total * xcd / 8, hi = total * (xcd + 1) / 8;
  while (true) {
    unsigned long long it = 0;
    if (lane == 0) it = atomicAdd(&counters[8 + xcd], 1ull);
    const int64_t item = uniform64(lo + (int64_t)__shfl((long long)it, 0));
    if (item >= hi) break;
    const int64_t d0 = item * kItemSlots;
    int cnt = 0;
    for (int j = 0; j < kItemSlots; ++j) {
      const int64_t u = d0 + j;
      if (u >= n) break;
      const int64_t e0 = uniform64(xptr[u]), e1 = uniform64(xptr[u + 1]);
      float t = 0.f, comp = 0.f;
      int wv = 0;  // 64 by-word indices at a time, one per lane
      for (int64_t e = e0; e < e1; e += kUnroll) {
        const int c8 = (int)min((int64_t)kUnroll, e1 - e);
        const int off = (int)((e - e0) & 63);
        if (off == 0) wv = e + lane < e1 ? (int)winv[e + lane] : 0;
        float x[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          const uint32_t wi = (uint32_t)__builtin_amdgcn_readlane(wv, off + k);
          x[k] = k < c8 ? cost[(int64_t)wi * 64 + lane] : 0.f;
        }
        const float g = ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
        const float y = g - comp;
        const float tt = t + y;
        comp = (tt - t) - y;
        t = tt;
      }
      sw[j][lane] = t;
      ++cnt;
    }
    float* o = out + (int64_t)lane * ld + d0;
    if (cnt == kItemSlots && (reinterpret_cast<uintptr_t>(o) & 15) == 0) {
#pragma unroll
      for (int t = 0; t < kItemSlots; t += 4)
        *reinterpret_cast<float4*>(o + t) = make_float4(sw[t][lane], sw[t + 1][lane], sw[t + 2][lane], sw[t + 3][lane]);
    } else {
      for (int t = 0; t < cnt; ++t) o[t] = sw[t][lane];
    }
  }
}

hipError_t launch_phase2_wordmajor(const int64_t* xptr, int64_t n, const int64_t* wptr, const float* wwt,
                                   const uint32_t* winv, int64_t nnz, int64_t v_used, const float2* ZW,
                                   int64_t zw_nq, int KT, float* cost, float* out, int64_t ld,
                                   unsigned long long* counters, hipStream_t s) {
  // one group of 64 queries: ZW and out start at the group's first query
  const int KP = (int)zw_pairs(KT);
  if (n <= 0 || nnz <= 0 || v_used <= 0) return hipSuccess;
  if (KP > 8 || nnz > 0xffffffffLL) return hipErrorInvalidValue;
  hipError_t e = launch_zero_ints((int*)counters, 32, s);
  if (e != hipSuccess) return e;
  const int64_t waves = (nnz + kWmSpan - 1) / kWmSpan;
  const dim3 ga((unsigned)((waves + kThreads / 64 - 1) / (kThreads / 64)));
  if (KP <= 4)
    hipLaunchKernelGGL(k_p2_word_costs<4>, ga, dim3(kThreads), 0, s, wptr, wwt, nnz, v_used, (const float4*)ZW,
                       zw_nq, KP, cost);
  else
    hipLaunchKernelGGL(k_p2_word_costs<8>, ga, dim3(kThreads), 0, s, wptr, wwt, nnz, v_used, (const float4*)ZW,
                       zw_nq, KP, cost);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t itemsB = (n + kItemSlots - 1) / kItemSlots;
  const int gb = persistent_grid((const void*)k_p2_doc_sums, kThreads, 0, (itemsB + 3) / 4);
  if (gb <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_p2_doc_sums, dim3(gb), dim3(kThreads), 0, s, xptr, n, winv, cost, out, ld, counters);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_max_inplace(float* a, const float* b, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < count) a[i] = fmaxf(a[i], b[i]);
}

hipError_t launch_max_inplace(float* a, const float* b, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_max_inplace, dim3((unsigned)((count + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, a, b, count);
  return hipGetLastError();
}

}  // namespace lcemd
