// Phase 2/3 of LC-ACT (Sec. 4, Eq. 6-9): for every non-zero X_ui of the
// database, the capacity-limited transfers of its mass against the query's
// table row for word i, summed per database row (document).
//
// Each table row holds (z, w) pairs in ascending distance order; its last
// valid entry carries w = +inf, so the walk below is Eq. (6)-(8) followed by
// Eq. (9) (the rest of the mass at the last distance) and always ends.
//
// Layout and mapping: a wave owns one database row at a time; its lanes
// stride over the row's non-zeros (coalesced 8-byte (word, weight) loads),
// apply a group of kQB queries' tables to each non-zero, then reduce across
// the wave with a fixed butterfly.  The per-row sum therefore has a fixed
// order that does not depend on which other queries or rows share the
// launch.
#include <algorithm>
#include <climits>
#include <mutex>
#include <vector>

#include "internal.h"

namespace lcemd {

// Queries per work item (one contiguous table run per non-zero): 16 when
// the database is large (fewer passes over X), 8 otherwise (half the
// registers, twice the resident waves for a latency-bound gather).
constexpr int kQBLarge = 16, kQBSmall = 8;
constexpr int64_t kLargeX = int64_t(64) << 20;  // bytes of X records
constexpr int kItemDocs = 16;  // database rows per work item of the persistent kernel

__device__ __forceinline__ float wave_sum(float t) {
  t += __shfl_xor(t, 32);
  t += __shfl_xor(t, 16);
  t += __shfl_xor(t, 8);
  t += __shfl_xor(t, 4);
  t += __shfl_xor(t, 2);
  t += __shfl_xor(t, 1);
  return t;
}

// One transfer step of Eq. (6)-(8) against table entry (z, w).
__device__ __forceinline__ void step(float& rem, float& acc, float z, float w) {
  const float r = fminf(rem, w);
  rem -= r;
  acc = fmaf(r, z, acc);
}

// Costs of database row u against queries q0 .. q0+nqb-1 (one wave).  For
// a non-zero of word r, the first pair of table entries of the kQB queries
// is one contiguous run (see zw_at); the kQB 16-byte loads are all issued
// before any is consumed (the walk along a row is a chain of dependent
// loads otherwise).  Entries past a row's sink are never used: the sink
// leaves no mass.
template <int kQB>
__device__ __forceinline__ void doc_costs(int lane, int64_t u, int64_t q0, int nqb,
                                          const int64_t* __restrict__ xptr,
                                          const int2* __restrict__ xcv,
                                          const float4* __restrict__ ZP, int64_t zw_nq, int KP,
                                          float* __restrict__ out, int64_t ld) {
  const int64_t e0 = xptr[u], e1 = xptr[u + 1];
  float t[kQB];
#pragma unroll
  for (int q = 0; q < kQB; ++q) t[q] = 0.f;
  for (int64_t e = e0 + lane; e < e1; e += 64) {
    const int2 cv = xcv[e];
    const float x = __int_as_float(cv.y);
    const float4* base = ZP + (int64_t)cv.x * KP * zw_nq + q0;
    float4 f[kQB];
#pragma unroll
    for (int q = 0; q < kQB; ++q) f[q] = base[min(q, nqb - 1)];
    // walk all queries one pair of entries at a time, so the loads of a
    // further pair for every query that still has mass go out together
    float rem[kQB], acc[kQB];
    bool any = false;
#pragma unroll
    for (int q = 0; q < kQB; ++q) {
      rem[q] = x;
      acc[q] = 0.f;
      step(rem[q], acc[q], f[q].x, f[q].y);
      if (rem[q] > 0.f) step(rem[q], acc[q], f[q].z, f[q].w);
      any = any || (q < nqb && rem[q] > 0.f);
    }
    for (int p = 1; any && p < KP; ++p) {
#pragma unroll
      for (int q = 0; q < kQB; ++q)
        if (q < nqb && rem[q] > 0.f) f[q] = base[p * zw_nq + q];
      any = false;
#pragma unroll
      for (int q = 0; q < kQB; ++q) {
        if (q < nqb && rem[q] > 0.f) {
          step(rem[q], acc[q], f[q].x, f[q].y);
          if (rem[q] > 0.f) step(rem[q], acc[q], f[q].z, f[q].w);
          any = any || rem[q] > 0.f;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kQB; ++q)
      if (q < nqb) t[q] += acc[q];
  }
#pragma unroll
  for (int q = 0; q < kQB; ++q) {
    const float s = wave_sum(t[q]);
    if (lane == 0 && q < nqb) out[(q0 + q) * ld + u] = s;
  }
}

// Persistent variant: a grid of resident workgroups whose waves pull
// (query group, kItemDocs database rows) items from eight work counters, one per
// XCD, each counter walking a contiguous eighth of the items (so an XCD
// keeps a few queries' tables hot in its L2).  For fixed-shape batches the
// live query count is read from device memory.  Every wave exits once its
// counter passes the end of its range.
template <int kQB>
__global__ __launch_bounds__(kThreads, kQB == kQBSmall ? 4 : 1) void k_phase2_persistent(
    const int64_t* __restrict__ xptr, const int2* __restrict__ xcv, int64_t n,
    const float4* __restrict__ ZP, int64_t zw_nq, int KP, int64_t nq_arg,
    const int* __restrict__ nq_dev, float* __restrict__ out, int64_t ld,
    unsigned long long* __restrict__ counters) {
  const int lane = threadIdx.x & 63;
  const int xcd = blockIdx.x & 7;
  const int64_t nq = nq_dev ? (int64_t)*nq_dev : nq_arg;
  const int64_t nd = (n + kItemDocs - 1) / kItemDocs;
  const int64_t total = (nq + kQB - 1) / kQB * nd;
  const int64_t lo = total * xcd / 8, hi = total * (xcd + 1) / 8;
  while (true) {
    unsigned long long it = 0;
    if (lane == 0) it = atomicAdd(&counters[xcd], 1ull);
    const int64_t item = lo + (int64_t)__shfl((long long)it, 0);
    if (item >= hi) break;
    const int64_t q0 = (item / nd) * kQB;
    const int nqb = (int)min((int64_t)kQB, nq - q0);
    const int64_t ubase = (item % nd) * kItemDocs;
    for (int j = 0; j < kItemDocs; ++j) {
      const int64_t u = ubase + j;
      if (u >= n) break;
      doc_costs<kQB>(lane, u, q0, nqb, xptr, xcv, ZP, zw_nq, KP, out, ld);
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
std::mutex g_occ_mu;
std::vector<OccEntry> g_occ;
int g_cus[64] = {0};
}  // namespace

int persistent_grid(const void* fn, int threads, size_t shmem, int64_t items) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  int per_cu = -1;
  {
    std::lock_guard<std::mutex> g(g_occ_mu);
    for (const OccEntry& e : g_occ)
      if (e.fn == fn && e.shmem == shmem && e.device == dev) per_cu = e.per_cu;
    if (!g_cus[dev] && hipDeviceGetAttribute(&g_cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -1;
    if (per_cu < 0) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, shmem) != hipSuccess) return -1;
      g_occ.push_back({fn, shmem, dev, per_cu});
    }
  }
  if (per_cu < 1) return -1;
  int64_t grid = (int64_t)per_cu * g_cus[dev];
  grid = std::min<int64_t>(grid, (items + 7) / 8 * 8);
  grid = std::max<int64_t>(8, (grid + 7) / 8 * 8);
  return (int)grid;
}

template <int kQB>
static hipError_t launch_p2(const int64_t* xptr, const int2* xcv, int64_t n, const float2* ZW,
                            int64_t zw_nq, int KT, int64_t nq, const int* nq_dev, float* out,
                            int64_t ld, unsigned long long* counters, hipStream_t s) {
  // items (one per wave) bound the grid when the batch size is known here
  const int64_t items = nq_dev ? INT64_MAX / 2 : (nq + kQB - 1) / kQB * ((n + kItemDocs - 1) / kItemDocs) * 64;
  const int grid = persistent_grid((const void*)k_phase2_persistent<kQB>, kThreads, 0, items);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_phase2_persistent<kQB>, dim3(grid), dim3(kThreads), 0, s, xptr, xcv, n,
                     (const float4*)ZW, zw_nq, (int)zw_pairs(KT), nq, nq_dev, out, ld, counters);
  return hipGetLastError();
}

hipError_t launch_phase2_persistent(const int64_t* xptr, const int2* xcv, int64_t n, int64_t nnz,
                                    const float2* ZW, int64_t zw_nq, int KT, int64_t nq,
                                    const int* nq_dev, float* out, int64_t ld,
                                    unsigned long long* counters, hipStream_t s) {
  if (n <= 0 || (!nq_dev && nq <= 0)) return hipSuccess;
  hipError_t e = launch_zero_ints((int*)counters, 16, s);
  if (e != hipSuccess) return e;
  if (nnz * 8 > kLargeX)
    return launch_p2<kQBLarge>(xptr, xcv, n, ZW, zw_nq, KT, nq, nq_dev, out, ld, counters, s);
  return launch_p2<kQBSmall>(xptr, xcv, n, ZW, zw_nq, KT, nq, nq_dev, out, ld, counters, s);
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
