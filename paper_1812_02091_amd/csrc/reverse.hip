// The reverse direction by the linear method (Q2D with the roles of Sec. 4
// swapped): the query batch becomes the histogram set whose non-zeros
// phase 2 walks.  These kernels build its records on the device -- the
// used words in ascending order (the batch's own vocabulary, Sec. 2.2), the
// (compact word id, weight) record of every non-zero, the largest weight of
// every used word (the depth bound of Lemma 1) and the rows ordered by
// length within windows of 128 -- so that no copy of the batch goes through
// the host.
#include "internal.h"

namespace lcemd {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;  // flags per thread
constexpr int kScanBlock = kScanThreads * kScanItems;

// wmax[w] = bits of the largest weight of word w in the batch (weights are
// > 0, so their bits order like the values and 0 means "unused")
__global__ __launch_bounds__(256) void k_rev_wmax(const int32_t* __restrict__ col, const float* __restrict__ val,
                                                  int64_t H, unsigned int* __restrict__ wmax) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < H) atomicMax(&wmax[col[i]], __float_as_uint(val[i]));
}

__global__ __launch_bounds__(256) void k_rev_zero(unsigned int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Block-local exclusive scan of the used flags; the block's total to bsum.
__global__ __launch_bounds__(kScanThreads) void k_rev_scan_local(const unsigned int* __restrict__ wmax, int64_t v,
                                                                 int* __restrict__ pos, int* __restrict__ bsum) {
  __shared__ int wsum[kScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)t * kScanItems;
  int f[kScanItems], s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    f[j] = (base + j < v && wmax[base + j] != 0u) ? 1 : 0;
    s += f[j];
  }
  // inclusive scan of the per-thread sums across the wave, then the waves
  int x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int w = lane < kScanThreads / 64 ? wsum[lane] : 0;
#pragma unroll
    for (int o = 1; o < kScanThreads / 64; o <<= 1) {
      const int y = __shfl_up(w, o);
      if (lane >= o) w += y;
    }
    if (lane < kScanThreads / 64) wsum[lane] = w;  // inclusive wave totals
  }
  __syncthreads();
  int run = x - s + (wave > 0 ? wsum[wave - 1] : 0);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < v) pos[base + j] = run;
    run += f[j];
  }
  if (t == kScanThreads - 1) bsum[blockIdx.x] = run;
}

// Exclusive scan of the block totals, one block, any count; the grand total
// (the used word count) to *nu.
__global__ __launch_bounds__(kScanThreads) void k_rev_scan_blocks(int* __restrict__ bsum, int nb,
                                                                  int* __restrict__ nu) {
  __shared__ int wsum[kScanThreads / 64];
  __shared__ int carry;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int s = b0 + t < nb ? bsum[b0 + t] : 0;
    int x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (wave == 0) {
      int w = lane < kScanThreads / 64 ? wsum[lane] : 0;
#pragma unroll
      for (int o = 1; o < kScanThreads / 64; o <<= 1) {
        const int y = __shfl_up(w, o);
        if (lane >= o) w += y;
      }
      if (lane < kScanThreads / 64) wsum[lane] = w;
    }
    __syncthreads();
    const int excl = carry + x - s + (wave > 0 ? wsum[wave - 1] : 0);
    if (b0 + t < nb) bsum[b0 + t] = excl;
    __syncthreads();  // every thread has read carry and wsum
    if (t == kScanThreads - 1) carry = excl + s;
    __syncthreads();
  }
  if (t == 0) *nu = carry;
}

// Used words in ascending order with their largest weights.
__global__ __launch_bounds__(256) void k_rev_used(const unsigned int* __restrict__ wmax, const int* __restrict__ pos,
                                                  const int* __restrict__ bsum, int64_t v, int32_t* __restrict__ used,
                                                  float* __restrict__ xmax) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= v || wmax[w] == 0u) return;
  const int p = pos[w] + bsum[w / kScanBlock];
  used[p] = (int32_t)w;
  xmax[p] = __uint_as_float(wmax[w]);
}

__global__ __launch_bounds__(256) void k_rev_records(const int32_t* __restrict__ col, const float* __restrict__ val,
                                                     int64_t H, const int* __restrict__ pos,
                                                     const int* __restrict__ bsum, int2* __restrict__ cv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= H) return;
  const int w = col[i];
  cv[i] = make_int2(pos[w] + bsum[w / kScanBlock], __float_as_int(val[i]));
}

// Rows by length within windows of 128 (stable: equal lengths keep their
// order), one window per block.
__global__ __launch_bounds__(128) void k_rev_perm(const int64_t* __restrict__ ptr, int64_t B,
                                                  int32_t* __restrict__ perm) {
  __shared__ int64_t len[128];
  const int64_t w0 = (int64_t)blockIdx.x * 128;
  const int t = threadIdx.x;
  const int cnt = (int)min<int64_t>(128, B - w0);
  if (t < cnt) len[t] = ptr[w0 + t + 1] - ptr[w0 + t];
  __syncthreads();
  if (t >= cnt) return;
  int r = 0;
  for (int j = 0; j < cnt; ++j) r += (len[j] < len[t] || (len[j] == len[t] && j < t)) ? 1 : 0;
  perm[w0 + r] = (int32_t)(w0 + t);
}

}  // namespace

int64_t reverse_scratch_ints(int64_t v) { return 2 * v + (v + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_reverse_records(const int64_t* ptr, const int32_t* col, const float* val, int64_t B, int64_t H,
                                  int64_t v, int* scratch, int2* cv, int32_t* used, float* xmax, int32_t* perm,
                                  int* nu, hipStream_t s) {
  if (B < 1 || H < 1 || v < 1) return hipErrorInvalidValue;
  unsigned int* wmax = reinterpret_cast<unsigned int*>(scratch);
  int* pos = scratch + v;
  int* bsum = scratch + 2 * v;
  const int nb = (int)((v + kScanBlock - 1) / kScanBlock);
  const unsigned g256v = (unsigned)((v + 255) / 256), g256h = (unsigned)((H + 255) / 256);
  hipLaunchKernelGGL(k_rev_zero, dim3(g256v), dim3(256), 0, s, wmax, v);
  hipLaunchKernelGGL(k_rev_wmax, dim3(g256h), dim3(256), 0, s, col, val, H, wmax);
  hipLaunchKernelGGL(k_rev_scan_local, dim3(nb), dim3(kScanThreads), 0, s, wmax, v, pos, bsum);
  hipLaunchKernelGGL(k_rev_scan_blocks, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, nu);
  hipLaunchKernelGGL(k_rev_used, dim3(g256v), dim3(256), 0, s, wmax, pos, bsum, v, used, xmax);
  hipLaunchKernelGGL(k_rev_records, dim3(g256h), dim3(256), 0, s, col, val, H, pos, bsum, cv);
  hipLaunchKernelGGL(k_rev_perm, dim3((unsigned)((B + 127) / 128)), dim3(128), 0, s, ptr, B, perm);
  return hipGetLastError();
}

}  // namespace lcemd
