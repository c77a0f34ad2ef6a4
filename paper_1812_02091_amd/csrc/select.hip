// Top-l selection (Sec. 5: the l nearest database histograms per query) and
// the exact symmetric search.
//
// Keys are packed as (order-preserving bits of the float32 distance) << 32
// | database row index, so one unsigned comparison orders by (distance,
// index) and ties go to the lower index.  Selection keeps a running best
// list at the front of an LDS buffer, refills the rest with the next chunk
// of a query's distances and bitonic-sorts the buffer.
//
// Symmetric top-l (Sec. 2.1/5: SYM = max(D2Q, Q2D) >= D2Q): the first L
// candidates by D2Q get their Q2D evaluated; the l best by SYM among them
// are exact as soon as the (L+1)-th candidate's D2Q key exceeds the l-th
// best SYM key, since every other row's SYM key is at least its D2Q key.
// Rows for which that certificate fails are flagged for a wider pass.
#include <algorithm>

#include "internal.h"

namespace lcemd {

__device__ __forceinline__ uint32_t order_bits_s(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint64_t pack_s(float f, uint32_t idx) {
  return ((uint64_t)order_bits_s(f) << 32) | (uint64_t)idx;
}
__device__ __forceinline__ float unpack_f(uint64_t k) {
  const uint32_t o = (uint32_t)(k >> 32);
  const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}

// Ascending bitonic sort of N (power of two) keys in LDS by all threads.
__device__ void bitonic_sort(uint64_t* buf, int N) {
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N / 2; i += kThreads) {
        const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const int hi = lo + j;
        const bool asc = (lo & k) == 0;
        const uint64_t x = buf[lo], y = buf[hi];
        if ((x > y) == asc) {
          buf[lo] = y;
          buf[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Threshold selection of the L smallest keys of one part of a row.  The
// buffer holds the best L keys found so far (sorted, at the front) followed
// by unsorted newcomers; a key enters only if it beats the threshold, so
// after the first round almost nothing is inserted and the pass runs at the
// speed of the coalesced reads.  The first threshold is the L-th smallest of
// the first round's per-thread minima (at least L keys lie at or below it,
// so every one of the L smallest does); later ones are the L-th best at a
// compaction, a bitonic sort of the occupied front of the buffer, which runs
// when the next round could overflow it.  Keys are unique (row index in the
// low bits), so the result is the exact L smallest in (distance, index)
// order.
constexpr int kSelBuf = 4096;
constexpr int kSelPer = 8;                      // keys per thread per round
constexpr int kSelRound = kSelPer * kThreads;   // 2048
constexpr int64_t kSelPart = 32768;             // keys per workgroup in the first pass

__device__ __forceinline__ void sel_compact(uint64_t* buf, int* cnt, uint64_t* thr, int L) {
  int N = 2;
  while (N < *cnt) N <<= 1;
  bitonic_sort(buf, N);  // entries at or past *cnt are ~0 and stay at the back
  const int old = *cnt, keep = min(old, L);
  __syncthreads();
  for (int i = keep + (int)threadIdx.x; i < old; i += kThreads) buf[i] = ~0ull;
  if (threadIdx.x == 0) {
    *cnt = keep;
    *thr = keep >= L ? buf[L - 1] : ~0ull;
  }
  __syncthreads();
}

// PACKED: keys are already packed (a second pass over first-pass results);
// otherwise float32 distances of row b, packed with their index here.
template <bool PACKED>
__global__ __launch_bounds__(kThreads) void k_select(const void* __restrict__ keys_, int64_t ld,
                                                     int64_t n, int L,
                                                     const int32_t* __restrict__ row_list,
                                                     int64_t exclude_base, int64_t part_len,
                                                     uint64_t* __restrict__ out) {
  __shared__ uint64_t buf[kSelBuf];
  __shared__ uint64_t mins[kThreads];
  __shared__ int cnt;
  __shared__ uint64_t thr;
  const int64_t ri = blockIdx.x, part = blockIdx.y;
  const int64_t b = row_list ? (int64_t)row_list[ri] : ri;
  const int64_t excl = exclude_base >= 0 ? exclude_base + b : -1;
  const int64_t lo = part * part_len, hi = min(n, lo + part_len);
  const float* kf = (const float*)keys_ + (PACKED ? 0 : b * ld);
  const uint64_t* kp = (const uint64_t*)keys_ + (PACKED ? ri * ld : 0);
  for (int i = threadIdx.x; i < kSelBuf; i += kThreads) buf[i] = ~0ull;
  if (threadIdx.x == 0) {
    cnt = 0;
    thr = ~0ull;
  }
  __syncthreads();
  for (int64_t base = lo; base < hi; base += kSelRound) {
    const int c = cnt;
    __syncthreads();  // every thread has read cnt before any append below
    if (c > kSelBuf - kSelRound) sel_compact(buf, &cnt, &thr, L);
    const uint64_t t = thr;
    uint64_t kk[kSelPer];
#pragma unroll
    for (int e = 0; e < kSelPer; ++e) {
      const int64_t u = base + e * kThreads + threadIdx.x;
      kk[e] = ~0ull;
      if (u < hi) {
        if constexpr (PACKED) kk[e] = kp[u];
        else if (u != excl) kk[e] = pack_s(kf[u], (uint32_t)u);
      }
    }
    uint64_t t_use = t;
    if (base == lo && L <= kThreads) {
      // first round: threshold = the L-th smallest per-thread minimum, + 1
      // so that it admits itself (keys are unique; ~0 if fewer than L)
      uint64_t m = ~0ull;
#pragma unroll
      for (int e = 0; e < kSelPer; ++e) m = kk[e] < m ? kk[e] : m;
      mins[threadIdx.x] = m;
      __syncthreads();
      bitonic_sort(mins, kThreads);
      t_use = mins[L - 1] == ~0ull ? ~0ull : mins[L - 1] + 1;
    }
#pragma unroll
    for (int e = 0; e < kSelPer; ++e)
      if (kk[e] < t_use) buf[atomicAdd(&cnt, 1)] = kk[e];
    if (base == lo && threadIdx.x == 0) thr = t_use;
    __syncthreads();
  }
  sel_compact(buf, &cnt, &thr, L);
  uint64_t* o = out + (ri * gridDim.y + part) * (int64_t)L;
  for (int i = threadIdx.x; i < L; i += kThreads) o[i] = buf[i];
}

int64_t select_parts(int64_t n) { return n > kSelPart ? (n + kSelPart - 1) / kSelPart : 1; }

int64_t select_tmp_elems(int64_t rows, int64_t n, int L) {
  const int64_t P = select_parts(n);
  return P > 1 ? rows * P * L : 0;
}

hipError_t launch_select(const float* keys, int64_t ld, int64_t n, int64_t rows, int L,
                         const int32_t* row_list, int64_t exclude_base, uint64_t* out,
                         uint64_t* tmp, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (L < 1 || L > kSelectBuf / 2 || rows > 0x7fffffffLL) return hipErrorInvalidValue;
  const int64_t P = select_parts(n);
  if (P == 1) {
    hipLaunchKernelGGL(k_select<false>, dim3((unsigned)rows, 1), dim3(kThreads), 0, s,
                       (const void*)keys, ld, n, L, row_list, exclude_base, n > 0 ? n : 1, out);
    return hipGetLastError();
  }
  if (!tmp || P > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_select<false>, dim3((unsigned)rows, (unsigned)P), dim3(kThreads), 0, s,
                     (const void*)keys, ld, n, L, row_list, exclude_base, kSelPart, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n2 = P * L;
  hipLaunchKernelGGL(k_select<true>, dim3((unsigned)rows, 1), dim3(kThreads), 0, s,
                     (const void*)tmp, n2, n2, L, nullptr, (int64_t)-1, n2, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_finalize_sym(
    const uint64_t* __restrict__ cand, int64_t cand_ld, int64_t cand_use,
    const float* __restrict__ q2d, const int32_t* __restrict__ row_list, int64_t n, int L,
    int64_t* __restrict__ idx, float* __restrict__ dist, int* __restrict__ flags) {
  __shared__ uint64_t buf[kSelectBuf];
  const int64_t ri = blockIdx.x;
  const int64_t b = row_list ? (int64_t)row_list[ri] : ri;
  const uint64_t* cr = cand + ri * cand_ld;
  for (int i = threadIdx.x; i < kSelectBuf; i += kThreads) {
    uint64_t kk = ~0ull;
    if (i < cand_use) {
      const uint64_t c = cr[i];
      if (c != ~0ull) {
        const float s = fmaxf(unpack_f(c), q2d[ri * cand_use + i]);
        kk = pack_s(s, (uint32_t)c);
      }
    }
    buf[i] = kk;
  }
  __syncthreads();
  bitonic_sort(buf, kSelectBuf);
  for (int i = threadIdx.x; i < L; i += kThreads) {
    const uint64_t kk = buf[i];
    idx[b * L + i] = kk == ~0ull ? -1 : (int64_t)(uint32_t)kk;
    dist[b * L + i] = kk == ~0ull ? INFINITY : unpack_f(kk);
  }
  if (threadIdx.x == 0) {
    int f = 0;
    if (cand_use < cand_ld) {
      const uint64_t next = cr[cand_use];
      if (next != ~0ull && next <= buf[L - 1]) f = 1;
    }
    flags[ri] = f;
  }
}

hipError_t launch_finalize_sym(const uint64_t* cand, int64_t cand_ld, int64_t cand_use,
                               const float* q2d, int64_t rows, const int32_t* row_list,
                               int64_t n, int L, int64_t* idx, float* dist, int* flags,
                               hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (cand_use > kSelectBuf || L > cand_use) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize_sym, dim3((unsigned)rows), dim3(kThreads), 0, s, cand, cand_ld,
                     cand_use, q2d, row_list, n, L, idx, dist, flags);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_unpack_topl(const uint64_t* __restrict__ cand,
                                                          int64_t cand_ld, int64_t rows,
                                                          const int32_t* __restrict__ row_list,
                                                          int L, int64_t* __restrict__ idx,
                                                          float* __restrict__ dist) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= rows * L) return;
  const int64_t ri = t / L, i = t % L;
  const int64_t b = row_list ? (int64_t)row_list[ri] : ri;
  const uint64_t kk = cand[ri * cand_ld + i];
  idx[b * L + i] = kk == ~0ull ? -1 : (int64_t)(uint32_t)kk;
  dist[b * L + i] = kk == ~0ull ? INFINITY : unpack_f(kk);
}

hipError_t launch_unpack_topl(const uint64_t* cand, int64_t cand_ld, int64_t rows,
                              const int32_t* row_list, int L, int64_t* idx, float* dist,
                              hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t total = rows * L;
  hipLaunchKernelGGL(k_unpack_topl, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, cand, cand_ld, rows, row_list, L, idx, dist);
  return hipGetLastError();
}

// The database weights (the second word of each 8-byte record).
__global__ __launch_bounds__(kThreads) void k_record_weights(const int2* __restrict__ xcv, int64_t nnz,
                                                             float* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < nnz) val[i] = __int_as_float(xcv[i].y);
}

hipError_t launch_record_weights(const int2* xcv, int64_t nnz, float* val, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_record_weights, dim3((unsigned)((nnz + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     xcv, nnz, val);
  return hipGetLastError();
}

// In-place n x n square matrix: mode 0 = transpose, 1 = symmetric maximum
// (D[i][j] = D[j][i] = max of the two).  One workgroup per pair of 64x64
// tiles (I <= J), both staged through LDS so reads and writes are coalesced.
constexpr int kTT = 64;
__global__ __launch_bounds__(kThreads) void k_square_pair(float* __restrict__ D, int64_t n, int mode) {
  __shared__ float a[kTT][kTT + 1], b[kTT][kTT + 1];
  const int64_t nt = (n + kTT - 1) / kTT;
  // blockIdx -> (I, J), I <= J, row-major over the upper triangle of tiles
  // rows 0..I-1 of the upper triangle hold I*nt - I(I-1)/2 tiles
  const int64_t t = blockIdx.x;
  auto before = [nt](int64_t r) { return r * nt - r * (r - 1) / 2; };
  const double f = (double)(2 * nt + 1);
  int64_t I = (int64_t)((f - sqrt(f * f - 8.0 * (double)t)) / 2.0);
  I = I < 0 ? 0 : (I >= nt ? nt - 1 : I);
  while (I > 0 && before(I) > t) --I;
  while (I + 1 < nt && before(I + 1) <= t) ++I;
  const int64_t J = I + (t - before(I));
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < kTT; r += kThreads / 64) {
    const int64_t i = I * kTT + r, j = J * kTT + tx;
    a[r][tx] = (i < n && j < n) ? D[i * n + j] : 0.f;
    const int64_t i2 = J * kTT + r, j2 = I * kTT + tx;
    b[r][tx] = (i2 < n && j2 < n) ? D[i2 * n + j2] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < kTT; r += kThreads / 64) {
    // (I, J) tile gets the transpose of (J, I) (or the max with it), and back
    const int64_t i = I * kTT + r, j = J * kTT + tx;
    const float v1 = mode == 0 ? b[tx][r] : fmaxf(a[r][tx], b[tx][r]);
    const int64_t i2 = J * kTT + r, j2 = I * kTT + tx;
    const float v2 = mode == 0 ? a[tx][r] : fmaxf(b[r][tx], a[tx][r]);
    if (i < n && j < n) D[i * n + j] = v1;
    if (I != J && i2 < n && j2 < n) D[i2 * n + j2] = v2;
  }
}

// Rectangular transpose through 64x64 LDS tiles (coalesced reads and
// writes): out[c * ld_out + r] = in[r * cols + c].
__global__ __launch_bounds__(kThreads) void k_transpose(const float* __restrict__ in, int64_t rows,
                                                        int64_t cols, float* __restrict__ out,
                                                        int64_t ld_out) {
  __shared__ float t[kTT][kTT + 1];
  const int64_t c0 = (int64_t)blockIdx.x * kTT;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // row tiles strided over the grid's y extent (which is capped)
  for (int64_t r0 = (int64_t)blockIdx.y * kTT; r0 < rows; r0 += (int64_t)gridDim.y * kTT) {
    for (int i = ty; i < kTT; i += kThreads / 64) {
      const int64_t r = r0 + i, c = c0 + tx;
      if (r < rows && c < cols) t[i][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int i = ty; i < kTT; i += kThreads / 64) {
      const int64_t c = c0 + i, r = r0 + tx;
      if (r < rows && c < cols) out[c * ld_out + r] = t[tx][i];
    }
    __syncthreads();
  }
}

hipError_t launch_transpose(const float* in, int64_t rows, int64_t cols, float* out, int64_t ld_out,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t gx = (cols + kTT - 1) / kTT, gy = std::min<int64_t>((rows + kTT - 1) / kTT, 32768);
  if (gx > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, s, in, rows, cols, out, ld_out);
  return hipGetLastError();
}

hipError_t launch_square_pair(float* D, int64_t n, int mode, hipStream_t s) {
  const int64_t nt = (n + kTT - 1) / kTT;
  const int64_t blocks = nt * (nt + 1) / 2;
  if (n <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_square_pair, dim3((unsigned)blocks), dim3(kThreads), 0, s, D, n, mode);
  return hipGetLastError();
}

}  // namespace lcemd
