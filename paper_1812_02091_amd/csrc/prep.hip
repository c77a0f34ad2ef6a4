// Load-time preparation of the resident embeddings and input validation.
//
// Embeddings (Sec. 4, matrix V): copied row-major into a zero-padded
// float32 array whose row stride m_pad is a multiple of the phase-1 K chunk
// (zero padding leaves dot products and distances unchanged).  Row norms
// |v|^2 are accumulated in float64 and stored as float32; with
// L2 normalisation (Sec. 5: word vectors are L2-normalised) the scale is
// also computed in float64 and each value is rounded once.
#include "internal.h"

namespace lcemd {

__global__ __launch_bounds__(kThreads) void k_prep_embeddings(const float* __restrict__ Vin,
                                                              int64_t v, int m, int m_pad,
                                                              int l2norm, float* __restrict__ Vpad,
                                                              float* __restrict__ vnorm) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (r >= v) return;
  const float* src = Vin + r * (int64_t)m;
  float* dst = Vpad + r * (int64_t)m_pad;
  double s = 0.0;
  for (int d = lane; d < m; d += 64) {
    const double x = (double)src[d];
    s += x * x;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  double scale = 1.0;
  if (l2norm && s > 0.0) scale = 1.0 / sqrt(s);
  double s2 = 0.0;
  for (int d = lane; d < m_pad; d += 64) {
    float y = 0.f;
    if (d < m) y = (float)((double)src[d] * scale);
    dst[d] = y;
    s2 += (double)y * (double)y;
  }
  for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
  if (lane == 0) vnorm[r] = (float)s2;
}

hipError_t launch_prep_embeddings(const float* Vin, int64_t v, int m, int m_pad, int l2norm,
                                  float* Vpad, float* vnorm, hipStream_t s) {
  const int64_t g = (v + 3) / 4;
  hipLaunchKernelGGL(k_prep_embeddings, dim3((unsigned)g), dim3(kThreads), 0, s, Vin, v, m, m_pad,
                     l2norm, Vpad, vnorm);
  return hipGetLastError();
}

// bfloat16 rows for the bf16 phase-1 kernel, round to nearest even
// (finite inputs), in two forms.  Row form (the vocabulary side): dims < m
// hold -2 v (bf16(-2 v) = -2 bf16(v), exactly), dims m..m+2 hold 1 and dims
// m+3..m+5 a three-piece split of |v|^2 (each piece the bf16 rounding of
// what the earlier ones leave: three bf16 significands hold the float32
// value exactly).  Query form (the query side): dims < m hold v, dims
// m..m+2 the split of |v|^2 and dims m+3..m+5 hold 1.  The rest are 0, so a
// row-form row times a query-form row is |v|^2 + |q|^2 - 2 <v_b, q_b>.
// vres gets |v - bf16(v)| from float64 sums, rounded up.  One wave per row.
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ __launch_bounds__(kThreads) void k_make_bf16_rows(const float* __restrict__ V,
                                                             const float* __restrict__ vnorm, int64_t v,
                                                             int m, int m_pad, int mb,
                                                             uint16_t* __restrict__ out_row,
                                                             uint16_t* __restrict__ out_query,
                                                             float* __restrict__ vres) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (r >= v) return;
  const float* x = V + r * (int64_t)m_pad;
  uint16_t* o = out_row + r * (int64_t)mb;
  uint16_t* oq = out_query + r * (int64_t)mb;
  const float vn = vnorm[r];
  const float p0 = bf16_val(bf16_rne(vn));
  const float p1 = bf16_val(bf16_rne(vn - p0));
  const float p2 = bf16_val(bf16_rne(vn - p0 - p1));
  double e2 = 0.0;
  for (int d = lane; d < mb; d += 64) {
    float y, yq;
    if (d < m) {
      const float f = x[d];
      const uint16_t b = bf16_rne(f);
      const double e = (double)f - (double)bf16_val(b);
      e2 += e * e;
      y = -2.f * bf16_val(b);
      yq = bf16_val(b);
    } else if (d < m + 6) {
      const int t = (d - m) % 3;
      const float piece = t == 0 ? p0 : (t == 1 ? p1 : p2);
      y = d < m + 3 ? 1.f : piece;
      yq = d < m + 3 ? piece : 1.f;
    } else {
      y = yq = 0.f;
    }
    o[d] = bf16_rne(y);
    oq[d] = bf16_rne(yq);
  }
  for (int k = 32; k > 0; k >>= 1) e2 += __shfl_xor(e2, k);
  if (lane == 0) vres[r] = (float)(sqrt(e2) * (1.0 + 1e-6)) + 1e-38f;
}

hipError_t launch_make_bf16_rows(const float* V, const float* vnorm, int64_t v, int m, int m_pad, int mb,
                                 uint16_t* out_row, uint16_t* out_query, float* vres, hipStream_t s) {
  const int64_t blocks = (v + kThreads / 64 - 1) / (kThreads / 64);
  hipLaunchKernelGGL(k_make_bf16_rows, dim3((unsigned)blocks), dim3(kThreads), 0, s, V, vnorm, v, m, m_pad, mb,
                     out_row, out_query, vres);
  return hipGetLastError();
}

// fp8 (OCP e4m3) copy with one float32 scale per row: scale = max|v_d| / 448
// (the largest finite e4m3 value), codes = round-to-nearest-even(v_d /
// scale).  One wave per row; rows are m8 bytes (zero codes past m_pad).
__global__ __launch_bounds__(kThreads) void k_make_fp8(const float* __restrict__ V, int64_t v, int m_pad,
                                                       int m8, uint8_t* __restrict__ out,
                                                       float* __restrict__ scale) {
  const int64_t row = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= v) return;
  const float* x = V + row * m_pad;
  float mx = 0.f;
  for (int d = lane; d < m_pad; d += 64) mx = fmaxf(mx, fabsf(x[d]));
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  const float sc = mx > 0.f ? mx / 448.f : 1.f;
  if (lane == 0) scale[row] = sc;
  uint32_t* o32 = (uint32_t*)(out + row * (int64_t)m8);
  for (int q = lane; q < m8 / 4; q += 64) {
    float f[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int d = 4 * q + j;
      f[j] = d < m_pad ? x[d] / sc : 0.f;
    }
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(f[0], f[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(f[2], f[3], w, true);
    o32[q] = (uint32_t)w;
  }
}

hipError_t launch_make_fp8(const float* V, int64_t v, int m_pad, int m8, uint8_t* out, float* scale,
                           hipStream_t s) {
  const int64_t blocks = (v + kThreads / 64 - 1) / (kThreads / 64);
  hipLaunchKernelGGL(k_make_fp8, dim3((unsigned)blocks), dim3(kThreads), 0, s, V, v, m_pad, m8, out, scale);
  return hipGetLastError();
}

// Validation of a CSR histogram batch resident on the device; each failing
// row sets a bit of err[0]: 1 = row pointers, 2 = column ids, 4 = weights,
// 8 = row sum (only when normalised rows are required); err[1] gets the
// longest row (both start at 0).
__global__ __launch_bounds__(kThreads) void k_validate_csr(const int64_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col,
                                                           const float* __restrict__ val,
                                                           int64_t rows, int64_t v, int normalized,
                                                           int* __restrict__ err) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= rows) return;
  const int64_t a = ptr[r], b = ptr[r + 1];
  int e = 0;
  if (b <= a || b - a > LCEMD_MAX_HIST || a < 0 || (r == 0 && a != 0)) e |= 1;
  else atomicMax(err + 1, (int)(b - a));
  if (!(e & 1)) {
    double sum = 0.0;
    int prev = -1;
    for (int64_t i = a; i < b; ++i) {
      const int c = col[i];
      if (c <= prev || c >= v) e |= 2;
      prev = c;
      const float x = val[i];
      if (!(x > 0.f) || !isfinite(x)) e |= 4;
      sum += (double)x;
    }
    if (normalized && fabs(sum - 1.0) > 1e-5) e |= 8;
  }
  if (e) atomicOr(err, e);
}

hipError_t launch_validate_csr(const int64_t* ptr, const int32_t* col, const float* val,
                               int64_t rows, int64_t v, int normalized, int* err,
                               hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)((rows + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, ptr, col, val, rows, v, normalized, err);
  return hipGetLastError();
}

}  // namespace lcemd
