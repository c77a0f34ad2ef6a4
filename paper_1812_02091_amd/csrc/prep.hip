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

// bfloat16 copy, round to nearest even (NaN-free inputs).
__global__ __launch_bounds__(kThreads) void k_make_bf16(const float* __restrict__ V, int64_t count,
                                                        uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= count) return;
  const uint32_t u = __float_as_uint(V[i]);
  const uint32_t rounded = u + 0x7fffu + ((u >> 16) & 1u);
  out[i] = (uint16_t)(rounded >> 16);
}

hipError_t launch_make_bf16(const float* V, int64_t count, uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_make_bf16, dim3((unsigned)((count + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, V, count, out);
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
// row sets a bit of *err: 1 = row pointers, 2 = column ids, 4 = weights,
// 8 = row sum (only when normalised rows are required).
__global__ __launch_bounds__(kThreads) void k_validate_csr(const int64_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col,
                                                           const float* __restrict__ val,
                                                           int64_t rows, int64_t v, int normalized,
                                                           int* __restrict__ err) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= rows) return;
  const int64_t a = ptr[r], b = ptr[r + 1];
  int e = 0;
  if (b <= a || b - a > LCEMD_MAX_HIST || a < 0) e |= 1;
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
