// Host-side checks of CSR histogram batches (the histograms of Sec. 2.2:
// rows of distinct word ids with positive weights, normalised to 1), free
// of any device code so that they also build and run under host sanitizers.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "../../include/lcemd.h"

namespace lcemd_host {

// Full check of rows [0, rows): rowptr[0] == 0, every row non-empty and at
// most LCEMD_MAX_HIST long, column ids strictly increasing in [0, v), weights
// finite and > 0, and (require_norm) each row summing to 1 within 1e-5 in
// float64.  Returns LCEMD_OK (and the longest row in *hmax) or an error code
// with a message in msg.
inline int csr_check(const char* what, const int64_t* ptr, const int32_t* col, const float* val, int64_t rows,
                     int64_t v, bool require_norm, int* hmax, char* msg, size_t cap) {
  if (ptr[0] != 0) {
    snprintf(msg, cap, "%s: rowptr[0] must be 0", what);
    return LCEMD_E_BAD_CSR;
  }
  int hm = 0;
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t a = ptr[r], b = ptr[r + 1];
    if (b <= a) {
      snprintf(msg, cap, "%s: row %lld is empty or rowptr decreases", what, (long long)r);
      return LCEMD_E_BAD_CSR;
    }
    if (b - a > LCEMD_MAX_HIST) {
      snprintf(msg, cap, "%s: row %lld has %lld non-zeros (limit %d)", what, (long long)r, (long long)(b - a),
               LCEMD_MAX_HIST);
      return LCEMD_E_CAPACITY;
    }
    hm = std::max<int>(hm, (int)(b - a));
    double sum = 0.0;
    int prev = -1;
    for (int64_t i = a; i < b; ++i) {
      if (col[i] <= prev || col[i] >= v) {
        snprintf(msg, cap, "%s: row %lld: column ids must be strictly increasing in [0, %lld)", what, (long long)r,
                 (long long)v);
        return LCEMD_E_BAD_CSR;
      }
      prev = col[i];
      if (!(val[i] > 0.f) || !std::isfinite(val[i])) {
        snprintf(msg, cap, "%s: row %lld: weights must be finite and > 0", what, (long long)r);
        return LCEMD_E_BAD_CSR;
      }
      sum += (double)val[i];
    }
    if (require_norm && std::fabs(sum - 1.0) > 1e-5) {
      snprintf(msg, cap, "%s: row %lld sums to %.9g, not 1", what, (long long)r, sum);
      return LCEMD_E_BAD_CSR;
    }
  }
  *hmax = hm;
  return LCEMD_OK;
}

// Row pointers only (the columns and weights of device-resident batches
// are checked by a kernel).
inline int ptr_check(const char* what, const int64_t* ptr, int64_t rows, int* hmax, char* msg, size_t cap) {
  if (ptr[0] != 0) {
    snprintf(msg, cap, "%s: rowptr[0] must be 0", what);
    return LCEMD_E_BAD_CSR;
  }
  int hm = 0;
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t d = ptr[r + 1] - ptr[r];
    if (d <= 0) {
      snprintf(msg, cap, "%s: row %lld is empty or rowptr decreases", what, (long long)r);
      return LCEMD_E_BAD_CSR;
    }
    if (d > LCEMD_MAX_HIST) {
      snprintf(msg, cap, "%s: row %lld has %lld non-zeros (limit %d)", what, (long long)r, (long long)d,
               LCEMD_MAX_HIST);
      return LCEMD_E_CAPACITY;
    }
    hm = std::max<int>(hm, (int)d);
  }
  *hmax = hm;
  return LCEMD_OK;
}

}  // namespace lcemd_host
