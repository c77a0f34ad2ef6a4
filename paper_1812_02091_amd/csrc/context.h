// Host-side context of the lcemd library and the helpers shared by the
// C-ABI entry points (api.cpp) and the serving engine (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
  double work;
};

// A call's buffers carved from a fixed device region instead of allocated
// (lcemd_topl_noalloc): fixed slots, no host or device allocation.
struct Arena {
  char* base = nullptr;  // null: scratch is allocated (grow-only, see wsget)
  size_t cap = 0, used = 0;
  struct Slot {
    const char* name;
    size_t off, bytes;
  } slot[32];
  int nslot = 0;
};

struct lcemd_ctx {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  std::string err;
  // embeddings (Sec. 4: V)
  int64_t v = 0;
  int m = 0, m_pad = 0;
  float* V = nullptr;
  float* vnorm = nullptr;
  uint16_t* Vb = nullptr;   // bfloat16 rows of mb dims (see P1Args::Vb)
  uint16_t* Vbq = nullptr;  // their query form (see P1Args::Vbq)
  float* vres = nullptr;    // |v - bf16(v)| per row
  int mb = 0;
  uint8_t* V8 = nullptr;    // fp8 codes, rows of m8 bytes
  float* vscale = nullptr;  // fp8 row scales
  int m8 = 0;
  // database (Sec. 4: X in CSR)
  int64_t n = 0, nnz = 0, v_used = 0;
  int db_hmax = 0;
  int64_t* xptr = nullptr;
  int2* xcv = nullptr;
  int32_t* xcol = nullptr;
  int32_t* xperm = nullptr;  // database rows by length within windows of 128
  // the weights grouped by compact word id (word-major phase 2): wptr[v_used
  // + 1] offsets into wwt (CSR order within a word); winv[i] = the by-word
  // index of CSR non-zero i
  int64_t* wptr = nullptr;
  float* wwt = nullptr;
  uint32_t* winv = nullptr;
  int32_t* used = nullptr;
  float* xmax = nullptr;
  std::vector<int32_t> used_host;
  std::vector<int64_t> xptr_host;  // database row pointers (host copy)
  // scratch, grow-only
  std::map<std::string, DevBuf> ws;
  size_t table_budget = size_t(12) << 30;  // test hook LCEMD_TABLE_BUDGET (bytes) sets it at creation
  int force_kernel = 0;   // test hook (LCEMD_FORCE_KERNEL): 1 = skip the 128-row kernel, 2 = deep kernel
  int sym_candidates = 0; // test hook (LCEMD_SYM_CANDIDATES): first candidate count of the SYM top-l
  int p2_mode = 0;        // test hook (LCEMD_PHASE2): 0 = by table size, 1 = word-major when possible, 2 = per document
  int fix_cap = 0;        // test hook (LCEMD_FIX_CAP): rows per table tile that may be redone exactly (0 = default)
  int64_t ws_fail_after = -1;  // test hook (LCEMD_SCRATCH_FAIL): scratch allocations granted before one is refused
  int64_t ws_allocs = 0;       // scratch allocations made (counted for that hook)
  int64_t fallbacks = 0;  // tiles redone with float32 keys / deeper lists
  unsigned long long* fix_total = nullptr;  // device: table rows redone exactly one by one
  // allocation-free calls: this device's scratch region and the arena over it
  void* scratch = nullptr;
  int scratch_rc = 0;
  Arena arena;
  // profiling
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<lcemd_phase_time> last;
};

namespace lcemd_host {

int fail(lcemd_ctx* c, int code, const char* fmt, ...);
int check_csr_host(lcemd_ctx* c, const char* what, const int64_t* ptr, const int32_t* col,
                   const float* val, int64_t rows, int64_t v, bool require_norm, int* hmax);
int ensure_precision(lcemd_ctx* c, int prec);
int p1_launch(lcemd_ctx* c, lcemd::P1Args& a, int mode, int prec, int depth, int seg_hmax,
              int row_hmax);
// this device's allocation-free scratch region (found once per device)
int noalloc_setup(int device, void** out);
size_t noalloc_capacity();
int pow2ceil(int x);

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, LCEMD_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

inline void dfree(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <typename T>
int dalloc(lcemd_ctx* c, T*& p, size_t count, const char* what) {
  void* q = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, LCEMD_E_OOM, "device allocation of %zu bytes for %s failed",
                count * sizeof(T), what);
  }
  p = static_cast<T*>(q);
  return LCEMD_OK;
}

int arena_get(lcemd_ctx* c, const char* name, size_t bytes, void** out);

// grow-only named scratch buffer (carved from the arena while one is set)
template <typename T>
int wsget(lcemd_ctx* c, const char* name, size_t count, T*& out) {
  if (c->arena.base) {
    void* p = nullptr;
    const int rc = arena_get(c, name, std::max<size_t>(count, 1) * sizeof(T), &p);
    out = static_cast<T*>(p);
    return rc;
  }
  DevBuf& b = c->ws[name];
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (b.bytes < bytes) {
    if (b.p) {
      (void)hipStreamSynchronize(c->stream);
      (void)hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
    }
    if (c->ws_fail_after >= 0 && c->ws_allocs++ >= c->ws_fail_after)
      return fail(c, LCEMD_E_OOM, "scratch allocation of %zu bytes (%s) refused (LCEMD_SCRATCH_FAIL)", bytes, name);
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, LCEMD_E_OOM, "scratch allocation of %zu bytes (%s) failed", bytes, name);
    }
    b.bytes = bytes;
  }
  out = static_cast<T*>(b.p);
  return LCEMD_OK;
}


}  // namespace lcemd_host
