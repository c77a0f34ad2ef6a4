// C-ABI entry points of lcemd (declared in include/lcemd.h): context and
// resident memory, argument validation, and the launch sequence of the hot
// path (Sec. 4 Phase 1 -> Phase 2/3 -> top-l of Sec. 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "context.h"
#include "validate.h"

using namespace lcemd;

namespace {
thread_local std::string g_create_error;
}  // namespace


namespace lcemd_host {

int arena_get(lcemd_ctx* c, const char* name, size_t bytes, void** out) {
  Arena& A = c->arena;
  for (int i = 0; i < A.nslot; ++i)
    if (strcmp(A.slot[i].name, name) == 0 && A.slot[i].bytes >= bytes) {
      *out = A.base + A.slot[i].off;
      return LCEMD_OK;
    }
  const size_t off = (A.used + 255) / 256 * 256;
  if (A.nslot >= 32 || off + bytes > A.cap)
    return fail(c, LCEMD_E_CAPACITY, "the call needs more than the %zu bytes of the allocation-free scratch (%s: %zu bytes)",
                A.cap, name, bytes);
  A.slot[A.nslot++] = Arena::Slot{name, off, bytes};
  A.used = off + bytes;
  *out = A.base + off;
  return LCEMD_OK;
}

int fail(lcemd_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

void free_db(lcemd_ctx* c) {
  dfree((void*&)c->xptr);
  dfree((void*&)c->xcv);
  dfree((void*&)c->xperm);
  dfree((void*&)c->xcol);
  dfree((void*&)c->used);
  dfree((void*&)c->xmax);
  dfree((void*&)c->wptr);
  dfree((void*&)c->wwt);
  dfree((void*&)c->winv);
  c->n = c->nnz = c->v_used = 0;
  c->db_hmax = 0;
  c->used_host.clear();
  c->xptr_host.clear();
}

void free_emb(lcemd_ctx* c) {
  dfree((void*&)c->V);
  dfree((void*&)c->vnorm);
  dfree((void*&)c->Vb);
  dfree((void*&)c->Vbq);
  dfree((void*&)c->vres);
  c->mb = 0;
  dfree((void*&)c->V8);
  dfree((void*&)c->vscale);
  c->v = 0;
  c->m = c->m_pad = 0;
}

// ------------------------------- profiling --------------------------------
void prof_reset(lcemd_ctx* c) {
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->recs.clear();
}

int prof_begin(lcemd_ctx* c, const char* name, double work) {
  if (!c->prof) return LCEMD_OK;
  ProfRec r;
  r.name = name;
  r.work = work;
  HIPCHK(c, hipEventCreate(&r.a));
  HIPCHK(c, hipEventCreate(&r.b));
  HIPCHK(c, hipEventRecord(r.a, c->stream));
  c->recs.push_back(r);
  return LCEMD_OK;
}

int prof_end(lcemd_ctx* c) {
  if (!c->prof || c->recs.empty()) return LCEMD_OK;
  HIPCHK(c, hipEventRecord(c->recs.back().b, c->stream));
  return LCEMD_OK;
}

int prof_collect(lcemd_ctx* c) {
  c->last.clear();
  if (!c->prof) return LCEMD_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::map<std::string, size_t> at;
  for (auto& r : c->recs) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
    auto it = at.find(r.name);
    if (it == at.end()) {
      lcemd_phase_time t{};
      snprintf(t.name, sizeof t.name, "%s", r.name.c_str());
      at[r.name] = c->last.size();
      c->last.push_back(t);
      it = at.find(r.name);
    }
    lcemd_phase_time& t = c->last[it->second];
    t.ms += ms;
    t.launches += 1;
    t.work += r.work;
  }
  prof_reset(c);
  return LCEMD_OK;
}

// ------------------------------- validation -------------------------------
// Host-side check of a CSR histogram batch (validate.h); returns LCEMD_OK
// or the error with its message.  hmax receives the longest row.
int check_csr_host(lcemd_ctx* c, const char* what, const int64_t* ptr, const int32_t* col,
                   const float* val, int64_t rows, int64_t v, bool require_norm, int* hmax) {
  char msg[256];
  const int rc = csr_check(what, ptr, col, val, rows, v, require_norm, hmax, msg, sizeof msg);
  return rc ? fail(c, rc, "%s", msg) : LCEMD_OK;
}

int check_ptr_host(lcemd_ctx* c, const char* what, const int64_t* ptr, int64_t rows, int* hmax) {
  char msg[256];
  const int rc = ptr_check(what, ptr, rows, hmax, msg, sizeof msg);
  return rc ? fail(c, rc, "%s", msg) : LCEMD_OK;
}

// Device-resident query: validated and (for host input) staged on device.
struct QDev {
  int64_t B = 0, nnz = 0;
  const int64_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const float* val = nullptr;
  std::vector<int64_t> hptr;
  int hmax = 0;
  bool device = false;
};

int stage_query(lcemd_ctx* c, const lcemd_query* q, QDev& Q) {
  if (!q || !q->rowptr || !q->col || !q->val) return fail(c, LCEMD_E_INVALID_ARG, "query arrays must not be NULL");
  if (q->B < 1) return fail(c, LCEMD_E_INVALID_ARG, "query batch must hold at least one histogram");
  if (q->B > (int64_t(1) << 24)) return fail(c, LCEMD_E_CAPACITY, "query batch too large");
  Q.B = q->B;
  Q.device = (q->flags & LCEMD_PTR_DEVICE) != 0;
  if (!c->arena.base) Q.hptr.resize(Q.B + 1);
  if (!Q.device) {
    memcpy(Q.hptr.data(), q->rowptr, sizeof(int64_t) * (Q.B + 1));
    int rc = check_csr_host(c, "query", q->rowptr, q->col, q->val, Q.B, c->v, true, &Q.hmax);
    if (rc) return rc;
    Q.nnz = Q.hptr[Q.B];
    int64_t* dp;
    int32_t* dc;
    float* dv;
    if ((rc = wsget(c, "q_ptr", Q.B + 1, dp)) || (rc = wsget(c, "q_col", Q.nnz, dc)) ||
        (rc = wsget(c, "q_val", Q.nnz, dv)))
      return rc;
    HIPCHK(c, hipMemcpyAsync(dp, q->rowptr, sizeof(int64_t) * (Q.B + 1), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dc, q->col, sizeof(int32_t) * Q.nnz, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dv, q->val, sizeof(float) * Q.nnz, hipMemcpyHostToDevice, c->stream));
    Q.ptr = dp;
    Q.col = dc;
    Q.val = dv;
  } else {
    int rc;
    int* derr;
    if ((rc = wsget(c, "q_err", 2, derr))) return rc;
    HIPCHK(c, launch_zero_ints(derr, 2, c->stream));
    if (c->arena.base) {
      // allocation-free: row pointers checked on the device too (no host
      // copy of them); the total and the longest row come back as numbers
      HIPCHK(c, hipMemcpyAsync(&Q.nnz, q->rowptr + Q.B, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    } else {
      HIPCHK(c, hipMemcpyAsync(Q.hptr.data(), q->rowptr, sizeof(int64_t) * (Q.B + 1), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      if ((rc = check_ptr_host(c, "query", Q.hptr.data(), Q.B, &Q.hmax))) return rc;
      Q.nnz = Q.hptr[Q.B];
    }
    HIPCHK(c, launch_validate_csr(q->rowptr, q->col, q->val, Q.B, c->v, 1, derr, c->stream));
    int herr[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(herr, derr, sizeof(int) * 2, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->arena.base) {
      if (herr[0] & 1) return fail(c, LCEMD_E_BAD_CSR, "query: malformed row pointers (empty, decreasing or over %d words)", LCEMD_MAX_HIST);
      Q.hmax = herr[1];
    }
    const int herr0 = herr[0];
    if (herr0 & 2) return fail(c, LCEMD_E_BAD_CSR, "query: column ids must be strictly increasing in [0, %lld)", (long long)c->v);
    if (herr0 & 4) return fail(c, LCEMD_E_BAD_CSR, "query: weights must be finite and > 0");
    if (herr0 & 8) return fail(c, LCEMD_E_BAD_CSR, "query: a row does not sum to 1");
    if (herr0) return fail(c, LCEMD_E_BAD_CSR, "query: malformed CSR");
    Q.ptr = q->rowptr;
    Q.col = q->col;
    Q.val = q->val;
  }
  return LCEMD_OK;
}

int check_opts(lcemd_ctx* c, const lcemd_opts* o) {
  if (!o) return fail(c, LCEMD_E_INVALID_ARG, "opts must not be NULL");
  if (o->method < LCEMD_RWMD || o->method > LCEMD_ICT) return fail(c, LCEMD_E_INVALID_ARG, "unknown method %d", o->method);
  if (o->method == LCEMD_ACT && (o->k < 1 || o->k > LCEMD_MAX_K))
    return fail(c, LCEMD_E_INVALID_ARG, "ACT needs 1 <= k <= %d (got %d)", LCEMD_MAX_K, o->k);
  if (o->direction < LCEMD_D2Q || o->direction > LCEMD_SYM) return fail(c, LCEMD_E_INVALID_ARG, "unknown direction %d", o->direction);
  if (o->precision < LCEMD_FP32 || o->precision > LCEMD_FP8) return fail(c, LCEMD_E_INVALID_ARG, "unknown precision %d", o->precision);
  for (int i = 0; i < 3; ++i)
    if (o->reserved[i]) return fail(c, LCEMD_E_INVALID_ARG, "reserved option fields must be 0");
  return LCEMD_OK;
}

constexpr int kMargin = 8;  // over-selection for approximate (bf16/fp8) keys
constexpr int kFixCap = 1 << 23;  // rows per launch that may be redone exactly (64 MB list)
constexpr int kFixCapNoAlloc = 1 << 16;  // the same in allocation-free calls
constexpr int kFixGrid = 4096;  // rows the exact-redo launch sizes its grid for (it strides over more)
constexpr int kNoAllocMaxQueries = 4096;   // queries per allocation-free call

int pow2ceil(int x) {
  int p = 2;
  while (p < x) p <<= 1;
  return p;
}

int ensure_precision(lcemd_ctx* c, int prec) {
  if (prec == LCEMD_BF16 && !c->Vb) {
    const int mb = bf16_row_dims(c->m);
    int rc = dalloc(c, c->Vb, (size_t)c->v * mb, "bfloat16 embeddings");
    if (!rc) rc = dalloc(c, c->Vbq, (size_t)c->v * mb, "bfloat16 query-form embeddings");
    if (!rc) rc = dalloc(c, c->vres, (size_t)c->v, "bfloat16 error norms");
    if (rc) {
      dfree((void*&)c->Vb);
      dfree((void*&)c->Vbq);
      return rc;
    }
    c->mb = mb;
    HIPCHK(c, launch_make_bf16_rows(c->V, c->vnorm, c->v, c->m, c->m_pad, mb, c->Vb, c->Vbq, c->vres, c->stream));
  }
  if (prec == LCEMD_FP8 && !c->V8) {
    c->m8 = (c->m_pad + 127) / 128 * 128;
    int rc = dalloc(c, c->V8, (size_t)c->v * c->m8, "fp8 embeddings");
    if (!rc) rc = dalloc(c, c->vscale, (size_t)c->v, "fp8 row scales");
    if (rc) {
      dfree((void*&)c->V8);
      return rc;
    }
    HIPCHK(c, launch_make_fp8(c->V, c->v, c->m_pad, c->m8, c->V8, c->vscale, c->stream));
  }
  return LCEMD_OK;
}

// Launch phase 1: rows of `a` may need up to `depth` list entries.  Lists of
// up to 32 entries (with the bf16 margin) run on the 128-row kernel, up to
// 64 (and float32 embeddings of at most 28 dims at any depth up to 64) on
// the 64-row streaming kernel, deeper rows on the kernel that keeps a
// whole row of keys in LDS (float32 keys).  Pair mode: a.rb_max is set to
// the row-block count of the chosen kernel for queries of up to row_hmax
// words (callers size `partial` for 64-row blocks, the largest count).
int p1_launch(lcemd_ctx* c, P1Args& a, int mode, int prec, int depth, int seg_hmax,
              int row_hmax) {
  // reduced-precision keys carry their selection certificate on the table
  // kernels for lists of up to 32 entries (bf16: its own kernel, rows of up
  // to kBf16MaxDims dims); deeper lists and the pair mode use float32 keys
  if (prec != LCEMD_FP32 && (depth + kMargin > 32 || c->force_kernel || mode == P1_PAIR || seg_hmax > kSegShort))
    prec = LCEMD_FP32;
  if (prec == LCEMD_BF16 && !(c->Vb && phase1_bf16_fits(c->mb, seg_hmax, depth))) prec = LCEMD_FP32;
  if (a.m4 < 1 || 4 * a.m4 > a.m_pad) return fail(c, LCEMD_E_INVALID_ARG, "internal: phase-1 arguments without their dims");
  if (!a.work_ctr) {
    int rc = wsget(c, "p1_counters", 8, a.work_ctr);
    if (rc) return rc;
  }
  const int margin = prec == LCEMD_FP32 ? 0 : kMargin;
  a.Vb = c->Vb;
  a.Vbq = c->Vbq;
  a.vres = c->vres;
  a.mb = c->mb;
  a.m = c->m;
  a.V8 = c->V8;
  a.vscale = c->vscale;
  a.m8 = c->m8;
  if (prec == LCEMD_BF16) {
    a.KT_margin = margin;
    a.rb_max = 0;
    // per-call row and query-word records (callers that capture graphs
    // bring their own buffers; a.qnnz covers the batch's query non-zeros)
    if (!a.rinfo) {
      int rc = wsget(c, "bf16_rinfo", (size_t)a.v_used, a.rinfo);
      if (rc) return rc;
    }
    if (!a.qinfo) {
      int rc = wsget(c, "bf16_qinfo", (size_t)std::max<int64_t>(a.qnnz, 1), a.qinfo);
      if (rc) return rc;
    }
    if (!a.qmx) {
      int rc = wsget(c, "bf16_qmax", (size_t)std::max<int64_t>(a.nq, 1), a.qmx);
      if (rc) return rc;
    }
    HIPCHK(c, launch_phase1_bf16(a, mode, depth, c->stream));
    return LCEMD_OK;
  }
  // float32 with at most 28 dims (image coordinates): the 64-row kernel,
  // whose row blocks waste less of ~160-word histograms and whose exact keys
  // need no redo of rows with tied grid distances.  Not for ICT tables: the
  // 128-row kernel redoes rows deeper than their list one by one, where the
  // 64-row kernel can only report overflow (and the tables are rebuilt at
  // full depth)
  const bool small_m = prec == LCEMD_FP32 && a.m4 <= 7 && !(mode == P1_TABLE && a.method == LCEMD_ICT);
  if (depth + margin <= 32 && !c->force_kernel && !small_m) {
    const int KL = pow2ceil(depth + margin);
    a.KT_margin = margin;
    a.rb_max = (row_hmax + phase1_wide_rows() - 1) / phase1_wide_rows();
    HIPCHK(c, launch_phase1_wide(a, mode, KL, prec, seg_hmax, c->stream));
  } else if (depth <= 64 && c->force_kernel != 2) {
    const int KL = pow2ceil(std::min(depth + margin, 64));
    a.KT_margin = margin;
    a.rb_max = (row_hmax + kRows - 1) / kRows;
    HIPCHK(c, launch_phase1_fast(a, mode, KL, prec, c->stream));
  } else {
    a.KT_margin = 0;
    a.rb_max = (row_hmax + kRows - 1) / kRows;
    if (seg_hmax > kSegShort && !a.deep_keys) {
      int rc = wsget(c, "deep_keys", (size_t)(kDeepSlots * kDeepSlotFloats), a.deep_keys);
      if (rc) return rc;
    }
    HIPCHK(c, launch_phase1_deep(a, mode, seg_hmax, PREC_F32, c->stream));
  }
  return LCEMD_OK;
}

int check_ready(lcemd_ctx* c) {
  if (!c) return LCEMD_E_INVALID_ARG;
  if (!c->V) return fail(c, LCEMD_E_NOT_LOADED, "embeddings not loaded");
  if (!c->xptr) return fail(c, LCEMD_E_NOT_LOADED, "database not loaded");
  return LCEMD_OK;
}

// table depth (entries per table row) for a method
int table_depth(const lcemd_opts* o, int hmax) {
  switch (o->method) {
    case LCEMD_RWMD: return 1;
    case LCEMD_OMR: return std::min(2, hmax);
    case LCEMD_ACT: return std::min(o->k, hmax);
    default: return std::min(64, hmax);  // ICT: first try; widened on overflow
  }
}

// The histograms whose non-zeros phase 2 walks (the "database" of Sec. 4):
// the loaded database, or for the reverse direction the query batch.
struct DbView {
  int64_t n = 0, nnz = 0, v_used = 0;
  const int64_t* xptr = nullptr;
  const int2* xcv = nullptr;     // (compact word id, weight bits)
  const int32_t* xcol = nullptr; // original word ids
  const int32_t* used = nullptr; // compact id -> word id
  const float* xmax = nullptr;   // largest weight of each used word
  const int32_t* perm = nullptr; // rows by length within windows of 128
  const int64_t* wptr = nullptr; // weights by word (the loaded database only)
  const float* wwt = nullptr;
  const uint32_t* winv = nullptr;
};

DbView db_view(lcemd_ctx* c) {
  DbView d;
  d.n = c->n;
  d.nnz = c->nnz;
  d.v_used = c->v_used;
  d.xptr = c->xptr;
  d.xcv = c->xcv;
  d.xcol = c->xcol;
  d.used = c->used;
  d.xmax = c->xmax;
  d.perm = c->xperm;
  d.wptr = c->wptr;
  d.wwt = c->wwt;
  d.winv = c->winv;
  return d;
}

// Word-major phase 2 for a tile: when the database has its by-word records,
// the lists fit (KT <= 16), and one 64-query group's tables (v_used x KP x
// 1 KiB) are far beyond the caches -- there the per-document walk re-reads
// a word's run from HBM for every document holding it -- and the cost
// scratch (nnz x 256 bytes) fits in free device memory.
bool use_word_major(lcemd_ctx* c, const DbView& db, int KT) {
  if (!db.wwt || c->p2_mode == 2 || KT > 16 || db.nnz > 0xffffffffLL) return false;
  if (c->p2_mode != 1 && (double)db.v_used * (double)zw_pairs(KT) * 1024.0 < 1e9) return false;
  const auto it = c->ws.find("p2_cost");
  const size_t need = (size_t)db.nnz * 64 * sizeof(float);
  if (it != c->ws.end() && it->second.bytes >= need) return true;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return fr > need + (size_t(2) << 30);
}

P1Args base_args(lcemd_ctx* c, const DbView& db, const QDev& Q, const lcemd_opts* o) {
  P1Args a;
  memset(&a, 0, sizeof a);
  a.V = c->V;
  a.vnorm = c->vnorm;
  a.Vb = c->Vb;
  a.m_pad = c->m_pad;
  a.m4 = (c->m + 3) / 4;
  a.method = o->method;
  a.k = o->method == LCEMD_ACT ? o->k : 1;
  a.n = db.n;
  a.xptr = db.xptr;
  a.xcv = db.xcv;
  a.xcol = db.xcol;
  a.v_used = db.v_used;
  a.used = db.used;
  a.xmax = db.xmax;
  a.qptr = Q.ptr;
  a.qcol = Q.col;
  a.qval = Q.val;
  return a;
}

P1Args base_args(lcemd_ctx* c, const QDev& Q, const lcemd_opts* o) { return base_args(c, db_view(c), Q, o); }

// Queries per table tile at list depth KT: the tables stay under the
// context's budget, or (allocation-free) half of what the scratch region
// has left.
int64_t d2q_tile_queries(lcemd_ctx* c, const DbView& db, int KT) {
  const size_t per_q = (size_t)db.v_used * sizeof(float2);
  const size_t tbudget = c->arena.base ? (c->arena.cap - std::min(c->arena.cap, c->arena.used)) / 2 : c->table_budget;
  int64_t Bt = (int64_t)std::max<size_t>(1, tbudget / (per_q * 2 * zw_pairs(KT)));
  Bt = std::min<int64_t>(Bt, 16384);  // also bounds the rows a tile may need to redo
  // whole 64-query groups per tile: phase 2 runs a wave per 64 queries of
  // a document, so a tile of 64 g + r queries pays a full group for r
  if (Bt >= 64) Bt = Bt / 64 * 64;
  return Bt;
}

// Phase 1 (Alg. 2-3 tables) of queries [q0, q0 + nq) into *ZW, with the
// exact redo of the rows it could not certify.  Nothing is read back: a row
// deeper than the lists raises *ovf on the device.
int d2q_tables(lcemd_ctx* c, const DbView& db, const QDev& Q, const lcemd_opts* o, int64_t q0, int64_t nq,
               int prec, bool full_lists, int KT, int* ovf, float2** ZWout) {
  int rc;
  float2* ZW;
  if ((rc = wsget(c, "zw", (size_t)zw_pitch(nq) * db.v_used * 2 * zw_pairs(KT), ZW))) return rc;
  *ZWout = ZW;
  P1Args a = base_args(c, db, Q, o);
  a.qnnz = Q.nnz;
  a.KT = KT;
  a.q0 = q0;
  a.nq = nq;
  a.ZW = ZW;
  a.zw_nq = zw_pitch(nq);
  a.overflow = ovf;
  // rows whose quantised selection is not certified are listed for an
  // exact redo (every precision on the 128-row kernel); the redo kernel
  // reads the listed count on the device
  int* fixc = nullptr;
  int fixcap = c->arena.base ? kFixCapNoAlloc : kFixCap;
  if (c->fix_cap > 0) fixcap = std::min(fixcap, c->fix_cap);
  if ((rc = wsget(c, "fix_count", 1, fixc)) || (rc = wsget(c, "fix_list", fixcap, a.fix_list))) return rc;
  HIPCHK(c, launch_zero_ints(fixc, 1, c->stream));
  a.fix_count = fixc;
  a.fix_cap = fixcap;
  a.fix_total = c->fix_total;
  const int64_t H = Q.hptr.empty() ? Q.nnz : Q.hptr[q0 + nq] - Q.hptr[q0];
  if ((rc = prof_begin(c, "phase1_table", 2.0 * (double)db.v_used * (double)H * (double)c->m))) return rc;
  const int list_depth = full_lists ? KT : std::min(KT, kIctList);
  if ((rc = p1_launch(c, a, P1_TABLE, prec, list_depth, Q.hmax, Q.hmax))) return rc;
  if ((rc = prof_end(c))) return rc;
  if ((rc = prof_begin(c, "fix_rows", 0.0))) return rc;
  HIPCHK(c, launch_fix_rows(a, P1_TABLE, kFixGrid, c->stream));
  if ((rc = prof_end(c))) return rc;
  return LCEMD_OK;
}

// Phase 2 (Eq. (6)-(9)) of queries [q0, q0 + nq) from their tables into out.
int d2q_phase2(lcemd_ctx* c, const DbView& db, int64_t q0, int64_t nq, int KT, const float2* ZW, float* out,
               int64_t ld) {
  int rc;
  const int64_t zw_nq = zw_pitch(nq);
  const double a2 = (double)nq * (8.0 * db.nnz + 8.0 * (db.n + 1) + 8.0 * (double)db.v_used * KT + 4.0 * db.n);
  if ((rc = prof_begin(c, "phase2", a2))) return rc;
  unsigned long long* p2c;
  if ((rc = wsget(c, "p2_counters", 16, p2c))) return rc;
  // whole 64-query groups word-major where that pays, the rest (and every
  // group otherwise) per document; both give the same bits
  const int64_t ng = !c->arena.base && use_word_major(c, db, KT) ? nq / 64 : 0;
  if (ng > 0) {
    float* cost;
    if ((rc = wsget(c, "p2_cost", (size_t)db.nnz * 64, cost))) return rc;
    for (int64_t g = 0; g < ng; ++g)
      HIPCHK(c, launch_phase2_wordmajor(db.xptr, db.n, db.wptr, db.wwt, db.winv, db.nnz, db.v_used,
                                        ZW + 2 * 64 * g, zw_nq, KT, cost, out + (q0 + 64 * g) * ld, ld, p2c,
                                        c->stream));
  }
  if (nq > 64 * ng)
    HIPCHK(c, launch_phase2_persistent(db.xptr, db.xcv, db.n, db.perm, ZW + 2 * 64 * ng, zw_nq, KT, nq - 64 * ng,
                                       nullptr, out + (q0 + 64 * ng) * ld, ld, p2c, c->stream));
  if ((rc = prof_end(c))) return rc;
  return LCEMD_OK;
}

// The list settings of a table tile, made one step deeper after an overflow:
// float32 keys first, then (float32 already) full-depth lists.
struct TileDepth {
  int prec, KT;
  bool full;
  bool deeper(lcemd_ctx* c, int hmax) {
    ++c->fallbacks;
    if (prec != LCEMD_FP32) {
      prec = LCEMD_FP32;
      return true;
    }
    if (!full || KT < hmax) {
      full = true;
      KT = hmax;
      return true;
    }
    return false;
  }
};

// Queries [t0, t1) tile by tile, each tile's overflow flag read back before
// its phase 2; a tile that overflowed is run again one step deeper (the
// deeper tables may split it).
int d2q_checked(lcemd_ctx* c, const DbView& db, const QDev& Q, const lcemd_opts* o, int64_t t0, int64_t t1,
                TileDepth d, int* ovf, float* out, int64_t ld) {
  int rc;
  for (int64_t r0 = t0; r0 < t1;) {
    const int64_t nq = std::min<int64_t>(d2q_tile_queries(c, db, d.KT), t1 - r0);
    float2* ZW;
    int h_ovf = 0;
    HIPCHK(c, launch_zero_ints(ovf, 1, c->stream));
    if ((rc = d2q_tables(c, db, Q, o, r0, nq, d.prec, d.full, d.KT, ovf, &ZW))) return rc;
    HIPCHK(c, hipMemcpyAsync(&h_ovf, ovf, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h_ovf) {  // the same queries again, one step deeper
      if (!d.deeper(c, Q.hmax))
        return fail(c, LCEMD_E_CAPACITY, "a table row of queries [%lld, %lld) is deeper than its lists at full depth",
                    (long long)r0, (long long)(r0 + nq));
      continue;
    }
    if ((rc = d2q_phase2(c, db, r0, nq, d.KT, ZW, out, ld))) return rc;
    r0 += nq;
  }
  return LCEMD_OK;
}

// D2Q distances of every query against every row of `db` (Sec. 4):
// out[b * ld + u].  ICT's short lists overflow often, so its tiles are
// checked one by one before their phase 2.  For the other measures, where
// an overflow is rare, the tiles run back to back, each with its own
// overflow flag; the flags are read once, after the last tile, and a tile
// that overflowed is run again, checked, one step deeper.  Phase 2 of an
// overflowed tile reads incomplete tables, but its loops are bounded by the
// list depth and the database records, and the rerun rewrites its rows.
int run_d2q(lcemd_ctx* c, const DbView& db, const QDev& Q, const lcemd_opts* o, float* out, int64_t ld) {
  // ICT: the tables hold up to KT entries per row, but the lists of phase 1
  // stop at kIctList (a row needs a few entries before its capacities cover
  // the word's largest weight, Lemma 1); deeper rows are redone exactly
  const TileDepth d0{o->precision, table_depth(o, Q.hmax), o->method != LCEMD_ICT};
  if (Q.B < 1) return LCEMD_OK;
  int* ovf;
  int rc;
  if (o->method == LCEMD_ICT) {
    if ((rc = wsget(c, "ovf", 1, ovf))) return rc;
    return d2q_checked(c, db, Q, o, 0, Q.B, d0, ovf, out, ld);
  }
  if ((rc = wsget(c, "ovf_tiles", (size_t)Q.B, ovf))) return rc;
  HIPCHK(c, launch_zero_ints(ovf, (int)Q.B, c->stream));
  std::vector<std::pair<int64_t, int64_t>> tiles;
  for (int64_t q0 = 0; q0 < Q.B;) {
    const int64_t nq = std::min<int64_t>(d2q_tile_queries(c, db, d0.KT), Q.B - q0);
    float2* ZW;
    if ((rc = d2q_tables(c, db, Q, o, q0, nq, d0.prec, d0.full, d0.KT, ovf + tiles.size(), &ZW))) return rc;
    if ((rc = d2q_phase2(c, db, q0, nq, d0.KT, ZW, out, ld))) return rc;
    tiles.emplace_back(q0, nq);
    q0 += nq;
  }
  std::vector<int> hf(tiles.size());
  HIPCHK(c, hipMemcpyAsync(hf.data(), ovf, sizeof(int) * hf.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (size_t t = 0; t < tiles.size(); ++t) {
    if (!hf[t]) continue;
    TileDepth d = d0;
    if (!d.deeper(c, Q.hmax))
      return fail(c, LCEMD_E_CAPACITY, "a table row of queries [%lld, %lld) is deeper than its lists at full depth",
                  (long long)tiles[t].first, (long long)(tiles[t].first + tiles[t].second));
    if ((rc = d2q_checked(c, db, Q, o, tiles[t].first, tiles[t].first + tiles[t].second, d, ovf, out, ld))) return rc;
  }
  return LCEMD_OK;
}

int run_d2q(lcemd_ctx* c, const QDev& Q, const lcemd_opts* o, float* out, int64_t ld) {
  return run_d2q(c, db_view(c), Q, o, out, ld);
}

// The L smallest keys of each row (scratch for the per-part first pass).
int select_rows(lcemd_ctx* c, const float* keys, int64_t ld, int64_t n, int64_t rows, int L,
                const int32_t* row_list, int64_t excl, uint64_t* out) {
  uint64_t* tmp = nullptr;
  const int64_t t = select_tmp_elems(rows, n, L);
  int rc;
  if (t > 0 && (rc = wsget(c, "select_tmp", (size_t)t, tmp))) return rc;
  HIPCHK(c, launch_select(keys, ld, n, rows, L, row_list, excl, out, tmp, c->stream));
  return LCEMD_OK;
}

// Q2D for an explicit list of pairs or candidates (see P1Args).
int run_pairs(lcemd_ctx* c, const QDev& Q, const lcemd_opts* o, P1Args a, float* out,
              int64_t out_ld, int64_t per_row) {
  const int rb_cap = (Q.hmax + kRows - 1) / kRows;
  float* partial;
  int rc;
  if ((rc = wsget(c, "partial", (size_t)a.npairs * rb_cap, partial))) return rc;
  int* ovf;
  if ((rc = wsget(c, "ovf_pair", 1, ovf))) return rc;
  a.partial = partial;
  a.overflow = ovf;
  const int depth = table_depth(o, c->db_hmax);
  HIPCHK(c, launch_zero_ints(ovf, 1, c->stream));
  if ((rc = prof_begin(c, "phase1_pair_q2d", (double)a.npairs))) return rc;
  if ((rc = p1_launch(c, a, P1_PAIR, o->precision, depth, c->db_hmax, Q.hmax))) return rc;
  if ((rc = prof_end(c))) return rc;
  if ((o->method == LCEMD_ICT && depth < c->db_hmax) || o->precision != LCEMD_FP32) {
    int h_ovf = 0;
    HIPCHK(c, hipMemcpyAsync(&h_ovf, ovf, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h_ovf) {
      ++c->fallbacks;
      const int d2 = o->method == LCEMD_ICT ? c->db_hmax : depth;
      if ((rc = p1_launch(c, a, P1_PAIR, LCEMD_FP32, d2, c->db_hmax, Q.hmax))) return rc;
    }
  }
  HIPCHK(c, launch_pair_reduce(partial, a.npairs, a.rb_max, out, out_ld, per_row, c->stream));
  return LCEMD_OK;
}

// Full Q2D matrix: out[b * ld + u], in query tiles that keep the pair grid
// within limits.
// The loaded database as a device-resident query batch (its weights copied
// out of the (word, weight) records).
int docs_as_queries(lcemd_ctx* c, QDev& Q) {
  Q.B = c->n;
  Q.nnz = c->nnz;
  Q.ptr = c->xptr;
  Q.col = c->xcol;
  Q.hmax = c->db_hmax;
  Q.device = true;
  float* dval;
  int rc = wsget(c, "db_val", (size_t)c->nnz, dval);
  if (rc) return rc;
  HIPCHK(c, launch_record_weights(c->xcv, c->nnz, dval, c->stream));
  Q.val = dval;
  Q.hptr = c->xptr_host;
  return LCEMD_OK;
}

// Q2D of every query against every database row (out[b * ld + u]) by the
// linear-complexity method with the roles swapped: the query batch is the
// histogram set whose non-zeros phase 2 walks (its used words are the table
// rows, its largest weight per word bounds ICT's depth, Lemma 1) and every
// database row is a query of phase 1; Q2D(b, u) moves query b's mass into
// row u, which is what that D2Q computes.
int run_q2d_lc(lcemd_ctx* c, const QDev& Q, const lcemd_opts* o, float* out, int64_t ld) {
  const int64_t B = Q.B, H = Q.nnz;
  const int64_t cap = std::min<int64_t>(H, c->v);
  int2* dcv;
  int32_t *dused, *dperm;
  float* dxmax;
  int *dscr, *dnu;
  int rc;
  if ((rc = wsget(c, "rev_xcv", (size_t)H, dcv)) || (rc = wsget(c, "rev_used", (size_t)cap, dused)) ||
      (rc = wsget(c, "rev_xmax", (size_t)cap, dxmax)) || (rc = wsget(c, "rev_perm", (size_t)B, dperm)) ||
      (rc = wsget(c, "rev_scratch", (size_t)reverse_scratch_ints(c->v), dscr)) || (rc = wsget(c, "rev_nu", 1, dnu)))
    return rc;
  HIPCHK(c, launch_reverse_records(Q.ptr, Q.col, Q.val, B, H, c->v, dscr, dcv, dused, dxmax, dperm, dnu, c->stream));
  // the used word count sizes the tables and phase 1's grid
  int nu = 0;
  HIPCHK(c, hipMemcpyAsync(&nu, dnu, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (nu < 1 || nu > cap) return fail(c, LCEMD_E_HIP, "internal: reverse records counted %d used words", nu);
  DbView d;
  d.n = B;
  d.nnz = H;
  d.v_used = nu;
  d.xptr = Q.ptr;
  d.xcv = dcv;
  d.xcol = Q.col;
  d.used = dused;
  d.xmax = dxmax;
  d.perm = dperm;
  QDev docs;
  if ((rc = docs_as_queries(c, docs))) return rc;
  float* T;
  if ((rc = wsget(c, "rev_out", (size_t)c->n * B, T))) return rc;
  if ((rc = run_d2q(c, d, docs, o, T, B))) return rc;  // T[u * B + b]
  HIPCHK(c, launch_transpose(T, c->n, B, out, ld, c->stream));
  return LCEMD_OK;
}

int finish_call(lcemd_ctx* c) {
  int rc = prof_collect(c);
  if (rc) return rc;
  HIPCHK(c, hipGetLastError());
  return LCEMD_OK;
}

}  // namespace lcemd_host

using namespace lcemd_host;

// ===========================================================================
extern "C" {

int lcemd_version(void) { return LCEMD_VERSION; }

int lcemd_create(lcemd_ctx** out, int device) {
  if (!out) return LCEMD_E_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    g_create_error = "no HIP device available";
    return LCEMD_E_NO_DEVICE;
  }
  if (device < 0 || device >= count) {
    g_create_error = "device index out of range";
    return LCEMD_E_NO_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    g_create_error = "hipGetDeviceProperties failed";
    return LCEMD_E_NO_DEVICE;
  }
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
    return LCEMD_E_NO_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) {
    g_create_error = "hipSetDevice failed";
    return LCEMD_E_NO_DEVICE;
  }
  lcemd_ctx* c = new lcemd_ctx();
  c->device = device;
  if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    g_create_error = "hipStreamCreate failed";
    return LCEMD_E_HIP;
  }
  c->stream = c->own_stream;
  if (hipMalloc((void**)&c->fix_total, sizeof(unsigned long long)) != hipSuccess ||
      hipMemsetAsync(c->fix_total, 0, sizeof(unsigned long long), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    if (c->fix_total) (void)hipFree(c->fix_total);
    (void)hipStreamDestroy(c->own_stream);
    delete c;
    g_create_error = "device allocation of the context's counters failed";
    return LCEMD_E_OOM;
  }
  // the allocation-free scratch region of this device (looked up once per
  // device, with the device current); a failure only disables that call
  c->scratch_rc = noalloc_setup(device, &c->scratch);
  if (const char* fk = getenv("LCEMD_FORCE_KERNEL")) c->force_kernel = atoi(fk);
  if (const char* sc = getenv("LCEMD_SYM_CANDIDATES")) c->sym_candidates = atoi(sc);
  if (const char* p2 = getenv("LCEMD_PHASE2")) c->p2_mode = atoi(p2);
  if (const char* tb = getenv("LCEMD_TABLE_BUDGET")) c->table_budget = (size_t)strtoull(tb, nullptr, 10);
  if (const char* fc = getenv("LCEMD_FIX_CAP")) c->fix_cap = atoi(fc);
  if (const char* sf = getenv("LCEMD_SCRATCH_FAIL")) c->ws_fail_after = atoll(sf);
  *out = c;
  return LCEMD_OK;
}

void lcemd_destroy(lcemd_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  prof_reset(c);
  free_db(c);
  free_emb(c);
  for (auto& kv : c->ws) dfree(kv.second.p);
  dfree((void*&)c->fix_total);
  c->ws.clear();
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

int lcemd_set_stream(lcemd_ctx* c, void* s) {
  if (!c) return LCEMD_E_INVALID_ARG;
  c->stream = (hipStream_t)s;
  return LCEMD_OK;
}

int lcemd_use_own_stream(lcemd_ctx* c) {
  if (!c) return LCEMD_E_INVALID_ARG;
  c->stream = c->own_stream;
  return LCEMD_OK;
}

const char* lcemd_last_error(const lcemd_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

int lcemd_load_embeddings(lcemd_ctx* c, const float* V, int64_t v, int32_t m, uint32_t flags) {
  if (!c) return LCEMD_E_INVALID_ARG;
  c->err.clear();
  if (!V) return fail(c, LCEMD_E_INVALID_ARG, "V must not be NULL");
  if (v < 1 || v >= (int64_t(1) << 31)) return fail(c, LCEMD_E_INVALID_ARG, "v out of range");
  if (m < 1 || m > 4096) return fail(c, LCEMD_E_INVALID_ARG, "m out of range (1..4096)");
  if (flags & ~(LCEMD_PTR_DEVICE | LCEMD_L2_NORMALIZE | LCEMD_MAKE_BF16 | LCEMD_MAKE_FP8))
    return fail(c, LCEMD_E_INVALID_ARG, "unknown flags");
  (void)hipSetDevice(c->device);
  const bool dev = flags & LCEMD_PTR_DEVICE;
  if (!dev) {
    for (int64_t i = 0; i < v * (int64_t)m; ++i)
      if (!std::isfinite(V[i])) return fail(c, LCEMD_E_INVALID_ARG, "embeddings must be finite");
  }
  free_db(c);
  free_emb(c);
  const int m_pad = ((m + 63) / 64) * 64;  // one 128-byte bf16 slice = 64 dims
  int rc;
  if ((rc = dalloc(c, c->V, (size_t)v * m_pad, "embeddings"))) return rc;
  if ((rc = dalloc(c, c->vnorm, (size_t)v, "row norms"))) return rc;
  const float* src = V;
  float* tmp = nullptr;
  hipError_t e = hipSuccess;
  if (!dev) {
    if ((rc = dalloc(c, tmp, (size_t)v * m, "embedding staging"))) return rc;
    e = hipMemcpyAsync(tmp, V, sizeof(float) * v * m, hipMemcpyHostToDevice, c->stream);
    src = tmp;
  }
  if (e == hipSuccess)
    e = launch_prep_embeddings(src, v, m, m_pad, (flags & LCEMD_L2_NORMALIZE) ? 1 : 0, c->V, c->vnorm,
                               c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (tmp) {
    if (e != hipSuccess) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
  }
  if (e != hipSuccess)
    return fail(c, LCEMD_E_HIP, "embedding preparation failed: %s", hipGetErrorString(e));
  c->v = v;
  c->m = m;
  c->m_pad = m_pad;
  if (flags & LCEMD_MAKE_BF16 && (rc = ensure_precision(c, LCEMD_BF16))) return rc;
  if (flags & LCEMD_MAKE_FP8 && (rc = ensure_precision(c, LCEMD_FP8))) return rc;
  if (flags & (LCEMD_MAKE_BF16 | LCEMD_MAKE_FP8)) HIPCHK(c, hipStreamSynchronize(c->stream));
  return LCEMD_OK;
}

int lcemd_load_database(lcemd_ctx* c, const int64_t* rowptr, const int32_t* col, const float* val,
                        int64_t n, uint32_t flags) {
  if (!c) return LCEMD_E_INVALID_ARG;
  c->err.clear();
  if (!c->V) return fail(c, LCEMD_E_NOT_LOADED, "load embeddings before the database");
  if (!rowptr || !col || !val) return fail(c, LCEMD_E_INVALID_ARG, "database arrays must not be NULL");
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(c, LCEMD_E_INVALID_ARG, "n out of range");
  if (flags & ~(LCEMD_PTR_DEVICE | LCEMD_NORMALIZE)) return fail(c, LCEMD_E_INVALID_ARG, "unknown flags");
  (void)hipSetDevice(c->device);
  const bool dev = flags & LCEMD_PTR_DEVICE;
  // host copies (the database is reorganised once, on the host)
  std::vector<int64_t> hp;
  std::vector<int32_t> hc;
  std::vector<float> hv;
  const int64_t* P = rowptr;
  const int32_t* Cc = col;
  const float* Vv = val;
  if (dev) {
    hp.resize(n + 1);
    HIPCHK(c, hipMemcpy(hp.data(), rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    int hm;
    int rc = check_ptr_host(c, "database", hp.data(), n, &hm);
    if (rc) return rc;
    hc.resize(hp[n]);
    hv.resize(hp[n]);
    HIPCHK(c, hipMemcpy(hc.data(), col, sizeof(int32_t) * hp[n], hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(hv.data(), val, sizeof(float) * hp[n], hipMemcpyDeviceToHost));
    P = hp.data();
    Cc = hc.data();
    Vv = hv.data();
  }
  const bool norm = flags & LCEMD_NORMALIZE;
  int hmax = 0;
  int rc = check_csr_host(c, "database", P, Cc, Vv, n, c->v, !norm, &hmax);
  if (rc) return rc;
  const int64_t nnz = P[n];
  // weights (optionally renormalised with float64 row sums)
  std::vector<float> w(Vv, Vv + nnz);
  if (norm) {
    for (int64_t r = 0; r < n; ++r) {
      double s = 0.0;
      for (int64_t i = P[r]; i < P[r + 1]; ++i) s += (double)w[i];
      for (int64_t i = P[r]; i < P[r + 1]; ++i) w[i] = (float)((double)w[i] / s);
    }
  }
  // used vocabulary (Sec. 2.2: union of the database's coordinates) and the
  // largest weight each used word carries anywhere in the database
  std::vector<int32_t> pos(c->v, -1);
  std::vector<char> seen(c->v, 0);
  for (int64_t i = 0; i < nnz; ++i) seen[Cc[i]] = 1;
  std::vector<int32_t> used;
  for (int64_t i = 0; i < c->v; ++i)
    if (seen[i]) {
      pos[i] = (int32_t)used.size();
      used.push_back((int32_t)i);
    }
  std::vector<float> xmax(used.size(), 0.f);
  std::vector<int2> cv(nnz);
  for (int64_t i = 0; i < nnz; ++i) {
    const int32_t p = pos[Cc[i]];
    cv[i].x = p;
    float wi = w[i];
    memcpy(&cv[i].y, &wi, sizeof(float));
    xmax[p] = std::max(xmax[p], wi);
  }
  free_db(c);
  if ((rc = dalloc(c, c->xptr, n + 1, "rowptr")) || (rc = dalloc(c, c->xcv, nnz, "database entries")) ||
      (rc = dalloc(c, c->xcol, nnz, "database word ids")) || (rc = dalloc(c, c->used, used.size(), "used vocabulary")) ||
      (rc = dalloc(c, c->xperm, n, "length order")) ||
      (rc = dalloc(c, c->xmax, used.size(), "word maxima"))) {
    free_db(c);
    return rc;
  }
  HIPCHK(c, hipMemcpy(c->xptr, P, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->xcv, cv.data(), sizeof(int2) * nnz, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->xcol, Cc, sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
  {
    // documents by length within aligned windows of 128 (phase 2 runs
    // documents of a similar length side by side; its outputs stay within a
    // window)
    std::vector<int32_t> perm(n);
    for (int64_t r = 0; r < n; ++r) perm[r] = (int32_t)r;
    for (int64_t w0 = 0; w0 < n; w0 += 128)
      std::stable_sort(perm.begin() + w0, perm.begin() + std::min<int64_t>(n, w0 + 128),
                       [&](int32_t x, int32_t y) { return P[x + 1] - P[x] < P[y + 1] - P[y]; });
    HIPCHK(c, hipMemcpy(c->xperm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  }
  HIPCHK(c, hipMemcpy(c->used, used.data(), sizeof(int32_t) * used.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->xmax, xmax.data(), sizeof(float) * used.size(), hipMemcpyHostToDevice));
  if (nnz <= 0xffffffffLL) {
    // the records grouped by word (CSR order within a word) for the
    // word-major phase 2
    const int64_t nu = (int64_t)used.size();
    std::vector<int64_t> wp(nu + 1, 0);
    for (int64_t i = 0; i < nnz; ++i) ++wp[cv[i].x + 1];
    for (int64_t p = 0; p < nu; ++p) wp[p + 1] += wp[p];
    std::vector<int64_t> fill(wp.begin(), wp.end() - 1);
    std::vector<float> ww(nnz);
    std::vector<uint32_t> inv(nnz);
    for (int64_t i = 0; i < nnz; ++i) {
      const int64_t e = fill[cv[i].x]++;
      memcpy(&ww[e], &cv[i].y, sizeof(float));
      inv[i] = (uint32_t)e;
    }
    if ((rc = dalloc(c, c->wptr, nu + 1, "word offsets")) || (rc = dalloc(c, c->wwt, nnz, "weights by word")) ||
        (rc = dalloc(c, c->winv, nnz, "by-word index"))) {
      free_db(c);
      return rc;
    }
    HIPCHK(c, hipMemcpy(c->wptr, wp.data(), sizeof(int64_t) * (nu + 1), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->wwt, ww.data(), sizeof(float) * nnz, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->winv, inv.data(), sizeof(uint32_t) * nnz, hipMemcpyHostToDevice));
  }
  c->n = n;
  c->nnz = nnz;
  c->v_used = (int64_t)used.size();
  c->db_hmax = hmax;
  c->used_host = std::move(used);
  c->xptr_host.assign(P, P + n + 1);
  return LCEMD_OK;
}

int lcemd_check_histograms(const int64_t* rowptr, const int32_t* col, const float* val,
                           int64_t rows, int64_t v, int require_normalized, char* msg,
                           size_t msg_cap) {
  lcemd_ctx scratch;  // only its error string is used
  int rc;
  int hmax = 0;
  if (!rowptr || !col || !val) rc = fail(&scratch, LCEMD_E_INVALID_ARG, "arrays must not be NULL");
  else if (rows < 1) rc = fail(&scratch, LCEMD_E_INVALID_ARG, "need at least one histogram");
  else if (v < 1) rc = fail(&scratch, LCEMD_E_INVALID_ARG, "vocabulary must not be empty");
  else rc = check_csr_host(&scratch, "histograms", rowptr, col, val, rows, v, require_normalized != 0, &hmax);
  if (msg && msg_cap) snprintf(msg, msg_cap, "%s", scratch.err.c_str());
  return rc;
}

int64_t lcemd_used_vocab(lcemd_ctx* c, int32_t* ids) {
  if (!c) return LCEMD_E_INVALID_ARG;
  if (ids && !c->used_host.empty()) memcpy(ids, c->used_host.data(), sizeof(int32_t) * c->used_host.size());
  return (int64_t)c->used_host.size();
}

int lcemd_profile(lcemd_ctx* c, int enable) {
  if (!c) return LCEMD_E_INVALID_ARG;
  c->prof = enable != 0;
  return LCEMD_OK;
}

int lcemd_counters(lcemd_ctx* c, int64_t* fallback_tiles, int64_t* exact_rows) {
  if (!c) return LCEMD_E_INVALID_ARG;
  if (fallback_tiles) *fallback_tiles = c->fallbacks;
  if (exact_rows) {
    unsigned long long t = 0;
    if (c->fix_total) {
      HIPCHK(c, hipMemcpyAsync(&t, c->fix_total, sizeof t, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    *exact_rows = (int64_t)t;
  }
  return LCEMD_OK;
}

int lcemd_profile_get(lcemd_ctx* c, lcemd_phase_time* out, int cap) {
  if (!c) return LCEMD_E_INVALID_ARG;
  const int cnt = (int)c->last.size();
  for (int i = 0; i < cnt && i < cap && out; ++i) out[i] = c->last[i];
  return cnt;
}

int lcemd_distances(lcemd_ctx* c, const lcemd_query* q, const lcemd_opts* o, float* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  c->err.clear();
  if ((rc = check_opts(c, o))) return rc;
  if (!out) return fail(c, LCEMD_E_INVALID_ARG, "out must not be NULL");
  (void)hipSetDevice(c->device);
  prof_reset(c);
  QDev Q;
  if ((rc = stage_query(c, q, Q))) return rc;
  if ((rc = ensure_precision(c, o->precision))) return rc;
  const int64_t n = c->n;
  float* dout = out;
  if (!Q.device && (rc = wsget(c, "dist_out", (size_t)Q.B * n, dout))) return rc;
  if (o->direction == LCEMD_D2Q || o->direction == LCEMD_SYM) {
    if ((rc = run_d2q(c, Q, o, dout, n))) return rc;
  }
  if (o->direction == LCEMD_Q2D) {
    if ((rc = run_q2d_lc(c, Q, o, dout, n))) return rc;
  } else if (o->direction == LCEMD_SYM) {
    float* tmp;
    if ((rc = wsget(c, "q2d_full", (size_t)Q.B * n, tmp))) return rc;
    if ((rc = run_q2d_lc(c, Q, o, tmp, n))) return rc;
    HIPCHK(c, launch_max_inplace(dout, tmp, Q.B * n, c->stream));
  }
  if (!Q.device) {
    HIPCHK(c, hipMemcpyAsync(out, dout, sizeof(float) * Q.B * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return finish_call(c);
}

int lcemd_topl(lcemd_ctx* c, const lcemd_query* q, const lcemd_opts* o, int32_t l, int64_t* idx,
               float* dist) {
  int rc = check_ready(c);
  if (rc) return rc;
  c->err.clear();
  if ((rc = check_opts(c, o))) return rc;
  if (!idx || !dist) return fail(c, LCEMD_E_INVALID_ARG, "idx/dist must not be NULL");
  const int64_t n = c->n;
  const int64_t avail = n - (o->exclude_self >= 0 ? 1 : 0);
  if (l < 1 || l > LCEMD_MAX_L || l > avail)
    return fail(c, LCEMD_E_INVALID_ARG, "need 1 <= l <= min(%d, %lld)", LCEMD_MAX_L, (long long)avail);
  (void)hipSetDevice(c->device);
  prof_reset(c);
  QDev Q;
  if ((rc = stage_query(c, q, Q))) return rc;
  if ((rc = ensure_precision(c, o->precision))) return rc;
  const int64_t B = Q.B;
  if (o->exclude_self >= 0 && o->exclude_self + B > n)
    return fail(c, LCEMD_E_INVALID_ARG, "exclude_self + B exceeds the database size");
  int64_t* didx = idx;
  float* ddist = dist;
  if (!Q.device) {
    if ((rc = wsget(c, "topl_idx", (size_t)B * l, didx)) || (rc = wsget(c, "topl_dist", (size_t)B * l, ddist))) return rc;
  }
  const int64_t excl = o->exclude_self >= 0 ? o->exclude_self : -1;
  float* d2q;
  if ((rc = wsget(c, "d2q_full", (size_t)B * n, d2q))) return rc;
  if (o->direction == LCEMD_Q2D) {
    if ((rc = run_q2d_lc(c, Q, o, d2q, n))) return rc;
  } else {
    if ((rc = run_d2q(c, Q, o, d2q, n))) return rc;
  }
  if (o->direction != LCEMD_SYM) {
    uint64_t* cand;
    if ((rc = wsget(c, "cand", (size_t)B * l, cand))) return rc;
    if ((rc = prof_begin(c, "select", (double)B * n))) return rc;
    if ((rc = select_rows(c, d2q, n, n, B, l, nullptr, excl, cand))) return rc;
    if ((rc = prof_end(c))) return rc;
    HIPCHK(c, launch_unpack_topl(cand, l, B, nullptr, l, didx, ddist, c->stream));
  } else {
    // exact symmetric top-l by lower-bound pruning (SYM >= D2Q)
    std::vector<int32_t> rows(B);
    for (int64_t b = 0; b < B; ++b) rows[b] = (int32_t)b;
    // first round: l + max(8, l/2) candidates (enough for every query of the
    // text and image workloads); queries whose certificate fails go again
    // with four times as many
    int64_t Lp = c->sym_candidates > 0 ? std::max<int64_t>(c->sym_candidates, l)
                                       : (int64_t)l + std::max<int64_t>(8, l / 2);
    int32_t* drows;
    int* dflags;
    if ((rc = wsget(c, "sym_rows", (size_t)B, drows)) || (rc = wsget(c, "sym_flags", (size_t)B, dflags))) return rc;
    std::vector<int> hflags;
    bool first = true;
    while (!rows.empty()) {
      const int64_t R = (int64_t)rows.size();
      const int64_t use = std::min<int64_t>(Lp, avail);
      const bool exhaustive = use >= avail;
      const int64_t cld = exhaustive ? use : use + 1;
      if (cld > kSelectBuf / 2 || (!first && R >= 8 && R * 8 > B)) {
        // too many candidates for the selection buffer, or the certificate
        // failed for many queries (at least 8 and an eighth of the batch:
        // measures whose two directions differ widely, such as RWMD): the
        // whole Q2D matrix by the swapped-role linear method, SYM = max, and
        // the remaining rows selected from it
        float* q2 = nullptr;
        if ((rc = wsget(c, "q2d_full", (size_t)B * n, q2))) return rc;
        if ((rc = run_q2d_lc(c, Q, o, q2, n))) return rc;
        HIPCHK(c, launch_max_inplace(d2q, q2, B * n, c->stream));
        HIPCHK(c, hipMemcpyAsync(drows, rows.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, c->stream));
        uint64_t* cand;
        if ((rc = wsget(c, "cand", (size_t)R * l, cand))) return rc;
        if ((rc = select_rows(c, d2q, n, n, R, l, drows, excl, cand))) return rc;
        HIPCHK(c, launch_unpack_topl(cand, l, R, drows, l, didx, ddist, c->stream));
        break;
      }
      HIPCHK(c, hipMemcpyAsync(drows, rows.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, c->stream));
      uint64_t* cand;
      float* q2v;
      if ((rc = wsget(c, "cand", (size_t)R * cld, cand)) || (rc = wsget(c, "cand_q2d", (size_t)R * use, q2v))) return rc;
      if ((rc = prof_begin(c, "select", (double)R * n))) return rc;
      if ((rc = select_rows(c, d2q, n, n, R, (int)cld, drows, excl, cand))) return rc;
      if ((rc = prof_end(c))) return rc;
      P1Args a = base_args(c, Q, o);
      a.cand = cand;
      a.cand_ld = cld;
      a.cand_use = use;
      a.qlist = drows;
      a.npairs = R * use;
      if ((rc = run_pairs(c, Q, o, a, q2v, use, use))) return rc;
      HIPCHK(c, launch_finalize_sym(cand, cld, use, q2v, R, drows, n, l, didx, ddist, dflags, c->stream));
      hflags.resize(R);
      HIPCHK(c, hipMemcpyAsync(hflags.data(), dflags, sizeof(int) * R, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      std::vector<int32_t> again;
      for (int64_t i = 0; i < R; ++i)
        if (hflags[i]) again.push_back(rows[i]);
      rows.swap(again);
      Lp *= 4;
      first = false;
    }
  }
  if (!Q.device) {
    HIPCHK(c, hipMemcpyAsync(idx, didx, sizeof(int64_t) * B * l, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(dist, ddist, sizeof(float) * B * l, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return finish_call(c);
}

// lcemd_topl for callers that cannot allocate: every buffer of the call is
// carved from this device's scratch region (noalloc.hip), which the arena
// hands out for the call and reclaims when it returns.
int lcemd_topl_noalloc(lcemd_ctx* c, const lcemd_query* q, const lcemd_opts* o, int32_t l, int64_t* idx,
                       float* dist) {
  int rc = check_ready(c);
  if (rc) return rc;
  c->err.clear();
  if ((rc = check_opts(c, o))) return rc;
  if (!q || !(q->flags & LCEMD_PTR_DEVICE))
    return fail(c, LCEMD_E_INVALID_ARG, "allocation-free top-l: queries and outputs must be device pointers");
  if (!idx || !dist) return fail(c, LCEMD_E_INVALID_ARG, "idx/dist must not be NULL");
  if (o->direction != LCEMD_D2Q) return fail(c, LCEMD_E_UNSUPPORTED, "allocation-free top-l: direction D2Q only");
  if ((o->precision == LCEMD_BF16 && !c->Vb) || (o->precision == LCEMD_FP8 && !c->V8))
    return fail(c, LCEMD_E_UNSUPPORTED,
                "allocation-free top-l: load the embeddings with LCEMD_MAKE_BF16 / LCEMD_MAKE_FP8 for that precision");
  if (!c->scratch) return fail(c, LCEMD_E_HIP, "no allocation-free scratch on this device (lookup failed: %d)", c->scratch_rc);
  const int64_t n = c->n;
  const int64_t avail = n - (o->exclude_self >= 0 ? 1 : 0);
  if (l < 1 || l > LCEMD_MAX_L || l > avail)
    return fail(c, LCEMD_E_INVALID_ARG, "need 1 <= l <= min(%d, %lld)", LCEMD_MAX_L, (long long)avail);
  if (q->B < 1 || q->B > kNoAllocMaxQueries)
    return fail(c, LCEMD_E_CAPACITY, "allocation-free top-l: 1..%d queries per call", kNoAllocMaxQueries);
  const double need = (double)q->B * (double)n * 4.0 + (double)q->B * l * 8.0;
  if (need > (double)noalloc_capacity() / 2)
    return fail(c, LCEMD_E_CAPACITY,
                "allocation-free top-l: %lld queries x %lld rows need %.0f bytes of distances, over half of the %zu-byte scratch",
                (long long)q->B, (long long)n, need, noalloc_capacity());
  (void)hipSetDevice(c->device);
  // the arena for this call; profiling (events) stays off
  struct Guard {
    lcemd_ctx* c;
    bool prof;
    Guard(lcemd_ctx* c_) : c(c_), prof(c_->prof) {
      c->arena = Arena();
      c->arena.base = static_cast<char*>(c->scratch);
      c->arena.cap = noalloc_capacity();
      c->prof = false;
    }
    ~Guard() {
      c->arena = Arena();
      c->prof = prof;
    }
  } guard(c);
  prof_reset(c);
  QDev Q;
  if ((rc = stage_query(c, q, Q))) return rc;
  if (Q.hmax > kSegShort)
    return fail(c, LCEMD_E_CAPACITY, "allocation-free top-l: queries of at most %d words", kSegShort);
  const int64_t excl = o->exclude_self >= 0 ? o->exclude_self : -1;
  if (excl >= 0 && excl + Q.B > n) return fail(c, LCEMD_E_INVALID_ARG, "exclude_self + B exceeds the database size");
  float* d2q;
  uint64_t* cand;
  if ((rc = wsget(c, "d2q_full", (size_t)Q.B * n, d2q)) || (rc = wsget(c, "cand", (size_t)Q.B * l, cand))) return rc;
  if ((rc = run_d2q(c, Q, o, d2q, n))) return rc;
  if ((rc = select_rows(c, d2q, n, n, Q.B, l, nullptr, excl, cand))) return rc;
  HIPCHK(c, launch_unpack_topl(cand, l, Q.B, nullptr, l, idx, dist, c->stream));
  HIPCHK(c, hipGetLastError());
  return LCEMD_OK;
}

int lcemd_tables(lcemd_ctx* c, const lcemd_query* q, const lcemd_opts* o, int32_t* S, float* Z,
                 float* W) {
  int rc = check_ready(c);
  if (rc) return rc;
  c->err.clear();
  if (!o) return fail(c, LCEMD_E_INVALID_ARG, "opts must not be NULL");
  if (o->k < 1 || o->k > LCEMD_MAX_K) return fail(c, LCEMD_E_INVALID_ARG, "need 1 <= k <= %d", LCEMD_MAX_K);
  if (o->precision < LCEMD_FP32 || o->precision > LCEMD_BF16)
    return fail(c, LCEMD_E_UNSUPPORTED, "tables: precision must be LCEMD_FP32 or LCEMD_BF16");
  if (!S || !Z || !W) return fail(c, LCEMD_E_INVALID_ARG, "S/Z/W must not be NULL");
  (void)hipSetDevice(c->device);
  prof_reset(c);
  QDev Q;
  if ((rc = stage_query(c, q, Q))) return rc;
  const size_t total = (size_t)Q.B * c->v_used * o->k;
  int32_t* dS = S;
  float *dZ = Z, *dW = W;
  if (!Q.device) {
    if ((rc = wsget(c, "tab_S", total, dS)) || (rc = wsget(c, "tab_Z", total, dZ)) || (rc = wsget(c, "tab_W", total, dW))) return rc;
  }
  lcemd_opts oo = *o;
  oo.method = LCEMD_ACT;
  P1Args a = base_args(c, Q, &oo);
  a.qnnz = Q.nnz;
  a.k = o->k;
  a.q0 = 0;
  a.nq = Q.B;
  a.S = dS;
  a.Z = dZ;
  a.W = dW;
  if (Q.B > 65535) return fail(c, LCEMD_E_CAPACITY, "tables: at most 65535 queries per call");
  if ((rc = ensure_precision(c, o->precision))) return rc;
  int* ovf;
  int* fixc;
  if ((rc = wsget(c, "ovf", 1, ovf)) || (rc = wsget(c, "fix_count", 1, fixc)) ||
      (rc = wsget(c, "fix_list", kFixCap, a.fix_list)))
    return rc;
  HIPCHK(c, launch_zero_ints(ovf, 1, c->stream));
  HIPCHK(c, launch_zero_ints(fixc, 1, c->stream));
  a.overflow = ovf;
  a.fix_count = fixc;
  a.fix_cap = kFixCap;
  a.fix_total = c->fix_total;
  if ((rc = p1_launch(c, a, P1_TABLE_FULL, o->precision, o->k, Q.hmax, Q.hmax))) return rc;
  {
    int h_ovf = 0, h_fix = 0;
    HIPCHK(c, hipMemcpyAsync(&h_ovf, ovf, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&h_fix, fixc, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h_ovf) {
      // redo everything with float32 keys: rows listed for an exact redo by
      // the first launch are dropped (the rerun lists its own), and an
      // overflow of the rerun itself is an error
      HIPCHK(c, launch_zero_ints(ovf, 1, c->stream));
      HIPCHK(c, launch_zero_ints(fixc, 1, c->stream));
      if ((rc = p1_launch(c, a, P1_TABLE_FULL, LCEMD_FP32, o->k, Q.hmax, Q.hmax))) return rc;
      ++c->fallbacks;
      HIPCHK(c, hipMemcpyAsync(&h_ovf, ovf, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(&h_fix, fixc, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      if (h_ovf) return fail(c, LCEMD_E_CAPACITY, "tables: rows need more candidates than the kernels keep");
    }
    if (h_fix > 0) {
      HIPCHK(c, launch_fix_rows(a, P1_TABLE_FULL, h_fix, c->stream));
      HIPCHK(c, hipMemcpyAsync(&h_ovf, ovf, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      if (h_ovf) return fail(c, LCEMD_E_CAPACITY, "tables: rows need more candidates than the kernels keep");
    }
  }
  if (!Q.device) {
    HIPCHK(c, hipMemcpyAsync(S, dS, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Z, dZ, sizeof(float) * total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(W, dW, sizeof(float) * total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return finish_call(c);
}

// Self-join (Sec. 5's all-pairs protocol): every database histogram is a
// query against all others, itself excluded.  The D2Q matrix of the
// database against itself is computed once; its transpose is the Q2D
// matrix, so the symmetric matrix is the element-wise maximum of the two.
int lcemd_selfjoin_topl(lcemd_ctx* c, const lcemd_opts* o, int32_t l, uint32_t flags, int64_t* idx,
                        float* dist) {
  int rc = check_ready(c);
  if (rc) return rc;
  c->err.clear();
  if ((rc = check_opts(c, o))) return rc;
  if (o->exclude_self != -1) return fail(c, LCEMD_E_INVALID_ARG, "exclude_self must be -1 (the self-join excludes itself)");
  if (!idx || !dist) return fail(c, LCEMD_E_INVALID_ARG, "idx/dist must not be NULL");
  if (flags & ~LCEMD_PTR_DEVICE) return fail(c, LCEMD_E_INVALID_ARG, "unknown flags");
  const int64_t n = c->n;
  if (n < 2) return fail(c, LCEMD_E_INVALID_ARG, "the database needs at least 2 histograms");
  if (l < 1 || l > LCEMD_MAX_L || l > n - 1)
    return fail(c, LCEMD_E_INVALID_ARG, "need 1 <= l <= min(%d, n - 1)", LCEMD_MAX_L);
  if ((double)n * (double)n * 4.0 > (double)(int64_t(64) << 30))
    return fail(c, LCEMD_E_CAPACITY, "self-join of %lld histograms needs more than 64 GB", (long long)n);
  (void)hipSetDevice(c->device);
  prof_reset(c);
  if ((rc = ensure_precision(c, o->precision))) return rc;
  // the database as a device-resident query batch
  QDev Q;
  if ((rc = docs_as_queries(c, Q))) return rc;
  float* D;
  if ((rc = wsget(c, "selfjoin", (size_t)n * n, D))) return rc;
  lcemd_opts od = *o;
  od.direction = LCEMD_D2Q;
  if ((rc = run_d2q(c, Q, &od, D, n))) return rc;
  if (o->direction != LCEMD_D2Q) {
    if ((rc = prof_begin(c, "square", (double)n * n * 8.0))) return rc;
    HIPCHK(c, launch_square_pair(D, n, o->direction == LCEMD_SYM ? 1 : 0, c->stream));
    if ((rc = prof_end(c))) return rc;
  }
  int64_t* didx = idx;
  float* ddist = dist;
  if (!(flags & LCEMD_PTR_DEVICE)) {
    if ((rc = wsget(c, "topl_idx", (size_t)n * l, didx)) || (rc = wsget(c, "topl_dist", (size_t)n * l, ddist))) return rc;
  }
  uint64_t* cand;
  if ((rc = wsget(c, "cand", (size_t)n * l, cand))) return rc;
  if ((rc = prof_begin(c, "select", (double)n * n))) return rc;
  if ((rc = select_rows(c, D, n, n, n, l, nullptr, 0, cand))) return rc;
  if ((rc = prof_end(c))) return rc;
  HIPCHK(c, launch_unpack_topl(cand, l, n, nullptr, l, didx, ddist, c->stream));
  if (!(flags & LCEMD_PTR_DEVICE)) {
    HIPCHK(c, hipMemcpyAsync(idx, didx, sizeof(int64_t) * n * l, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(dist, ddist, sizeof(float) * n * l, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return finish_call(c);
}

// serving entry points: implemented in server.cpp
}  // extern "C"
