// Serving engine: continuous batching of a query stream against the resident
// database (entry points lcemd_server_* in include/lcemd.h).
//
// The memory budget is split at start into K lanes: a lane is a stream with
// its own preallocated device and pinned host buffers for up to B queries
// and W words.  Submitted queries wait in one FIFO (admission.h); a worker
// thread owns the context while the server runs, and whenever a lane is free
// and queries wait it hands the lane the FIFO head's queries at once and
// launches the lane's batch: phase 1 (tables), the exact redo of
// uncertified bf16 rows, phase 2 on a persistent kernel fed by per-XCD work
// counters, the D2Q candidate selection, Q2D for the candidates, the
// symmetric max and top-l.  Up to K batches overlap on the device.  All of a
// batch has fixed launch shapes (padding slots are empty queries; the live
// query count is read from device memory), so with use_graph it is captured
// once per lane as a hipGraph and replayed for every batch.  A query whose
// symmetric top-l certificate fails (or whose lists overflowed) is
// finished by the exact widening path of lcemd_topl.
//
// Each query's result depends only on that query: tables, per-document
// sums and the top-l selection are computed per query in a fixed order, and
// the candidate count is fixed, so a query alone and the same query in any
// mix give identical bits (and the same bits as lcemd_topl on it alone).
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "admission.h"
#include "context.h"

using namespace lcemd;
using namespace lcemd_host;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Pending {
  uint64_t ticket;
  std::vector<int32_t> col;
  std::vector<float> val;
  double t_submit;
  int words;
};

struct Done {
  std::vector<int64_t> idx;
  std::vector<float> dist;
  double latency;
  int status;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  hipGraphExec_t gexec = nullptr;
  // device
  int64_t* qptr = nullptr;
  int32_t* qcol = nullptr;
  float* qval = nullptr;
  int* nq = nullptr;
  int* ints = nullptr;  // [8] overflow, [9] rows to redo
  unsigned long long* ctr = nullptr;  // work counters of the persistent kernels
  int64_t* fixl = nullptr;
  float2* ZW = nullptr;
  float* d2q = nullptr;
  uint64_t* cand = nullptr;
  uint64_t* seltmp = nullptr;
  float* q2dv = nullptr;
  float* partial = nullptr;
  float4* rinfo = nullptr;  // bf16 phase-1 records (lane-owned: graphs capture the pointers)
  float4* qinfo = nullptr;
  float2* qmx = nullptr;
  int64_t* idx = nullptr;
  float* dist = nullptr;
  int* flags = nullptr;
  // pinned host
  int64_t* h_qptr = nullptr;
  int32_t* h_qcol = nullptr;
  float* h_qval = nullptr;
  int* h_nq = nullptr;
  int64_t* h_idx = nullptr;
  float* h_dist = nullptr;
  int* h_flags = nullptr;
  int* h_ints = nullptr;
  std::vector<Pending> batch;
  bool busy = false;
};

constexpr int kFixCapLane = 1 << 16;
constexpr int kFixBlocks = 256;

}  // namespace

struct lcemd_server {
  lcemd_ctx* ctx = nullptr;
  lcemd_server_cfg cfg{};
  int prec = LCEMD_FP32;
  int KT = 1, depth_pair = 1, use = 0, cld = 0, l = 0;
  int B = 1, W = LCEMD_SERVE_MAX_HIST;
  std::vector<Lane> lanes;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  lcemd_serve::Admission<Pending>* adm = nullptr;  // FIFO + free lanes (guarded by mu)
  std::unordered_map<uint64_t, Done> done;
  std::unordered_set<uint64_t> live;  // submitted, not yet waited for
  uint64_t next_ticket = 1;
  bool stopping = false;
  int dead = 0;  // first device error of the worker (status code)
};

namespace {

int method_depth(int method, int k, int hmax) {
  switch (method) {
    case LCEMD_RWMD: return 1;
    case LCEMD_OMR: return std::min(2, hmax);
    case LCEMD_ACT: return std::min(k, hmax);
    default: return std::min(64, hmax);
  }
}

template <typename T>
int halloc(lcemd_ctx* c, T*& p, size_t count) {
  void* q = nullptr;
  if (hipHostMalloc(&q, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, LCEMD_E_OOM, "pinned host allocation failed");
  }
  p = static_cast<T*>(q);
  return LCEMD_OK;
}

void free_lane(Lane& L) {
  if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
  void* dev[] = {L.qptr, L.qcol, L.qval, L.nq, L.ints, L.ctr, L.fixl, L.ZW, L.d2q, L.cand, L.seltmp, L.q2dv, L.partial, L.rinfo, L.qinfo, L.qmx, L.idx, L.dist, L.flags};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  void* host[] = {L.h_qptr, L.h_qcol, L.h_qval, L.h_nq, L.h_idx, L.h_dist, L.h_flags, L.h_ints};
  for (void* p : host)
    if (p) (void)hipHostFree(p);
  if (L.ev) (void)hipEventDestroy(L.ev);
  if (L.stream) (void)hipStreamDestroy(L.stream);
  L = Lane();
}

// Issue one batch's kernels on the lane's stream (also used for capture).
struct StreamSwap {
  lcemd_ctx* c;
  hipStream_t saved;
  StreamSwap(lcemd_ctx* c_, hipStream_t s) : c(c_), saved(c_->stream) { c->stream = s; }
  ~StreamSwap() { c->stream = saved; }
};

int issue(lcemd_server* s, Lane& L) {
  lcemd_ctx* c = s->ctx;
  StreamSwap swap(c, L.stream);  // p1_launch issues on the context's stream
  int rc = LCEMD_OK;
  do {
    HIPCHK(c, launch_zero_ints(L.ints, 10, L.stream));
    P1Args a;
    memset(&a, 0, sizeof a);
    a.V = c->V;
    a.vnorm = c->vnorm;
    a.m_pad = c->m_pad;
    a.m4 = (c->m + 3) / 4;
    a.method = s->cfg.method;
    a.k = s->cfg.method == LCEMD_ACT ? s->cfg.k : 1;
    a.n = c->n;
    a.xptr = c->xptr;
    a.xcv = c->xcv;
    a.xcol = c->xcol;
    a.v_used = c->v_used;
    a.used = c->used;
    a.xmax = c->xmax;
    a.qptr = L.qptr;
    a.qcol = L.qcol;
    a.qval = L.qval;
    a.q0 = 0;
    a.nq = s->B;
    a.KT = s->KT;
    a.ZW = L.ZW;
    a.zw_nq = zw_pitch(s->B);
    a.overflow = L.ints + 8;
    a.work_ctr = L.ctr;
    a.fix_count = L.ints + 9;
    a.fix_list = L.fixl;
    a.fix_cap = kFixCapLane;
    a.rinfo = L.rinfo;
    a.qinfo = L.qinfo;
    a.qmx = L.qmx;
    a.qnnz = s->W;  // the lane's word capacity (padding words are never read)
    // ICT lists stop at 16 entries as in lcemd_topl; deeper rows go to the
    // exact redo below (tables hold s->KT entries)
    const int list_depth = s->cfg.method == LCEMD_ICT ? std::min(s->KT, kIctList) : s->KT;
    if ((rc = p1_launch(c, a, P1_TABLE, s->prec, list_depth, LCEMD_SERVE_MAX_HIST, LCEMD_SERVE_MAX_HIST))) break;
    HIPCHK(c, launch_fix_rows(a, P1_TABLE, kFixBlocks, L.stream));
    HIPCHK(c, launch_phase2_persistent(c->xptr, c->xcv, c->n, c->xperm, L.ZW, zw_pitch(s->B), s->KT, s->B, L.nq,
                                       L.d2q, c->n, L.ctr + 8, L.stream));
    HIPCHK(c, launch_select(L.d2q, c->n, c->n, s->B, s->cld, nullptr, -1, L.cand, L.seltmp, L.stream));
    P1Args p = a;
    p.ZW = nullptr;
    p.fix_count = nullptr;
    p.fix_list = nullptr;
    p.fix_cap = 0;
    p.cand = L.cand;
    p.cand_ld = s->cld;
    p.cand_use = s->use;
    p.npairs = (int64_t)s->B * s->use;
    p.partial = L.partial;
    if ((rc = p1_launch(c, p, P1_PAIR, LCEMD_FP32, s->depth_pair, c->db_hmax, LCEMD_SERVE_MAX_HIST))) break;
    HIPCHK(c, launch_pair_reduce(L.partial, p.npairs, p.rb_max, L.q2dv, s->use, s->use, L.stream));
    HIPCHK(c, launch_finalize_sym(L.cand, s->cld, s->use, L.q2dv, s->B, nullptr, c->n, s->l, L.idx,
                                  L.dist, L.flags, L.stream));
  } while (0);
  return rc;
}

int setup_lane(lcemd_server* s, Lane& L) {
  lcemd_ctx* c = s->ctx;
  int rc;
  const size_t B = s->B, W = s->W, n = c->n;
  const int rbcap = (LCEMD_SERVE_MAX_HIST + kRows - 1) / kRows;
  HIPCHK(c, hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
  HIPCHK(c, hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
  if ((rc = dalloc(c, L.qptr, B + 1, "lane")) || (rc = dalloc(c, L.qcol, W, "lane")) ||
      (rc = dalloc(c, L.qval, W, "lane")) || (rc = dalloc(c, L.nq, 1, "lane")) ||
      (rc = dalloc(c, L.ints, 16, "lane")) || (rc = dalloc(c, L.ctr, 16, "lane")) || (rc = dalloc(c, L.fixl, kFixCapLane, "lane")) ||
      (rc = dalloc(c, L.ZW, zw_pitch(B) * c->v_used * 2 * zw_pairs(s->KT), "lane tables")) ||
      (rc = dalloc(c, L.d2q, B * n, "lane")) || (rc = dalloc(c, L.cand, B * s->cld, "lane")) ||
      (rc = dalloc(c, L.seltmp, select_tmp_elems(B, n, s->cld), "lane")) ||
      (rc = dalloc(c, L.q2dv, B * s->use, "lane")) ||
      (rc = dalloc(c, L.partial, B * s->use * rbcap, "lane")) ||
      (rc = dalloc(c, L.rinfo, c->v_used, "lane")) || (rc = dalloc(c, L.qinfo, W, "lane")) ||
      (rc = dalloc(c, L.qmx, B, "lane")) ||
      (rc = dalloc(c, L.idx, B * s->l, "lane")) || (rc = dalloc(c, L.dist, B * s->l, "lane")) ||
      (rc = dalloc(c, L.flags, B, "lane")))
    return rc;
  if ((rc = halloc(c, L.h_qptr, B + 1)) || (rc = halloc(c, L.h_qcol, W)) || (rc = halloc(c, L.h_qval, W)) ||
      (rc = halloc(c, L.h_nq, 1)) || (rc = halloc(c, L.h_idx, B * s->l)) ||
      (rc = halloc(c, L.h_dist, B * s->l)) || (rc = halloc(c, L.h_flags, B)) || (rc = halloc(c, L.h_ints, 16)))
    return rc;
  // an empty batch: every slot is a padding slot
  for (size_t i = 0; i <= B; ++i) L.h_qptr[i] = 0;
  *L.h_nq = 0;
  HIPCHK(c, hipMemcpyAsync(L.qptr, L.h_qptr, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, L.stream));
  HIPCHK(c, hipMemcpyAsync(L.nq, L.h_nq, sizeof(int), hipMemcpyHostToDevice, L.stream));
  if ((rc = issue(s, L))) return rc;  // warm-up (sets kernel attributes outside any capture)
  HIPCHK(c, hipStreamSynchronize(L.stream));
  if (s->cfg.use_graph) {
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(L.stream, hipStreamCaptureModeThreadLocal));
    rc = issue(s, L);
    hipError_t e = hipStreamEndCapture(L.stream, &g);
    if (rc) return rc;
    if (e != hipSuccess) return fail(c, LCEMD_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&L.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, LCEMD_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  return LCEMD_OK;
}

int launch_batch(lcemd_server* s, Lane& L) {
  lcemd_ctx* c = s->ctx;
  const int nb = (int)L.batch.size();
  int64_t nnz = 0;
  L.h_qptr[0] = 0;
  for (int i = 0; i < nb; ++i) {
    const Pending& p = L.batch[i];
    memcpy(L.h_qcol + nnz, p.col.data(), sizeof(int32_t) * p.col.size());
    memcpy(L.h_qval + nnz, p.val.data(), sizeof(float) * p.val.size());
    nnz += (int64_t)p.col.size();
    L.h_qptr[i + 1] = nnz;
  }
  for (int i = nb + 1; i <= s->B; ++i) L.h_qptr[i] = nnz;  // padding slots are empty
  *L.h_nq = nb;
  HIPCHK(c, hipMemcpyAsync(L.qptr, L.h_qptr, sizeof(int64_t) * (s->B + 1), hipMemcpyHostToDevice, L.stream));
  HIPCHK(c, hipMemcpyAsync(L.qcol, L.h_qcol, sizeof(int32_t) * std::max<int64_t>(nnz, 1), hipMemcpyHostToDevice, L.stream));
  HIPCHK(c, hipMemcpyAsync(L.qval, L.h_qval, sizeof(float) * std::max<int64_t>(nnz, 1), hipMemcpyHostToDevice, L.stream));
  HIPCHK(c, hipMemcpyAsync(L.nq, L.h_nq, sizeof(int), hipMemcpyHostToDevice, L.stream));
  if (L.gexec) {
    HIPCHK(c, hipGraphLaunch(L.gexec, L.stream));
  } else {
    int rc = issue(s, L);
    if (rc) return rc;
  }
  HIPCHK(c, hipMemcpyAsync(L.h_idx, L.idx, sizeof(int64_t) * nb * s->l, hipMemcpyDeviceToHost, L.stream));
  HIPCHK(c, hipMemcpyAsync(L.h_dist, L.dist, sizeof(float) * nb * s->l, hipMemcpyDeviceToHost, L.stream));
  HIPCHK(c, hipMemcpyAsync(L.h_flags, L.flags, sizeof(int) * nb, hipMemcpyDeviceToHost, L.stream));
  HIPCHK(c, hipMemcpyAsync(L.h_ints, L.ints, sizeof(int) * 10, hipMemcpyDeviceToHost, L.stream));
  HIPCHK(c, hipEventRecord(L.ev, L.stream));
  L.busy = true;
  return LCEMD_OK;
}

// Results of a finished lane; queries without a certificate go through the
// exact widening path of lcemd_topl.
void finish_lane(lcemd_server* s, Lane& L) {
  const int nb = (int)L.batch.size();
  const bool overflow = L.h_ints[8] != 0;
  std::vector<Done> res(nb);
  for (int i = 0; i < nb; ++i) {
    Done& d = res[i];
    d.status = LCEMD_OK;
    if (!overflow && !L.h_flags[i]) {
      d.idx.assign(L.h_idx + (size_t)i * s->l, L.h_idx + (size_t)(i + 1) * s->l);
      d.dist.assign(L.h_dist + (size_t)i * s->l, L.h_dist + (size_t)(i + 1) * s->l);
    } else {
      const Pending& p = L.batch[i];
      int64_t ptr[2] = {0, (int64_t)p.col.size()};
      lcemd_query q{ptr, p.col.data(), p.val.data(), 1, 0};
      lcemd_opts o{};
      o.method = s->cfg.method;
      o.k = s->cfg.k;
      o.direction = LCEMD_SYM;
      o.precision = s->prec;
      o.exclude_self = -1;
      d.idx.resize(s->l);
      d.dist.resize(s->l);
      d.status = lcemd_topl(s->ctx, &q, &o, s->l, d.idx.data(), d.dist.data());
    }
  }
  const double t = now_s();
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (int i = 0; i < nb; ++i) {
      res[i].latency = t - L.batch[i].t_submit;
      s->done[L.batch[i].ticket] = std::move(res[i]);
    }
  }
  s->cv_done.notify_all();
  L.batch.clear();
  L.busy = false;
}

void worker_main(lcemd_server* s) {
  (void)hipSetDevice(s->ctx->device);
  std::vector<Pending> batch;
  while (true) {
    bool any_busy = false;
    for (int li = 0; li < (int)s->lanes.size(); ++li) {
      Lane& L = s->lanes[li];
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.ev);
      if (q == hipSuccess) {
        finish_lane(s, L);
        std::lock_guard<std::mutex> g(s->mu);
        s->adm->done(li);
      } else if (q != hipErrorNotReady) {
        std::lock_guard<std::mutex> g(s->mu);
        s->dead = LCEMD_E_HIP;
        s->stopping = true;
        for (const Pending& p : L.batch) s->done[p.ticket] = Done{{}, {}, 0.0, LCEMD_E_HIP};
        L.batch.clear();
        L.busy = false;
        s->adm->done(li);
        s->cv_done.notify_all();
      } else {
        any_busy = true;
      }
    }
    int lane = -1;
    {
      std::unique_lock<std::mutex> g(s->mu);
      if (s->dead) {
        for (const Pending& p : s->adm->queue()) s->done[p.ticket] = Done{{}, {}, 0.0, s->dead};
        s->adm->queue().clear();
        s->cv_done.notify_all();
        if (!any_busy) break;
      }
      if (s->stopping && s->adm->waiting() == 0 && !any_busy) break;
      // continuous batching: a free lane takes the FIFO head's queries at once
      if (!s->dead) lane = s->adm->next(batch);
      if (lane < 0 && !any_busy) {
        s->cv_work.wait(g, [s] { return s->stopping || s->adm->waiting() > 0; });
        continue;
      }
    }
    if (lane >= 0) {
      Lane& L = s->lanes[lane];
      L.batch = std::move(batch);
      batch.clear();
      const int rc = launch_batch(s, L);
      if (rc) {
        std::lock_guard<std::mutex> g(s->mu);
        for (const Pending& p : L.batch) s->done[p.ticket] = Done{{}, {}, 0.0, rc};
        L.batch.clear();
        L.busy = false;
        s->adm->done(lane);
        s->dead = rc;
        s->cv_done.notify_all();
      }
      continue;
    }
    // lanes are busy and nothing can be admitted: wait briefly for a
    // completion or a new submission
    std::unique_lock<std::mutex> g(s->mu);
    s->cv_work.wait_for(g, std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

int lcemd_server_start(lcemd_ctx* c, const lcemd_server_cfg* cfg, lcemd_server** out) {
  if (out) *out = nullptr;
  if (!c || !cfg || !out) return LCEMD_E_INVALID_ARG;
  c->err.clear();
  if (!c->V || !c->xptr) return fail(c, LCEMD_E_NOT_LOADED, "load embeddings and database first");
  if (cfg->method < LCEMD_RWMD || cfg->method > LCEMD_ICT) return fail(c, LCEMD_E_INVALID_ARG, "unknown method");
  if (cfg->method == LCEMD_ACT && (cfg->k < 1 || cfg->k > LCEMD_MAX_K)) return fail(c, LCEMD_E_INVALID_ARG, "bad k");
  if (cfg->precision < LCEMD_FP32 || cfg->precision > LCEMD_FP8)
    return fail(c, LCEMD_E_INVALID_ARG, "unknown precision %d", cfg->precision);
  if (cfg->l < 1 || cfg->l > LCEMD_MAX_L || cfg->l > c->n) return fail(c, LCEMD_E_INVALID_ARG, "bad l");
  if (cfg->max_slots < 1) return fail(c, LCEMD_E_INVALID_ARG, "max_slots must be >= 1");
  if (cfg->lanes < 0 || cfg->lanes > 16) return fail(c, LCEMD_E_INVALID_ARG, "lanes must be 0..16");
  for (int i = 0; i < 4; ++i)
    if (cfg->reserved[i]) return fail(c, LCEMD_E_INVALID_ARG, "reserved fields must be 0");
  if (c->db_hmax > LCEMD_SERVE_MAX_HIST)
    return fail(c, LCEMD_E_CAPACITY, "serving needs database histograms of at most %d words (longest: %d)",
                LCEMD_SERVE_MAX_HIST, c->db_hmax);
  (void)hipSetDevice(c->device);
  int rc = ensure_precision(c, cfg->precision);
  if (rc) return rc;
  // the lanes' streams do not order after the context's stream
  HIPCHK(c, hipStreamSynchronize(c->stream));
  lcemd_server* s = new lcemd_server();
  s->ctx = c;
  s->cfg = *cfg;
  s->prec = cfg->precision;
  s->l = cfg->l;
  s->KT = method_depth(cfg->method, cfg->k, LCEMD_SERVE_MAX_HIST);
  s->depth_pair = method_depth(cfg->method, cfg->k, c->db_hmax);
  // candidates per query (twice the text workload's need at l = 16): a query
  // whose certificate fails is finished by lcemd_topl
  s->use = (int)std::min<int64_t>(std::max(2 * cfg->l, cfg->l + 16), c->n);
  s->cld = s->use < c->n ? s->use + 1 : s->use;
  if (s->cld > kSelectBuf / 2) s->use = kSelectBuf / 2 - 1, s->cld = s->use + 1;
  // admission by device memory: lanes x slots x per-query state <= budget
  const int nlanes = cfg->lanes > 0 ? cfg->lanes : 1;
  const double per_q = (double)c->v_used * zw_pairs(s->KT) * 16 + (double)c->n * 4 + (double)s->cld * 8 +
                       (double)s->use * 4 * (1 + (LCEMD_SERVE_MAX_HIST + kRows - 1) / kRows) + 64.0 * s->l +
                       (double)LCEMD_SERVE_MAX_HIST * 32;
  const double per_lane = (double)c->v_used * 16 + (double)kFixCapLane * 8 +
                          (double)select_tmp_elems(cfg->max_slots, c->n, s->cld) * 8;
  const int64_t budget = cfg->memory_budget > 0 ? cfg->memory_budget : (int64_t(4) << 30);
  const int fit = lcemd_serve::plan_slots(budget, per_q, per_lane, nlanes, cfg->max_slots);
  if (fit < 1) {
    delete s;
    return fail(c, LCEMD_E_CAPACITY, "memory budget %lld B holds no query (%.0f B per query, %d lanes)",
                (long long)budget, per_q, nlanes);
  }
  s->B = fit;
  s->W = cfg->max_batch_words > 0 ? std::max(cfg->max_batch_words, (int32_t)LCEMD_SERVE_MAX_HIST)
                                   : s->B * LCEMD_SERVE_MAX_HIST;
  s->adm = new lcemd_serve::Admission<Pending>(nlanes, s->B, s->W);
  s->lanes.resize(nlanes);
  for (Lane& L : s->lanes) {
    if ((rc = setup_lane(s, L))) {
      for (Lane& M : s->lanes) free_lane(M);
      delete s->adm;
      delete s;
      return rc;
    }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return LCEMD_OK;
}

int lcemd_server_submit(lcemd_server* s, const int32_t* col, const float* val, int32_t h,
                        uint64_t* ticket) {
  if (!s || !col || !val || !ticket) return LCEMD_E_INVALID_ARG;
  if (h < 1) return LCEMD_E_BAD_CSR;
  if (h > LCEMD_SERVE_MAX_HIST) return LCEMD_E_CAPACITY;
  int64_t ptr[2] = {0, h};
  lcemd_ctx scratch;
  int hm = 0;
  int rc = check_csr_host(&scratch, "query", ptr, col, val, 1, s->ctx->v, true, &hm);
  if (rc) return rc;
  Pending p;
  p.col.assign(col, col + h);
  p.val.assign(val, val + h);
  p.t_submit = now_s();
  p.words = h;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stopping) return LCEMD_E_INVALID_ARG;
    if (s->dead) return s->dead;
    if (!s->adm->fits(h)) return LCEMD_E_CAPACITY;
    p.ticket = s->next_ticket++;
    *ticket = p.ticket;
    s->live.insert(p.ticket);
    s->adm->push(std::move(p));
  }
  s->cv_work.notify_one();
  return LCEMD_OK;
}

int lcemd_server_wait(lcemd_server* s, uint64_t ticket, int64_t* idx, float* dist, double* latency_s) {
  if (!s) return LCEMD_E_INVALID_ARG;
  std::unique_lock<std::mutex> g(s->mu);
  if (!s->live.count(ticket)) return LCEMD_E_INVALID_ARG;  // unknown or already waited for
  s->live.erase(ticket);
  s->cv_done.wait(g, [&] { return s->done.count(ticket) != 0; });
  Done d = std::move(s->done[ticket]);
  s->done.erase(ticket);
  g.unlock();
  if (d.status) return d.status;
  if (idx) memcpy(idx, d.idx.data(), sizeof(int64_t) * d.idx.size());
  if (dist) memcpy(dist, d.dist.data(), sizeof(float) * d.dist.size());
  if (latency_s) *latency_s = d.latency;
  return LCEMD_OK;
}

void lcemd_server_stop(lcemd_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->ctx->device);
  for (Lane& L : s->lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    free_lane(L);
  }
  delete s->adm;
  delete s;
}

}  // extern "C"
