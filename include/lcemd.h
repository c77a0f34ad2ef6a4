/*
 * lcemd: linear-complexity lower bounds of the Earth Mover's Distance on one
 * MI355X (gfx950), after Atasu & Mittelholzer, "Low-Complexity Data-Parallel
 * Earth Mover's Distance Approximations" (ICML 2019).
 *
 * Problem (Sec. 2.2 and Sec. 4): a vocabulary of v words with m-dimensional
 * embeddings V (v x m), a database X of n histograms over that vocabulary
 * (sparse rows, weights summing to 1), and a batch of B query histograms over
 * the same vocabulary.  For every (query, database histogram) pair the
 * library computes a lower bound of the EMD with Euclidean ground cost
 * (Sec. 5):
 *
 *   RWMD  one-sided relaxed WMD (Sec. 2.1); equal to ACT with k = 1
 *   OMR   overlapping mass reduction (Alg. 1)
 *   ACT   approximate iterative constrained transfers, k >= 1 (Alg. 3)
 *   ICT   iterative constrained transfers (Alg. 2)
 *
 * in direction D2Q (move the database histogram into the query: the LC
 * direction of Sec. 4), Q2D (move the query into the database histogram) or
 * SYM (the maximum of the two, Sec. 2.1 and Sec. 5), and returns either the
 * full B x n distance matrix or the l nearest database histograms per query
 * (Sec. 5, top-l search).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Return value: LCEMD_OK (0) on success, a negative LCEMD_E_* code on
 *   failure; lcemd_last_error() then describes the failure.  No C++
 *   exception crosses this interface.  On failure, caller-owned outputs are
 *   left untouched unless the failure is LCEMD_E_HIP (a device error after
 *   work was issued).
 * - Validation of every argument (shapes, CSR structure, weights) happens
 *   before any device work is issued.
 * - Histograms are CSR: rowptr (int64, rows+1, rowptr[0] == 0,
 *   non-decreasing, no empty rows), col (int32 word ids in [0, v), strictly
 *   increasing within a row), val (float32, finite and > 0, each row sums to
 *   1 within 1e-5).  Explicit zeros are rejected: a zero-weight bin would take
 *   a top-k slot in Alg. 3.
 * - Pointer residency: without LCEMD_PTR_DEVICE every array argument is host
 *   memory and every call returns with its outputs complete.  With
 *   LCEMD_PTR_DEVICE every array argument of that call (inputs and outputs)
 *   is device memory on the context's device; outputs are then ordered on
 *   the context's stream.
 * - Ownership: loads copy into library-owned device memory (the caller may
 *   free its arrays on return); queries and outputs stay caller-owned.
 *   Scratch (tables, distance matrices, candidate lists) is allocated by the
 *   context on first need, grows but never shrinks, and is freed by
 *   lcemd_destroy: a self-join of n histograms keeps its n^2 floats.
 * - A context is not thread-safe; calls on one context must be serialised.
 */
#ifndef LCEMD_H
#define LCEMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LCEMD_VERSION 1

/* status codes */
#define LCEMD_OK 0
#define LCEMD_E_INVALID_ARG (-1) /* bad scalar argument or NULL pointer */
#define LCEMD_E_BAD_CSR (-2)     /* malformed histogram CSR or weights */
#define LCEMD_E_NOT_LOADED (-3)  /* embeddings or database not loaded yet */
#define LCEMD_E_OOM (-4)         /* device allocation failed */
#define LCEMD_E_HIP (-5)         /* HIP runtime / kernel launch failure */
#define LCEMD_E_UNSUPPORTED (-6) /* option combination not implemented */
#define LCEMD_E_CAPACITY (-7)    /* a size exceeds a documented limit */
#define LCEMD_E_NO_DEVICE (-8)   /* no usable GPU */

/* distance measures */
#define LCEMD_RWMD 0
#define LCEMD_OMR 1
#define LCEMD_ACT 2
#define LCEMD_ICT 3

/* directions */
#define LCEMD_D2Q 0
#define LCEMD_Q2D 1
#define LCEMD_SYM 2

/* arithmetic of the phase-1 distance contraction (candidate selection);
 * the selected candidates' distances are always recomputed in float32 from
 * the float32 embeddings.  LCEMD_FP32 and LCEMD_BF16 select exactly (bf16
 * keys keep every candidate within a worst-case error band and rows whose
 * certificate fails are redone in float32).  LCEMD_FP8 (OCP e4m3 codes,
 * one float32 scale per embedding row) uses a statistical band instead of
 * the worst-case one (which would keep nearly every candidate): its
 * results agree with the float32 path with high probability, not always. */
#define LCEMD_FP32 0
#define LCEMD_BF16 1
#define LCEMD_FP8 2

/* flags */
#define LCEMD_PTR_DEVICE 0x1u  /* array arguments are device pointers */
#define LCEMD_NORMALIZE 0x2u   /* load_database: renormalise rows (float64 sums) */
#define LCEMD_L2_NORMALIZE 0x4u /* load_embeddings: scale rows to unit L2 norm */
#define LCEMD_MAKE_BF16 0x8u    /* load_embeddings: build the bfloat16 copy now */
#define LCEMD_MAKE_FP8 0x10u    /* load_embeddings: build the fp8 copy now */

/* limits */
#define LCEMD_MAX_HIST 1024 /* max non-zeros of one query or database row (dense
                               28x28 images with background: 784) */
#define LCEMD_SERVE_MAX_HIST 512 /* serving: max words of a query or database row */
#define LCEMD_MAX_L 1024    /* max l of lcemd_topl */
#define LCEMD_MAX_K 512     /* max k of ACT */

typedef struct lcemd_ctx lcemd_ctx;

typedef struct {
  const int64_t* rowptr; /* B+1 row pointers */
  const int32_t* col;    /* word ids */
  const float* val;      /* weights */
  int64_t B;             /* number of queries, >= 1 */
  uint32_t flags;        /* LCEMD_PTR_DEVICE: rowptr/col/val and the call's
                            outputs are device pointers */
} lcemd_query;

typedef struct {
  int32_t method;       /* LCEMD_RWMD / OMR / ACT / ICT */
  int32_t k;            /* ACT only: 1 <= k <= LCEMD_MAX_K; ignored otherwise */
  int32_t direction;    /* LCEMD_D2Q / Q2D / SYM */
  int32_t precision;    /* LCEMD_FP32 / BF16 / FP8 */
  int32_t exclude_self; /* lcemd_topl: if >= 0, query b never returns
                           database row (exclude_self + b) (self-join use) */
  int32_t reserved[3];  /* must be 0 */
} lcemd_opts;

/* Library version (LCEMD_VERSION). */
int lcemd_version(void);

/* Create a context on HIP device `device` (its own default-priority stream
 * until lcemd_set_stream).  *out receives the context.  Errors:
 * LCEMD_E_NO_DEVICE if the device does not exist or is not gfx950,
 * LCEMD_E_INVALID_ARG if out is NULL, LCEMD_E_OOM if its 8-byte device
 * counter cannot be allocated.  Test hooks, read from the environment here:
 * LCEMD_FORCE_KERNEL (1: skip the 128-row phase-1 kernel, 2: deep kernel),
 * LCEMD_SYM_CANDIDATES (first candidate count of the symmetric top-l),
 * LCEMD_PHASE2 (1: word-major phase 2 where possible, 2: per document),
 * LCEMD_TABLE_BUDGET (bytes of phase-1 tables per tile; default 12 GiB),
 * LCEMD_FIX_CAP (rows per table tile that may be redone exactly; a tile
 * with more uncertified rows is run again with float32 keys),
 * LCEMD_SCRATCH_FAIL (scratch allocations granted before the next one is
 * refused with LCEMD_E_OOM, as if the device were out of memory). */
int lcemd_create(lcemd_ctx** out, int device);

/* Free all library-owned device memory and the context.  NULL-safe. */
void lcemd_destroy(lcemd_ctx* ctx);

/* Issue all further work of this context on `hip_stream` (a hipStream_t;
 * NULL is HIP's null stream, not the library's own).  The caller keeps
 * ownership.  Device-pointer calls are ordered on this stream only. */
int lcemd_set_stream(lcemd_ctx* ctx, void* hip_stream);
/* Go back to the context's own (non-blocking) stream. */
int lcemd_use_own_stream(lcemd_ctx* ctx);

/* Message of the last failing call on this context (context-owned string;
 * "" if none).  Also valid for ctx == NULL (then: last lcemd_create error). */
const char* lcemd_last_error(const lcemd_ctx* ctx);

/* Load the vocabulary embeddings V: v rows of m float32 (row-major, finite),
 * the coordinates of Sec. 4's matrix V.  Replaces earlier embeddings (and
 * drops a loaded database).  Builds the device-side padded copy, the row
 * norms (accumulated in float64) and the bfloat16 / fp8 copies: at load
 * with LCEMD_MAKE_BF16 / LCEMD_MAKE_FP8, else at the first call that asks
 * for that precision (the copies are the same either way).  Flags:
 * LCEMD_PTR_DEVICE, LCEMD_L2_NORMALIZE, LCEMD_MAKE_BF16, LCEMD_MAKE_FP8;
 * other bits are LCEMD_E_INVALID_ARG.  If a copy asked for by a MAKE flag
 * cannot be allocated (LCEMD_E_OOM), the float32 embeddings stay loaded.
 * Limits: 1 <= v < 2^31, 1 <= m <= 4096. */
int lcemd_load_embeddings(lcemd_ctx* ctx, const float* V, int64_t v, int32_t m,
                          uint32_t flags);

/* Load the database X (Sec. 4: n histograms over the vocabulary, kept in
 * CSR).  Requires embeddings.  Derives the used vocabulary (the union of
 * the database's words, Sec. 2.2) and, per used word, the largest weight
 * any database row gives it (bounds how deep a transfer can go).  Flags:
 * LCEMD_PTR_DEVICE, LCEMD_NORMALIZE (other bits: LCEMD_E_INVALID_ARG).
 * Limits: n >= 1, at most
 * LCEMD_MAX_HIST non-zeros per row. */
int lcemd_load_database(lcemd_ctx* ctx, const int64_t* rowptr, const int32_t* col,
                        const float* val, int64_t n, uint32_t flags);

/* All B x n distances (row-major float32, out[b*n + u]) between the query
 * batch and the database for one measure and direction (Sec. 2.1, Alg. 1-3,
 * Sec. 4).  Queries: at most LCEMD_MAX_HIST words each. */
int lcemd_distances(lcemd_ctx* ctx, const lcemd_query* q, const lcemd_opts* o,
                    float* out);

/* The l nearest database rows per query (Sec. 5 top-l search), ascending by
 * (distance, database row index): idx[b*l + r] (int64) and dist[b*l + r]
 * (float32).  1 <= l <= min(n, LCEMD_MAX_L).  SYM is evaluated exactly with
 * lower-bound pruning: SYM >= D2Q, so only rows whose D2Q value can still
 * enter the result get a Q2D evaluation. */
int lcemd_topl(lcemd_ctx* ctx, const lcemd_query* q, const lcemd_opts* o,
               int32_t l, int64_t* idx, float* dist);

/* lcemd_topl for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * top-l, but every buffer of the call (tables, the D2Q distance rows,
 * candidate lists, counters) comes from a fixed 256 MiB device region that
 * the library holds per GPU from its first use there to process end; the
 * call itself allocates nothing, host or device.  Restrictions:
 * LCEMD_PTR_DEVICE (queries and outputs in device memory), direction D2Q,
 * 1..4096 queries of at most 512 words, B x n distances within half the
 * region, and one query's tables (512 x ceil(KT / 2) bytes per used
 * vocabulary word: about 260,000 words at k <= 2, 65,000 at k = 8) within
 * what is left (LCEMD_E_CAPACITY otherwise); bf16 / fp8 keys need their copy built at load
 * (LCEMD_MAKE_BF16 / LCEMD_MAKE_FP8), else LCEMD_E_UNSUPPORTED.  Results
 * equal lcemd_topl's (same kernels).  Every call on a GPU shares that GPU's
 * region and leaves its contents behind (what must start at zero is cleared
 * by each call): calls that overlap on one GPU -- from several contexts or
 * threads -- race and must be serialised by the caller. */
int lcemd_topl_noalloc(lcemd_ctx* ctx, const lcemd_query* q, const lcemd_opts* o, int32_t l,
                       int64_t* idx, float* dist);

/* Phase-1 tables of Sec. 4 for every query and every used vocabulary word
 * (used words in ascending word id order; lcemd_used_vocab lists them):
 * S = positions (0-based, within the query row) of the k_eff = min(k, h_b)
 * nearest query words, ascending by (distance, position); Z = their
 * distances; W = their query weights.  Layout [b][used word][k]; entries
 * l >= k_eff hold S = -1, Z = 0, W = 0.  Uses o->k and o->precision; method
 * and direction are ignored.  Meant for verification: B x used x k entries. */
int lcemd_tables(lcemd_ctx* ctx, const lcemd_query* q, const lcemd_opts* o,
                 int32_t* S, float* Z, float* W);

/* Host-only check (no device needed) that `rows` histograms in host memory
 * follow the CSR conventions above over a vocabulary of v words, with row
 * sums checked when require_normalized != 0.  Returns LCEMD_OK,
 * LCEMD_E_BAD_CSR, LCEMD_E_CAPACITY or LCEMD_E_INVALID_ARG; a description of
 * the first violation is written to msg (msg_cap bytes, may be NULL).  The
 * same check guards every call that takes histograms. */
int lcemd_check_histograms(const int64_t* rowptr, const int32_t* col, const float* val,
                           int64_t rows, int64_t v, int require_normalized, char* msg,
                           size_t msg_cap);

/* Number of used vocabulary words (after lcemd_load_database); if ids is
 * non-NULL also writes them (host int32, ascending). */
int64_t lcemd_used_vocab(lcemd_ctx* ctx, int32_t* ids);

/* Self-join (Sec. 5, the all-pairs protocol): the l nearest neighbours of
 * every database histogram among the others (itself excluded), by the
 * measure, direction and precision of `opts` (exclude_self must be -1).
 * The D2Q matrix of the database against itself is formed once in device
 * memory (n^2 float32, at most 64 GB); Q2D is its transpose and SYM the
 * element-wise maximum of the two.  idx/dist: n * l entries, row b holding
 * database row b's neighbours in ascending (distance, index) order; host
 * arrays, or device arrays with flags = LCEMD_PTR_DEVICE (filled on the
 * context's stream).  LCEMD_E_CAPACITY if n^2 floats exceed 64 GB. */
int lcemd_selfjoin_topl(lcemd_ctx* ctx, const lcemd_opts* opts, int32_t l, uint32_t flags,
                        int64_t* idx, float* dist);

/* Per-kernel timing of the most recent lcemd_distances / lcemd_topl call
 * when enabled: device time measured with HIP events on the context's
 * stream.  lcemd_profile(ctx, 1) enables recording; lcemd_profile_get fills
 * up to `cap` entries and returns how many there are. */
typedef struct {
  char name[48];     /* kernel / phase name */
  double ms;         /* summed device time of its launches in the call */
  int64_t launches;  /* launches in the call */
  double work;       /* algorithmic units processed (bytes or flops) */
} lcemd_phase_time;
int lcemd_profile(lcemd_ctx* ctx, int enable);
/* Cumulative counts since lcemd_create: query tiles whose phase 1 was redone
 * with float32 keys or deeper lists (a row needed more candidates than the
 * fast kernels keep), and bfloat16 table rows whose exactness certificate
 * failed and that were redone one by one with float32 distances (counted on
 * the device: reading it waits for the context's stream).  Either pointer
 * may be NULL. */
int lcemd_counters(lcemd_ctx* ctx, int64_t* fallback_tiles, int64_t* exact_rows);
int lcemd_profile_get(lcemd_ctx* ctx, lcemd_phase_time* out, int cap);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of a query stream against the resident
 * database, returning each query's symmetric top-l (the top-l search of
 * Sec. 5, with the exact pruning of lcemd_topl).  The device memory budget
 * is split at start into `lanes` launch lanes, each a stream with
 * preallocated device and pinned host buffers for up to B queries and W
 * words.  Submitted queries wait in one FIFO; whenever a lane is free and
 * queries wait, the lane takes the FIFO head's queries (as many as fit its
 * B slots and W words) and launches at once -- no batch waits to fill, and
 * queries that arrive while other batches run join the next free lane, so
 * up to `lanes` batches overlap on the device.  One lane is the default: a
 * batch's phase-1 and phase-2 kernels each fill every CU, so overlapping
 * batches add no throughput and lengthen each other; with one lane the
 * next batch starts the moment the previous one ends, with every query
 * that arrived meanwhile.  A batch runs phase 1
 * tables, the exact redo of uncertified rows, phase 2 on persistent
 * kernels fed by per-XCD work counters (one per query-lane width; the one
 * whose band holds the live query count does the work), D2Q candidate
 * selection, Q2D of the
 * candidates and the symmetric top-l, and completes each query
 * independently.  A query whose top-l certificate fails, or whose lists
 * overflowed, is finished by lcemd_topl.  lcemd_serve_sim runs the same
 * admission policy on the host against a fake executor.
 *
 * Results depend only on the query, never on the others sharing a batch.
 * For RWMD, OMR and ACT (k <= the query's word count) they are also the
 * bits lcemd_topl gives for the query alone; ICT serves with 64-entry
 * tables on every query, so its results can differ from lcemd_topl's
 * (whose first-try depth follows the batch) by float32 rounding.
 *
 * While a server runs, its worker thread owns the context: make no other
 * call on that context until lcemd_server_stop returns.
 * --------------------------------------------------------------------- */
typedef struct lcemd_server lcemd_server;

typedef struct {
  int32_t method;          /* as lcemd_opts */
  int32_t k;               /* ACT only, 1..LCEMD_MAX_K */
  int32_t precision;       /* LCEMD_FP32, LCEMD_BF16 or LCEMD_FP8 */
  int32_t l;               /* neighbours returned per query, 1..min(LCEMD_MAX_L, n) */
  int32_t max_slots;       /* queries per batch (>= 1); lowered to fit memory_budget */
  int32_t max_batch_words; /* words per batch (raised to LCEMD_SERVE_MAX_HIST); 0 = no limit */
  int64_t memory_budget;   /* device bytes for all lanes' buffers; 0 = 4 GiB */
  int32_t use_graph;       /* nonzero: each lane's batch replayed as a captured hipGraph;
                              zero: kernels launched per batch */
  int32_t lanes;           /* batches in flight, 0..16; 0 = 1 (see above) */
  int32_t reserved[4];     /* must be 0 */
} lcemd_server_cfg;

/* Allocates every lane buffer up front: B = the slots per lane that the
 * budget allows (lanes x B x per-query bytes within memory_budget), at most
 * max_slots.  LCEMD_E_CAPACITY if the budget holds no query or a database
 * histogram has more than LCEMD_SERVE_MAX_HIST words.  *out is NULL on
 * error. */
int lcemd_server_start(lcemd_ctx* ctx, const lcemd_server_cfg* cfg, lcemd_server** out);
/* Queue one query (host arrays of h words: ascending distinct ids < v,
 * finite weights > 0 summing to 1 within 1e-5; copied before return).  *ticket gets its id.
 * LCEMD_E_BAD_CSR for a malformed query, LCEMD_E_CAPACITY for h >
 * LCEMD_SERVE_MAX_HIST.  Thread-safe. */
int lcemd_server_submit(lcemd_server* s, const int32_t* col, const float* val, int32_t h,
                        uint64_t* ticket);
/* Block until `ticket` completes; writes l (idx, dist) pairs in ascending
 * distance and the seconds from submit to completion (any output pointer
 * may be NULL).  Each ticket is waited for once; unknown or already waited
 * tickets give LCEMD_E_INVALID_ARG.  Thread-safe. */
int lcemd_server_wait(lcemd_server* s, uint64_t ticket, int64_t* idx, float* dist,
                      double* latency_s);
/* Finish every queued query, stop the worker and free the server (results
 * not yet waited for are dropped).  NULL-safe. */
void lcemd_server_stop(lcemd_server* s);

/* The serving admission policy run on the host (no GPU) against a fake
 * executor on a virtual clock, for testing it: nq queries arriving at
 * arrival_s[i] (non-decreasing) with words[i] words; `lanes` lanes whose
 * slots per lane are planned from budget and per_query_bytes like the
 * server's (at most max_slots), max_words words per lane; a launch of q
 * queries lasts t_fixed_s + t_per_query_s * q.  Per query: status
 * (LCEMD_OK, or LCEMD_E_CAPACITY when it has more than max_words words and
 * is refused), lane and launch index (-1 if refused), start and finish time.
 * Returns the slots per lane (> 0), LCEMD_E_CAPACITY if the budget holds
 * no query, LCEMD_E_INVALID_ARG for bad arguments.  All arrays are host
 * memory of nq entries, caller-owned. */
int lcemd_serve_sim(int32_t nq, const double* arrival_s, const int32_t* words, int32_t lanes,
                    int32_t max_slots, int32_t max_words, int64_t budget, double per_query_bytes,
                    double t_fixed_s, double t_per_query_s, int32_t* status, int32_t* lane,
                    int32_t* launch, double* start_s, double* finish_s);

#ifdef __cplusplus
}
#endif
#endif /* LCEMD_H */
