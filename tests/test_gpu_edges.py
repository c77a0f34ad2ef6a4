"""Degenerate and boundary cases through the C-ABI, against closed forms and
the float64 oracle: single-word histograms, a one-histogram database,
queries of the maximum length, k beyond the histogram length, embedding
widths that are not multiples of the padding, and skewed weights."""
import sys

import numpy as np
import pytest

from oracle import emd_oracle as O
from synth.generators import CSR
import parity as P

pytestmark = pytest.mark.gpu

MEASURES = [("rwmd", 1), ("omr", 1), ("act", 1), ("act", 3), ("ict", 1)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_02091_amd import lcemd

    lcemd.load_library()
    return lcemd


def _csr(rows):
    """rows: list of (cols, weights) with ascending distinct cols."""
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(c) for c, _ in rows])
    col = np.concatenate([np.asarray(c, dtype=np.int32) for c, _ in rows])
    val = np.concatenate([np.asarray(w, dtype=np.float64) / np.sum(w) for _, w in rows]).astype(np.float32)
    return CSR(ptr, col, val)


def test_single_word_histograms_are_word_distances(L):
    """One word on each side: every measure moves all mass along the single
    edge, so it equals the Euclidean distance of the two words (both
    directions, SYM)."""
    rng = np.random.default_rng(21)
    V = rng.standard_normal((50, 7)).astype(np.float32)
    db = _csr([([i], [1.0]) for i in range(0, 50, 3)])
    q = _csr([([i], [1.0]) for i in (1, 3, 49)])
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    want = np.linalg.norm(V[q.col].astype(np.float64)[:, None, :] - V[db.col].astype(np.float64)[None], axis=2)
    for method, k in MEASURES:
        for d in ("d2q", "q2d", "sym"):
            say(f"[gpu] single words {method} k={k} {d}")
            g = ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction=d)
            P.assert_distances(g, want, f"{method} {d}")
            assert g[1, 1] == 0.0  # query word 3 is database row 1's word


def test_one_histogram_database(L):
    rng = np.random.default_rng(22)
    V = rng.standard_normal((30, 16)).astype(np.float32)
    db = _csr([([2, 5, 11, 29], [0.1, 0.2, 0.3, 0.4])])
    q = _csr([([1, 5], [1.0, 3.0]), ([0, 2, 5, 11, 29], [1.0, 1.0, 2.0, 3.0, 4.0])])
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    orc = O.Oracle(V, db.rowptr, db.col, db.val)
    for method, k in MEASURES:
        o = orc.matrix(q.rowptr, q.col, q.val, method, k, "sym")
        P.assert_distances(ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction="sym"), o, method)
        idx, dist = ctx.topl(q.rowptr, q.col, q.val, 1, method=method, k=k, direction="sym")
        assert idx.ravel().tolist() == [0, 0]
        P.assert_distances(dist[:, 0], o[:, 0], method)


@pytest.mark.parametrize("m", [1, 5, 37])
def test_embedding_widths(L, m):
    """Widths far from the 64-dim padding (one slice, partial float4 groups)."""
    rng = np.random.default_rng(23 + m)
    v = 400
    V = rng.standard_normal((v, m)).astype(np.float32)
    rows = []
    for _ in range(40):
        h = int(rng.integers(1, 30))
        cols = np.sort(rng.choice(v, h, replace=False))
        rows.append((cols, rng.random(h) + 0.05))
    db = _csr(rows[:32])
    q = _csr(rows[32:])
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    orc = O.Oracle(V, db.rowptr, db.col, db.val)
    for method, k in MEASURES:
        say(f"[gpu] m={m} {method} k={k}")
        o = orc.matrix(q.rowptr, q.col, q.val, method, k, "sym")
        P.assert_distances(ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction="sym"), o,
                           f"m={m} {method}")


def test_k_beyond_histogram_length_is_ict(L):
    """ACT with k at least the query length takes every destination: ICT
    (Alg. 3 with k_eff = h)."""
    rng = np.random.default_rng(24)
    V = rng.standard_normal((200, 12)).astype(np.float32)
    cols = [np.sort(rng.choice(200, int(rng.integers(2, 9)), replace=False)) for _ in range(30)]
    rows = [(c, rng.random(c.size) + 0.1) for c in cols]
    db = _csr(rows[:24])
    q = _csr(rows[24:])
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    ict = ctx.distances(q.rowptr, q.col, q.val, method="ict", direction="d2q")
    for k in (8, 16, 64):
        g = ctx.distances(q.rowptr, q.col, q.val, method="act", k=k, direction="d2q")
        P.assert_distances(g, ict.astype(np.float64), f"k={k}")


@pytest.mark.parametrize("m", [8, 40])
def test_maximum_length_queries(L, m):
    """Queries of LCEMD_MAX_HIST words (every word of a 1,024-word
    vocabulary) against short and long database rows; m = 8 runs the 64-row
    phase-1 kernel, m = 40 the long-segment variant of the 128-row one."""
    rng = np.random.default_rng(25)
    v = L.MAX_HIST
    V = rng.standard_normal((v, m)).astype(np.float32)
    cols = [np.sort(rng.choice(v, h, replace=False)) for h in (1, 40, 700, 1024)]
    rows = [(c, rng.random(c.size) + 0.05) for c in cols]
    db = _csr(rows)
    q = _csr([(np.arange(v), rng.random(v) + 0.05), (np.arange(0, v, 2), rng.random(v // 2) + 0.05)])
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    orc = O.Oracle(V, db.rowptr, db.col, db.val)
    for method, k in (("rwmd", 1), ("act", 4), ("ict", 1)):
        say(f"[gpu] 1024-word queries m={m} {method} k={k}")
        o = orc.matrix(q.rowptr, q.col, q.val, method, k, "sym")
        P.assert_distances(ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction="sym"), o,
                           f"max length {method}")


def test_skewed_weights(L):
    """One word carries almost all the mass: capacity cuts after the first
    entry, long walks for the rest."""
    rng = np.random.default_rng(26)
    V = rng.standard_normal((300, 10)).astype(np.float32)
    rows = []
    for _ in range(36):
        h = int(rng.integers(3, 40))
        cols = np.sort(rng.choice(300, h, replace=False))
        w = np.full(h, 1e-4)
        w[int(rng.integers(h))] = 1.0
        rows.append((cols, w))
    db = _csr(rows[:30])
    q = _csr(rows[30:])
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    orc = O.Oracle(V, db.rowptr, db.col, db.val)
    for method, k in MEASURES:
        o = orc.matrix(q.rowptr, q.col, q.val, method, k, "sym")
        P.assert_distances(ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction="sym"), o,
                           f"skewed {method}")


def test_reduced_precision_copies_built_at_load(L):
    """LCEMD_MAKE_BF16 / LCEMD_MAKE_FP8 build the reduced-precision copies at
    load; the results are those of copies built at the first call that asks."""
    from synth import make_workload

    w = make_workload("text", n=150, B=5, v=4000)
    q = (w.queries.rowptr, w.queries.col, w.queries.val)
    lazy = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    eager = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, precisions=("bf16", "fp8"))
    for prec in ("bf16", "fp8"):
        say(f"[gpu] copies at load, {prec}")
        for method, k in (("act", 4), ("ict", 1)):
            i0, d0 = lazy.topl(*q, 8, method=method, k=k, direction="sym", precision=prec)
            i1, d1 = eager.topl(*q, 8, method=method, k=k, direction="sym", precision=prec)
            assert np.array_equal(i0, i1) and np.array_equal(d0, d1), (prec, method)
    with pytest.raises(ValueError):
        eager.load_embeddings(w.V, precisions=("fp16",))


def test_unknown_load_flags_rejected(L):
    """Flag bits the header does not define are LCEMD_E_INVALID_ARG, checked
    before anything loaded is dropped."""
    import ctypes as C

    rng = np.random.default_rng(27)
    V = rng.standard_normal((40, 6)).astype(np.float32)
    db = _csr([([1, 4, 9], [1.0, 2.0, 3.0]), ([0, 39], [1.0, 1.0])])
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    before = ctx.distances(db.rowptr, db.col, db.val, method="act", k=2, direction="sym")
    rc = ctx.lib.lcemd_load_embeddings(ctx.h, C.c_void_p(V.ctypes.data), 40, 6, 0x100)
    assert rc == L.E_INVALID_ARG
    rc = ctx.lib.lcemd_load_database(ctx.h, C.c_void_p(db.rowptr.ctypes.data), C.c_void_p(db.col.ctypes.data),
                                     C.c_void_p(db.val.ctypes.data), 2, 0x100)
    assert rc == L.E_INVALID_ARG
    after = ctx.distances(db.rowptr, db.col, db.val, method="act", k=2, direction="sym")
    assert np.array_equal(before, after)


MEASURES_WM = [("act", 3), ("act", 8), ("act", 16), ("rwmd", 1), ("omr", 1)]


def test_word_major_phase2_matches_per_document(L, monkeypatch):
    """Phase 2 word-major (forced here; chosen by itself when a query
    group's tables outgrow the caches): 150 queries -- two whole 64-query
    groups word-major, a 22-query tail per document -- against 300
    documents, ACT k = 3, 8 and 16 (one, four and eight table pairs per
    float4 run), RWMD and OMR: bit for bit the per-document kernel's
    distances, and the oracle's."""
    from synth import make_workload

    w = make_workload("text", n=300, B=150, v=3000)
    q = w.queries
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    got = {}
    for mode in ("1", "2"):
        monkeypatch.setenv("LCEMD_PHASE2", mode)
        ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
        for method, k in MEASURES_WM:
            say(f"[gpu] phase-2 mode {mode}: 150 x 300 {method} k={k} d2q")
            got[mode, method, k] = ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction="d2q")
        ctx.close()
    for method, k in MEASURES_WM:
        assert np.array_equal(got["1", method, k], got["2", method, k]), (method, k)
    sel = [0, 1, 63, 64, 100, 127, 128, 149]
    s = q.take(sel)
    for method, k in (("act", 8), ("rwmd", 1)):
        P.assert_distances(got["1", method, k][sel], orc.matrix(s.rowptr, s.col, s.val, method, k, "d2q"),
                           f"word-major {method}")


def test_batch_lanes_with_unaligned_rows_and_short_tail(L):
    """More than 32 queries (64 query lanes, results staged and stored 16 at
    a time) against 150 documents: output rows of odd queries start off a
    16-byte boundary and the last item of each row holds 6 documents.  The
    distances equal the oracle's, and bit for bit those of 5-query batches
    (8 query lanes, stored one by one) and of 1-4-query batches (1, 2 or 4
    query lanes, records loaded per lane)."""
    from synth import make_workload

    w = make_workload("tiny", n=150, B=40)
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    q = w.queries
    for method, k in (("rwmd", 1), ("act", 3)):
        say(f"[gpu] 40 queries x 150 documents {method} k={k} d2q")
        g = ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction="d2q")
        P.assert_distances(g, orc.matrix(q.rowptr, q.col, q.val, method, k, "d2q"), f"{method} d2q")
        for b0 in range(0, 40, 5):
            s = q.take(list(range(b0, b0 + 5)))
            part = ctx.distances(s.rowptr, s.col, s.val, method=method, k=k, direction="d2q")
            assert np.array_equal(part, g[b0:b0 + 5]), (method, b0)
        # batches of 1-4 queries: one, two or four query lanes per document
        # (each lane loads its document's records itself)
        b0 = 0
        for size in (1, 2, 3, 4, 1, 4):
            s = q.take(list(range(b0, b0 + size)))
            part = ctx.distances(s.rowptr, s.col, s.val, method=method, k=k, direction="d2q")
            assert np.array_equal(part, g[b0:b0 + size]), (method, b0, size)
            b0 += size


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_deep_ict_rows_redo_their_tile(L, prec, monkeypatch):
    """ICT rows deeper than any list the table kernels keep (Lemma 1: a word
    of weight 1 in a database histogram needs every entry of a long, flat
    query) overflow their tile, which is run again with float32 keys and
    then full-depth lists.  A small table budget (test hook) splits the batch
    into tiles of two queries, so only the middle tile overflows and its
    rerun is split again; every distance still matches the oracle."""
    rng = np.random.default_rng(31)
    nv, m = 600, 32
    V = rng.standard_normal((nv, m)).astype(np.float32)
    rows = [([w], [1.0]) for w in range(10)]  # single-word histograms: capacity 1
    for _ in range(30):
        c = np.sort(rng.choice(nv, size=int(rng.integers(5, 21)), replace=False))
        rows.append((c, rng.uniform(0.5, 2.0, size=len(c))))
    db = _csr(rows)
    qrows = []
    for h in (5, 7, 200, 300, 6, 4):
        c = np.sort(rng.choice(nv, size=h, replace=False))
        qrows.append((c, rng.uniform(0.9, 1.1, size=h)))
    q = _csr(qrows)
    monkeypatch.setenv("LCEMD_TABLE_BUDGET", str(700 * 1024))
    ctx = L.open_context(V, db.rowptr, db.col, db.val, precisions=("bf16",))
    monkeypatch.delenv("LCEMD_TABLE_BUDGET")
    orc = O.Oracle(V, db.rowptr, db.col, db.val)
    fb0, _ = ctx.counters()
    for d in ("d2q", "sym"):
        say(f"[gpu] deep ICT rows {prec} {d}")
        g = ctx.distances(q.rowptr, q.col, q.val, method="ict", k=1, direction=d, precision=prec)
        P.assert_distances(g, orc.matrix(q.rowptr, q.col, q.val, "ict", 1, d), f"ict {prec} {d}")
    fb1, fixed = ctx.counters()
    assert fb1 > fb0, "no tile was redone"
    assert fixed >= 0
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_overflowed_tiles_are_redone_after_the_pass(L, prec, monkeypatch):
    """ACT table tiles run back to back and their overflow flags are read
    once, after the last tile.  A query of 20 near-identical words (closer
    than the bf16 keys resolve) fills every row's 16-entry list with ties, so
    every row goes to the exact redo; a redo capacity of one row per tile
    (test hook) then makes each tile holding such a query overflow, and
    tiles of two queries (test hook) put those tiles beside clean ones
    (one-word queries).  The flagged tiles are run again deeper, and every
    distance and top-5 list matches the oracle."""
    rng = np.random.default_rng(32)
    nv, m = 500, 64
    V = rng.standard_normal((nv, m)).astype(np.float32)
    V[1:20] = V[0] + 1e-3 * rng.standard_normal((19, m)).astype(np.float32)
    rows = []
    for _ in range(60):
        c = np.sort(rng.choice(np.arange(20, nv), size=int(rng.integers(10, 31)), replace=False))
        rows.append((c, rng.uniform(0.5, 2.0, size=len(c))))
    db = _csr(rows)
    used = np.unique(db.col)
    dup = (np.arange(20), rng.uniform(0.5, 1.5, size=20))
    qrows = [dup if i % 3 == 0 else ([int(rng.integers(20, nv))], [1.0]) for i in range(6)]
    q = _csr(qrows)
    monkeypatch.setenv("LCEMD_TABLE_BUDGET", str(2 * len(used) * 16 + 8))
    monkeypatch.setenv("LCEMD_FIX_CAP", "1")
    ctx = L.open_context(V, db.rowptr, db.col, db.val, precisions=("bf16",))
    monkeypatch.delenv("LCEMD_TABLE_BUDGET")
    monkeypatch.delenv("LCEMD_FIX_CAP")
    orc = O.Oracle(V, db.rowptr, db.col, db.val)
    fb0, _ = ctx.counters()
    for d in ("d2q", "sym"):
        say(f"[gpu] overflowed tiles {prec} {d}")
        o = orc.matrix(q.rowptr, q.col, q.val, "act", 2, d)
        g = ctx.distances(q.rowptr, q.col, q.val, method="act", k=2, direction=d, precision=prec)
        P.assert_distances(g, o, f"act {prec} {d}")
        idx, dist = ctx.topl(q.rowptr, q.col, q.val, 5, method="act", k=2, direction=d, precision=prec)
        for b in range(q.rowptr.size - 1):
            P.check_topl(idx[b], dist[b], o[b], 5, f"act {prec} {d} query {b}")
    fb1, _ = ctx.counters()
    say(f"[gpu] overflowed tiles {prec}: {fb1 - fb0} tile redos")
    if prec == "bf16":
        assert fb1 > fb0, "no tile was redone"
    ctx.close()


@pytest.mark.parametrize("after", [0, 2, 4])
def test_refused_scratch_allocation_is_reported(L, after, monkeypatch):
    """A device allocation that fails inside a call (forced from the host:
    the test hook refuses the context's scratch allocation number `after`)
    ends the call with LCEMD_E_OOM and a message naming the buffer, leaves
    the context closable, and a context without the hook computes the same
    call correctly."""
    rng = np.random.default_rng(33)
    V = rng.standard_normal((300, 24)).astype(np.float32)
    rows = []
    for _ in range(40):
        c = np.sort(rng.choice(300, size=int(rng.integers(3, 12)), replace=False))
        rows.append((c, rng.uniform(0.5, 2.0, size=len(c))))
    db = _csr(rows)
    q = _csr(rows[:5])
    monkeypatch.setenv("LCEMD_SCRATCH_FAIL", str(after))
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    monkeypatch.delenv("LCEMD_SCRATCH_FAIL")
    say(f"[gpu] refused scratch allocation {after}")
    with pytest.raises(L.LcemdError) as ei:
        ctx.topl(q.rowptr, q.col, q.val, 3, method="act", k=2, direction="sym")
    assert ei.value.code == L.E_OOM and "refused" in str(ei.value), str(ei.value)
    ctx.close()
    ctx = L.open_context(V, db.rowptr, db.col, db.val)
    idx, dist = ctx.topl(q.rowptr, q.col, q.val, 3, method="act", k=2, direction="sym")
    o = O.Oracle(V, db.rowptr, db.col, db.val).matrix(q.rowptr, q.col, q.val, "act", 2, "sym")
    for b in range(5):
        P.check_topl(idx[b], dist[b], o[b], 3, f"after refused scratch, query {b}")
    ctx.close()
