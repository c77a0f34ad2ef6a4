"""Parity at the full workload sizes, in the configuration bench.py times
(one lcemd_topl call over the whole query batch, device-resident inputs):
the oracle computes sampled outputs one by one -- whole distance rows for
a few queries (exact top-16 check) and single (query, neighbour) pairs."""
import sys

import numpy as np
import pytest

from oracle import emd_oracle as O
from synth import make_workload
from synth.generators import sample_pairs
import parity as P

pytestmark = pytest.mark.gpu


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


def _device_topl(L, w, ell, **kw):
    import torch

    dev = torch.device("cuda:0")
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    q = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    idx, dist = ctx.topl(*q, ell, **kw)
    torch.cuda.synchronize()
    return ctx, idx.cpu().numpy(), dist.cpu().numpy()


def _check_pairs(orc, w, idx, dist, method, k, picks):
    for b, j in picks:
        qc, qw = w.queries.row(int(b))
        o = orc.pair(qc, qw, int(idx[b, j]), method, k, "sym")
        P.assert_distances(np.array([dist[b, j]]), np.array([o]), f"query {b} rank {j}")


def _check_list(idx, dist, n, ell):
    assert idx.shape[1] == ell
    assert np.all((idx >= 0) & (idx < n))
    assert np.all(np.diff(dist, axis=1) >= 0)
    for b in range(idx.shape[0]):
        assert len(set(idx[b].tolist())) == ell


def test_text_full_size(L):
    """Text workload (70,000 x 300 vocabulary, 18,000 documents, 1,000
    queries), ACT k=16 symmetric top-16, float32 and bf16 keys."""
    import torch

    w = make_workload("text")
    say("[gpu] full-size text, ACT k=16 sym top-16, fp32")
    ctx, idx, dist = _device_topl(L, w, 16, method="act", k=16, direction="sym", precision="fp32")
    _check_list(idx, dist, w.db.n, 16)
    dev = torch.device("cuda:0")
    q = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    say("[gpu] full-size text, bf16")
    ib, db = ctx.topl(*q, 16, method="act", k=16, direction="sym", precision="bf16")
    ib, db = ib.cpu().numpy(), db.cpu().numpy()
    _check_list(ib, db, w.db.n, 16)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    bs, js = sample_pairs(2, w.queries.n, 16, 24)
    _check_pairs(orc, w, idx, dist, "act", 16, zip(bs, js))
    _check_pairs(orc, w, ib, db, "act", 16, zip(bs, js))
    for b in (int(bs[0]), int(bs[1])):  # whole rows: the top-16 itself
        qc, qw = w.queries.row(b)
        row = orc.row_distances(qc, qw, "act", 16, "sym")
        swaps = P.check_topl(idx[b], dist[b], row, 16, f"query {b} fp32")
        swaps += P.check_topl(ib[b], db[b], row, 16, f"query {b} bf16")
        assert swaps <= 2, (b, swaps)
    say("[gpu] full-size text done")


def test_image_full_size(L):
    """Image workload (28x28 grid, 60,000 documents, 10,000 queries), ACT
    k=2 symmetric top-16: sampled (query, neighbour) distances."""
    w = make_workload("image")
    say("[gpu] full-size image, ACT k=2 sym top-16")
    ctx, idx, dist = _device_topl(L, w, 16, method="act", k=2, direction="sym")
    _check_list(idx, dist, w.db.n, 16)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    bs, js = sample_pairs(3, w.queries.n, 16, 24)
    _check_pairs(orc, w, idx, dist, "act", 2, zip(bs, js))
    swaps = 0
    for b in (int(bs[0]), int(bs[1])):  # whole oracle rows: all 60,000 documents
        say(f"[gpu] full-size image: oracle row of query {b}")
        qc, qw = w.queries.row(b)
        row = orc.row_distances(qc, qw, "act", 2, "sym")
        swaps += P.check_topl(idx[b], dist[b], row, 16, f"query {b}")
    assert swaps <= 2, swaps
    say("[gpu] full-size image done")


def test_text_1m_vocabulary(L):
    """1M-word vocabulary and 1M documents (the serving database), 64 of
    its queries, ACT k=8 symmetric top-16 in float32 and bf16: sampled
    (query, neighbour) distances and agreement of the two paths."""
    w = make_workload("text-1M", B=64)
    say("[gpu] 1M-word workload, 64 queries, ACT k=8 sym top-16")
    ctx, idx, dist = _device_topl(L, w, 16, method="act", k=8, direction="sym", precision="fp32")
    _check_list(idx, dist, w.db.n, 16)
    import torch

    dev = torch.device("cuda:0")
    q = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    ib, db = ctx.topl(*q, 16, method="act", k=8, direction="sym", precision="bf16")
    ib = ib.cpu().numpy()
    agree = np.mean([len(set(idx[b]) & set(ib[b])) / 16 for b in range(idx.shape[0])])
    assert agree == 1.0, agree
    bs, js = sample_pairs(4, w.queries.n, 16, 16)
    docs = sorted({int(idx[b, j]) for b, j in zip(bs, js)})
    sub = w.db.take(docs)
    pos = {u: i for i, u in enumerate(docs)}
    orc = O.Oracle(w.V, sub.rowptr, sub.col, sub.val)
    for b, j in zip(bs, js):
        qc, qw = w.queries.row(int(b))
        o = orc.pair(qc, qw, pos[int(idx[b, j])], "act", 8, "sym")
        P.assert_distances(np.array([dist[b, j]]), np.array([o]), f"query {b} rank {j}")
    say("[gpu] 1M-word workload done")


def test_text_1m_word_major_phase2(L, monkeypatch):
    """At the 1M-word size one 64-query group's tables (4 GB at k = 8) are
    far beyond the caches and phase 2 runs word-major (costs per non-zero,
    then per-document sums); 130 queries (two whole groups and a 2-query
    tail on the per-document kernel): the D2Q distances equal the
    per-document kernel's bit for bit, for ACT k=8 and RWMD."""
    import torch

    w = make_workload("text-1M", B=130)
    dev = torch.device("cuda:0")
    q = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    out = {}
    for mode in ("0", "2"):
        monkeypatch.setenv("LCEMD_PHASE2", mode)
        ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
        for method, k in (("act", 8), ("rwmd", 1)):
            say(f"[gpu] 1M-word D2Q, 130 queries, {method} k={k}, phase-2 mode {mode}")
            out[mode, method] = ctx.distances(*q, method=method, k=k, direction="d2q")
        ctx.close()
    for method in ("act", "rwmd"):
        a, b = out["0", method], out["2", method]
        assert torch.equal(a, b), (method, int((a != b).sum()))
    # and against the float64 oracle on sampled pairs of both groups and the tail
    bs, us = sample_pairs(6, 130, w.db.n, 12)
    bs = np.concatenate([bs, [0, 63, 64, 127, 128, 129]])
    us = np.concatenate([us, [5, 77, 123456, 999999, 314159, 42]])
    docs = sorted(set(int(u) for u in us))
    sub = w.db.take(docs)
    pos = {u: i for i, u in enumerate(docs)}
    orc = O.Oracle(w.V, sub.rowptr, sub.col, sub.val)
    d = out["0", "act"]
    for b, u in zip(bs, us):
        qc, qw = w.queries.row(int(b))
        o = orc.pair(qc, qw, pos[int(u)], "act", 8, "d2q")
        P.assert_distances(np.array([float(d[int(b), int(u)])]), np.array([o]), f"query {b} doc {u}")


def test_text_1m_serving_and_noalloc(L):
    """The serving path and the allocation-free call at the 1M-document
    size: queries of the arrival trace (10-500 words) served in one batch on
    one lane (the 8-lane phase-2 kernel of its live-count band) and on
    three, equal bit for bit to lcemd_topl on each query alone; and
    lcemd_topl_noalloc, whose 256 MiB region cannot hold one query's tables
    over a million used words (512 bytes per word and table pair run, 2 GB
    here), refusing with LCEMD_E_CAPACITY and leaving the context usable."""
    import torch

    from synth import arrival_trace

    w = make_workload("text-1M", B=24)
    say("[gpu] 1M-word serving and allocation-free calls")
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, precisions=("bf16",))
    _, qs = arrival_trace(1000.0, 7, w.V.shape[0], lmin=10, lmax=500)
    ref = []
    for b in range(qs.n):
        one = qs.take([b])
        i, d = ctx.topl(one.rowptr, one.col, one.val, 16, method="act", k=8, direction="sym", precision="bf16")
        ref.append((i[0], d[0]))
    for lanes in (1, 3):
        srv = L.Server(ctx, method="act", k=8, precision="bf16", l=16, max_slots=8, lanes=lanes)
        try:
            got = [srv.wait(t) for t in [srv.submit(*qs.row(b)) for b in range(qs.n)]]
        finally:
            srv.stop()
        for b, (i, d, _) in enumerate(got):
            assert np.array_equal(i, ref[b][0]) and np.array_equal(d, ref[b][1]), (lanes, b)
    dev = torch.device("cuda:0")
    s = w.queries.take([3, 9, 17])
    q = [torch.from_numpy(x).to(dev) for x in (s.rowptr, s.col, s.val)]
    out = (torch.full((s.n, 16), -1, dtype=torch.int64, device=dev),
           torch.full((s.n, 16), -1.0, dtype=torch.float32, device=dev))
    with pytest.raises(L.LcemdError) as e:
        ctx.topl_noalloc(*q, 16, out, method="act", k=8, precision="bf16")
    assert e.value.code == L.E_CAPACITY and "allocation-free" in str(e.value)
    r = ctx.topl(*q, 16, method="act", k=8, direction="d2q", precision="bf16")
    i0, d0 = ctx.topl(s.rowptr, s.col, s.val, 16, method="act", k=8, direction="d2q", precision="bf16")
    assert np.array_equal(r[0].cpu().numpy(), i0) and np.array_equal(r[1].cpu().numpy(), d0)
    ctx.close()


def certified_row(orc, qc, qw, method, k, tau, tol_frac=1e-5):
    """The oracle's symmetric distances of one query against the whole
    database wherever they can reach the top-l: every document whose
    one-sided RWMD (moving the document into the query) is at most tau plus
    tolerance is evaluated exactly; every other document is provably farther
    (SYM >= D2Q >= RWMD, Thm 2) and keeps its bound.  Returns (row, exact):
    the row and a mask of the exactly evaluated documents."""
    R = orc.query_block(qc)
    bound = orc.rwmd_d2q_all(qc, R)
    exact = bound <= tau * (1 + 4 * tol_frac) + 1e-6
    row = bound.copy()
    for u in np.nonzero(exact)[0]:
        row[u] = orc.pair(qc, qw, int(u), method, k, "sym", R)
    return row, exact


def test_text_1m_whole_rows(L):
    """1M-word vocabulary, 1M documents, ACT k=8 symmetric top-16 (the
    precision workload's shape): for one query the float32 and bf16 lists
    against its whole oracle row, certified by RWMD lower bounds -- the
    oracle evaluates exactly every document that could enter the top-16,
    and no other document can."""
    import torch

    w = make_workload("text-1M", B=16)
    say("[gpu] 1M-word workload, 16 queries, whole-row certificate")
    ctx, idx, dist = _device_topl(L, w, 16, method="act", k=8, direction="sym", precision="fp32")
    dev = torch.device("cuda:0")
    q = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    ib, db = ctx.topl(*q, 16, method="act", k=8, direction="sym", precision="bf16")
    ib, db = ib.cpu().numpy(), db.cpu().numpy()
    ctx.close()
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    # the shortest of the 16 queries keeps the oracle's vocabulary block
    # (every used word against the query's words) to a few seconds
    b = int(np.argmin(np.diff(w.queries.rowptr)))
    qc, qw = w.queries.row(b)
    tau = float(max(dist[b, -1], db[b, -1]))
    say(f"[gpu] 1M-word whole row: oracle certificate for query {b} ({qc.size} words)")
    row, exact = certified_row(orc, qc, qw, "act", 8, tau)
    say(f"  query {b}: {int(exact.sum())} documents evaluated exactly")
    assert exact[idx[b]].all() and exact[ib[b]].all()
    swaps = P.check_topl(idx[b], dist[b], row, 16, f"query {b} fp32")
    swaps += P.check_topl(ib[b], db[b], row, 16, f"query {b} bf16")
    assert swaps <= 2, swaps
