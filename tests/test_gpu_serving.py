"""Serving engine (continuous batching) through the C ABI.  A query's result
is the same whether it ran alone or mixed with others, with or without
hipGraph capture; for RWMD/OMR/ACT it equals lcemd_topl on the query alone
bit for bit, for ICT (64-entry tables on every query) up to float32
rounding of the distances."""
import sys
import threading

import numpy as np
import pytest

from oracle import emd_oracle as O
from synth import arrival_trace, make_workload
import parity as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_02091_amd import lcemd

    w = make_workload("text", n=300, B=2, v=4000)
    _, qs = arrival_trace(1000.0, 40, 4000, lmin=10, lmax=500)
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    say("[gpu] serving setup: v=4000 n=300, 40 queries of 10-500 words")
    return lcemd, w, qs, ctx


def _same(got, ref, method, tag):
    i, d = got
    ri, rd = ref
    if method != "ict":
        assert np.array_equal(i, ri) and np.array_equal(d, rd), tag
        return
    np.testing.assert_allclose(d, rd, rtol=1e-5, atol=1e-7, err_msg=str(tag))
    # indices may only differ where distances tie within rounding
    for j in np.nonzero(i != ri)[0]:
        assert abs(float(d[j]) - float(rd[j])) <= 1e-5 * abs(float(rd[j])) + 1e-7, (tag, j)


def _reference(ctx, qs, method, k, prec, ell):
    ref = []
    for b in range(qs.n):
        one = qs.take([b])
        i, d = ctx.topl(one.rowptr, one.col, one.val, ell, method=method, k=k, direction="sym",
                        precision=prec)
        ref.append((i[0].copy(), d[0].copy()))
    return ref


@pytest.mark.parametrize("prec,graph,method,k,lanes", [("fp32", True, "act", 8, 1), ("fp32", True, "act", 8, 3),
                                                       ("fp32", False, "act", 8, 1), ("bf16", True, "act", 8, 1),
                                                       ("bf16", True, "act", 8, 4), ("fp8", True, "act", 8, 1),
                                                       ("fp32", True, "ict", 1, 2), ("fp32", True, "omr", 1, 1)])
def test_server_matches_topl_alone_and_mixed(setup, prec, graph, method, k, lanes):
    L, w, qs, ctx = setup
    ell = 16
    say(f"[gpu] server {prec} graph={graph} {method} k={k} lanes={lanes}")
    ref = _reference(ctx, qs, method, k, prec, ell)
    srv = L.Server(ctx, method=method, k=k, precision=prec, l=ell, max_slots=16, use_graph=graph, lanes=lanes)
    try:
        # each query alone
        alone = {}
        for b in (0, 7, 23):
            c, v = qs.row(b)
            i, d, lat = srv.wait(srv.submit(c, v))
            _same((i, d), ref[b], method, b)
            alone[b] = (i, d)
            assert lat > 0
        # all queries at once from two threads (batches overlap, slots recycle)
        tickets = [None] * qs.n

        def feed(lo, hi):
            for b in range(lo, hi):
                c, v = qs.row(b)
                tickets[b] = srv.submit(c, v)

        th = [threading.Thread(target=feed, args=(0, 20)), threading.Thread(target=feed, args=(20, qs.n))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for b in range(qs.n):
            i, d, lat = srv.wait(tickets[b])
            _same((i, d), ref[b], method, b)
            if b in alone:
                assert np.array_equal(i, alone[b][0]) and np.array_equal(d, alone[b][1]), b
        with pytest.raises(L.LcemdError):
            srv.wait(tickets[0])  # each ticket is waited for once
    finally:
        srv.stop()


def test_server_rejects_bad_queries(setup):
    L, w, qs, ctx = setup
    srv = L.Server(ctx, method="act", k=4, l=8, max_slots=4)
    try:
        with pytest.raises(L.LcemdError) as e:
            srv.submit(np.arange(513), np.full(513, 1 / 513))
        assert e.value.code == L.E_CAPACITY
        with pytest.raises(L.LcemdError) as e:
            srv.submit(np.array([3, 1]), np.array([0.5, 0.5]))
        assert e.value.code == L.E_BAD_CSR
        c, v = qs.row(1)
        i, d, _ = srv.wait(srv.submit(c, v))
        assert i.shape == (8,)
    finally:
        srv.stop()


def test_server_memory_budget_too_small(setup):
    L, w, qs, ctx = setup
    with pytest.raises(L.LcemdError) as e:
        L.Server(ctx, method="act", k=8, l=8, memory_budget=1024)
    assert e.value.code == L.E_CAPACITY


@pytest.mark.parametrize("prec,graph,lanes", [("bf16", True, 1), ("bf16", True, 4), ("fp32", False, 1)])
def test_server_matches_oracle(setup, prec, graph, lanes):
    """Serving results against whole float64 oracle rows (Sec. 5 top-l,
    ACT k=8 symmetric, m = 300): ten queries of the arrival trace, the
    longest ones (300-500 words) among them, submitted together so that
    they share batches."""
    L, w, qs, ctx = setup
    lens = np.diff(qs.rowptr)
    picks = sorted(set(np.argsort(lens)[-5:].tolist()) | {0, 1, 2, 3, 4})
    assert lens[picks].max() >= 300
    say(f"[gpu] server vs oracle {prec} graph={graph} lanes={lanes}: queries of {sorted(lens[picks].tolist())} words")
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    srv = L.Server(ctx, method="act", k=8, precision=prec, l=16, max_slots=8, use_graph=graph, lanes=lanes)
    try:
        tickets = [srv.submit(*qs.row(b)) for b in picks]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.stop()
    swaps = 0
    for b, (i, d, _) in zip(picks, got):
        qc, qw = qs.row(b)
        row = orc.row_distances(qc, qw, "act", 8, "sym")
        swaps += P.check_topl(i, d, row, 16, f"query {b} ({qc.size} words)")
    assert swaps <= 2, swaps
