"""Parity of the HIP path (through the C ABI) with the float64 oracle.

Sizes here finish in seconds on the oracle and still span several phase-1
row blocks, several 64-column passes (text workload: 50-300 words per
histogram, m = 300 so ten K chunks) and ragged tails; the image workload
has exact integer ties everywhere.
"""
import sys

import numpy as np
import pytest

from oracle import emd_oracle as O
from synth import make_workload
import parity as P

pytestmark = pytest.mark.gpu

METHODS = [("rwmd", 1), ("omr", 1), ("act", 1), ("act", 2), ("act", 3), ("act", 8), ("ict", 1)]


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


def _ctx(L, w):
    return L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)


@pytest.fixture(scope="module")
def tiny(L):
    w = make_workload("tiny")
    say("[gpu] tiny workload: v=2000 m=64 n=200 B=8")
    return w, _ctx(L, w), O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)


@pytest.fixture(scope="module")
def text_small(L):
    w = make_workload("text", n=150, B=5, v=4000)
    say("[gpu] text-shaped workload: v=4000 m=300 n=150 B=5")
    return w, _ctx(L, w), O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)


@pytest.fixture(scope="module")
def image_small(L):
    w = make_workload("image", n=160, B=5)
    say("[gpu] image workload: 28x28 grid n=160 B=5")
    return w, _ctx(L, w), O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)


def _q(w):
    return w.queries.rowptr, w.queries.col, w.queries.val


def _oracle_matrix(orc, w, method, k, direction):
    return orc.matrix(w.queries.rowptr, w.queries.col, w.queries.val, method, k, direction)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 3, 16])
def test_tables_tiny(tiny, k):
    w, ctx, orc = tiny
    say(f"[gpu] tables tiny k={k}")
    S, Z, W = ctx.tables(*_q(w), k=k)
    assert np.array_equal(ctx.used_vocab(), orc.used)
    diff = 0
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        So, Zo, Wo, R = orc.tables(qc, qw, k)
        d, _ = P.check_table_rows(S[b], Z[b], W[b], So, R, qw, k, qc.size)
        diff += d
    say(f"  rows differing inside the float32 tie band: {diff}")
    assert diff <= 2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("k", [4, 16])
def test_tables_text_default_kernel(text_small, k, prec):
    """Phase-1 tables at the text shape (m = 300, 50-300-word queries, several
    64-column passes and a ragged last row block) on the kernel the library
    picks by default for that precision: index sets equal the oracle's
    tie-broken sets except inside the float32 tie band, Z and W per entry."""
    w, ctx, orc = text_small
    say(f"[gpu] tables text m=300 k={k} {prec}")
    S, Z, W = ctx.tables(*_q(w), k=k, precision=prec)
    assert np.array_equal(ctx.used_vocab(), orc.used)
    diff = rows = 0
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        So, Zo, Wo, R = orc.tables(qc, qw, k)
        d, r = P.check_table_rows(S[b], Z[b], W[b], So, R, qw, k, qc.size)
        diff += d
        rows += r
    say(f"  rows differing inside the float32 tie band: {diff} of {rows}")
    assert diff <= 2


@pytest.mark.parametrize("k", [1, 4, 16])
def test_tables_image_exact_ties(image_small, k):
    """Integer grid: squared distances are exact in float32, so the index
    sets must equal the oracle's tie-broken sets bit for bit."""
    w, ctx, orc = image_small
    say(f"[gpu] tables image k={k}")
    S, Z, W = ctx.tables(*_q(w), k=k)
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        So, Zo, Wo, R = orc.tables(qc, qw, k)
        assert np.array_equal(S[b].astype(np.int64), So), b
        assert np.array_equal(W[b], Wo.astype(np.float32)), b
        assert np.allclose(Z[b], Zo, rtol=1e-6, atol=0), b


@pytest.mark.parametrize("method,k", METHODS)
@pytest.mark.parametrize("direction", ["d2q", "q2d", "sym"])
def test_distances_tiny(tiny, method, k, direction):
    w, ctx, orc = tiny
    say(f"[gpu] distances tiny {method} k={k} {direction}")
    g = ctx.distances(*_q(w), method=method, k=k, direction=direction)
    o = _oracle_matrix(orc, w, method, k, direction)
    rel = P.assert_distances(g, o, f"tiny {method}{k} {direction}")
    say(f"  max rel err {rel:.2e}")


@pytest.mark.parametrize("method,k", [("rwmd", 1), ("omr", 1), ("act", 2), ("act", 16), ("ict", 1)])
@pytest.mark.parametrize("direction", ["d2q", "sym"])
def test_distances_text(text_small, method, k, direction):
    w, ctx, orc = text_small
    say(f"[gpu] distances text {method} k={k} {direction}")
    g = ctx.distances(*_q(w), method=method, k=k, direction=direction)
    o = _oracle_matrix(orc, w, method, k, direction)
    P.assert_distances(g, o, f"text {method}{k} {direction}")


@pytest.mark.parametrize("method,k", [("rwmd", 1), ("omr", 1), ("act", 4), ("ict", 1)])
def test_distances_image(image_small, method, k):
    w, ctx, orc = image_small
    say(f"[gpu] distances image {method} k={k} sym")
    g = ctx.distances(*_q(w), method=method, k=k, direction="sym")
    o = _oracle_matrix(orc, w, method, k, "sym")
    P.assert_distances(g, o, f"image {method}{k}")


def test_act1_is_rwmd_bitwise(tiny):
    w, ctx, _ = tiny
    say("[gpu] ACT(1) == RWMD")
    for d in ("d2q", "q2d", "sym"):
        a = ctx.distances(*_q(w), method="act", k=1, direction=d)
        r = ctx.distances(*_q(w), method="rwmd", k=1, direction=d)
        assert np.array_equal(a, r), d


def test_identical_histograms_give_exact_zero(L):
    w = make_workload("tiny", n=60, B=4)
    # the queries are copies of database rows 3, 10, 11, 59
    rows = [3, 10, 11, 59]
    sub = w.db.take(rows)
    ctx = _ctx(L, w)
    say("[gpu] identical histograms -> 0")
    for method, k in METHODS:
        for d in ("d2q", "q2d", "sym"):
            g = ctx.distances(sub.rowptr, sub.col, sub.val, method=method, k=k, direction=d)
            for b, u in enumerate(rows):
                assert g[b, u] == 0.0, (method, k, d, b)
    idx, dist = ctx.topl(sub.rowptr, sub.col, sub.val, 3, method="act", k=2, direction="sym")
    assert idx[:, 0].tolist() == rows and np.all(dist[:, 0] == 0.0)


def test_ordering_chain_on_gpu(tiny):
    """Thm 2 on the GPU results: RWMD <= OMR <= ACT(2) <= ACT(3) <= ICT."""
    w, ctx, orc = tiny
    say("[gpu] ordering chain")
    for d in ("d2q", "q2d", "sym"):
        vals = [ctx.distances(*_q(w), method=m, k=k, direction=d).astype(np.float64)
                for m, k in (("rwmd", 1), ("omr", 1), ("act", 2), ("act", 3), ("ict", 1))]
        for lo, hi in zip(vals[:-1], vals[1:]):
            assert np.all(lo <= hi * (1 + 1e-5) + 1e-6), d


def test_gpu_below_exact_emd(tiny):
    """ICT <= EMD (Thm 1) on 20 seeded pairs, EMD by linear programming."""
    w, ctx, orc = tiny
    say("[gpu] ICT <= EMD on 20 pairs")
    g = ctx.distances(*_q(w), method="ict", direction="sym")
    rng = np.random.default_rng(1003)
    for _ in range(20):
        b, u = int(rng.integers(0, w.queries.n)), int(rng.integers(0, w.db.n))
        qc, qw = w.queries.row(b)
        dc, dw = w.db.row(u)
        C, _ = O.cost_matrix(w.V[dc], w.V[qc])
        p = dw.astype(np.float64) / dw.astype(np.float64).sum()
        q = qw.astype(np.float64) / qw.astype(np.float64).sum()
        assert g[b, u] <= O.emd_lp(p, q, C) * (1 + 1e-5) + 1e-6


@pytest.mark.parametrize("method,k,direction", [("act", 2, "sym"), ("act", 3, "d2q"), ("ict", 1, "sym"),
                                                ("rwmd", 1, "sym"), ("omr", 1, "q2d")])
def test_topl_tiny(tiny, method, k, direction):
    w, ctx, orc = tiny
    say(f"[gpu] top-5 tiny {method} k={k} {direction}")
    idx, dist = ctx.topl(*_q(w), 5, method=method, k=k, direction=direction)
    o = _oracle_matrix(orc, w, method, k, direction)
    swaps = sum(P.check_topl(idx[b], dist[b], o[b], 5, f"b={b}") for b in range(w.queries.n))
    assert swaps <= 2, swaps  # at most one pair of neighbours tied within tolerance


@pytest.mark.parametrize("ell", [1, 16, 150])
def test_topl_text_sym(text_small, ell):
    w, ctx, orc = text_small
    say(f"[gpu] top-{ell} text act8 sym")
    idx, dist = ctx.topl(*_q(w), ell, method="act", k=8, direction="sym")
    o = _oracle_matrix(orc, w, "act", 8, "sym")
    swaps = sum(P.check_topl(idx[b], dist[b], o[b], ell, f"b={b}") for b in range(w.queries.n))
    assert swaps <= 2, swaps


def test_topl_exclude_self(L):
    w = make_workload("tiny", n=80, B=6)
    ctx = _ctx(L, w)
    q = w.db.take(range(10, 16))
    say("[gpu] top-l with exclude_self")
    idx, dist = ctx.topl(q.rowptr, q.col, q.val, 4, method="act", k=2, direction="sym", exclude_self=10)
    for b in range(6):
        assert 10 + b not in idx[b].tolist()
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    o = orc.matrix(q.rowptr, q.col, q.val, "act", 2, "sym")
    swaps = 0
    for b in range(6):
        o[b, 10 + b] = np.inf
        swaps += P.check_topl(idx[b], dist[b], o[b], 4, f"b={b}")
    assert swaps <= 2, swaps


def test_device_pointer_path_matches_host(tiny):
    import torch

    w, ctx, _ = tiny
    say("[gpu] device-pointer path")
    dev = torch.device("cuda:0")
    qp = torch.from_numpy(w.queries.rowptr).to(dev)
    qc = torch.from_numpy(w.queries.col).to(dev)
    qv = torch.from_numpy(w.queries.val).to(dev)
    gd = ctx.distances(qp, qc, qv, method="act", k=3, direction="sym")
    torch.cuda.synchronize()
    gh = ctx.distances(*_q(w), method="act", k=3, direction="sym")
    assert np.array_equal(gd.cpu().numpy(), gh)
    i1, d1 = ctx.topl(qp, qc, qv, 5, method="ict", direction="sym")
    i2, d2 = ctx.topl(*_q(w), 5, method="ict", direction="sym")
    assert np.array_equal(i1.cpu().numpy(), i2) and np.array_equal(d1.cpu().numpy(), d2)


def test_results_do_not_depend_on_batch(tiny):
    """Each query alone gives bit-identical results to the same query inside
    the batch (fixed per-query reduction order)."""
    w, ctx, _ = tiny
    say("[gpu] alone vs batch")
    full = ctx.distances(*_q(w), method="act", k=3, direction="sym")
    for b in (0, 5, 7):
        one = w.queries.take([b])
        g = ctx.distances(one.rowptr, one.col, one.val, method="act", k=3, direction="sym")
        assert np.array_equal(g[0], full[b]), b


def test_invalid_query_rejected_before_device_work(tiny, L):
    w, ctx, _ = tiny
    bad = w.queries.val.copy()
    bad[0] = 0.0
    with pytest.raises(L.LcemdError) as e:
        ctx.distances(w.queries.rowptr, w.queries.col, bad, method="act", k=2)
    assert e.value.code == L.E_BAD_CSR
    with pytest.raises(L.LcemdError) as e:
        ctx.distances(*_q(w), method="act", k=0)
    assert e.value.code == L.E_INVALID_ARG


# ---------------------------------------------------------------------------
# bfloat16 phase-1 contraction: candidates ranked on bf16 keys with a margin,
# every listed distance recomputed exactly in float32 and re-sorted
@pytest.mark.parametrize("k", [1, 4, 16])
def test_tables_bf16_image_exact(image_small, k):
    """Grid coordinates <= 27 are exact in bfloat16 and their products sum
    exactly in float32, so even bf16 keys give the exact tie-broken sets."""
    w, ctx, orc = image_small
    say(f"[gpu] bf16 tables image k={k}")
    S, Z, W = ctx.tables(*_q(w), k=k, precision="bf16")
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        So, Zo, Wo, R = orc.tables(qc, qw, k)
        assert np.array_equal(S[b].astype(np.int64), So), b
        assert np.allclose(Z[b], Zo, rtol=1e-6, atol=0), b


@pytest.mark.parametrize("method,k", [("rwmd", 1), ("omr", 1), ("act", 3), ("act", 16), ("ict", 1)])
@pytest.mark.parametrize("wl", ["tiny", "text"])
def test_distances_bf16(tiny, text_small, method, k, wl):
    w, ctx, orc = tiny if wl == "tiny" else text_small
    say(f"[gpu] bf16 distances {wl} {method} k={k} sym")
    g = ctx.distances(*_q(w), method=method, k=k, direction="sym", precision="bf16")
    o = _oracle_matrix(orc, w, method, k, "sym")
    P.assert_distances(g, o, f"bf16 {wl} {method}{k}")


def test_topl_bf16_text(text_small):
    w, ctx, orc = text_small
    say("[gpu] bf16 top-16 text act8 sym")
    idx, dist = ctx.topl(*_q(w), 16, method="act", k=8, direction="sym", precision="bf16")
    o = _oracle_matrix(orc, w, "act", 8, "sym")
    swaps = sum(P.check_topl(idx[b], dist[b], o[b], 16, f"b={b}") for b in range(w.queries.n))
    assert swaps <= 2, swaps


@pytest.mark.parametrize("force", ["1", "2"])
def test_other_phase1_kernels(L, force, monkeypatch):
    """The 64-row streaming kernel (force=1) and the whole-row kernel
    (force=2) give the same results as the default kernel choice."""
    monkeypatch.setenv("LCEMD_FORCE_KERNEL", force)
    w = make_workload("text", n=90, B=3, v=3000)
    ctx = _ctx(L, w)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    say(f"[gpu] phase-1 kernel variant {force}")
    for method, k in (("act", 3), ("ict", 1), ("omr", 1), ("rwmd", 1)):
        g = ctx.distances(*_q(w), method=method, k=k, direction="sym")
        o = _oracle_matrix(orc, w, method, k, "sym")
        P.assert_distances(g, o, f"variant {force} {method}{k}")
    S, Z, W = ctx.tables(*_q(w), k=4)
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        So, Zo, Wo, R = orc.tables(qc, qw, 4)
        P.check_table_rows(S[b], Z[b], W[b], So, R, qw, 4, qc.size)


@pytest.mark.parametrize("direction,ell", [("d2q", 16), ("d2q", 1000), ("sym", 16), ("sym", 200)])
def test_topl_many_documents(L, direction, ell):
    """More database rows than one selection workgroup takes (two-pass
    selection): the top-l equals the first l of the full distance row
    ordered by (distance, index) -- bit for bit for D2Q; for SYM within the
    float32 tie band, since lcemd_distances computes the reverse direction
    by the swapped-role linear method and lcemd_topl per candidate pair --
    and its distances match the oracle pair by pair."""
    w = make_workload("text", n=70000, B=3, v=3000)
    ctx = _ctx(L, w)
    say(f"[gpu] top-{ell} {direction} over n=70000 (two-pass selection)")
    excl = 40000  # query b excludes row excl + b, which sits in the second part
    idx, dist = ctx.topl(*_q(w), ell, method="act", k=4, direction=direction, exclude_self=excl)
    full = ctx.distances(*_q(w), method="act", k=4, direction=direction)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    swaps = 0
    for b in range(w.queries.n):
        row = full[b].astype(np.float64).copy()
        row[excl + b] = np.inf
        order = np.lexsort((np.arange(row.size), row))[:ell]
        if direction == "d2q":
            assert np.array_equal(idx[b], order), b
            assert np.array_equal(dist[b], full[b][order]), b
        else:
            swaps += P.check_topl(idx[b], dist[b], row, ell, f"query {b}")
        qc, qw = w.queries.row(b)
        for j in range(0, ell, max(1, ell // 8)):
            o = orc.pair(qc, qw, int(idx[b, j]), "act", 4, direction)
            assert abs(float(dist[b, j]) - o) <= 1e-5 * abs(o) + 1e-7, (b, j)
    assert swaps <= 4, swaps  # the two reverse computations round differently


@pytest.mark.parametrize("wl", ["tiny", "text"])
@pytest.mark.parametrize("method,k", [("rwmd", 1), ("act", 3), ("act", 8)])
def test_distances_fp8_agreement(tiny, text_small, wl, method, k):
    """fp8 keys with a statistical band: distances are float32 values of
    the selected candidates; nearly all agree with the oracle."""
    w, ctx, orc = tiny if wl == "tiny" else text_small
    say(f"[gpu] fp8 distances {wl} {method}{k}")
    g = ctx.distances(*_q(w), method=method, k=k, direction="sym", precision="fp8")
    o = _oracle_matrix(orc, w, method, k, "sym")
    tol = 1e-5 * np.abs(o) + 1e-7 * np.mean(np.abs(o))
    ok = np.abs(g.astype(np.float64) - o) <= tol
    assert np.mean(ok) >= 0.99, np.mean(ok)
    assert np.all(np.isfinite(g)) and np.all(g >= 0)


def test_topl_fp8_text_agreement(text_small):
    w, ctx, _ = text_small
    say("[gpu] fp8 top-16 agreement with fp32")
    i32, _ = ctx.topl(*_q(w), 16, method="act", k=8, direction="sym", precision="fp32")
    i8, d8 = ctx.topl(*_q(w), 16, method="act", k=8, direction="sym", precision="fp8")
    agree = np.mean([len(set(i32[b]) & set(i8[b])) / 16 for b in range(w.queries.n)])
    assert agree >= 0.95, agree
    assert np.all(np.diff(d8, axis=1) >= 0)


def test_device_results_ordered_on_torch_stream(tiny):
    """Device-pointer calls run on torch's current stream (its default stream
    has the null handle): a copy to the host right after the call, with no
    explicit synchronisation, sees the finished results."""
    import torch

    w, ctx, _ = tiny
    dev = torch.device("cuda:0")
    q = [torch.from_numpy(x).to(dev) for x in _q(w)]
    gh = ctx.distances(*_q(w), method="act", k=2, direction="d2q")
    for _ in range(3):
        gd = ctx.distances(*q, method="act", k=2, direction="d2q")
        assert np.array_equal(gd.cpu().numpy(), gh)


@pytest.mark.parametrize("wl", ["text", "image"])
def test_phase2_lane_layouts_agree_bitwise(L, wl):
    """Phase 2 puts 64 queries of one document in a wave for batches of more
    than 32, and 32/16/8 queries of several documents (taken by length)
    below; the per-pair sums have one fixed order, so every batch size gives
    the same bits."""
    w = make_workload(wl, n=300, B=40) if wl == "image" else make_workload(wl, n=300, B=40, v=4000)
    say(f"[gpu] phase-2 lane layouts, {wl}")
    ctx = _ctx(L, w)
    big = w.queries
    full = ctx.distances(big.rowptr, big.col, big.val, method="act", k=4, direction="d2q")
    for size in (20, 12, 5, 1):
        sub = w.queries.take(list(range(size)))
        g = ctx.distances(sub.rowptr, sub.col, sub.val, method="act", k=4, direction="d2q")
        assert np.array_equal(g, full[:size]), size
