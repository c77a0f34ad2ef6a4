"""Dense images with their background (Sec. 5): every one of the 784 pixels
is a coordinate of every histogram, so rows are longer than the 512 words
the short kernel variants keep in LDS.  Parity against the float64 oracle
on a small batch (all measures, directions and phase-1 kernels), and at the
full 60,000-image size against the closed forms the oracle pins: RWMD is
exactly 0 and OMR = ACT(2) = sum_i max(p_i - q_i, 0) for source p."""
import sys

import numpy as np
import pytest

from oracle import emd_oracle as O
from synth import make_workload
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


@pytest.fixture(scope="module")
def small():
    w = make_workload("image-bg", n=24, B=2)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    q = (w.queries.rowptr, w.queries.col, w.queries.val)
    ref = {}
    for method, k in (("rwmd", 1), ("omr", 1), ("act", 2), ("act", 16), ("ict", 1)):
        for d in ("d2q", "q2d"):
            ref[(method, k, d)] = orc.matrix(*q, method, k, d)
        ref[(method, k, "sym")] = np.maximum(ref[(method, k, "d2q")], ref[(method, k, "q2d")])
    return w, ref


CASES = [(m, k, d) for m, k in (("rwmd", 1), ("omr", 1), ("act", 2), ("act", 16), ("ict", 1))
         for d in ("d2q", "q2d", "sym")]


@pytest.mark.parametrize("force", ["0", "1", "2"])
def test_dense_distances_match_oracle(L, small, force, monkeypatch):
    """784-word rows through the 128-row, 64-row and keys-in-device-memory
    phase-1 kernels (LCEMD_FORCE_KERNEL 0/1/2)."""
    monkeypatch.setenv("LCEMD_FORCE_KERNEL", force)
    w, ref = small
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    q = (w.queries.rowptr, w.queries.col, w.queries.val)
    for method, k, d in CASES:
        say(f"[gpu] dense 784-word rows, kernel {force}, {method} k={k} {d}")
        g = ctx.distances(*q, method=method, k=k, direction=d)
        o = ref[(method, k, d)]
        if method == "rwmd":
            assert np.all(g == 0.0), (d, g.max())
        else:
            P.assert_distances(g, o, f"{method} k={k} {d} kernel {force}")


def test_dense_topl_and_tables(L, small):
    w, ref = small
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    q = (w.queries.rowptr, w.queries.col, w.queries.val)
    for method, k in (("act", 2), ("act", 16), ("ict", 1)):
        say(f"[gpu] dense top-5 {method} k={k} sym")
        idx, dist = ctx.topl(*q, 5, method=method, k=k, direction="sym")
        swaps = sum(P.check_topl(idx[b], dist[b], ref[(method, k, "sym")][b], 5, f"{method} query {b}")
                    for b in range(w.queries.n))
        assert swaps <= 2, (method, k, swaps)
    for prec in ("bf16", "fp8"):  # long rows fall back to float32 keys: same lists
        i2, d2 = ctx.topl(*q, 5, method="act", k=2, direction="sym", precision=prec)
        i1, d1 = ctx.topl(*q, 5, method="act", k=2, direction="sym")
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)


def test_dense_selfjoin(L, small):
    w, _ = small
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    say("[gpu] dense self-join act k=2 sym")
    idx, dist = ctx.selfjoin_topl(4, method="act", k=2, direction="sym")
    swaps = 0
    for b in (0, 13):
        c, v = w.db.row(b)
        row = np.asarray(orc.row_distances(c, v, "act", 2, "sym"), dtype=np.float64)
        row[b] = np.inf
        swaps += P.check_topl(idx[b], dist[b], row, 4, f"row {b}")
    assert swaps <= 2, swaps


def test_dense_full_size_closed_forms(L):
    """60,000 dense images, 4 queries: RWMD all exactly 0; OMR and ACT(2)
    against the closed form on every one of the 240,000 pairs."""
    import torch

    w = make_workload("image-bg", B=4)
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    dev = torch.device("cuda:0")
    q = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    say("[gpu] dense full size rwmd sym")
    r = ctx.distances(*q, method="rwmd", direction="sym")
    assert bool((r == 0).all())
    # closed form for all pairs, float64: database rows are all 784 long
    X = w.db.val.astype(np.float64).reshape(w.db.n, 784)
    for method, k in (("omr", 1), ("act", 2)):
        for d in ("d2q", "q2d"):
            say(f"[gpu] dense full size {method} {d}")
            g = ctx.distances(*q, method=method, k=k, direction=d).cpu().numpy()
            for b in range(w.queries.n):
                qv = w.queries.row(b)[1].astype(np.float64)
                cf = np.maximum(X - qv, 0).sum(1) if d == "d2q" else np.maximum(qv - X, 0).sum(1)
                P.assert_distances(g[b], cf, f"{method} {d} query {b}")
    say("[gpu] dense full size top-16 act k=2 sym")
    idx, dist = ctx.topl(*q, 16, method="act", k=2, direction="sym")
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    swaps = 0
    for b in range(w.queries.n):
        qv = w.queries.row(b)[1].astype(np.float64)
        cf = np.maximum(np.maximum(X - qv, 0).sum(1), np.maximum(qv - X, 0).sum(1))
        swaps += P.check_topl(idx[b], dist[b], cf, 16, f"query {b}")
    assert swaps <= 2, swaps


def test_serving_rejects_long_database_rows(L, small):
    """Serving is sized for histograms of at most 512 words: a database of
    784-word rows is refused at start, with the context left usable."""
    w, ref = small
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    with pytest.raises(L.LcemdError):
        L.Server(ctx, method="act", k=2, l=4, max_slots=4)
    q = (w.queries.rowptr, w.queries.col, w.queries.val)
    P.assert_distances(ctx.distances(*q, method="act", k=2, direction="d2q"), ref[("act", 2, "d2q")], "after refusal")


@pytest.mark.parametrize("k", [1, 4, 16])
def test_dense_tables_exact_ties(L, small, k):
    """Phase-1 tables of 784-word queries (the long-segment kernel variant):
    on the integer grid squared distances are exact in float32, so the index
    sets equal the oracle's tie-broken sets bit for bit."""
    w, _ = small
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    say(f"[gpu] dense tables k={k}")
    S, Z, W = ctx.tables(w.queries.rowptr, w.queries.col, w.queries.val, k=k)
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        So, Zo, Wo, R = orc.tables(qc, qw, k)
        assert np.array_equal(S[b].astype(np.int64), So), b
        assert np.array_equal(W[b], Wo.astype(np.float32)), b
        assert np.allclose(Z[b], Zo, rtol=1e-6, atol=0), b
