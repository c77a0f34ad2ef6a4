"""Self-join (Sec. 5's all-pairs protocol): every database histogram against
all others, itself excluded.  Checked against the float64 oracle's full
matrix (self distances masked) and against lcemd_topl with the database
rows as the query batch and exclude_self = 0."""
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
def tiny():
    w = make_workload("tiny", n=300)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    return w, orc


def _masked(M):
    M = np.array(M, dtype=np.float64)
    np.fill_diagonal(M, np.inf)
    return M


def _check_against_rows(idx, dist, rows, ell, what):
    reordered = 0
    for b in range(idx.shape[0]):
        reordered += P.check_topl(idx[b], dist[b], rows[b], ell, f"{what} row {b}")
        assert b not in set(idx[b].tolist()), f"{what}: row {b} lists itself"
    return reordered


@pytest.mark.parametrize("method,k,direction", [("act", 3, "sym"), ("rwmd", 1, "d2q"), ("omr", 1, "q2d"),
                                                ("ict", 1, "sym")])
def test_selfjoin_matches_oracle(L, tiny, method, k, direction):
    w, orc = tiny
    say(f"[gpu] self-join tiny n=300 {method} k={k} {direction}")
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    idx, dist = ctx.selfjoin_topl(5, method=method, k=k, direction=direction)
    M = _masked(orc.matrix(w.db.rowptr, w.db.col, w.db.val, method, k, direction))
    swaps = _check_against_rows(idx, dist, M, 5, f"{method} {direction}")
    assert swaps <= 6, swaps  # list positions: at most three adjacent pairs tied within tolerance


def test_selfjoin_equals_topl_on_database_rows(L, tiny):
    """Same lists as lcemd_topl over the database rows with exclude_self=0:
    D2Q bit for bit (the same kernels), symmetric within tolerance."""
    w, _ = tiny
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    q = (w.db.rowptr, w.db.col, w.db.val)
    for direction in ("d2q", "q2d", "sym"):
        say(f"[gpu] self-join vs topl, act k=2 {direction}")
        si, sd = ctx.selfjoin_topl(8, method="act", k=2, direction=direction)
        ti, td = ctx.topl(*q, 8, method="act", k=2, direction=direction, exclude_self=0)
        if direction == "d2q":
            assert np.array_equal(si, ti) and np.array_equal(sd, td)
        else:
            P.assert_distances(sd, td, direction)
            same = np.mean([len(set(si[b]) & set(ti[b])) / 8 for b in range(si.shape[0])])
            assert same >= 0.99, same


def test_selfjoin_precisions(L, tiny):
    """bf16 and fp8 keys: distances recomputed in float32, lists agree with
    the float32 self-join."""
    w, orc = tiny
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    fi, fd = ctx.selfjoin_topl(5, method="act", k=3, direction="sym", precision="fp32")
    for prec in ("bf16", "fp8"):
        say(f"[gpu] self-join tiny act k=3 sym {prec}")
        pi, pd = ctx.selfjoin_topl(5, method="act", k=3, direction="sym", precision=prec)
        agree = np.mean([len(set(fi[b]) & set(pi[b])) / 5 for b in range(fi.shape[0])])
        assert agree >= 0.98, (prec, agree)
        for b in range(0, fi.shape[0], 37):
            c, v = w.db.row(b)
            row = np.asarray(orc.row_distances(c, v, "act", 3, "sym"), dtype=np.float64)
            P.assert_distances(pd[b], row[pi[b]], f"{prec} row {b}")


def test_selfjoin_image_rows(L):
    """Image shape (28x28 grid, ACT k=2 symmetric) with 1,500 histograms:
    two whole oracle rows and the device-pointer output form."""
    import torch

    w = make_workload("image", n=1500, B=4)
    say("[gpu] self-join image n=1500 act k=2 sym")
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    idx, dist = ctx.selfjoin_topl(16, method="act", k=2, direction="sym", device=True)
    torch.cuda.synchronize()
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    hi, hd = ctx.selfjoin_topl(16, method="act", k=2, direction="sym")
    assert np.array_equal(idx, hi) and np.array_equal(dist, hd)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    swaps = 0
    for b in (7, 1234):
        c, v = w.db.row(b)
        row = np.asarray(orc.row_distances(c, v, "act", 2, "sym"), dtype=np.float64)
        row[b] = np.inf
        swaps += P.check_topl(idx[b], dist[b], row, 16, f"image row {b}")
    assert swaps <= 2, swaps
    assert np.all(np.diff(dist, axis=1) >= 0)


def test_selfjoin_rejects(L, tiny):
    w, _ = tiny
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    for kw in (dict(l=0), dict(l=300), dict(l=5, exclude_self=0)):
        l = kw.pop("l")
        with pytest.raises(L.LcemdError):
            ctx.selfjoin_topl(l, method="act", k=2, direction="sym", **kw)
    i, d = ctx.selfjoin_topl(299, method="rwmd", direction="d2q")  # l = n - 1: every other row
    assert all(sorted(i[b].tolist()) == [x for x in range(300) if x != b] for b in range(0, 300, 50))


def test_selfjoin_two_histograms(L):
    """The smallest self-join: each of two histograms has the other as its
    only neighbour, at the oracle's symmetric distance."""
    w = make_workload("tiny", n=2, B=1)
    ctx = L.open_context(w.V, w.db.rowptr, w.db.col, w.db.val)
    idx, dist = ctx.selfjoin_topl(1, method="act", k=2, direction="sym")
    assert idx[:, 0].tolist() == [1, 0]
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    c, v = w.db.row(0)
    o = orc.row_distances(c, v, "act", 2, "sym")[1]
    P.assert_distances(dist[:, 0], np.array([o, o]), "two histograms")
