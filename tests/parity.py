"""Comparison rules between the HIP path and the float64 oracle.

Float32 distances: |gpu - oracle| <= 1e-5 * |oracle| + 1e-7 * mean_nonzero,
and exactly 0 where the oracle is exactly 0 (identical histograms).

Index sets (phase-1 tables S, top-l lists) must match exactly, except inside
a tie band: where the oracle's float64 keys of two candidates differ by less
than float32 can resolve, either order is accepted (and counted).
"""
import numpy as np

REL = 1e-5
ABS_FRAC = 1e-7


def dist_tol(oracle: np.ndarray) -> np.ndarray:
    o = np.abs(np.asarray(oracle, dtype=np.float64))
    nz = o[o > 0]
    cbar = float(nz.mean()) if nz.size else 1.0
    return REL * o + ABS_FRAC * cbar


def assert_distances(gpu, oracle, what=""):
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(oracle, dtype=np.float64)
    assert g.shape == o.shape, (what, g.shape, o.shape)
    assert np.all(np.isfinite(g)), what
    tol = dist_tol(o)
    err = np.abs(g - o)
    bad = err > tol
    if bad.any():
        i = np.unravel_index(np.argmax(err - tol), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {g.size} outside tolerance; worst at {i}: "
                             f"gpu={g[i]!r} oracle={o[i]!r} tol={tol[i]!r}")
    zero = o == 0.0
    assert np.all(g[zero] == 0.0), f"{what}: oracle zero but gpu not exactly 0"
    rel = err / np.maximum(o, 1e-30)
    return float(rel[o > 0].max()) if (o > 0).any() else 0.0


def check_table_rows(S_gpu, Z_gpu, W_gpu, S_or, R_or, qw, k, hq):
    """One query's tables.  R_or: oracle squared distances (used rows x hq).
    Returns (rows with a different S, rows compared)."""
    ke = min(k, hq)
    band = 2.0 ** -20 * float(R_or.max()) + 1e-30
    diff_rows = 0
    for i in range(S_or.shape[0]):
        sg = S_gpu[i, :ke].astype(np.int64)
        so = S_or[i, :ke]
        assert np.all(S_gpu[i, ke:] == -1) and np.all(Z_gpu[i, ke:] == 0) and np.all(W_gpu[i, ke:] == 0)
        assert np.all((sg >= 0) & (sg < hq)) and len(set(sg.tolist())) == ke
        # weights are the query's weights at the selected positions, bit for bit
        assert np.array_equal(W_gpu[i, :ke], np.asarray(qw, dtype=np.float32)[sg])
        # distances of the selected positions match the oracle's distances
        zo = np.sqrt(R_or[i, sg])
        tol = REL * zo + 1e-7
        assert np.all(np.abs(Z_gpu[i, :ke].astype(np.float64) - zo) <= tol), (i, Z_gpu[i, :ke], zo)
        if not np.array_equal(sg, so):
            diff_rows += 1
            # every selected key is within the band of the oracle's k_eff-th key,
            # every unselected one is not below it by more than the band, and the
            # order is ascending up to the band
            kth = np.sort(R_or[i])[ke - 1]
            sel = np.zeros(hq, dtype=bool)
            sel[sg] = True
            assert np.all(R_or[i, sg] <= kth + band), ("S outside tie band", i)
            assert np.all(R_or[i, ~sel] >= kth - band), ("S misses a nearer word", i)
            assert np.all(np.diff(R_or[i, sg]) >= -band), ("S order", i)
    return diff_rows, S_or.shape[0]


def check_topl(idx_gpu, dist_gpu, oracle_row, ell, what="", tol_row=None):
    """GPU top-l list against the oracle's full distance row (entries the
    caller wants excluded set to +inf).  Returns the number of list
    positions whose index differs from the oracle's (distance, index)
    order; callers cap it.

    Whatever the tie order, the list must be a valid top-l:
    * l distinct in-range rows, ascending by (GPU distance, index);
    * each returned distance equal to the oracle's for that row within
      tolerance;
    * no returned row beyond the oracle's l-th distance by more than the
      tolerance of both, and no row left out that is nearer than the
      farthest returned one by more than the tolerance of both -- so a list
      that drops a clearly nearer row fails even when the next row ties
      with the l-th.
    tol_row: per-row distance tolerance (default: dist_tol of the row)."""
    o = np.asarray(oracle_row, dtype=np.float64)
    order = np.lexsort((np.arange(o.size), o))[:ell]
    ig = np.asarray(idx_gpu, dtype=np.int64)
    dg = np.asarray(dist_gpu, dtype=np.float64)
    assert ig.shape == (ell,) and dg.shape == (ell,), (what, ig.shape, dg.shape)
    assert len(set(ig.tolist())) == ell and ig.min() >= 0 and ig.max() < o.size, what
    assert np.all(np.isfinite(o[ig])), (what, "returned an excluded row")
    # ascending by (distance, index) in the returned values themselves
    for j in range(ell - 1):
        assert (dg[j], ig[j]) < (dg[j + 1], ig[j + 1]), (what, "list not ascending", j)
    fin = np.isfinite(o)
    tol = np.full(o.shape, np.inf)
    tol[fin] = dist_tol(o[fin]) if tol_row is None else np.asarray(tol_row, dtype=np.float64)[fin]
    bad = np.abs(dg - o[ig]) > tol[ig]
    assert not bad.any(), (what, "distance off", ig[bad][:4], dg[bad][:4], o[ig][bad][:4])
    swaps = int(np.sum(ig != order))
    if swaps == 0:
        return 0
    kth = order[-1]
    assert np.all(o[ig] <= o[kth] + tol[ig] + tol[kth]), (what, "returned a row beyond the l-th")
    far = ig[np.argmax(o[ig])]
    left = np.ones(o.size, dtype=bool)
    left[ig] = False
    left &= fin
    nearer = left & (o < o[far] - tol - tol[far])
    assert not nearer.any(), (what, "left out a nearer row", np.nonzero(nearer)[0][:4], o[far])
    return swaps
