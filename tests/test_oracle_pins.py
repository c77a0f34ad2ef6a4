"""Pins for the float64 oracle, independent of the oracle's own code paths.

Each check ties the oracle to something the paper or the mathematics fixes:
hand-worked examples (tests/golden), the linear programs the greedy
algorithms solve (Thm 1, Lemma 2), the ordering chain (Thm 2), effectiveness
(Thm 3 and its remark), the overlapping-support failure of RWMD (Sec. 3),
the 1-D EMD closed form, brute-force distances and the LC table form of
Sec. 4 (Eq. 6-9) evaluated by code written here, not in the oracle.
"""
import json
import os

import numpy as np
import pytest

from oracle import emd_oracle as O
from synth import make_workload

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

TOL = 1e-12


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _c1d(a, b):
    a = np.asarray(a, dtype=np.float64)[:, None]
    b = np.asarray(b, dtype=np.float64)[None, :]
    return np.abs(a - b)


def _emd_1d(xp, wp, xq, wq):
    """Textbook 1-D EMD: integral of |F_p - F_q| over the line."""
    pts = np.unique(np.concatenate([xp, xq]).astype(np.float64))
    total = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        Fp = np.sum(np.asarray(wp)[np.asarray(xp) <= a])
        Fq = np.sum(np.asarray(wq)[np.asarray(xq) <= a])
        total += abs(Fp - Fq) * (b - a)
    return total


def _measure_by_key(key, p, q, C):
    if key == "rwmd":
        return O.rwmd(p, q, C)
    if key == "omr":
        return O.omr(p, q, C)
    if key == "ict":
        return O.ict(p, q, C)
    if key.startswith("act"):
        return O.act(p, q, C, int(key[3:]))
    raise KeyError(key)


# --------------------------------------------------------------------------
# hand-worked examples
# --------------------------------------------------------------------------
def test_hand_examples(golden_dir):
    data = _load(golden_dir, "hand_examples.json")
    for ex in data["examples"]:
        p, q = np.array(ex["p_w"]), np.array(ex["q_w"])
        C = _c1d(ex["p_coord"], ex["q_coord"])
        for key, want in ex.get("d2q", {}).items():
            assert abs(_measure_by_key(key, p, q, C) - want) < 1e-12, (ex["name"], "d2q", key)
        for key, want in ex.get("q2d", {}).items():
            assert abs(_measure_by_key(key, q, p, C.T) - want) < 1e-12, (ex["name"], "q2d", key)
        for key, want in ex.get("sym", {}).items():
            got = max(_measure_by_key(key, p, q, C), _measure_by_key(key, q, p, C.T))
            assert abs(got - want) < 1e-12, (ex["name"], "sym", key)
        assert abs(O.emd_lp(p, q, C) - ex["emd"]) < 1e-9, ex["name"]
        assert abs(_emd_1d(ex["p_coord"], p, ex["q_coord"], q) - ex["emd"]) < 1e-12


def test_hand_examples_through_batch_driver(golden_dir):
    """The same examples through the CSR batch driver (doc = p, query = q)."""
    data = _load(golden_dir, "hand_examples.json")
    for ex in data["examples"]:
        coords = sorted(set(ex["p_coord"]) | set(ex["q_coord"]))
        V = np.array(coords, dtype=np.float64)[:, None]
        wid = {c: i for i, c in enumerate(coords)}
        pc = [wid[c] for c in ex["p_coord"]]
        qc = [wid[c] for c in ex["q_coord"]]
        orc = O.Oracle(V, [0, len(pc)], pc, ex["p_w"])
        for direction in ("d2q", "q2d", "sym"):
            for key, want in ex.get(direction, {}).items():
                method, k = (key, 1) if not key.startswith("act") else ("act", int(key[3:]))
                got = orc.pair(qc, ex["q_w"], 0, method, k, direction)
                assert abs(got - want) < 1e-12, (ex["name"], direction, key)


def test_tie_table(golden_dir):
    t = _load(golden_dir, "tie_table.json")
    V = np.array(t["vocab_coord"], dtype=np.float64)[:, None]
    nv = V.shape[0]
    orc = O.Oracle(V, [0, nv], np.arange(nv), np.full(nv, 1.0 / nv))
    S, Z, W, _ = orc.tables(t["query_words"], t["query_w"], t["k"])
    for row, want in t["rows"].items():
        i = int(row)
        assert S[i].tolist() == want["S"]
        assert np.allclose(Z[i], want["Z"], rtol=0, atol=1e-15)
        assert np.allclose(W[i], want["W"], rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# random tiny instances
# --------------------------------------------------------------------------
def _instances(count, seed=7, grid=False, max_bins=6, m=2):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        hp, hq = rng.integers(1, max_bins + 1, 2)
        if grid:  # integer coordinates: exact ties and shared coordinates
            A = rng.integers(0, 4, (hp, m)).astype(np.float64)
            B = rng.integers(0, 4, (hq, m)).astype(np.float64)
        else:
            A = rng.standard_normal((hp, m))
            B = rng.standard_normal((hq, m))
        p = rng.random(hp) + 0.05
        q = rng.random(hq) + 0.05
        p /= p.sum()
        q /= q.sum()
        C, R = O.cost_matrix(A, B)
        yield p, q, C, R


@pytest.mark.parametrize("grid", [False, True])
def test_act1_is_rwmd(grid):
    for p, q, C, R in _instances(200, seed=1, grid=grid):
        assert O.act(p, q, C, 1, R) == O.rwmd(p, q, C, R)


@pytest.mark.parametrize("grid", [False, True])
def test_act_saturates_at_ict(grid):
    for p, q, C, R in _instances(200, seed=2, grid=grid):
        hq = C.shape[1]
        ref = O.ict(p, q, C, R)
        for k in range(hq, hq + 3):
            assert O.act(p, q, C, k, R) == ref


@pytest.mark.parametrize("grid", [False, True])
def test_ordering_chain_and_emd(grid):
    """Thm 2: RWMD <= OMR <= ACT(2) <= ... <= ICT <= EMD, both directions."""
    for p, q, C, R in _instances(150, seed=3, grid=grid):
        for (a, b, M, RM) in ((p, q, C, R), (q, p, C.T, R.T)):
            chain = [O.rwmd(a, b, M, RM), O.omr(a, b, M, RM)]
            chain += [O.act(a, b, M, k, RM) for k in range(2, M.shape[1] + 1)]
            chain += [O.ict(a, b, M, RM), O.emd_lp(a, b, M)]
            for lo, hi in zip(chain[:-1], chain[1:]):
                assert lo <= hi + 1e-9, chain


@pytest.mark.parametrize("grid", [False, True])
def test_ict_solves_relaxed_lp(grid):
    """Thm 1: ICT is the optimum of Eq. (1), (2), (4)."""
    for p, q, C, R in _instances(120, seed=4, grid=grid):
        lp = O.relaxed_lp(p, q, C, np.ones_like(C, dtype=bool))
        assert abs(O.ict(p, q, C, R) - lp) < 1e-9


@pytest.mark.parametrize("grid", [False, True])
def test_act_solves_partially_capped_lp(grid):
    """Lemma 2: ACT(k) is the optimum of Eq. (1), (2) with Eq. (4) imposed only
    on each row's k-1 nearest destinations."""
    for p, q, C, R in _instances(120, seed=5, grid=grid):
        order = np.argsort(R, axis=1, kind="stable")
        for k in range(1, C.shape[1] + 1):
            mask = np.zeros_like(C, dtype=bool)
            for i in range(C.shape[0]):
                mask[i, order[i, :k - 1]] = True
            lp = O.relaxed_lp(p, q, C, mask)
            assert abs(O.act(p, q, C, k, R) - lp) < 1e-9, k


@pytest.mark.parametrize("grid", [False, True])
def test_rwmd_and_omr_lps(grid):
    """RWMD = out-flow-only LP (Sec. 2.1); OMR = capacities only where the cost
    is zero (Sec. 3.1), for effective costs (distinct coordinates)."""
    for p, q, C, R in _instances(120, seed=6, grid=grid):
        assert abs(O.rwmd(p, q, C) - O.relaxed_lp(p, q, C, np.zeros_like(C, dtype=bool))) < 1e-9
        distinct_q = np.all((C == 0).sum(axis=1) <= 1)
        if distinct_q:
            assert abs(O.omr(p, q, C, R) - O.relaxed_lp(p, q, C, C == 0)) < 1e-9


def test_identical_histograms_are_zero_and_effectiveness():
    """Thm 3 + remark: identical histograms give 0; different weights on the
    same distinct coordinates give OMR, ACT(k>=2), ICT > 0."""
    rng = np.random.default_rng(11)
    for _ in range(100):
        h = int(rng.integers(1, 8))
        A = rng.standard_normal((h, 3))
        p = rng.random(h) + 0.1
        p /= p.sum()
        C, R = O.cost_matrix(A, A)
        assert np.all(np.diag(C) == 0.0)
        for m in O.METHODS:
            assert O.measure(m, p, p, C, 3, R) == 0.0
        if h >= 2:
            q = rng.random(h) + 0.1
            q /= q.sum()
            if np.max(np.abs(p - q)) > 1e-6:
                assert O.omr(p, q, C, R) > 0
                assert O.act(p, q, C, 2, R) > 0
                assert O.ict(p, q, C, R) > 0


def test_overlapping_supports_defeat_rwmd():
    """Sec. 3 and the with-background image experiment: when every coordinate
    of p is also a coordinate of q, RWMD is 0 in both directions while ACT(2)
    is not."""
    rng = np.random.default_rng(12)
    V = np.stack(np.divmod(np.arange(49), 7), 1).astype(np.float64)  # 7x7 grid
    for _ in range(20):
        p = rng.random(49) + 0.01
        q = rng.random(49) + 0.01
        p /= p.sum()
        q /= q.sum()
        C, R = O.cost_matrix(V, V)
        assert O.rwmd(p, q, C) == 0.0 and O.rwmd(q, p, C.T) == 0.0
        assert O.act(p, q, C, 2, R) > 0 and O.act(q, p, C.T, 2, R.T) > 0


def test_emd_lp_matches_1d_closed_form():
    rng = np.random.default_rng(13)
    for _ in range(60):
        hp, hq = rng.integers(1, 7, 2)
        xp = rng.integers(0, 20, hp).astype(np.float64)
        xq = rng.integers(0, 20, hq).astype(np.float64)
        p = rng.random(hp) + 0.05
        q = rng.random(hq) + 0.05
        p /= p.sum()
        q /= q.sum()
        assert abs(O.emd_lp(p, q, _c1d(xp, xq)) - _emd_1d(xp, p, xq, q)) < 1e-9


def test_single_source_ict_equals_emd():
    """Lemma 1 with one source bin: ICT moves q_j to every destination, which is
    the only feasible (hence optimal) EMD flow."""
    rng = np.random.default_rng(14)
    for _ in range(50):
        hq = int(rng.integers(1, 9))
        B = rng.standard_normal((hq, 4))
        A = rng.standard_normal((1, 4))
        q = rng.random(hq) + 0.05
        q /= q.sum()
        C, R = O.cost_matrix(A, B)
        want = float(np.sum(q * C[0]))
        assert abs(O.ict([1.0], q, C, R) - want) < 1e-12
        assert abs(O.emd_lp(np.array([1.0]), q, C) - want) < 1e-9


@pytest.mark.parametrize("grid", [False, True])
def test_tie_order_does_not_change_distances(grid):
    """Reversing the tie rule (ties to the higher position) changes S/W but
    not the ACT/ICT/OMR value (up to float64 rounding)."""
    for p, q, C, R in _instances(200, seed=15, grid=grid):
        flipped = (slice(None), slice(None, None, -1))
        Cf, Rf, qf = C[flipped], R[flipped], q[::-1]
        for k in (1, 2, 3, 5):
            assert abs(O.act(p, q, C, k, R) - O.act(p, qf, Cf, k, Rf)) < TOL
        assert abs(O.omr(p, q, C, R) - O.omr(p, qf, Cf, Rf)) < TOL


def test_symmetric_measure_is_symmetric():
    rng = np.random.default_rng(16)
    V = rng.standard_normal((30, 5))
    for _ in range(50):
        a = np.sort(rng.choice(30, int(rng.integers(1, 8)), replace=False))
        b = np.sort(rng.choice(30, int(rng.integers(1, 8)), replace=False))
        wa = rng.random(a.size) + 0.1
        wb = rng.random(b.size) + 0.1
        wa /= wa.sum()
        wb /= wb.sum()
        o1 = O.Oracle(V, [0, a.size], a, wa)
        o2 = O.Oracle(V, [0, b.size], b, wb)
        for method, k in (("rwmd", 1), ("omr", 1), ("act", 3), ("ict", 1)):
            assert abs(o1.pair(b, wb, 0, method, k, "sym") - o2.pair(a, wa, 0, method, k, "sym")) < TOL


def test_squared_distances_brute_force():
    rng = np.random.default_rng(17)
    A = rng.standard_normal((7, 5))
    B = rng.standard_normal((4, 5))
    R = O.squared_distances(A, B)
    for i in range(7):
        for j in range(4):
            want = sum((float(A[i, d]) - float(B[j, d])) ** 2 for d in range(5))
            assert abs(R[i, j] - want) < 1e-12
    assert np.all(np.diag(O.squared_distances(A, A)) == 0.0)


# --------------------------------------------------------------------------
# the LC form of Sec. 4 (Eq. 6-9), written here against the oracle's tables
# --------------------------------------------------------------------------
def _lc_act_from_tables(Z, W, X_rows, k):
    """Phase 2/3 of LC-ACT for one query, written from Eq. (6)-(9): for every
    non-zero X_ui, k-1 rounds of Y = min(X, w^(l)), X -= Y, t += Y z^(l), then
    t += X z^(k).  Z, W are indexed by used-vocabulary row."""
    out = []
    for rows, x in X_rows:
        t = 0.0
        Xr = np.array(x, dtype=np.float64)
        for l in range(k - 1):
            Y = np.minimum(Xr, W[rows, l])
            Xr = Xr - Y
            t += float(np.sum(Y * Z[rows, l]))
        t += float(np.sum(Xr * Z[rows, k - 1]))
        out.append(t)
    return np.array(out)


@pytest.mark.parametrize("k", [1, 2, 3, 8])
def test_lc_form_matches_per_pair(k):
    w = make_workload("tiny", n=40, B=3)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    pos = {int(c): i for i, c in enumerate(orc.used)}
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        ke = min(k, qc.size)
        S, Z, W, _ = orc.tables(qc, qw, k)
        X_rows = []
        for u in range(w.db.n):
            dc, dw = w.db.row(u)
            X_rows.append((np.array([pos[int(c)] for c in dc]), dw))
        lc = _lc_act_from_tables(Z, W, X_rows, ke)
        direct = orc.row_distances(qc, qw, "act", k, "d2q")
        assert np.max(np.abs(lc - direct)) < 1e-12


def test_memoised_block_matches_fresh_pairs():
    w = make_workload("tiny", n=30, B=2)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    qc, qw = w.queries.row(1)
    Rb = orc.query_block(qc)
    for u in range(w.db.n):
        for method, k in (("act", 3), ("ict", 1), ("omr", 1)):
            a = orc.pair(qc, qw, u, method, k, "sym", Rb)
            b = orc.pair(qc, qw, u, method, k, "sym", None)
            assert a == b


def test_cost_matrix_is_euclidean_not_squared():
    """Sec. 5: the ground cost is the L2 distance (3-4-5 triangle, 1-D case)."""
    C, R = O.cost_matrix(np.array([[0.0, 0.0], [1.0, 1.0]]), np.array([[3.0, 4.0], [1.0, 1.0]]))
    assert C[0, 0] == 5.0 and R[0, 0] == 25.0 and C[1, 1] == 0.0
    C1, _ = O.cost_matrix(np.array([[0.0], [1.0]]), np.array([[0.0], [3.0]]))
    assert np.array_equal(C1, _c1d([0, 1], [0, 3]))


def test_dense_background_images_closed_forms():
    """Images with their background (every one of the 28x28 pixels is a
    coordinate of every histogram, Sec. 5): RWMD is exactly 0 both ways; each
    pixel's nearest other pixel is at distance 1, so OMR (Alg. 1) and ACT(2)
    (Alg. 3) keep min(p_i, q_i) in place and move the rest one grid step:
    both equal sum_i max(p_i - q_i, 0) for source p (the total variation
    distance when both sum to 1).  Deeper measures grow along Thm 2's
    chain."""
    from synth import make_workload

    w = make_workload("image-bg", n=3, B=2)
    assert np.all(np.diff(w.db.rowptr) == 784) and np.all(np.diff(w.queries.rowptr) == 784)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    for b in range(2):
        c, qv = w.queries.row(b)
        for d in ("d2q", "q2d"):
            assert np.all(orc.row_distances(c, qv, "rwmd", 1, d) == 0.0)
            omr = orc.row_distances(c, qv, "omr", 1, d)
            act2 = orc.row_distances(c, qv, "act", 2, d)
            q64 = qv.astype(np.float64)
            src = [(w.db.row(u)[1].astype(np.float64), q64) for u in range(3)]
            tv = np.array([np.maximum(a - b, 0).sum() if d == "d2q" else np.maximum(b - a, 0).sum()
                           for a, b in src])
            assert np.allclose(omr, tv, rtol=1e-12, atol=0) and np.allclose(act2, tv, rtol=1e-12, atol=0)
            act4 = orc.row_distances(c, qv, "act", 4, d)
            ict = orc.row_distances(c, qv, "ict", 1, d)
            assert np.all(tv > 0) and np.all(act2 <= act4 + 1e-12) and np.all(act4 <= ict + 1e-12)


# --------------------------------------------------------------------------
# top-l order, the bulk RWMD bound, OMR with repeated coordinates
# --------------------------------------------------------------------------
def test_top_l_ties_go_to_lower_index():
    """Sec. 5 top-l: ascending distance, equal distances by ascending
    document index -- checked on a worked row and against brute force
    (Python's tuple sort) on integer rows full of ties."""
    row = np.array([3.0, 1.0, 2.0, 1.0, 0.0, 2.0, 1.0])
    idx, dist = O.Oracle.top_l(row, 4)
    assert idx.tolist() == [4, 1, 3, 6] and dist.tolist() == [0.0, 1.0, 1.0, 1.0]
    rng = np.random.default_rng(41)
    for _ in range(200):
        n = int(rng.integers(1, 40))
        r = rng.integers(0, 5, n).astype(np.float64)
        ell = int(rng.integers(1, n + 1))
        want = sorted(range(n), key=lambda i: (r[i], i))[:ell]
        got, d = O.Oracle.top_l(r, ell)
        assert got.tolist() == want and np.array_equal(d, r[want])


def test_rwmd_bound_for_all_documents():
    """The bulk one-sided RWMD equals the per-pair RWMD of every document
    (Sec. 2.1 / Sec. 2.2) and lower-bounds ACT and the symmetric measure
    (Thm 2, and SYM >= D2Q)."""
    w = make_workload("tiny", n=60, B=3)
    orc = O.Oracle(w.V, w.db.rowptr, w.db.col, w.db.val)
    for b in range(w.queries.n):
        qc, qw = w.queries.row(b)
        bulk = orc.rwmd_d2q_all(qc)
        pairs = orc.row_distances(qc, qw, "rwmd", 1, "d2q")
        assert np.allclose(bulk, pairs, rtol=1e-12, atol=0)
        for method, k, d in (("act", 4, "d2q"), ("ict", 1, "d2q"), ("act", 2, "sym")):
            assert np.all(bulk <= orc.row_distances(qc, qw, method, k, d) * (1 + 1e-12))


def test_omr_with_repeated_coordinates_follows_sec_3_1():
    """A destination coordinate that occurs twice (not a valid histogram,
    but the grid instances above make them): the nearest overlapping
    destination is capped and the rest goes to the second closest, which
    here overlaps too -- so OMR stays at ACT(2) (Thm 2's order holds), below
    the program that caps every zero-cost pair.  Distinct coordinates: OMR
    is that program's optimum (test_rwmd_and_omr_lps)."""
    C = _c1d([0.0], [0.0, 0.0, 2.0])
    p, q = np.array([1.0]), np.array([0.3, 0.3, 0.4])
    assert O.omr(p, q, C) == 0.0 and O.act(p, q, C, 2) == 0.0
    assert abs(O.relaxed_lp(p, q, C, C == 0) - 0.8) < 1e-9
    assert abs(O.ict(p, q, C) - 0.8) < 1e-12
    # overlap with a second, distinct destination: 0.3 free, 0.7 at cost 2
    C2 = _c1d([0.0], [0.0, 2.0])
    assert abs(O.omr(p, np.array([0.3, 0.7]), C2) - 1.4) < 1e-12
    # one destination only, at the same coordinate: nothing to pay (the last
    # destination absorbs the rest)
    assert O.omr(np.array([1.0]), np.array([1.0]), _c1d([0.0], [0.0])) == 0.0
