"""Plain float64 CPU oracle for the EMD lower bounds of Atasu & Mittelholzer,
"Low-Complexity Data-Parallel Earth Mover's Distance Approximations" (ICML 2019).

TEST INFRASTRUCTURE ONLY.  This module exists to check the HIP library; only
the tests, the smoke check and the benchmark's CPU-baseline leg may import it.
It shares no code with the library (no kernels, headers, tables or helpers).

Everything is computed per histogram pair, directly from the definitions:

* ground cost (Sec. 5): Euclidean distance between embedding vectors,
  computed by direct coordinate differences in float64, so identical words
  are at distance exactly 0;
* per-pair measures on an explicit h_p x h_q cost matrix C:
  RWMD one-sided bound (Sec. 2.1), OMR (Alg. 1), ICT (Alg. 2), ACT (Alg. 3);
* the reverse direction is the same measure with the roles of p and q
  swapped and C transposed; the symmetric measure is the maximum of the two
  one-sided bounds (Sec. 2.1, Sec. 5);
* exact EMD and its relaxations as linear programs (Eq. 1-5), solved with
  scipy's HiGHS, for tiny inputs only.

Readings taken where the text is silent or garbled:

* ranking inside a row is ascending (squared distance, destination position):
  the position breaks ties; the distances themselves do not depend on the
  tie order;
* ACT with k larger than the destination count uses k_eff = min(k, h_q); the
  k-th (last) nearest destination absorbs whatever mass is left, which is also
  how ICT is closed when float rounding leaves a residue after the last
  destination (ICT := ACT with k = h_q; Lemma 1 makes them equal in exact
  arithmetic);
* Alg. 3's cost update uses C[i, s[l]] (its printed index is a typo; Alg. 2
  has the intended form);
* OMR with a single destination uses s[min(2, h_q)].

The LC reorganisation of Sec. 4 computes the same per-pair values, so the
batch drivers below simply loop over pairs; per query they memoise the
vocabulary-to-query distance block, which holds the same float64 values the
per-pair cost matrices would.
"""
from __future__ import annotations

import numpy as np

try:  # scipy's cdist evaluates sum((a-b)^2) by direct differences in C
    from scipy.spatial.distance import cdist as _cdist
except Exception:  # pragma: no cover
    _cdist = None

METHODS = ("rwmd", "omr", "act", "ict")
DIRECTIONS = ("d2q", "q2d", "sym")


# --------------------------------------------------------------------------
# ground cost (Sec. 5: Euclidean distance between embedding vectors)
# --------------------------------------------------------------------------
def squared_distances(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """|a - b|^2 for every row a of A and row b of B, by direct differences
    in float64 (never the |a|^2 + |b|^2 - 2ab form)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if _cdist is not None:
        return _cdist(A, B, metric="sqeuclidean")
    out = np.empty((A.shape[0], B.shape[0]))
    for i in range(A.shape[0]):
        d = A[i][None, :] - B
        out[i] = np.einsum("ij,ij->i", d, d)
    return out


def cost_matrix(A: np.ndarray, B: np.ndarray):
    """(C, R): C = Euclidean cost matrix, R = squared distances used for
    ranking (ranking on R avoids ties created by rounding in the sqrt)."""
    R = squared_distances(A, B)
    return np.sqrt(R), R


def _order(R: np.ndarray) -> np.ndarray:
    """Per row, destination indices sorted ascending by (R, position).  A
    stable sort keeps equal keys in position order."""
    return np.argsort(R, axis=1, kind="stable")


# --------------------------------------------------------------------------
# per-pair measures on an explicit cost matrix
# --------------------------------------------------------------------------
def rwmd(p, q, C, R=None) -> float:
    """One-sided RWMD (Sec. 2.1): drop the in-flow constraints (Eq. 3); every
    source bin sends all its mass to its nearest destination."""
    p = np.asarray(p, dtype=np.float64)
    return float(np.sum(p * C.min(axis=1)))


def omr(p, q, C, R=None) -> float:
    """Overlapping Mass Reduction (Sec. 3.1): the relaxed in-flow cap of
    Eq. (4) is kept only between overlapping coordinates.  A source bin whose
    nearest destination overlaps it (cost exactly 0) moves at most that
    destination's weight there for free and the rest to its second closest
    destination; every other bin moves all of its mass to its nearest
    destination.  Row by row this is ACT with k = 2 where the nearest
    destination overlaps and ACT with k = 1 elsewhere (Lemma 2's program
    with the cap on that one pair), so it is computed from ``act_rows``."""
    p = np.asarray(p, dtype=np.float64)
    order = _order(C if R is None else R)
    nearest = C[np.arange(C.shape[0]), order[:, 0]]
    capped = act_rows(p, q, C, 2, R)
    plain = act_rows(p, q, C, 1, R)
    return float(np.sum(np.where(nearest == 0.0, capped, plain)))


def act_rows(p, q, C, k: int, R=None) -> np.ndarray:
    """Per-source-bin costs of ACT (Alg. 3) with k_eff = min(k, h_q): k_eff-1
    capacity-limited transfers to the nearest destinations in ascending
    order (transfer r = min(remaining, q_s[l]), cost r * C[i, s[l]]), then the
    remaining mass to the k_eff-th nearest destination."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    hp, hq = C.shape
    if k < 1:
        raise ValueError("k must be >= 1")
    ke = min(k, hq)
    s = _order(C if R is None else R)[:, :ke]
    Cs = np.take_along_axis(C, s, axis=1)
    caps = q[s]
    rem = p.copy()
    t = np.zeros(hp)
    for l in range(ke - 1):
        r = np.minimum(rem, caps[:, l])
        rem = rem - r
        t += r * Cs[:, l]
    t += rem * Cs[:, ke - 1]
    return t


def act(p, q, C, k: int, R=None) -> float:
    """ACT (Alg. 3): sum over source bins of ``act_rows``."""
    return float(np.sum(act_rows(p, q, C, k, R)))


def ict(p, q, C, R=None) -> float:
    """ICT (Alg. 2): per source bin, capacity-limited transfers to the
    destinations in ascending cost order until its mass is exhausted; equal
    to ACT with k = h_q (the last destination absorbs a rounding residue)."""
    return act(p, q, C, C.shape[1], R)


def measure(method: str, p, q, C, k: int = 1, R=None) -> float:
    if method == "rwmd":
        return rwmd(p, q, C, R)
    if method == "omr":
        return omr(p, q, C, R)
    if method == "act":
        return act(p, q, C, k, R)
    if method == "ict":
        return ict(p, q, C, R)
    raise ValueError(method)


# --------------------------------------------------------------------------
# linear programs (Eq. 1-5), tiny inputs only
# --------------------------------------------------------------------------
def _lp(p, q, C, inflow: bool, cap_mask=None):
    from scipy.optimize import linprog

    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    hp, hq = C.shape
    nv = hp * hq
    A_eq, b_eq = [], []
    for i in range(hp):  # out-flow, Eq. (2)
        row = np.zeros(nv)
        row[i * hq:(i + 1) * hq] = 1.0
        A_eq.append(row)
        b_eq.append(p[i])
    if inflow:  # in-flow, Eq. (3)
        for j in range(hq):
            row = np.zeros(nv)
            row[j::hq] = 1.0
            A_eq.append(row)
            b_eq.append(q[j])
    bounds = []
    for i in range(hp):
        for j in range(hq):
            ub = None
            if cap_mask is not None and cap_mask[i, j]:
                ub = q[j]  # Eq. (4): F_ij <= q_j
            bounds.append((0.0, ub))
    res = linprog(C.reshape(-1), A_eq=np.array(A_eq), b_eq=np.array(b_eq),
                  bounds=bounds, method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return float(res.fun)


def emd_lp(p, q, C) -> float:
    """Exact EMD, Eq. (1)-(3); p and q must have equal total mass."""
    return _lp(p, q, C, inflow=True)


def relaxed_lp(p, q, C, cap_mask) -> float:
    """min sum F*C subject to the out-flow constraints (Eq. 2) and
    F_ij <= q_j wherever cap_mask is true (Eq. 4); no in-flow constraints."""
    return _lp(p, q, C, inflow=False, cap_mask=cap_mask)


# --------------------------------------------------------------------------
# batch drivers: a query batch against a CSR database (Sec. 4 problem setting)
# --------------------------------------------------------------------------
class Oracle:
    """Float64 per-pair evaluation of a query batch against a database.

    V: (v, m) embeddings; db: rows of (column ids, weights) histograms given
    as (rowptr, col, val).  Inputs are promoted to float64 as stored; no
    renormalisation.
    """

    def __init__(self, V, rowptr, col, val):
        self.V = np.asarray(V, dtype=np.float64)
        self.ptr = np.asarray(rowptr, dtype=np.int64)
        self.col = np.asarray(col, dtype=np.int64)
        self.val = np.asarray(val, dtype=np.float64)
        self.n = self.ptr.shape[0] - 1
        self.used = np.unique(self.col)  # the LC vocabulary (Sec. 2.2)
        self._pos = np.full(self.V.shape[0], -1, dtype=np.int64)
        self._pos[self.used] = np.arange(self.used.shape[0])

    def doc(self, u: int):
        a, b = self.ptr[u], self.ptr[u + 1]
        return self.col[a:b], self.val[a:b]

    def query_block(self, qcols):
        """Squared distances from every used vocabulary word to the query's
        words: the float64 values every per-pair cost matrix of this query
        draws from."""
        return squared_distances(self.V[self.used], self.V[np.asarray(qcols)])

    def pair(self, qcols, qw, u, method, k, direction, R_block=None):
        """One (query, document) distance."""
        qcols = np.asarray(qcols, dtype=np.int64)
        qw = np.asarray(qw, dtype=np.float64)
        dc, dw = self.doc(u)
        if R_block is None:
            R = squared_distances(self.V[dc], self.V[qcols])
        else:
            R = R_block[self._pos[dc]]
        C = np.sqrt(R)
        d2q = q2d = None
        if direction in ("d2q", "sym"):  # move the document's mass into the query
            d2q = measure(method, dw, qw, C, k, R)
        if direction in ("q2d", "sym"):  # move the query's mass into the document
            q2d = measure(method, qw, dw, C.T, k, R.T)
        if direction == "d2q":
            return d2q
        if direction == "q2d":
            return q2d
        return max(d2q, q2d)

    def rwmd_d2q_all(self, qcols, R_block=None) -> np.ndarray:
        """One-sided RWMD (Sec. 2.1) moving every database document into the
        query, for all documents at once: each document word sends its whole
        weight to its nearest query word.  Per document this is exactly
        ``rwmd`` on its cost matrix; the nearest distance of a word is
        shared by every document that holds it (Sec. 2.2)."""
        if R_block is None:
            R_block = self.query_block(qcols)
        nearest = np.sqrt(R_block.min(axis=1))
        contrib = self.val * nearest[self._pos[self.col]]
        out = np.zeros(self.n)
        lens = np.diff(self.ptr)
        nz = lens > 0
        out[nz] = np.add.reduceat(contrib, self.ptr[:-1][nz])
        return out

    def row_distances(self, qcols, qw, method, k, direction, docs=None):
        """Distances from one query to the given documents (default: all)."""
        docs = range(self.n) if docs is None else docs
        Rb = self.query_block(qcols)
        return np.array([self.pair(qcols, qw, int(u), method, k, direction, Rb) for u in docs])

    def matrix(self, qptr, qcol, qval, method, k, direction, docs=None):
        """B x n (or B x len(docs)) float64 distance matrix."""
        qptr = np.asarray(qptr)
        out = []
        for b in range(qptr.shape[0] - 1):
            a, e = int(qptr[b]), int(qptr[b + 1])
            out.append(self.row_distances(qcol[a:e], qval[a:e], method, k, direction, docs))
        return np.array(out)

    @staticmethod
    def top_l(dist_row, ell: int):
        """The ell nearest documents: ascending (distance, document index)."""
        idx = np.arange(dist_row.shape[0])
        order = np.lexsort((idx, dist_row))[:ell]
        return order, dist_row[order]

    def tables(self, qcols, qw, k: int):
        """Phase-1 tables of Sec. 4 for one query, over the used vocabulary
        (ascending word id): S = query positions of the k nearest query words
        (ascending squared distance, then position), Z = their distances,
        W = their query weights.  Entries past min(k, h_q) are padding
        (S = -1, Z = 0, W = 0)."""
        qw = np.asarray(qw, dtype=np.float64)
        R = self.query_block(qcols)
        hq = R.shape[1]
        ke = min(k, hq)
        s = _order(R)[:, :ke]
        S = np.full((R.shape[0], k), -1, dtype=np.int64)
        Z = np.zeros((R.shape[0], k))
        W = np.zeros((R.shape[0], k))
        S[:, :ke] = s
        Z[:, :ke] = np.sqrt(np.take_along_axis(R, s, axis=1))
        W[:, :ke] = qw[s]
        return S, Z, W, R
