"""Seeded synthetic histogram databases, query batches and embeddings.

The shapes follow the workloads the method is evaluated on: text documents
as sparse word histograms over a large embedding vocabulary (Sec. 5, Tab. 4:
20 Newsgroups, 300-d word vectors, ~80-120 distinct words per document) and
greyscale images as histograms over a 28x28 pixel grid whose embedding is the
pixel coordinate (Sec. 2, Fig. 1; Sec. 5, Tab. 4: MNIST, ~150 non-zero pixels).
None of those datasets is reproduced: everything here is drawn from seeded
distributions of the same shape.

Every random stream is ``np.random.default_rng(1000 * config + stream)`` with
streams 0 = embeddings, 1 = database, 2 = queries, 3 = parity sample,
4 = arrival trace.  Histograms are returned in canonical CSR form: int64 row
pointers, strictly increasing int32 column ids per row, float32 weights > 0
that sum to 1 per row (normalised in float64, then rounded once).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, Optional

import numpy as np

STREAM_V, STREAM_DB, STREAM_Q, STREAM_SAMPLE, STREAM_ARRIVAL = 0, 1, 2, 3, 4
# background pixel value of the dense image workload, on the scale where a
# disc pixel's intensity is in (0, 1]: one grey level of an 8-bit image
BACKGROUND = 1.0 / 255.0


@dataclass
class CSR:
    """Row-compressed histograms: row r owns entries rowptr[r]:rowptr[r+1]."""

    rowptr: np.ndarray  # int64 (n+1)
    col: np.ndarray  # int32 (nnz), strictly increasing inside a row
    val: np.ndarray  # float32 (nnz), > 0, rows sum to 1

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row(self, r: int):
        a, b = int(self.rowptr[r]), int(self.rowptr[r + 1])
        return self.col[a:b], self.val[a:b]

    def lengths(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def take(self, rows) -> "CSR":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.lengths()[rows]
        ptr = np.zeros(rows.shape[0] + 1, dtype=np.int64)
        np.cumsum(lens, out=ptr[1:])
        cols = np.empty(int(ptr[-1]), dtype=np.int32)
        vals = np.empty(int(ptr[-1]), dtype=np.float32)
        for i, r in enumerate(rows):
            c, v = self.row(int(r))
            cols[ptr[i]:ptr[i + 1]] = c
            vals[ptr[i]:ptr[i + 1]] = v
        return CSR(ptr, cols, vals)


@dataclass
class Workload:
    name: str
    V: np.ndarray  # float32 (v, m)
    db: CSR
    queries: CSR
    ks: tuple = (1, 2, 3)
    ell: int = 5
    meta: Dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# embeddings
# --------------------------------------------------------------------------
def gaussian_embeddings(rng, v: int, m: int, unit: bool, chunk: int = 1 << 16) -> np.ndarray:
    """v x m standard normal rows; if ``unit`` each row is scaled to unit L2
    norm in float64 before the single rounding to float32 (Sec. 5: word
    vectors are L2-normalised)."""
    out = np.empty((v, m), dtype=np.float32)
    for a in range(0, v, chunk):
        b = min(v, a + chunk)
        x = rng.standard_normal((b - a, m))
        if unit:
            x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[a:b] = x
    return out


def grid_embeddings(side: int = 28) -> np.ndarray:
    """Pixel (row, col) coordinates of a side x side image, pixel id
    row*side+col; not normalised (Sec. 5: image embeddings are raw)."""
    r, c = np.divmod(np.arange(side * side), side)
    return np.stack([r, c], axis=1).astype(np.float32)


# --------------------------------------------------------------------------
# histogram databases
# --------------------------------------------------------------------------
def _zipf_cdf(v: int, s: float) -> np.ndarray:
    w = np.arange(1, v + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    return cdf / cdf[-1]


class _ZipfSampler:
    """Inverse-CDF sampling of word ranks: the same result as
    searchsorted(cdf, u, side="right"), found from a guide table of the
    CDF at K evenly spaced points and a short walk."""

    def __init__(self, cdf: np.ndarray):
        self.cdf = cdf
        self.K = 4 * cdf.shape[0]
        self.g = np.searchsorted(cdf, np.arange(self.K + 1) / self.K, side="right")

    def __call__(self, u: np.ndarray) -> np.ndarray:
        cdf, v = self.cdf, self.cdf.shape[0]
        shape = u.shape
        u = u.reshape(-1)
        idx = self.g[np.minimum((u * self.K).astype(np.int64), self.K)]
        np.minimum(idx, v - 1, out=idx)
        act = np.nonzero(cdf[idx] <= u)[0]
        while act.size:  # walk up to the first cdf entry above u
            idx[act] += 1
            act = act[(idx[act] < v - 1) & (cdf[idx[act]] <= u[act])]
        act = np.nonzero((idx > 0) & (cdf[np.maximum(idx - 1, 0)] > u))[0]
        while act.size:  # (u*K rounded up) walk down
            idx[act] -= 1
            act = act[(idx[act] > 0) & (cdf[idx[act] - 1] > u[act])]
        return idx.reshape(shape)


def _first_distinct(T: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Mask of the first L[r] distinct values of each row of T, in draw order."""
    order = np.argsort(T, axis=1, kind="stable")
    st = np.take_along_axis(T, order, 1)
    fs = np.ones_like(st, dtype=bool)
    fs[:, 1:] = st[:, 1:] != st[:, :-1]
    first = np.empty_like(fs)
    np.put_along_axis(first, order, fs, 1)
    return first & (np.cumsum(first, axis=1) <= L[:, None])


def _distinct_words(rng, cdf: np.ndarray, lengths: np.ndarray, chunk: int = 8192,
                    threads: int = 8):
    """For each row, the first L distinct word ids of i.i.d. Zipf draws,
    returned sorted.  Rows are processed in groups of similar length (each
    group with its own generator seeded from ``rng``, so the result does not
    depend on the thread count); a group draws 2*max(L)+16 tokens per row
    and redraws the rare rows that fall short with twice as many."""
    n = lengths.shape[0]
    v = cdf.shape[0]
    if n and int(lengths.max()) > v:
        raise ValueError("a row asks for more distinct words than the vocabulary has")
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=rowptr[1:])
    cols = np.empty(int(rowptr[-1]), dtype=np.int32)
    sample = _ZipfSampler(cdf)
    order = np.argsort(lengths, kind="stable")
    starts = list(range(0, n, chunk))
    seeds = rng.integers(0, 2**63 - 1, len(starts))

    def group(gi):
        rows = order[starts[gi]:starts[gi] + chunk]
        L = lengths[rows]
        crng = np.random.default_rng(int(seeds[gi]))
        todo = np.arange(rows.shape[0])
        M = 2 * int(L.max()) + 16
        while todo.size:
            Lt = L[todo]
            T = sample(crng.random((todo.size, M)))
            keep = _first_distinct(T, Lt)
            full = keep.sum(1) == Lt
            r_loc, c_loc = np.nonzero(keep[full])
            ids = T[full][r_loc, c_loc]
            key = r_loc.astype(np.int64) * v + ids
            key.sort()
            r_s = key // v
            done = todo[full]
            off = np.zeros(done.size + 1, dtype=np.int64)
            np.cumsum(L[done], out=off[1:])
            dest = rowptr[rows[done]][r_s] + (np.arange(key.size) - off[r_s])
            cols[dest] = (key - r_s * v).astype(np.int32)
            todo = todo[~full]
            M *= 2

    if threads > 1 and len(starts) > 1:
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(min(threads, len(starts))) as ex:
            list(ex.map(group, range(len(starts))))
    else:
        for gi in range(len(starts)):
            group(gi)
    return rowptr, cols


def _normalise_rows(rowptr: np.ndarray, raw: np.ndarray) -> np.ndarray:
    raw = raw.astype(np.float64)
    sums = np.add.reduceat(raw, rowptr[:-1]) if raw.size else np.zeros(0)
    lens = np.diff(rowptr)
    return (raw / np.repeat(sums, lens)).astype(np.float32)


def zipf_histograms(rng, n: int, v: int, s: float, length_fn: Callable, weight: str) -> CSR:
    """n sparse histograms over a v-word vocabulary.

    length_fn(rng, n) gives the distinct-word count per row; words are Zipf(s)
    over ranks 1..v (word id = rank-1); ``weight`` is "uniform" (1 - U[0,1))
    or "tf" (term frequency ~ Geometric(1/2) on {1,2,...}); rows are then
    L1-normalised.
    """
    lengths = np.asarray(length_fn(rng, n), dtype=np.int64)
    rowptr, cols = _distinct_words(rng, _zipf_cdf(v, s), lengths)
    nnz = int(rowptr[-1])
    if weight == "uniform":
        raw = 1.0 - rng.random(nnz)
    elif weight == "tf":
        raw = rng.geometric(0.5, nnz).astype(np.float64)
    else:
        raise ValueError(weight)
    return CSR(rowptr, cols, _normalise_rows(rowptr, raw))


def blob_histograms(rng, n: int, side: int = 28, rmin: int = 4, rmax: int = 10, chunk: int = 8192,
                    background: float = 0.0) -> CSR:
    """n greyscale 'blob' images: radius ~ U{rmin..rmax}, centre ~
    U{r..side-1-r}^2, pixels inside the disc get intensity 1 - U[0,1);
    L1-normalised (pixel weights = normalised pixel values, Sec. 5).

    background > 0: every pixel is a coordinate (Sec. 5, images with their
    background): each pixel's value is background + its disc intensity, so
    all side*side pixels carry weight (the same random draws as without)."""
    yy, xx = np.divmod(np.arange(side * side), side)
    ptrs, cols_l, raws = [np.zeros(1, dtype=np.int64)], [], []
    base = 0
    for a in range(0, n, chunk):
        c = min(n, a + chunk) - a
        r = rng.integers(rmin, rmax + 1, c)
        cy = rng.integers(r, side - r)
        cx = rng.integers(r, side - r)
        mask = (yy[None, :] - cy[:, None]) ** 2 + (xx[None, :] - cx[:, None]) ** 2 <= (r[:, None] ** 2)
        rows, px = np.nonzero(mask)
        lens = mask.sum(1)
        raw = 1.0 - rng.random(px.shape[0])
        if background > 0:
            dense = np.full((c, side * side), float(background))
            dense[rows, px] += raw
            lens = np.full(c, side * side, dtype=np.int64)
            px = np.tile(np.arange(side * side), c)
            raw = dense.ravel()
        cols_l.append(px.astype(np.int32))
        raws.append(raw)
        ptrs.append(base + np.cumsum(lens))
        base += int(lens.sum())
    rowptr = np.concatenate(ptrs).astype(np.int64)
    cols = np.concatenate(cols_l)
    return CSR(rowptr, cols, _normalise_rows(rowptr, np.concatenate(raws)))


def _uniform_len(lo, hi):
    return lambda rng, n: rng.integers(lo, hi + 1, n)


def _lognormal_len(mean=120.0, sigma=0.5, lo=50, hi=300):
    mu = np.log(mean) - sigma * sigma / 2.0
    return lambda rng, n: np.clip(np.round(rng.lognormal(mu, sigma, n)), lo, hi).astype(np.int64)


def _rng(config: int, stream: int):
    return np.random.default_rng(1000 * config + stream)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def _tiny(n=200, B=8, v=2000, m=64, **_):
    V = gaussian_embeddings(_rng(1, STREAM_V), v, m, unit=False)
    f = _uniform_len(10, 40)
    db = zipf_histograms(_rng(1, STREAM_DB), n, v, 1.1, f, "uniform")
    q = zipf_histograms(_rng(1, STREAM_Q), B, v, 1.1, f, "uniform")
    return Workload("tiny-fp32", V, db, q, ks=(1, 2, 3), ell=5,
                    meta=dict(config=1, v=v, m=m, n=n, B=B))


def _text(n=18000, B=1000, v=70000, m=300, cfg=2, **_):
    V = gaussian_embeddings(_rng(cfg, STREAM_V), v, m, unit=True)
    f = _lognormal_len()
    db = zipf_histograms(_rng(cfg, STREAM_DB), n, v, 1.0, f, "tf")
    q = zipf_histograms(_rng(cfg, STREAM_Q), B, v, 1.0, f, "tf")
    ks = tuple(range(1, 17)) if cfg == 2 else (8,)
    return Workload("text" if cfg == 2 else "text-1M", V, db, q, ks=ks, ell=16,
                    meta=dict(config=cfg, v=v, m=m, n=n, B=B))


def _image(n=60000, B=10000, **_):
    V = grid_embeddings(28)
    db = blob_histograms(_rng(3, STREAM_DB), n)
    q = blob_histograms(_rng(3, STREAM_Q), B)
    return Workload("image", V, db, q, ks=(1, 4, 8, 16), ell=16,
                    meta=dict(config=3, v=784, m=2, n=n, B=B))


def _image_bg(n=60000, B=10000, **_):
    V = grid_embeddings(28)
    db = blob_histograms(_rng(5, STREAM_DB), n, background=BACKGROUND)
    q = blob_histograms(_rng(5, STREAM_Q), B, background=BACKGROUND)
    return Workload("image-bg", V, db, q, ks=(1, 2, 4, 16), ell=16,
                    meta=dict(config=5, v=784, m=2, n=n, B=B, background=BACKGROUND))


def _precision(n=1_000_000, B=4096, v=1_000_000, m=300, **_):
    return _text(n=n, B=B, v=v, m=m, cfg=4)


WORKLOADS = {
    "tiny": _tiny,        # 2,000 x 64 N(0,1); 200 docs of 10-40 words; 8 queries
    "text": _text,        # 70,000 x 300 unit; 18,000 docs ~120 words; 1,000 queries
    "image": _image,      # 28x28 grid; 60,000 blobs; 10,000 queries
    "text-1M": _precision,  # 1e6 x 300 unit; 1e6 docs; 4,096 queries
    "image-bg": _image_bg,  # 28x28 grid, every pixel a coordinate; 60,000 x 10,000
}


def make_workload(name: str, **overrides) -> Workload:
    """Build a named workload; keyword overrides (n, B, v, m) shrink it for
    tests while keeping its distributions."""
    return WORKLOADS[name](**overrides)


def arrival_trace(rate_qps: float, count: int, v: int, seed_config: int = 5,
                  lmin: int = 10, lmax: int = 500):
    """Open-loop Poisson arrivals: (arrival times in s, query CSR) with
    U{lmin..lmax} distinct Zipf(1.0) words per query and tf weights."""
    rng = _rng(seed_config, STREAM_ARRIVAL)
    t = np.cumsum(rng.exponential(1.0 / rate_qps, count))
    q = zipf_histograms(rng, count, v, 1.0, _uniform_len(lmin, lmax), "tf")
    return t, q


def sample_pairs(config: int, B: int, n: int, count: int, seed_stream: int = STREAM_SAMPLE):
    """Seeded (query, doc) index pairs for spot checks at full size."""
    rng = _rng(config, seed_stream)
    return rng.integers(0, B, count), rng.integers(0, n, count)
