"""Synthetic inputs: determinism and canonical CSR form."""
import numpy as np

from synth import make_workload, arrival_trace


def _canonical(c, v):
    assert c.rowptr.dtype == np.int64 and c.col.dtype == np.int32 and c.val.dtype == np.float32
    assert c.rowptr[0] == 0 and np.all(np.diff(c.rowptr) > 0)
    assert c.col.min() >= 0 and c.col.max() < v
    assert np.all(c.val > 0) and np.all(np.isfinite(c.val))
    for r in range(c.n):
        cc, vv = c.row(r)
        assert np.all(np.diff(cc) > 0)
        assert abs(float(vv.astype(np.float64).sum()) - 1.0) < 1e-5


def test_tiny_is_deterministic_and_canonical():
    a = make_workload("tiny")
    b = make_workload("tiny")
    assert np.array_equal(a.V, b.V)
    for x, y in ((a.db, b.db), (a.queries, b.queries)):
        assert np.array_equal(x.rowptr, y.rowptr) and np.array_equal(x.col, y.col)
        assert np.array_equal(x.val, y.val)
    _canonical(a.db, a.V.shape[0])
    _canonical(a.queries, a.V.shape[0])
    assert a.db.n == 200 and a.queries.n == 8 and a.V.shape == (2000, 64)
    L = a.db.lengths()
    assert L.min() >= 10 and L.max() <= 40


def test_text_and_image_shapes_small():
    t = make_workload("text", n=300, B=20, v=5000)
    _canonical(t.db, 5000)
    L = t.db.lengths()
    assert L.min() >= 50 and L.max() <= 300 and 90 < L.mean() < 150
    assert np.allclose(np.linalg.norm(t.V.astype(np.float64), axis=1), 1.0, atol=1e-6)
    im = make_workload("image", n=500, B=10)
    _canonical(im.db, 784)
    assert im.V.shape == (784, 2) and np.all(im.V == np.round(im.V))
    assert 100 < im.db.lengths().mean() < 220


def test_arrival_trace():
    t, q = arrival_trace(1000.0, 200, 5000)
    assert np.all(np.diff(t) > 0) and q.n == 200
    L = q.lengths()
    assert L.min() >= 10 and L.max() <= 500


def test_zipf_sampler_is_inverse_cdf():
    """The guide-table sampler returns exactly searchsorted(cdf, u, 'right'),
    also at CDF values and just below them."""
    from synth.generators import _ZipfSampler, _zipf_cdf

    for v, s in ((2000, 1.1), (70000, 1.0)):
        cdf = _zipf_cdf(v, s)
        u = np.random.default_rng(v).random((50, 200))
        u[0, :6] = [0.0, cdf[0], cdf[10], np.nextafter(cdf[10], 0), cdf[-2], np.nextafter(1.0, 0)]
        assert np.array_equal(_ZipfSampler(cdf)(u), np.searchsorted(cdf, u, side="right"))


def test_distinct_words_independent_of_threads():
    from synth.generators import _distinct_words, _zipf_cdf

    cdf = _zipf_cdf(300, 1.0)
    lengths = np.random.default_rng(3).integers(1, 300, 3000)
    a = _distinct_words(np.random.default_rng(9), cdf, lengths, chunk=256, threads=1)
    b = _distinct_words(np.random.default_rng(9), cdf, lengths, chunk=256, threads=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for r in range(0, 3000, 13):
        c = a[1][a[0][r]:a[0][r + 1]]
        assert c.size == lengths[r] and np.all(np.diff(c) > 0) and c.max() < 300


def test_image_background_histograms():
    """Images with their background: every histogram has all 784 pixels, rows
    sum to 1, the foreground draws are those of the same generator without
    background, and the workload is seeded (same arrays on a second build)."""
    import numpy as np

    from synth import make_workload
    from synth.generators import blob_histograms, _rng, STREAM_DB

    w = make_workload("image-bg", n=50, B=3)
    assert np.all(np.diff(w.db.rowptr) == 784) and np.all(np.diff(w.queries.rowptr) == 784)
    sums = np.add.reduceat(w.db.val.astype(np.float64), w.db.rowptr[:-1])
    assert np.allclose(sums, 1.0, atol=1e-5) and np.all(w.db.val > 0)
    again = make_workload("image-bg", n=50, B=3)
    assert np.array_equal(w.db.val, again.db.val) and np.array_equal(w.queries.val, again.queries.val)
    sparse = blob_histograms(_rng(5, STREAM_DB), 50)
    dense = w.db
    for r in range(0, 50, 7):
        cols = sparse.col[sparse.rowptr[r]:sparse.rowptr[r + 1]]
        d = dense.val[dense.rowptr[r]:dense.rowptr[r + 1]]
        bg = np.setdiff1d(np.arange(784), cols)
        # background pixels share one (smallest) weight; disc pixels are heavier
        assert np.allclose(d[bg], d[bg][0]) and np.all(d[cols] > d[bg][0])
