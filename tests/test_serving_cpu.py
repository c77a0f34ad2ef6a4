"""The serving admission policy (continuous batching) on the host, through
lcemd_serve_sim: the serving worker's own admission code run against a fake
executor on a virtual clock and a fake memory budget.  No GPU needed."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def L():
    from paper_1812_02091_amd import lcemd

    lcemd.load_library()
    return lcemd


def _run(L, arrivals, words, lanes=4, slots=8, max_words=512, budget=1 << 30, per_q=1 << 20, t_fixed=0.010,
         t_per=0.001):
    return L.serve_sim(np.asarray(arrivals, dtype=np.float64), np.asarray(words, dtype=np.int32), lanes, slots,
                       max_words, budget, per_q, t_fixed, t_per)


def _check_launches(words, status, lane, launch, start, finish, slots, max_words, lanes):
    ok = status == 0
    for lid in np.unique(launch[ok]):
        m = ok & (launch == lid)
        assert m.sum() <= slots, ("launch over its slots", lid)
        assert words[m].sum() <= max_words, ("launch over its words", lid)
        assert len(set(lane[m].tolist())) == 1 and len(set(start[m].tolist())) == 1
        assert len(set(finish[m].tolist())) == 1
    # at any time at most `lanes` launches run, and a lane runs one at a time
    ev = sorted({(float(start[i]), int(launch[i]), int(lane[i]), float(finish[i])) for i in np.nonzero(ok)[0]})
    for i, (s0, lid, ln, f0) in enumerate(ev):
        running = [e for e in ev if e[0] <= s0 < e[3]]
        assert len(running) <= lanes
        assert len({e[2] for e in running}) == len(running), "two launches on one lane at once"


def test_idle_lanes_take_queries_at_once(L):
    """Arrivals spaced apart while lanes are free: every query starts the
    moment it arrives (no batch waits to fill), each on its own launch."""
    arr = np.arange(4) * 0.001  # 4 lanes, each launch lasts >= 11 ms
    words = np.full(4, 100)
    slots, status, lane, launch, start, finish = _run(L, arr, words)
    assert slots == 8
    assert np.all(status == 0)
    assert np.array_equal(start, arr)
    assert len(set(launch.tolist())) == 4 and len(set(lane.tolist())) == 4


def test_queries_join_the_next_free_lane_in_fifo_order(L):
    """A burst larger than the lanes hold: the first launches fill every
    lane, and the waiting queries start on the first lane that frees up,
    in submission order; no launch exceeds its slots or words."""
    rng = np.random.default_rng(3)
    n = 200
    arr = np.sort(rng.uniform(0, 0.05, n))
    words = rng.integers(10, 501, n)
    lanes, slots, maxw = 4, 8, 2048
    s, status, lane, launch, start, finish = _run(L, arr, words, lanes=lanes, slots=slots, max_words=maxw)
    assert np.all(status == 0)
    assert np.all(np.diff(start) >= 0), "queries must start in submission order"
    assert np.all(start >= arr) and np.all(finish > start)
    _check_launches(words, status, lane, launch, start, finish, slots, maxw, lanes)
    # under load every lane is used and batches overlap
    assert len(set(lane.tolist())) == lanes
    # continuity: a query that waited started exactly when some launch finished
    waited = start > arr + 1e-12
    ends = set(np.round(finish, 12).tolist())
    assert all(round(float(t), 12) in ends for t in start[waited])


def test_no_starvation_of_long_queries(L):
    """Long queries among many short ones: the FIFO head always fits an
    empty lane, so every query completes."""
    n = 120
    arr = np.linspace(0, 0.02, n)
    words = np.where(np.arange(n) % 7 == 0, 500, 12)
    s, status, lane, launch, start, finish = _run(L, arr, words, lanes=2, slots=16, max_words=512)
    assert np.all(status == 0) and np.all(np.isfinite(finish))
    assert np.all(np.diff(start) >= 0)
    _check_launches(words, status, lane, launch, start, finish, 16, 512, 2)


def test_query_longer_than_a_lane_is_refused(L):
    arr = [0.0, 0.0, 0.001]
    words = [100, 600, 100]
    s, status, lane, launch, start, finish = _run(L, arr, words, max_words=512)
    assert status.tolist() == [0, L.E_CAPACITY, 0]
    assert lane[1] == -1 and launch[1] == -1


def test_memory_budget_sets_the_slots(L):
    """Slots per lane = budget / lanes / per-query bytes (at most max_slots);
    a budget that holds no query is refused."""
    per_q = 64 << 20
    s, *_ = _run(L, [0.0], [10], lanes=4, slots=64, budget=4 * 5 * per_q, per_q=per_q)
    assert s == 5
    s, *_ = _run(L, [0.0], [10], lanes=4, slots=3, budget=4 * 5 * per_q, per_q=per_q)
    assert s == 3
    with pytest.raises(L.LcemdError) as e:
        _run(L, [0.0], [10], lanes=4, slots=8, budget=per_q, per_q=per_q)
    assert e.value.code == L.E_CAPACITY


def test_one_lane_is_a_plain_fifo(L):
    """One lane: launches never overlap, and each takes everything that
    waited (up to its slots) when the previous one ends."""
    arr = np.linspace(0, 0.01, 30)
    words = np.full(30, 50)
    s, status, lane, launch, start, finish = _run(L, arr, words, lanes=1, slots=8, max_words=4096)
    _check_launches(words, status, lane, launch, start, finish, 8, 4096, 1)
    assert set(lane.tolist()) == {0}
