"""The comparison rules of tests/parity.py, on the CPU: a correct top-l
list passes, and the mistakes a GPU list could make fail."""
import numpy as np
import pytest

import parity as P


def _row():
    # rows 0..9; rows 3 and 8 tie exactly at the 4th/5th place
    return np.array([5.0, 1.0, 9.0, 3.0, 7.0, 2.0, 8.0, 6.0, 3.0, 4.0])


def test_exact_list_passes():
    o = _row()
    idx = np.array([1, 5, 3, 8])
    assert P.check_topl(idx, o[idx], o, 4) == 0


def test_tie_order_swap_is_counted():
    o = _row()
    o[8] = 3.0 * (1 + 1e-7)  # within tolerance of row 3, but after it
    idx = np.array([1, 5, 8, 3])
    d = np.array([1.0, 2.0, 3.0, 3.0 * (1 + 2e-7)])  # ascending as returned
    assert P.check_topl(idx, d, o, 4) == 2


def test_dropped_nearest_row_fails_even_when_the_next_one_ties():
    """The true nearest (row 1) is left out and replaced by row 9, the 5th,
    which ties the 4th: every returned row is within the l-th distance, yet
    the list is wrong."""
    o = _row()
    o[9] = 3.0
    idx = np.array([5, 3, 8, 9])
    with pytest.raises(AssertionError, match="nearer"):
        P.check_topl(idx, o[idx], o, 4)


def test_unsorted_list_fails():
    o = _row()
    idx = np.array([5, 1, 3, 8])
    with pytest.raises(AssertionError, match="ascending"):
        P.check_topl(idx, o[idx], o, 4)


def test_wrong_distance_fails():
    o = _row()
    idx = np.array([1, 5, 3, 8])
    d = o[idx].copy()
    d[3] *= 1 + 1e-3
    with pytest.raises(AssertionError, match="distance off"):
        P.check_topl(idx, d, o, 4)


def test_excluded_row_fails():
    o = _row()
    o[1] = np.inf  # e.g. the query itself in a self-join
    idx = np.array([1, 5, 3, 8])
    with pytest.raises(AssertionError):
        P.check_topl(idx, np.array([0.5, 2.0, 3.0, 3.0]), o, 4)
    o[9] = 3.0
    idx = np.array([5, 3, 8, 9])
    assert P.check_topl(idx, o[idx], o, 4) == 0
