"""Pins of the oracle's ranking, prune count and compaction (CPU only)."""
import numpy as np
import pytest


def test_n_prune_rounding(oracle_lib):
    assert oracle_lib.n_prune(5, 0.5) == 3          # 2.5 rounds away from zero
    assert oracle_lib.n_prune(5, 0.1) == 1          # 0.5 -> 1
    assert oracle_lib.n_prune(10, 0.34) == 3
    assert oracle_lib.n_prune(3_000_000, 0.5) == 1_500_000
    assert oracle_lib.n_prune(3_000_000, 0.9) == 2_700_000
    assert oracle_lib.n_prune(6_000_000, 0.66) == 3_960_000
    assert oracle_lib.n_prune(0, 0.5) == 0
    assert oracle_lib.n_prune(7, 0.999) == 7


@pytest.mark.parametrize("n,k", [(0, 0), (1, 0), (1, 1), (50, 0), (50, 25), (50, 50), (1000, 333)])
def test_select_matches_brute_force_sort(oracle_lib, n, k):
    rng = np.random.default_rng(n + k)
    D = rng.integers(0, 7, size=n).astype(np.float64) * 0.25    # many ties
    keep, order = oracle_lib.select(D, k)
    ref = sorted(range(n), key=lambda i: (D[i], i))
    assert list(order) == ref
    expect = np.ones(n, dtype=np.uint8)
    expect[ref[:k]] = 0
    np.testing.assert_array_equal(keep, expect)
    assert int(keep.sum()) == n - k


def test_select_ties_prune_lower_index_first(oracle_lib):
    D = np.zeros(10)
    keep, _ = oracle_lib.select(D, 4)
    assert list(keep) == [0, 0, 0, 0, 1, 1, 1, 1, 1, 1]


def test_compact_matches_boolean_indexing(oracle_lib):
    from paper_2606_09074_amd import synth
    pl = synth.make_planes(synth.SMALL.with_n(777), stride=800)
    keep = (np.random.default_rng(4).random(800) < 0.4).astype(np.uint8)
    out, idx = oracle_lib.compact(pl, keep, n=777)
    sel = keep[:777].astype(bool)
    np.testing.assert_array_equal(out, pl[:, :777][:, sel])
    np.testing.assert_array_equal(idx, np.nonzero(sel)[0])
    out0, idx0 = oracle_lib.compact(pl, np.zeros(800, np.uint8), n=777)
    assert out0.shape == (59, 0) and idx0.size == 0
