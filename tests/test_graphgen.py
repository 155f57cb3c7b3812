"""Pins of the input generator: the degree sampler follows the Pld([a,b),gamma)
pmf (chi-squared), the configuration model pairs stubs uniformly (exact laws
on tiny degree sequences), and erasure leaves a simple symmetric sorted CSR
whose degrees never exceed the drawn ones."""
import numpy as np
import pytest
from scipy import stats

import graphgen

ALPHA = 1e-3


def _simple_symmetric_sorted(rp, col):
    n = len(rp) - 1
    rows = [col[rp[x]:rp[x + 1]] for x in range(n)]
    for x, r in enumerate(rows):
        if len(r) and (np.any(np.diff(r) <= 0) or np.any(r == x) or r.min() < 0 or r.max() >= n):
            return False
    src = np.repeat(np.arange(n), np.diff(rp))
    fwd = set(zip(src.tolist(), col.tolist()))
    return all((y, x) in fwd for x, y in fwd)


@pytest.mark.parametrize("a,b,gamma", [(5, 50, 2.0), (2, 30, 2.6), (10, 40, 1.8)])
def test_pld_degrees_follow_the_pmf(a, b, gamma):
    n = 200000
    deg, total = graphgen.pld_degrees(n, a, b, gamma, seed=3)
    assert total == int(deg.sum()) and total % 2 == 0
    assert deg.min() >= a and deg.max() < b
    ks = np.arange(a, b)
    pmf = ks.astype(float) ** -gamma
    pmf /= pmf.sum()
    obs = np.bincount(deg - a, minlength=b - a)
    assert stats.chisquare(obs, pmf * n).pvalue > ALPHA


def test_pld_degrees_thread_count_independent():
    d1, _ = graphgen.pld_degrees(50000, 3, 300, 2.1, seed=9, threads=1)
    d8, _ = graphgen.pld_degrees(50000, 3, 300, 2.1, seed=9, threads=7)
    assert np.array_equal(d1, d8)


def _graph_key(rp, col):
    n = len(rp) - 1
    return tuple((x, int(y)) for x in range(n) for y in col[rp[x]:rp[x + 1]] if x < y)


def test_configuration_model_pairs_stubs_uniformly():
    # degrees (1,1,1,1): the three perfect matchings of four stubs, 1/3 each
    counts = {}
    for s in range(3000):
        rp, col = graphgen.configuration_model(np.array([1, 1, 1, 1]), seed=s)
        k = _graph_key(rp, col)
        counts[k] = counts.get(k, 0) + 1
    assert sorted(counts) == [((0, 1), (2, 3)), ((0, 2), (1, 3)), ((0, 3), (1, 2))]
    assert stats.chisquare(list(counts.values()), [1000] * 3).pvalue > ALPHA


def test_configuration_model_erases_loops_with_their_probability():
    # degrees (2,1,1), stubs a a' b c: {aa', bc} (1/3) loses the loop and keeps
    # {b,c}; the other two pairings (2/3) give the path b-a-c
    counts = {}
    for s in range(3000):
        rp, col = graphgen.configuration_model(np.array([2, 1, 1]), seed=s)
        k = _graph_key(rp, col)
        counts[k] = counts.get(k, 0) + 1
    assert sorted(counts) == [((0, 1), (0, 2)), ((1, 2),)]
    assert stats.chisquare([counts[((0, 1), (0, 2))], counts[((1, 2),)]], [2000, 1000]).pvalue > ALPHA


def test_erased_graph_is_simple_and_below_drawn_degrees():
    deg, _ = graphgen.pld_degrees(3000, 2, 400, 1.9, seed=4)
    rp, col = graphgen.configuration_model(deg, seed=4 + 0x5EED)
    assert _simple_symmetric_sorted(rp, col)
    got = np.diff(rp)
    assert np.all(got <= deg)
    # erasure removes few stubs on a sparse graph
    assert got.sum() >= 0.9 * deg.sum()
