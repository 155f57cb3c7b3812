"""The statistics of the chain-quality study on series whose answer is known:
an independent Bernoulli series is classified independent, a sticky Markov
series correlated, and thinning a Markov series far beyond its correlation
time makes it independent again. Edge presence is recovered exactly."""
import numpy as np

import graphgen
from paper_1804_08487_amd import quality


def _markov(rows, T, p01, p11, seed):
    rng = np.random.default_rng(seed)
    Z = np.zeros((rows, T), bool)
    Z[:, 0] = rng.random(rows) < 0.5
    for t in range(1, T):
        u = rng.random(rows)
        Z[:, t] = np.where(Z[:, t - 1], u < p11, u < p01)
    return Z


def test_independent_series_are_classified_independent():
    Z = np.random.default_rng(1).random((2000, 600)) < 0.3
    assert quality.correlated_by_bic(Z).mean() < 0.1


def test_sticky_series_are_classified_correlated_and_thinning_decorrelates():
    Z = _markov(400, 20000, 0.02, 0.98, 2)      # correlation time about 25 steps
    frac = quality.correlated_fraction(Z, [1, 4, 200])
    assert frac[1] > 0.99
    assert frac[200] < 0.1
    assert frac[1] >= frac[4] >= frac[200]


def test_edge_presence_matrix():
    rp, col = graphgen.edge_list_to_csr(4, [(0, 1), (2, 3)])
    rp2, col2 = graphgen.edge_list_to_csr(4, [(0, 2), (1, 3)])
    assert np.array_equal(rp, rp2)
    keys, Z = quality.edge_presence(rp, [col, col2, col])
    assert keys.tolist() == [0 * 4 + 1, 0 * 4 + 2, 1 * 4 + 3, 2 * 4 + 3]
    assert Z.tolist() == [[True, False, True], [False, True, False], [False, True, False], [True, False, True]]
