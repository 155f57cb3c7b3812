"""Pins of the oracle's uniform single-trade chain (Simple Undirected
Curveball, Sec. 3.2): the pair law, a hand-derived exact row, exact
enumeration (symmetric, stochastic, mixing to uniform), the oracle's one-step
frequencies against the exact row, and invariants."""
import json
import os
from fractions import Fraction
from itertools import permutations

import numpy as np
import pytest
from scipy import stats

import graphgen
from tests import exact_enum

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA = 1e-3


def _key(rp, col, n):
    return tuple(sorted((x, int(y)) for x in range(n) for y in col[rp[x]:rp[x + 1]] if x < y))


@pytest.mark.parametrize("n", [2, 5, 9])
def test_pair_is_uniform_over_ordered_pairs(orc, n):
    pairs = {(u, v): i for i, (u, v) in enumerate((u, v) for u in range(n) for v in range(n) if u != v)}
    counts = np.zeros(len(pairs))
    for s in range(300 * len(pairs)):
        u, v = orc.cbu_pair(n, 17, s)
        assert 0 <= u < n and 0 <= v < n and u != v
        counts[pairs[(u, v)]] += 1
    assert stats.chisquare(counts, np.full(len(pairs), counts.sum() / len(pairs))).pvalue > ALPHA


def test_enumerator_reproduces_hand_derived_cbu_row():
    g = json.load(open(os.path.join(GOLDEN, "cbu_four_node_row.json")))
    row = exact_enum.cbu_row(exact_enum.from_edges(g["n"], g["start"]))
    assert row == {tuple(map(tuple, s)): Fraction(p) for s, p in g["row"]}


@pytest.mark.parametrize("degrees", [(1, 1, 2, 2), (2, 2, 2, 2), (1, 2, 2, 2, 1), (1, 1, 2, 2, 2, 2)])
def test_cbu_matrix_symmetric_stochastic_mixing(degrees):
    states, P = exact_enum.cbu_matrix(degrees)
    k = len(states)
    for i in range(k):
        assert sum(P[i]) == 1 and P[i][i] > 0
        for j in range(k):
            assert P[i][j] == P[j][i]
    R = np.linalg.matrix_power(np.array([[float(x) for x in r] for r in P]), 400)
    assert np.allclose(R, 1.0 / k, atol=1e-9)


@pytest.mark.parametrize("n,edges,samples", [
    (4, [(0, 1), (2, 3)], 6000),
    (5, [(0, 1), (1, 2), (2, 3), (3, 4)], 12000),
])
def test_oracle_single_step_frequencies_match_exact_row(orc, n, edges, samples):
    exact = exact_enum.cbu_row(exact_enum.from_edges(n, edges))
    rp, col = graphgen.edge_list_to_csr(n, edges)
    counts = {}
    for s in range(samples):
        out, st = orc.cbu(rp, col, seed=s, step0=0, steps=1)
        assert st["trades"] == 1
        k = _key(rp, out, n)
        counts[k] = counts.get(k, 0) + 1
    assert set(counts) <= set(exact)
    keys = sorted(exact)
    obs = [counts.get(k, 0) for k in keys]
    assert stats.chisquare(obs, [float(exact[k]) * samples for k in keys]).pvalue > ALPHA


def test_oracle_chain_invariants_and_resume(orc):
    rp, col = graphgen.pld_graph(600, 2, 80, 2.0, 9)
    a, sa = orc.cbu(rp, col, 5, 0, 2000)
    assert orc.check_graph(rp, a) == 0 and sa["trades"] == 2000
    assert (a != col).any()
    b, _ = orc.cbu(rp, col, 5, 0, 700)
    b, _ = orc.cbu(rp, b, 5, 700, 1300)
    assert np.array_equal(a, b)
    c, _ = orc.cbu(rp, col, 6, 0, 2000)
    assert not np.array_equal(a, c)
    assert sa["moved"] % 2 == 0 and 0 < sa["moved"] <= sa["disjoint"]


def test_oracle_chain_degenerate(orc):
    for n in (0, 1):
        rp = np.zeros(n + 1, np.int64)
        out, st = orc.cbu(rp, np.zeros(0, np.int32), 1, 0, 10)
        assert out.size == 0 and st["trades"] == 0
    rp, col = graphgen.edge_list_to_csr(2, [(0, 1)])
    out, st = orc.cbu(rp, col, 1, 0, 10)          # the only pair's edge is never traded
    assert np.array_equal(out, col) and st["moved"] == 0
