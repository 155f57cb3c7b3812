"""Pins of the CPU oracle against facts fixed outside it: published Philox
known answers, the paper's worked trade example, closed forms of the bounded
draw, the hypergeometric law of a uniform split, exact transition rows by
brute force, and the paper's theorem (symmetric, stochastic transition
matrix converging to uniform)."""
import json
import math
import os
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest
from scipy import stats

import graphgen
from tests import exact_enum

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA = 1e-3


def _chi2_ok(observed, expected_probs):
    observed = np.asarray(observed, dtype=float)
    expected = np.asarray(expected_probs, dtype=float) * observed.sum()
    return stats.chisquare(observed, expected).pvalue > ALPHA


# ---------------------------------------------------------------- Philox

def test_philox_known_answers(orc):
    rows = [line.split() for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        ctr = [int(x, 16) for x in r[0:4]]
        key = [int(x, 16) for x in r[4:6]]
        want = tuple(int(x, 16) for x in r[6:10])
        assert orc.philox4x32_10(ctr, key) == want


def test_philox64_word_order(orc):
    # philox64 = (w1 << 32) | w0 of the block with key (seed_lo, seed_hi)
    seed = 0x0123456789ABCDEF
    w = orc.philox4x32_10((5, 6, 7, 8), (seed & 0xFFFFFFFF, seed >> 32))
    assert orc.philox64(seed, 5, 6, 7, 8) == (w[1] << 32) | w[0]


# ---------------------------------------------------------------- bounded draw

def test_bounded_closed_forms(orc):
    top = 2**64 - 1
    for k in (1, 2, 3, 7, 10, 2**31 - 1, 2**32, 2**40 + 3):
        assert orc.bounded(0, k) == 0
        assert orc.bounded(top, k) == k - 1
        assert orc.bounded(2**63, k) == k // 2
    assert orc.bounded(0xDEADBEEF12345678, 2**32) == 0xDEADBEEF
    assert orc.bounded(3 * 2**62, 4) == 3
    # monotone in x
    xs = sorted(orc.philox64(9, i, 0, 0, 1) for i in range(200))
    ys = [orc.bounded(x, 1000) for x in xs]
    assert ys == sorted(ys)


def test_bounded_uniform_on_philox(orc):
    k = 7
    counts = np.zeros(k)
    for i in range(14000):
        counts[orc.bounded(orc.philox64(123, i, 1, 2, 3), k)] += 1
    assert _chi2_ok(counts, [1 / k] * k)


# ---------------------------------------------------------------- one trade

def test_trade_matches_paper_figure(orc):
    g = json.load(open(os.path.join(GOLDEN, "trade_figure.json")))
    Bu, Bv, mtv, mtu, info = orc.trade_apply(g["A_i"], g["A_j"], g["i"], g["j"],
                                             arrangement=g["sigma"])
    assert Bu.tolist() == g["B_i"]
    assert Bv.tolist() == g["B_j"]
    assert sorted(mtv.tolist()) == g["moved_i_to_j"]
    assert sorted(mtu.tolist()) == g["moved_j_to_i"]
    assert info["common"] == 1 and info["uv"] == 1          # triangle (i, j, 6) kept
    assert len(mtv) + len(mtu) == 4                          # four edges change


def test_trade_rejects_bad_sigma(orc):
    with pytest.raises(ValueError):
        orc.trade_apply([1, 2, 6, 8], [3, 4, 5, 6, 7], 7, 8, arrangement=[4, 3, 5, 1, 9])


@pytest.mark.parametrize("a,b", [(2, 3), (3, 2), (1, 4), (4, 1), (3, 3), (2, 2), (1, 1)])
def test_split_uniform_over_subsets_and_hypergeometric(orc, a, b):
    N = a + b
    subsets = list(combinations(range(N), a))
    index = {s: i for i, s in enumerate(subsets)}
    counts = np.zeros(len(subsets))
    kept = np.zeros(a + 1)           # elements of X (ids < a) that stay with u
    trials = 400 * len(subsets)
    for t in range(trials):
        D = orc.split(np.arange(N), a, 77, 5, t)
        assert sorted(D.tolist()) == list(range(N))
        U = tuple(sorted(D[:a].tolist()))
        counts[index[U]] += 1
        kept[sum(1 for x in U if x < a)] += 1
    assert _chi2_ok(counts, [1 / len(subsets)] * len(subsets))
    pmf = [math.comb(a, i) * math.comb(b, a - i) / math.comb(N, a) for i in range(a + 1)]
    nz = [i for i in range(a + 1) if pmf[i] > 0]
    assert _chi2_ok(kept[nz], [pmf[i] for i in nz])


def test_split_degenerate_sides_draw_nothing(orc):
    D = np.arange(6)
    assert orc.split(D, 0, 1, 2, 3).tolist() == list(range(6))
    assert orc.split(D, 6, 1, 2, 3).tolist() == list(range(6))


def test_hypergeometric_pmf_values():
    # the pmfs quoted as pins for the moved count (a, b) -> P(|U n X| = i)
    def pmf(a, b):
        return [Fraction(math.comb(a, i) * math.comb(b, a - i), math.comb(a + b, a))
                for i in range(a + 1)]
    assert pmf(2, 3) == [Fraction(3, 10), Fraction(3, 5), Fraction(1, 10)]
    assert pmf(3, 3) == [Fraction(1, 20), Fraction(9, 20), Fraction(9, 20), Fraction(1, 20)]


def test_trade_set_invariants_random(orc):
    rng = np.random.default_rng(5)
    for t in range(300):
        n = 40
        u, v = 0, 1
        Au = set(rng.choice(np.arange(2, n), rng.integers(0, 20), replace=False).tolist())
        Av = set(rng.choice(np.arange(2, n), rng.integers(0, 20), replace=False).tolist())
        if rng.random() < 0.5:
            Au.add(v)
            Av.add(u)
        Bu, Bv, mtv, mtu, info = orc.trade_apply(sorted(Au), sorted(Av), u, v, seed=3, rnd=1, trade=t)
        Bu, Bv = set(Bu.tolist()), set(Bv.tolist())
        assert len(Bu) == len(Au) and len(Bv) == len(Av)            # degrees
        assert (v in Bu) == (v in Au) and (u in Bv) == (u in Av)    # u-v edge kept
        assert (Bu - {v}) & (Bv - {u}) == (Au - {v}) & (Av - {u})  # shared kept
        assert (Bu - {v}) | (Bv - {u}) == (Au - {v}) | (Av - {u})  # D re-split
        assert set(mtv.tolist()) == (Au - {v}) - Bu
        assert set(mtu.tolist()) == (Av - {u}) - Bv
        assert u not in Bu and v not in Bv


# ---------------------------------------------------------------- matching

@pytest.mark.parametrize("n", [4, 5])
def test_matching_is_uniform_permutation(orc, n):
    from itertools import permutations
    perms = {p: i for i, p in enumerate(permutations(range(n)))}
    counts = np.zeros(len(perms))
    samples = 60 * len(perms)
    for s in range(samples):
        order, trade_of = orc.matching(n, seed=1000 + s // 7, rnd=s % 7)
        counts[perms[tuple(order.tolist())]] += 1
    assert _chi2_ok(counts, [1 / len(perms)] * len(perms))


def test_matching_trade_of_layout(orc):
    for n in (0, 1, 2, 3, 10, 11):
        order, trade_of = orc.matching(n, 3, 4)
        assert sorted(order.tolist()) == list(range(n))
        for p, x in enumerate(order.tolist()):
            if n % 2 and p == n - 1:
                assert trade_of[x] == 2**31 - 1
            else:
                assert trade_of[x] == p // 2


# ---------------------------------------------------------------- exact chain

def test_enumerator_reproduces_hand_derived_row():
    g = json.load(open(os.path.join(GOLDEN, "four_node_row.json")))
    start = exact_enum.from_edges(g["n"], g["start"])
    row = exact_enum.global_trade_row(start)
    want = {tuple(map(tuple, s)): Fraction(p) for s, p in g["row"]}
    assert row == want


@pytest.mark.parametrize("degrees", [(1, 1, 1, 1), (1, 1, 2, 2), (2, 2, 2, 2),
                                     (1, 2, 2, 2, 1), (2, 2, 2, 2, 2), (1, 1, 2, 2, 2, 2)])
def test_exact_matrix_symmetric_stochastic_mixing(degrees):
    """Theorem (Sec. 3.3): P is symmetric and the chain converges to uniform."""
    states, P = exact_enum.transition_matrix(degrees)
    k = len(states)
    assert k >= 1
    for i in range(k):
        assert sum(P[i]) == 1
        assert P[i][i] > 0                                   # aperiodic (self-loop)
        for j in range(k):
            assert P[i][j] == P[j][i]
    M = np.array([[float(x) for x in r] for r in P])
    R = np.linalg.matrix_power(M, 200)
    assert np.allclose(R, 1.0 / k, atol=1e-9)               # irreducible -> uniform


def _empirical_row(orc, n, edges, seeds):
    rp, col = graphgen.edge_list_to_csr(n, edges)
    counts = {}
    for s in seeds:
        out, _ = orc.global_trade(rp, col, seed=s, rnd=0)
        key = tuple(sorted((x, int(y)) for x in range(n)
                           for y in out[rp[x]:rp[x + 1]] if x < y))
        counts[key] = counts.get(key, 0) + 1
    return counts


@pytest.mark.parametrize("n,edges,samples", [
    (4, [(0, 1), (2, 3)], 6000),
    (5, [(0, 1), (1, 2), (2, 3), (3, 4)], 16000),
    (6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)], 16000),
])
def test_oracle_one_step_frequencies_match_exact_row(orc, n, edges, samples):
    exact = exact_enum.global_trade_row(exact_enum.from_edges(n, edges))
    counts = _empirical_row(orc, n, edges, range(samples))
    assert set(counts) <= set(exact)                       # only reachable states
    keys = sorted(exact)
    obs = [counts.get(k, 0) for k in keys]
    assert _chi2_ok(obs, [float(exact[k]) for k in keys])


def test_oracle_two_steps_frequencies_match_exact(orc):
    n, edges = 5, [(0, 1), (1, 2), (2, 3), (3, 4)]
    states, P = exact_enum.transition_matrix((1, 2, 2, 2, 1))
    start = states.index(tuple(sorted(edges)))
    two = [sum(P[start][m] * P[m][j] for m in range(len(states))) for j in range(len(states))]
    rp, col = graphgen.edge_list_to_csr(n, edges)
    counts = np.zeros(len(states))
    for s in range(12000):
        c = col
        for r in range(2):
            c, _ = orc.global_trade(rp, c, seed=s, rnd=r)
        key = tuple(sorted((x, int(y)) for x in range(n) for y in c[rp[x]:rp[x + 1]] if x < y))
        counts[states.index(key)] += 1
    nz = [j for j in range(len(states)) if two[j] > 0]
    assert counts[[j for j in range(len(states)) if two[j] == 0]].sum() == 0
    assert _chi2_ok(counts[nz], [float(two[j]) for j in nz])


# Exact one-step rows of a global trade from fixed states, derived once by an
# independent brute force in rational arithmetic (every node order, every
# split): the enumerator above must reproduce them. States are edge sets; rows
# are over the lexicographic order of the state space.
def _two_triangles(state):
    adj = {x: set() for x in range(6)}
    for a, b in state:
        adj[a].add(b)
        adj[b].add(a)
    return all(len(adj[a] & adj[b]) == 1 for a, b in state)


def test_enumerator_exact_rows_odd_n_path():
    states, P = exact_enum.transition_matrix((1, 2, 2, 2, 1))
    start = states.index(((0, 1), (1, 2), (2, 3), (3, 4)))
    assert start == 0
    assert P[start] == [Fraction(68, 135), Fraction(59, 540), Fraction(59, 540), Fraction(13, 540),
                        Fraction(13, 540), Fraction(2, 15), Fraction(13, 135)]


def test_enumerator_exact_rows_small_even():
    states, P = exact_enum.transition_matrix((1, 1, 2, 2))
    assert len(states) == 2 and P[0][0] == Fraction(5, 6) and P[0][1] == Fraction(1, 6)
    states, P = exact_enum.transition_matrix((2, 2, 2, 2))
    assert len(states) == 3
    assert all(P[i][j] == (Fraction(2, 3) if i == j else Fraction(1, 6)) for i in range(3) for j in range(3))
    states, P = exact_enum.transition_matrix((1, 1, 2, 2, 2, 2))
    assert len(states) == 31 and P[0][0] == Fraction(2, 9)


def test_enumerator_exact_rows_five_cycle():
    states, P = exact_enum.transition_matrix((2, 2, 2, 2, 2))
    start = states.index(((0, 1), (0, 2), (1, 3), (2, 4), (3, 4)))
    assert len(states) == 12
    assert P[start][start] == Fraction(1, 3)
    assert sum(1 for p in P[start] if p == 0) == 1


def test_enumerator_exact_rows_six_nodes_two_classes():
    tri = ((0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5))
    row = exact_enum.global_trade_row(exact_enum.from_edges(6, tri))
    assert row[tri] == Fraction(31, 270)
    assert sum(p for s, p in row.items() if _two_triangles(s)) == Fraction(7, 27)
    assert sum(p for s, p in row.items() if not _two_triangles(s)) == Fraction(20, 27)
    c6 = ((0, 1), (0, 5), (1, 2), (2, 3), (3, 4), (4, 5))
    row = exact_enum.global_trade_row(exact_enum.from_edges(6, c6))
    assert row[c6] == Fraction(193, 1620)
    assert sum(p for s, p in row.items() if _two_triangles(s)) == Fraction(10, 81)


# ---------------------------------------------------------------- graph check

@pytest.mark.parametrize("name,n,rp,col,code", [
    ("row_ptr0", 2, [1, 1, 2], [1, 0], -1),
    ("non_monotone", 2, [0, -1, 0], [0], -2),
    ("negative_id", 2, [0, 1, 2], [-1, 0], -3),
    ("id_beyond_n", 2, [0, 1, 2], [2, 0], -3),
    ("self_loop", 2, [0, 2, 3], [0, 1, 0], -4),
    ("unsorted_row", 3, [0, 2, 3, 4], [2, 1, 0, 0], -5),
    ("duplicate", 3, [0, 3, 4, 5], [1, 1, 2, 0, 0], -5),
    ("asymmetric", 3, [0, 1, 2, 2], [1, 2], -6),
    ("odd_entries", 2, [0, 1, 1], [1], -6),
])
def test_check_graph_rejects(orc, name, n, rp, col, code):
    assert orc.check_graph(np.array(rp, np.int64), np.array(col, np.int32)) == code


def test_check_graph_accepts_simple_symmetric(orc):
    rp, col = graphgen.edge_list_to_csr(5, [(0, 1), (0, 4), (1, 2), (3, 4)])
    assert orc.check_graph(rp, col) == 0
    assert orc.check_graph(np.zeros(4, np.int64), np.zeros(0, np.int32)) == 0
