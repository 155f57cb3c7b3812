"""Oracle self-consistency: O1 (definition-literal) and O2 (IM-CB form) give
the same bytes; every round keeps degrees, simplicity and symmetry; the
dependency count equals a brute-force edge count and what O2 actually
receives; work per round is 2m - deg(unmatched); degenerate graphs."""
import numpy as np
import pytest

import graphgen


def _graphs():
    yield "empty0", (np.zeros(1, np.int64), np.zeros(0, np.int32))
    yield "single", (np.zeros(2, np.int64), np.zeros(0, np.int32))
    yield "pair", graphgen.edge_list_to_csr(2, [(0, 1)])
    yield "three", graphgen.edge_list_to_csr(3, [(0, 1), (1, 2)])
    yield "isolated", graphgen.edge_list_to_csr(7, [(0, 1), (2, 3)])
    yield "star", graphgen.edge_list_to_csr(9, [(0, i) for i in range(1, 9)])
    yield "clique", graphgen.edge_list_to_csr(7, [(i, j) for i in range(7) for j in range(i + 1, 7)])
    yield "bipartite", graphgen.edge_list_to_csr(9, [(i, j) for i in range(4) for j in range(4, 9)])
    for s in range(12):
        yield f"er{s}", graphgen.random_simple_graph(20 + s, 0.1 + 0.03 * s, s)
    yield "pld", graphgen.pld_graph(500, 2, 60, 2.0, 7)
    yield "pld_odd", graphgen.pld_graph(501, 2, 60, 2.0, 8)


GRAPHS = list(_graphs())


def _brute_dep(row_ptr, col, trade_of, n):
    dep = np.zeros(n // 2, np.int64)
    for x in range(n):
        for y in col[row_ptr[x]:row_ptr[x + 1]]:
            if x < y:
                tx, ty = trade_of[x], trade_of[y]
                if tx != ty and max(tx, ty) != 2**31 - 1:
                    dep[max(tx, ty)] += 1
    return dep


@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_o1_equals_o2_and_invariants(orc, name, g):
    row_ptr, col = g
    n = len(row_ptr) - 1
    assert orc.check_graph(row_ptr, col) == 0
    c1 = c2 = col
    for rnd in range(4):
        order, trade_of = orc.matching(n, 11, rnd)
        dep = orc.depcount(row_ptr, c1, trade_of, order)
        assert np.array_equal(dep, _brute_dep(row_ptr, c1, trade_of, n))
        c1, s1 = orc.global_trade(row_ptr, c1, 11, rnd, "o1")
        c2, s2 = orc.global_trade(row_ptr, c2, 11, rnd, "o2")
        assert np.array_equal(c1, c2)
        assert s1["dep_mismatch"] == 0 and s2["dep_mismatch"] == 0
        for k in ("trades", "work", "common", "disjoint", "moved", "uv_edges", "max_s"):
            assert s1[k] == s2[k], k
        assert orc.check_graph(row_ptr, c1) == 0
        unmatched_deg = 0
        if n % 2:
            assert s1["unmatched"] == order[-1]
            unmatched_deg = row_ptr[order[-1] + 1] - row_ptr[order[-1]]
        else:
            assert s1["unmatched"] == -1
        assert s1["work"] == len(col) - unmatched_deg
        assert s1["trades"] == n // 2


def test_clique_and_star_are_fixed_points(orc):
    for edges, n in (([(i, j) for i in range(9) for j in range(i + 1, 9)], 9),
                     ([(0, i) for i in range(1, 12)], 12)):
        rp, col = graphgen.edge_list_to_csr(n, edges)
        out, st = orc.global_trade(rp, col, 5, 0)
        assert np.array_equal(out, col)
        assert st["moved"] == 0


def test_determinism_and_round_dependence(orc):
    rp, col = graphgen.pld_graph(300, 3, 40, 2.0, 3)
    a, _ = orc.global_trade(rp, col, 9, 0)
    b, _ = orc.global_trade(rp, col, 9, 0)
    c, _ = orc.global_trade(rp, col, 9, 1)
    d, _ = orc.global_trade(rp, col, 10, 0)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)


def test_resume_equals_uninterrupted(orc):
    rp, col = graphgen.pld_graph(400, 3, 40, 2.0, 4)
    x = col
    for r in range(6):
        x, _ = orc.global_trade(rp, x, 21, r)
    y = col
    for r in range(3):
        y, _ = orc.global_trade(rp, y, 21, r)
    y = np.array(y)          # "download" and continue from a copy
    for r in range(3, 6):
        y, _ = orc.global_trade(rp, y, 21, r)
    assert np.array_equal(x, y)


def test_small_workload_many_rounds(orc):
    rp, col = graphgen.workload("small")
    x = col
    for r in range(10):
        x, st = orc.global_trade(rp, x, 1, r, "o2")
        assert st["dep_mismatch"] == 0
    assert orc.check_graph(rp, x) == 0
    # edges really move: most of the graph differs from the start
    assert (x != col).mean() > 0.5
