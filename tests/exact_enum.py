"""Brute-force exact transition probabilities of one global trade on tiny
graphs, written directly from the paper's definitions with Python sets and
rational arithmetic.  Independent of the C oracle (no shared code): it
enumerates every node order (uniform permutation, Def. "Undirected Global
Trade") and, for every trade, every way to hand |A_{u-v}| of the disjoint
neighbours to u (sigma uniform, Sec. 3.2 / Sec. 4), each with its exact
probability.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations, permutations


def canon(adj):
    """Graph state as a sorted tuple of edges (x < y)."""
    return tuple(sorted((x, y) for x in range(len(adj)) for y in adj[x] if x < y))


def from_edges(n, edges):
    adj = [set() for _ in range(n)]
    for x, y in edges:
        adj[x].add(y)
        adj[y].add(x)
    return tuple(frozenset(s) for s in adj)


def trade_outcomes(adj, u, v):
    """All results of trading u and v, with their probabilities."""
    su = adj[u] - {v}
    sv = adj[v] - {u}
    common = su & sv
    x_only = su - common
    y_only = sv - common
    disjoint = sorted(x_only | y_only)
    a = len(x_only)
    choices = list(combinations(disjoint, a))
    p = Fraction(1, len(choices))
    out = []
    for pick in choices:
        to_u = set(pick)
        to_v = set(disjoint) - to_u
        new = [set(s) for s in adj]
        new[u] = common | to_u | ({v} if v in adj[u] else set())
        new[v] = common | to_v | ({u} if u in adj[v] else set())
        for x in x_only - to_u:      # passive lists follow the moved edges
            new[x].discard(u)
            new[x].add(v)
        for y in y_only - to_v:
            new[y].discard(v)
            new[y].add(u)
        out.append((p, tuple(frozenset(s) for s in new)))
    return out


def global_trade_row(adj):
    """Exact distribution of canon(state) after one global trade from adj."""
    n = len(adj)
    orders = list(permutations(range(n)))
    p_order = Fraction(1, len(orders))
    dist = {}
    for order in orders:
        states = {adj: Fraction(1)}
        for i in range(n // 2):
            u, v = order[2 * i], order[2 * i + 1]
            nxt = {}
            for s, ps in states.items():
                for p, t in trade_outcomes(s, u, v):
                    nxt[t] = nxt.get(t, 0) + ps * p
            states = nxt
        for s, ps in states.items():
            key = canon(s)
            dist[key] = dist.get(key, 0) + p_order * ps
    return dist


def state_space(degrees):
    """All simple graphs on len(degrees) labelled nodes with these degrees."""
    n = len(degrees)
    pairs = [(x, y) for x in range(n) for y in range(x + 1, n)]
    m2 = sum(degrees)
    if m2 % 2:
        return []
    m = m2 // 2
    out = []
    for es in combinations(pairs, m):
        deg = [0] * n
        for x, y in es:
            deg[x] += 1
            deg[y] += 1
        if deg == list(degrees):
            out.append(tuple(es))
    return out


def transition_matrix(degrees):
    """(states, P) with P[i][j] = exact probability state i -> state j."""
    states = state_space(degrees)
    index = {s: i for i, s in enumerate(states)}
    n = len(degrees)
    P = [[Fraction(0)] * len(states) for _ in states]
    for i, s in enumerate(states):
        for t, p in global_trade_row(from_edges(n, s)).items():
            P[i][index[t]] += p
    return states, P


def cbu_row(adj):
    """Exact distribution of canon(state) after one uniform single trade
    (Simple Undirected Curveball): an ordered pair of distinct nodes drawn
    uniformly (so a uniform unordered pair), then the trade with a uniform
    split."""
    n = len(adj)
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    p_pair = Fraction(1, len(pairs))
    dist = {}
    for u, v in pairs:
        for p, t in trade_outcomes(adj, u, v):
            key = canon(t)
            dist[key] = dist.get(key, 0) + p_pair * p
    return dist


def cbu_matrix(degrees):
    states = state_space(degrees)
    index = {s: i for i, s in enumerate(states)}
    n = len(degrees)
    P = [[Fraction(0)] * len(states) for _ in states]
    for i, s in enumerate(states):
        for t, p in cbu_row(from_edges(n, s)).items():
            P[i][index[t]] += p
    return states, P
