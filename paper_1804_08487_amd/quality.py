"""Chain-quality measurements on the GPU chains (the paper's mixing study,
Sec. 5.1 "Mixing of Edge-Switching, Curveball and Global Curveball", and its
appendix on swaps performed by Curveball and Global Curveball).

The chains run in the HIP library through the C ABI (global trades, or n/2
uniform single trades per super-step); this module only downloads states and
does the statistics on the host:

* ``correlated_fraction``: the thinning criterion. Every edge that occurs in
  the chain gets its presence series Z_e; the k-thinned series keeps every
  k-th entry; it is fitted by an independent (Bernoulli) model and by a
  first-order Markov model, each scored by the Bayesian information criterion
  on the same transitions, and the edge counts as still correlated when the
  Markov model scores better. Reported per k as the fraction of edges.
* ``swap_fraction``: disjoint neighbours that changed sides over the sum of
  deg u + deg v of the trades (a swap exchanges two neighbours, and all
  possible swaps of a trade are (deg u + deg v) / 2), per super-step.
"""
from __future__ import annotations

import numpy as np

from . import Graph, OPT_GIANT_DEG, OPT_HELP_MIN


def run_chain(row_ptr, col, scheme: str, supersteps: int, seed: int):
    """States of the chain after each super-step (index 0: the start).
    scheme "global": one global trade per super-step; "single": n/2 uniform
    single trades per super-step. Returns a list of int32 arrays (CSR cols)."""
    n = len(row_ptr) - 1
    g = Graph(row_ptr, col)
    g.set_option(OPT_GIANT_DEG, 0)
    states = [np.array(col, np.int32, copy=True)]
    for t in range(supersteps):
        if scheme == "global":
            g.global_trade(seed, t)
        elif scheme == "single":
            g.single_trades(seed, t * (n // 2), n // 2)
        else:
            raise ValueError(scheme)
        states.append(g.download())
    g.close()
    return states


def edge_presence(row_ptr, states):
    """(keys, Z): keys of every edge {x < y} that occurs (x * n + y), and the
    boolean matrix Z[e, t] of its presence in state t."""
    n = len(row_ptr) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    per_state = []
    for c in states:
        c = np.asarray(c, np.int64)
        m = src < c
        per_state.append(src[m] * n + c[m])
    keys = np.unique(np.concatenate(per_state))
    Z = np.zeros((len(keys), len(states)), dtype=bool)
    for t, k in enumerate(per_state):
        Z[np.searchsorted(keys, k), t] = True
    return keys, Z


def _xlogy(x, y):
    out = np.zeros_like(y, dtype=float)
    m = x > 0
    out[m] = x[m] * np.log(y[m])
    return out


def correlated_by_bic(Z: np.ndarray) -> np.ndarray:
    """Per row of the boolean matrix Z (one series per edge): True when a
    first-order Markov model explains the transitions better than an
    independent Bernoulli model, by BIC on the same N - 1 observations
    (1 parameter against 2)."""
    a, b = Z[:, :-1], Z[:, 1:]
    N = b.shape[1]
    n01 = (~a & b).sum(1).astype(float)
    n00 = (~a & ~b).sum(1).astype(float)
    n11 = (a & b).sum(1).astype(float)
    n10 = (a & ~b).sum(1).astype(float)
    ones = n01 + n11
    p = ones / N
    ll_ind = _xlogy(ones, p) + _xlogy(N - ones, 1 - p)
    r0 = n00 + n01
    r1 = n10 + n11
    p01 = np.divide(n01, r0, out=np.zeros_like(n01), where=r0 > 0)
    p11 = np.divide(n11, r1, out=np.zeros_like(n11), where=r1 > 0)
    ll_mk = _xlogy(n01, p01) + _xlogy(n00, 1 - p01) + _xlogy(n11, p11) + _xlogy(n10, 1 - p11)
    bic_ind = -2 * ll_ind + 1 * np.log(N)
    bic_mk = -2 * ll_mk + 2 * np.log(N)
    return bic_mk < bic_ind


def correlated_fraction(Z: np.ndarray, ks) -> dict:
    """Fraction of edges still correlated in the k-thinned series, per k."""
    out = {}
    for k in ks:
        Zk = Z[:, ::k]
        out[int(k)] = float(correlated_by_bic(Zk).mean()) if Zk.shape[1] >= 3 and len(Zk) else float("nan")
    return out


def swap_fraction(row_ptr, col, scheme: str, supersteps: int, seed: int):
    """Per super-step: moved neighbours / sum of deg u + deg v (every trade
    counted: write phases are not shared)."""
    n = len(row_ptr) - 1
    g = Graph(row_ptr, col)
    g.set_option(OPT_GIANT_DEG, 0)
    g.set_option(OPT_HELP_MIN, 0)
    out = []
    for t in range(supersteps):
        if scheme == "global":
            g.global_trade(seed, t)
        else:
            g.single_trades(seed, t * (n // 2), n // 2)
        s = g.stats()
        out.append(s["moved"] / s["work"] if s["work"] else 0.0)
    g.close()
    return out


def correlated_fraction_states(row_ptr, states, ks, chunk: int = 1 << 16) -> dict:
    """correlated_fraction over every edge that occurs in `states`, built in
    chunks of edges (the presence matrix of all of them can be large)."""
    n = len(row_ptr) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    per_state = []
    for c in states:
        c = np.asarray(c, np.int64)
        m = src < c
        per_state.append(np.sort(src[m] * n + c[m]))
    keys = np.unique(np.concatenate(per_state))
    hits = {int(k): 0 for k in ks}
    for lo in range(0, len(keys), chunk):
        kk = keys[lo:lo + chunk]
        Z = np.zeros((len(kk), len(states)), dtype=bool)
        for t, ps in enumerate(per_state):
            sel = ps[(ps >= kk[0]) & (ps <= kk[-1])]
            Z[np.searchsorted(kk, sel), t] = True
        for k in ks:
            Zk = Z[:, ::k]
            if Zk.shape[1] >= 3:
                hits[int(k)] += int(correlated_by_bic(Zk).sum())
    return {k: hits[k] / len(keys) for k in hits}, len(keys)


def study(supersteps: int = 300, seed: int = 1, ks=(1, 2, 3, 4, 6, 8, 12, 16, 24, 32)):
    """The quality workload: thinning on Pld([5, b), 2) graphs with n = 2000,
    b in {25, 750}, for global trades and n/2 single trades per super-step;
    swap fractions on 10-regular and Pld([10, n/20), 2) graphs of growing n."""
    import graphgen
    out = {"thinning": [], "swap_fraction": []}
    for b in (25, 750):
        rp, col = graphgen.pld_graph(2000, 5, b, 2.0, 40 + b)
        for scheme in ("global", "single"):
            states = run_chain(rp, col, scheme, supersteps, seed)
            frac, edges = correlated_fraction_states(rp, states, ks)
            out["thinning"].append({"graph": f"n=2000 Pld([5,{b}),2)", "m": len(col) // 2, "scheme": scheme,
                                    "supersteps": supersteps, "edges_seen": edges, "correlated_fraction": frac})
    for n in (1 << 8, 1 << 10, 1 << 12, 1 << 14, 1 << 16):
        reg = graphgen.configuration_model(np.full(n, 10, np.int32), seed=n)
        pl = graphgen.pld_graph(n, 10, max(11, n // 20), 2.0, 70 + n)
        for name, (rp, col) in (("10-regular", reg), ("Pld([10,n/20),2)", pl)):
            for scheme in ("global", "single"):
                f = swap_fraction(rp, col, scheme, 4, seed)
                out["swap_fraction"].append({"graph": name, "n": n, "m": len(col) // 2, "scheme": scheme,
                                             "fraction": float(np.mean(f))})
    return out
