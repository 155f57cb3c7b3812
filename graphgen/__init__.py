"""Seeded synthetic inputs: power-law degree sequences and erased
configuration-model graphs as symmetric CSR (numpy arrays).

This package is shared by the tests, the oracle checks and the benchmark; it
holds none of the Curveball arithmetic (see ``graphgen.c``).

Workloads (degrees i.i.d. from Pld([a,b), gamma), P[k] ~ k^-gamma):

* ``small``:  n = 8192,  Pld([5, 500), 2.0),      graph seed 1
* ``mid``:    n = 2^20,  Pld([10, 2^16), 2.0),    graph seed 1
* ``large``:  n = 2^24,  Pld([20, 2^20), 2.2),    graph seed 1
* ``hubs``:   n = 2^24,  Pld([1, 2^16), 2.5),     graph seed 3 (sparse, about ten
  nodes of degree above 8192: the bitmap-set path at the full id range)
* batched:    ``batch_specs`` / ``batch_chain``: 512 chains of 2^10..2^16 nodes
* served:     ``serve_specs``: requests of 2^12..2^24 edges, 1..32 samples, 5..20 rounds
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
LIB_PATH = os.path.join(_HERE, "libgraphgen.so")

WORKLOADS = {
    "small": dict(n=8192, a=5, b=500, gamma=2.0, seed=1),
    "mid": dict(n=1 << 20, a=10, b=1 << 16, gamma=2.0, seed=1),
    "large": dict(n=1 << 24, a=20, b=1 << 20, gamma=2.2, seed=1),
    # sparse graph over 2^24 ids with a handful of nodes above degree 8192
    "hubs": dict(n=1 << 24, a=1, b=1 << 16, gamma=2.5, seed=3),
}

_lib = None


def build(out: str = LIB_PATH) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-fPIC", "-shared", "-pthread",
           "-o", out + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.gg_degrees.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_int, i32p]
        lib.gg_degrees.restype = ctypes.c_int64
        lib.gg_configuration_model.argtypes = [ctypes.c_int64, i32p, ctypes.c_uint64, ctypes.c_int,
                                               i64p, i32p, ctypes.c_int64]
        lib.gg_configuration_model.restype = ctypes.c_int64
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def pld_degrees(n: int, a: int, b: int, gamma: float, seed: int, threads: int | None = None):
    lib = _load()
    deg = np.empty(max(n, 1), np.int32)
    total = lib.gg_degrees(n, a, b, gamma, seed, threads or default_threads(),
                           deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if total < 0:
        raise ValueError(f"gg_degrees failed ({total})")
    return deg[:n], int(total)


def configuration_model(deg: np.ndarray, seed: int, threads: int | None = None):
    """Erased configuration model for an even-sum degree sequence."""
    lib = _load()
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    n = len(deg)
    total = int(deg.sum(dtype=np.int64))
    row_ptr = np.empty(n + 1, np.int64)
    col = np.empty(max(total, 1), np.int32)
    nnz = lib.gg_configuration_model(n, deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), seed,
                                     threads or default_threads(),
                                     row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(col))
    if nnz < 0:
        raise ValueError(f"gg_configuration_model failed ({nnz})")
    if nnz < len(col) // 2:
        col = col[:nnz].copy()
    else:
        col = col[:nnz]
    return row_ptr, col


def pld_graph(n: int, a: int, b: int, gamma: float, seed: int, threads: int | None = None,
              cache_dir: str | None = None):
    """Power-law erased configuration-model graph (row_ptr int64, col int32).

    With ``cache_dir`` (or the ``CB_GRAPH_CACHE`` environment variable) the
    arrays are kept as .npy files keyed by the parameters."""
    cache_dir = cache_dir or os.environ.get("CB_GRAPH_CACHE")
    key = hashlib.sha1(repr((n, a, b, float(gamma), seed, "v1")).encode()).hexdigest()[:16]
    if cache_dir:
        rp_path = os.path.join(cache_dir, f"g_{key}_rp.npy")
        col_path = os.path.join(cache_dir, f"g_{key}_col.npy")
        if os.path.exists(rp_path) and os.path.exists(col_path):
            return np.load(rp_path), np.load(col_path, mmap_mode=None)
    deg, _ = pld_degrees(n, a, b, gamma, seed, threads)
    row_ptr, col = configuration_model(deg, seed + 0x5EED, threads)
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        np.save(rp_path + ".tmp.npy", row_ptr)
        np.save(col_path + ".tmp.npy", col)
        os.replace(rp_path + ".tmp.npy", rp_path)
        os.replace(col_path + ".tmp.npy", col_path)
    return row_ptr, col


def workload(name: str, **kw):
    p = dict(WORKLOADS[name])
    p.update(kw)
    return pld_graph(p["n"], p["a"], p["b"], p["gamma"], p["seed"])


def batch_specs(chains: int = 512, seed: int = 4):
    """The batched workload: chain c has n_c = round(2^U[10,16]) nodes, degrees
    Pld([2, n_c / 8), gamma_c) with gamma_c ~ U[1.8, 2.6], graph seed 1000 + c
    and chain seed c. The uniforms come from numpy's PCG64 with `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((chains, 2))
    out = []
    for c in range(chains):
        n = int(round(2.0 ** (10 + 6 * u[c, 0])))
        out.append(dict(n=n, a=2, b=max(3, n // 8), gamma=float(1.8 + 0.8 * u[c, 1]),
                        graph_seed=1000 + c, chain_seed=c))
    return out


def batch_chain(spec):
    return pld_graph(spec["n"], spec["a"], spec["b"], spec["gamma"], spec["graph_seed"], threads=1)


def pld_mean(a: int, b: int, gamma: float) -> float:
    ks = np.arange(a, b, dtype=float)
    w = ks ** -gamma
    return float((ks * w).sum() / w.sum())


def serve_specs(count: int, seed: int = 5):
    """The served workload: request q has m_target = 2^U[12,24] edges, n chosen
    so that n * E[Pld([5, sqrt n), 2)] / 2 is about m_target, graph seed
    10^6 + q, k ~ U{1..32} samples and r ~ U{5..20} rounds (numpy PCG64 with
    `seed`)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for q in range(count):
        m_target = 2.0 ** (12 + 12 * rng.random())
        lo, hi = 16, 1 << 26
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if mid * pld_mean(5, max(6, int(mid ** 0.5)), 2.0) / 2 < m_target:
                lo = mid
            else:
                hi = mid
        n = hi
        out.append(dict(n=n, a=5, b=max(6, int(n ** 0.5)), gamma=2.0, graph_seed=10**6 + q,
                        samples=int(rng.integers(1, 33)), rounds=int(rng.integers(5, 21)),
                        chain_seed=7919 * (q + 1)))
    return out


def edge_list_to_csr(n: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric sorted CSR from an undirected simple edge list (tests)."""
    rows = [set() for _ in range(n)]
    for x, y in edges:
        if x == y:
            raise ValueError("self-loop")
        rows[x].add(y)
        rows[y].add(x)
    row_ptr = np.zeros(n + 1, np.int64)
    for x in range(n):
        row_ptr[x + 1] = row_ptr[x] + len(rows[x])
    col = np.array([y for x in range(n) for y in sorted(rows[x])], dtype=np.int32)
    return row_ptr, col


def random_simple_graph(n: int, p: float, seed: int):
    """Erdos-Renyi G(n, p) as CSR (small test graphs)."""
    rng = np.random.default_rng(seed)
    edges = [(x, y) for x in range(n) for y in range(x + 1, n) if rng.random() < p]
    return edge_list_to_csr(n, edges)
