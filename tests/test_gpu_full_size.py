"""Parity of the HIP path with the oracle at the full workload sizes, on the GPU.

The oracle's whole-chain results at these sizes are stored as SHA-256
digests (``tests/golden/digests_<workload>.json``, written by
``tests/golden/make_digests.py``, which calls only ``oracle/`` and
``graphgen/``). After every round the whole downloaded adjacency is hashed
and compared: equal digests of the whole int32 array mean the arrays are
equal element by element. The round-0 matching (``perm``, ``trade_of``) and
dependency counts are compared in full the same way.

Workloads (inputs regenerated here from their seeds, checked against the
stored input digest first):

* mid:   n = 2^20, Pld([10, 2^16), 2.0): all 20 rounds of chain seed 1 and
  3 rounds of chain seed 2;
* large: n = 2^24, Pld([20, 2^20), 2.2): all 10 rounds of chain seed 1, in the
  launch configuration the benchmark times;
* hubs:  n = 2^24, Pld([1, 2^16), 2.5): sparse, with nodes above degree 8192
  whose arrivals go to bitmap sets over all 2^24 ids (4096 superblocks).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen
import paper_1804_08487_amd as cb

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(f"[gpu-full] {msg}", flush=True)


def _sha(a):
    return hashlib.sha256(memoryview(np.ascontiguousarray(a)).cast("B")).hexdigest()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def _digests(name):
    path = os.path.join(GOLDEN, f"digests_{name}.json")
    if not os.path.exists(path):
        pytest.fail(f"{path} is missing: run tests/golden/make_digests.py {name}")
    with open(path) as f:
        return json.load(f)


def _check_chain(name, rp, col, chain, rounds=None, options=None):
    seed = chain["seed"]
    want = chain["col_sha256"][:rounds] if rounds else chain["col_sha256"]
    n = len(rp) - 1
    g = cb.Graph(rp, col, validate=False)
    for opt, val in (options or {}).items():
        g.set_option(opt, val)
    # round 0, step by step: matching and dependency counts in full
    g.run_steps(seed, 0, cb.STEP_DEPSCAN)
    assert _sha(g.state(cb.STATE_PERM)) == chain["round0_perm_sha256"], "round-0 perm"
    assert _sha(g.state(cb.STATE_TRADE_OF)) == chain["round0_trade_of_sha256"], "round-0 trade_of"
    assert _sha(g.state(cb.STATE_DEP)) == chain["round0_dep_sha256"], "round-0 dependency counts"
    _say(f"{name} seed {seed}: round-0 matching and dependency counts equal (n={n})")
    for r, digest in enumerate(want):
        g.global_trade(seed, r)
        got = g.download()
        assert _sha(got) == digest, f"{name} seed {seed} round {r}: adjacency differs from the oracle"
        _say(f"{name} seed {seed} round {r}: equal")
    st = g.stats()
    assert st["trades"] == n // 2
    g.close()


@pytest.mark.timeout(900)
def test_mid_workload_all_rounds_two_seeds():
    rec = _digests("mid")
    rp, col = graphgen.workload("mid")
    assert _sha(col) == rec["input_sha256"] and _sha(rp) == rec["rp_sha256"], "generator output differs"
    _say(f"mid n={len(rp) - 1} m={len(col) // 2}")
    for chain in rec["chains"]:
        _check_chain("mid", rp, col, chain)


@pytest.mark.timeout(1200)
def test_large_workload_all_rounds():
    rec = _digests("large")
    rp, col = graphgen.workload("large")
    assert _sha(col) == rec["input_sha256"] and _sha(rp) == rec["rp_sha256"], "generator output differs"
    _say(f"large n={len(rp) - 1} m={len(col) // 2}")
    for chain in rec["chains"]:
        _check_chain("large", rp, col, chain)


@pytest.mark.timeout(900)
def test_hubs_workload_bitmap_sets_at_full_id_range():
    rec = _digests("hubs")
    rp, col = graphgen.workload("hubs")
    assert _sha(col) == rec["input_sha256"] and _sha(rp) == rec["rp_sha256"], "generator output differs"
    deg = np.diff(rp)
    assert (deg >= 8192).sum() >= 4, "the workload should hold several nodes above the bitmap threshold"
    _say(f"hubs n={len(rp) - 1} m={len(col) // 2}, {(deg >= 8192).sum()} nodes of degree >= 8192")
    for chain in rec["chains"]:
        _check_chain("hubs", rp, col, chain)


@pytest.mark.parametrize("n", [0, 1])
def test_degenerate_sizes_end_to_end(orc, n):
    rp, col = np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
    g = cb.Graph(rp, col)
    for r in range(3):
        g.global_trade(5, r)
    got = g.download()
    assert got.size == 0
    st = g.stats()
    assert st["trades"] == 0
    g.close()


@pytest.mark.parametrize("seed", [2, 0xDEADBEEFCAFE])
def test_small_workload_other_chain_seeds(orc, seed):
    rp, col = graphgen.workload("small")
    g = cb.Graph(rp, col)
    ref = col
    for r in range(6):
        ref, _ = orc.global_trade(rp, ref, seed, r, "o1")
        g.global_trade(seed, r)
        assert np.array_equal(g.download(), ref), f"seed {seed} round {r}"
    g.close()
