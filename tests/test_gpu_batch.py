"""Batched chains on the GPU: many independent chains advance together (one
global trade of each per round, launched as one captured graph), and every
chain's adjacency must equal, byte for byte, the oracle's chain run alone with
that chain's seed and rounds. The autotuner must leave results unchanged."""
import numpy as np
import pytest

import graphgen
import paper_1804_08487_amd as cb

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-batch] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def _mixed_chains():
    gs = [
        graphgen.edge_list_to_csr(2, [(0, 1)]),
        (np.zeros(1, np.int64), np.zeros(0, np.int32)),            # n = 0
        (np.zeros(2, np.int64), np.zeros(0, np.int32)),            # n = 1
        graphgen.edge_list_to_csr(3, [(0, 1), (1, 2)]),
        graphgen.edge_list_to_csr(41, [(0, i) for i in range(1, 41)]),
        graphgen.edge_list_to_csr(24, [(i, j) for i in range(24) for j in range(i + 1, 24)]),
        graphgen.edge_list_to_csr(30, [(i, j) for i in range(10) for j in range(10, 30)]),
    ]
    for s in range(5):
        gs.append(graphgen.random_simple_graph(40 + 7 * s, 0.08 + 0.05 * s, 300 + s))
    gs.append(graphgen.pld_graph(3000, 2, 300, 2.0, 11))
    gs.append(graphgen.pld_graph(3001, 3, 400, 1.9, 12))
    gs.append(graphgen.pld_graph(1025, 2, 128, 2.2, 13))
    return gs


def _oracle_chain(orc, rp, col, seed, first, rounds, form="o1"):
    x = col
    for r in range(first, first + rounds):
        x, _ = orc.global_trade(rp, x, seed, r, form)
    return x


OPTS = {"default": {}, "all_workgroup": {cb.OPT_SMALL_MAX: 0},
        "all_global": {cb.OPT_SMALL_MAX: 0, cb.OPT_BIG_LDS_MAX: 0},
        "help_all": {cb.OPT_SMALL_MAX: 0, cb.OPT_HELP_MIN: 1, cb.OPT_HELP_CHUNK: 64},
        "giant20": {cb.OPT_GIANT_DEG: 20}}


@pytest.mark.parametrize("opt", list(OPTS))
def test_mixed_batch_each_chain_equals_oracle(orc, opt):
    gs = _mixed_chains()
    seeds = [7 + 13 * c for c in range(len(gs))]
    first = [c % 3 for c in range(len(gs))]
    _say(f"mixed batch of {len(gs)} chains, options {opt}")
    b = cb.Batch(gs, seeds, first)
    for o, v in OPTS[opt].items():
        b.set_option(o, v)
    b.run(2)
    b.run(1)          # a second captured graph of another length
    for c, (rp, col) in enumerate(gs):
        n, nnz, nxt = b.info(c)
        assert (n, nnz, nxt) == (len(rp) - 1, len(col), first[c] + 3)
        want = _oracle_chain(orc, rp, col, seeds[c], first[c], 3)
        assert np.array_equal(b.download_chain(c), want), f"chain {c}"
    b.close()


def test_batch_repeated_runs_replay_the_graph(orc):
    gs = [graphgen.pld_graph(500 + 37 * c, 2, 60, 2.0, 40 + c) for c in range(9)]
    seeds = [100 + c for c in range(9)]
    b = cb.Batch(gs, seeds)
    for _ in range(4):
        b.run(2)      # the same captured graph launched four times
    for c, (rp, col) in enumerate(gs):
        assert np.array_equal(b.download_chain(c), _oracle_chain(orc, rp, col, seeds[c], 0, 8)), f"chain {c}"
    b.close()


def test_batch_equals_single_chain_kernel(orc):
    gs = [graphgen.pld_graph(2000 + 300 * c, 2, 200, 2.1, 60 + c) for c in range(5)]
    seeds = [3 * c + 1 for c in range(5)]
    b = cb.Batch(gs, seeds)
    b.run(4)
    for c, (rp, col) in enumerate(gs):
        g = cb.Graph(rp, col)
        for r in range(4):
            g.global_trade(seeds[c], r)
        assert np.array_equal(b.download_chain(c), g.download()), f"chain {c}"
        g.close()
    b.close()


def test_autotune_keeps_results(orc):
    gs = [graphgen.pld_graph(4096 + 512 * c, 2, 600, 2.0, 80 + c) for c in range(12)]
    seeds = list(range(12))
    b = cb.Batch(gs, seeds)
    res = b.autotune(trial_rounds=1, use_cache=False)
    _say(f"tuned {res}")
    assert res["evaluated"] > 2 and res["ms_per_round"] <= res["default_ms_per_round"]
    assert b.info(0)[2] == 0           # the tuner's trial rounds are undone
    b.run(3)
    for c, (rp, col) in enumerate(gs):
        assert np.array_equal(b.download_chain(c), _oracle_chain(orc, rp, col, seeds[c], 0, 3, "o2")), f"chain {c}"
    again = b.autotune(trial_rounds=1, use_cache=True)
    assert again["cached"] == 1 and again["small_max"] == res["small_max"]
    b.close()


def test_batch_workload_sample_matches_oracle(orc):
    """A sample of the batched workload's chains (its generator and seeds),
    four rounds, every chain against the oracle."""
    spec = graphgen.batch_specs(64)
    gs = [graphgen.batch_chain(s) for s in spec]
    seeds = [s["chain_seed"] for s in spec]
    _say(f"batch sample: {len(gs)} chains, {sum(len(c) for _, c in gs) // 2} edges")
    b = cb.Batch(gs, seeds, validate=False)
    b.run(4)
    for c, (rp, col) in enumerate(gs):
        assert np.array_equal(b.download_chain(c), _oracle_chain(orc, rp, col, seeds[c], 0, 4, "o2")), f"chain {c}"
    b.close()


def test_batch_rejects_cross_chain_ids():
    gs = [graphgen.edge_list_to_csr(3, [(0, 1), (1, 2)]), (np.array([0, 1, 2]), np.array([1, 2]))]
    with pytest.raises(cb.CurveballError) as e:
        cb.Batch(gs, [1, 2])
    assert e.value.status == cb.CB_ENOTSIMPLE
