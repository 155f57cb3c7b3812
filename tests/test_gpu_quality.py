"""The chain-quality workload on the GPU: the uniform single-trade chain
(Simple Undirected Curveball) equals the oracle's step by step sequence byte
for byte, and the per-round count of disjoint neighbours that changed sides
(the swap fraction's numerator) equals the oracle's."""
import numpy as np
import pytest

import graphgen
import paper_1804_08487_amd as cb

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-quality] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


TIERS = {"default": {}, "all_workgroup": {cb.OPT_SMALL_MAX: 0},
         "all_global": {cb.OPT_SMALL_MAX: 0, cb.OPT_BIG_LDS_MAX: 0},
         "help_all": {cb.OPT_SMALL_MAX: 0, cb.OPT_HELP_MIN: 1}}


def _graphs():
    yield "pair", graphgen.edge_list_to_csr(2, [(0, 1)])
    yield "three", graphgen.edge_list_to_csr(3, [(0, 1), (1, 2)])
    yield "isolated", graphgen.edge_list_to_csr(9, [(0, 1), (2, 3), (3, 4)])
    yield "star", graphgen.edge_list_to_csr(41, [(0, i) for i in range(1, 41)])
    yield "er", graphgen.random_simple_graph(70, 0.15, 8)
    yield "pld", graphgen.pld_graph(2000, 5, 300, 2.0, 13)


@pytest.mark.parametrize("tier", list(TIERS))
@pytest.mark.parametrize("name,g", list(_graphs()), ids=[n for n, _ in _graphs()])
def test_single_trades_equal_oracle(orc, name, g, tier):
    rp, col = g
    n = len(rp) - 1
    _say(f"single trades {name} tier {tier}")
    gr = cb.Graph(rp, col)
    gr.set_option(cb.OPT_GIANT_DEG, 0)
    for o, v in TIERS[tier].items():
        gr.set_option(o, v)
    ref = col
    step = 0
    for chunk in (1, 7, max(n, 2) // 2, 3 * n):
        gr.single_trades(11, step, chunk)
        ref, st = orc.cbu(rp, ref, 11, step, chunk)
        step += chunk
        assert np.array_equal(gr.download(), ref), f"after step {step}"
        s = gr.stats()
        if n >= 2:
            assert s["small_trades"] + s["big_trades"] == chunk
    gr.close()


def test_single_then_global_trades(orc):
    rp, col = graphgen.pld_graph(1500, 3, 200, 2.1, 14)
    gr = cb.Graph(rp, col)
    gr.set_option(cb.OPT_GIANT_DEG, 0)
    ref = col
    for r in range(3):
        gr.global_trade(2, r)
        ref, _ = orc.global_trade(rp, ref, 2, r)
        gr.single_trades(5, 750 * r, 750)
        ref, _ = orc.cbu(rp, ref, 5, 750 * r, 750)
        assert np.array_equal(gr.download(), ref), f"round {r}"
    gr.close()


@pytest.mark.parametrize("tier", ["default", "all_workgroup", "all_global"])
def test_moved_count_equals_oracle(orc, tier):
    rp, col = graphgen.pld_graph(3000, 2, 300, 2.0, 11)
    gr = cb.Graph(rp, col)
    gr.set_option(cb.OPT_HELP_MIN, 0)        # no shared write phase: every trade counted
    gr.set_option(cb.OPT_GIANT_DEG, 20)
    for o, v in TIERS[tier].items():
        gr.set_option(o, v)
    ref = col
    for r in range(3):
        gr.global_trade(9, r)
        ref, st = orc.global_trade(rp, ref, 9, r)
        s = gr.stats()
        assert s["counted_trades"] == s["trades"]
        assert s["moved"] == st["moved"], f"round {r}"
    gr.set_option(cb.OPT_GIANT_DEG, 0)
    gr.single_trades(3, 0, 1500)
    _, st = orc.cbu(rp, ref, 3, 0, 1500)
    s = gr.stats()
    assert s["counted_trades"] == 1500 and s["moved"] == st["moved"]
    gr.close()
