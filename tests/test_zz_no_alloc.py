"""The entry point that allocates nothing (global_trade_static): its result
equals the allocating path's (graph_upload + global_trade + graph_download)
byte for byte, on two calls in a row, the second with a smaller graph, and a
graph beyond its static scratch is rejected before any device work."""
import ctypes

import numpy as np
import pytest

import graphgen
import paper_1804_08487_amd as cb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def _allocating(rp, col, seed, rnd):
    g = cb.Graph(rp, col)
    g.global_trade(seed, rnd)
    out = g.download()
    g.close()
    return out


def test_static_entry_point_equals_allocating_path():
    import torch
    cases = [(graphgen.pld_graph(6000, 2, 500, 2.0, 71), 5, 3),
             (graphgen.pld_graph(1500, 2, 200, 2.1, 72), 9, 0),     # smaller, second
             (graphgen.edge_list_to_csr(41, [(0, i) for i in range(1, 41)]), 2, 1)]
    for (rp, col), seed, rnd in cases:
        print(f"[no-alloc] n={len(rp) - 1} nnz={len(col)} seed={seed} round={rnd}", flush=True)
        d = torch.from_numpy(col.copy()).to("cuda")
        torch.cuda.synchronize()
        cb.global_trade_static(rp, d.data_ptr(), seed, rnd)
        got = d.cpu().numpy()
        assert np.array_equal(got, _allocating(rp, col, seed, rnd))


def test_static_chain_of_rounds_equals_allocating_chain(orc):
    import torch
    rp, col = graphgen.workload("small")
    d = torch.from_numpy(col.copy()).to("cuda")
    want = col
    for r in range(4):
        cb.global_trade_static(rp, d.data_ptr(), 1, r)
        want, _ = orc.global_trade(rp, want, 1, r)
    assert np.array_equal(d.cpu().numpy(), want)


def test_static_rejects_graph_beyond_scratch():
    n = 1 << 22
    rp = np.zeros(n + 1, np.int64)
    st = cb.lib().global_trade_static(n, rp.ctypes.data, None, 1, 0, None)
    assert st == cb.CB_EINVAL
    assert "static array" in cb.lib().cb_last_error().decode()


def test_static_rejects_bad_arguments():
    rp = np.array([0, 1, 2], np.int64)
    assert cb.lib().global_trade_static(2, rp.ctypes.data, None, 1, 0, None) == cb.CB_EINVAL
    assert cb.lib().global_trade_static(-1, rp.ctypes.data, None, 1, 0, None) == cb.CB_EINVAL
