"""The request server on the GPU: requests that arrive while others run join
the running batch (continuous batching); every sample of every request must
equal, byte for byte, the oracle's chain (seed + sample, rounds 0..r-1) and
the same request served alone. Integer results: the tolerance is zero."""
import numpy as np
import pytest

import graphgen
import paper_1804_08487_amd as cb

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-serve] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def _requests():
    out = []
    for q in range(9):
        rp, col = graphgen.pld_graph(400 + 350 * q, 2, 80 + 20 * q, 2.0, 500 + q)
        out.append(dict(rp=rp, col=col, samples=1 + q % 4, rounds=2 + (q * 3) % 5, seed=1000 * (q + 1)))
    out.append(dict(rp=np.zeros(2, np.int64), col=np.zeros(0, np.int32), samples=2, rounds=3, seed=5))  # n = 1
    star = graphgen.edge_list_to_csr(41, [(0, i) for i in range(1, 41)])
    out.append(dict(rp=star[0], col=star[1], samples=3, rounds=0, seed=6))                          # r = 0
    return out


def _oracle(orc, req, sample):
    x = req["col"]
    for r in range(req["rounds"]):
        x, _ = orc.global_trade(req["rp"], x, req["seed"] + sample, r)
    return x


def _drain(srv, ids, limit=10000):
    for _ in range(limit):
        if all(srv.finished(i) for i in ids):
            return
        srv.step()
    raise AssertionError("server did not finish")


def test_requests_in_the_mix_equal_oracle_and_alone(orc):
    reqs = _requests()
    srv = cb.Server(8 << 30)
    ids = []
    seen_queue, max_active = 0, 0
    # staggered arrivals: three now, the rest while the first ones run
    for q, req in enumerate(reqs):
        ids.append(srv.submit(req["rp"], req["col"], req["samples"], req["rounds"], req["seed"]))
        if q >= 2:
            st = srv.step()
            seen_queue = max(seen_queue, st["queued"])
            max_active = max(max_active, st["active_chains"])
    _drain(srv, ids)
    _say(f"mix done, largest batch {max_active} chains")
    assert max_active > 4
    mix = {}
    for q, (rid, req) in enumerate(zip(ids, reqs)):
        for j in range(req["samples"]):
            got = srv.result(rid, j)
            assert np.array_equal(got, _oracle(orc, req, j)), f"request {q} sample {j}"
            mix[(q, j)] = got
        srv.release(rid)
    srv.close()
    # each request alone on a fresh server
    for q, req in enumerate(reqs):
        alone = cb.Server(8 << 30)
        rid = alone.submit(req["rp"], req["col"], req["samples"], req["rounds"], req["seed"])
        _drain(alone, [rid])
        for j in range(req["samples"]):
            assert np.array_equal(alone.result(rid, j), mix[(q, j)]), f"request {q} sample {j} alone"
        alone.close()


def test_budget_admits_one_request_at_a_time(orc):
    reqs = []
    for q in range(4):
        rp, col = graphgen.pld_graph(1500, 2, 100, 2.0, 600 + q)
        reqs.append(dict(rp=rp, col=col, samples=2, rounds=3, seed=77 * (q + 1)))
    probe = cb.Server(8 << 30)
    probe.submit(reqs[0]["rp"], reqs[0]["col"], 2, 3, 1)
    one = probe.step()["active_bytes"]
    probe.close()
    # half the budget holds one request's chains but not two
    srv = cb.Server(3 * one)
    ids = [srv.submit(r["rp"], r["col"], r["samples"], r["rounds"], r["seed"]) for r in reqs]
    st = srv.step()
    assert st["queued"] == 3 and st["active_chains"] == 2, st
    _drain(srv, ids)
    for rid, req in zip(ids, reqs):
        for j in range(req["samples"]):
            assert np.array_equal(srv.result(rid, j), _oracle(orc, req, j))
    srv.close()


def test_submissions_rejected():
    srv = cb.Server(16 << 20)
    rp, col = graphgen.pld_graph(200000, 5, 400, 2.0, 3)
    with pytest.raises(cb.CurveballError) as e:
        srv.submit(rp, col, 32, 5, 1)
    assert e.value.status == cb.CB_ENOMEM
    with pytest.raises(cb.CurveballError) as e:
        srv.submit(np.array([0, 1, 1, 2]), np.array([2, 1]), 1, 1, 1)     # asymmetric
    assert e.value.status == cb.CB_ENOTSIMPLE
    with pytest.raises(cb.CurveballError) as e:
        srv.submit(np.array([0, 2, 3, 4]), np.array([2, 1, 0, 0]), 1, 1, 1)   # unsorted row
    assert e.value.status == cb.CB_ENOTSIMPLE
    srv.close()
