#!/usr/bin/env python3
"""Write the oracle's SHA-256 digests of whole-workload chains.

The GPU parity tests at the full workload sizes compare the downloaded
adjacency after every round with these digests (equal digests of the whole
int32 array mean equal arrays, element by element). Every stored value comes
from the CPU oracle (IM-CB form, which equals the definition-literal form on
every graph the oracle tests cover) applied to graphs from `graphgen`; nothing
here reads the HIP library.

    python tests/golden/make_digests.py mid      # 20 rounds of n = 2^20
    python tests/golden/make_digests.py large    # 10 rounds of n = 2^24 (about 20 min)
    python tests/golden/make_digests.py hubs     # 4 rounds of the sparse 2^24 graph with hubs

Each run writes tests/golden/digests_<name>.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

# workload name -> (chain seeds, rounds per seed)
PLAN = {
    "mid": ((1, 20), (2, 3)),
    "large": ((1, 10),),
    "hubs": ((1, 4),),
}


def sha(a: np.ndarray) -> str:
    """SHA-256 of the array's bytes (native little-endian order)."""
    return hashlib.sha256(memoryview(np.ascontiguousarray(a)).cast("B")).hexdigest()


def main(name: str) -> int:
    t0 = time.time()
    rp, col = graphgen.workload(name)
    n, m = len(rp) - 1, len(col) // 2
    deg = np.diff(rp)
    print(f"[digests] {name}: n={n} m={m} max deg {int(deg.max())} generated in {time.time() - t0:.1f} s",
          flush=True)
    orc = oracle.default()
    rec = {"workload": name, "params": graphgen.WORKLOADS[name], "n": n, "m": m,
           "input_sha256": sha(col), "rp_sha256": sha(rp), "chains": []}
    for seed, rounds in PLAN[name]:
        order, trade_of = orc.matching(n, seed, 0)
        dep = orc.depcount(rp, col, trade_of, order)
        chain = {"seed": seed, "round0_perm_sha256": sha(order), "round0_trade_of_sha256": sha(trade_of),
                 "round0_dep_sha256": sha(dep), "col_sha256": []}
        del order, trade_of, dep
        x = col
        for r in range(rounds):
            t = time.time()
            x, st = orc.global_trade(rp, x, seed, r, "o2")
            if st["dep_mismatch"] != 0:
                raise RuntimeError(f"round {r}: dependency count mismatch")
            chain["col_sha256"].append(sha(x))
            print(f"[digests] {name} seed {seed} round {r}: {time.time() - t:.1f} s", flush=True)
        rec["chains"].append(chain)
    with open(os.path.join(HERE, f"digests_{name}.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
