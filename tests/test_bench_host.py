"""Host-side pieces of bench.py: the committed rocprofv3 traffic record is
read back into the bench line (no GPU needed)."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _record(workload="large"):
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")) as f:
        return json.load(f)


def test_traffic_record_gives_the_trade_kernel_bytes():
    rec = _record()
    k_trade = bench.kernel_bytes(rec, "k_trade")
    assert k_trade is not None and k_trade > 0
    # the trade kernel is one of the kernels summed into the step
    assert rec["step_bytes"] >= k_trade
    assert abs(sum(rec["kernels"].values()) - rec["step_bytes"]) <= 1e-6 * rec["step_bytes"]
    assert bench.kernel_bytes(rec, "no_such_kernel") is None


def test_traffic_record_commands_run_committed_files():
    rec = _record()
    assert rec["commands"], "the record names the commands that made it"
    for cmd in rec["commands"]:
        assert cmd.startswith("rocprofv3 ") and "_work/" not in cmd
        # the profiled program comes right after "--" and is the committed bench
        assert cmd.split(" -- ", 1)[1].split()[:2] == ["python3", "bench.py"]


def test_stale_record_is_not_used(tmp_path, monkeypatch):
    rec = _record()
    rec["source_sha1"] = "0" * 40
    path = tmp_path / "traffic_large.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic_{workload}.json"))
    assert bench.measured_traffic("large") is None
