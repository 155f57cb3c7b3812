"""The help-job ticket protocol of the trade kernel (shared write phases and
giant passes), modelled on the host with std::atomic and many threads that
yield at random points: every chunk of every generation is worked exactly
once with that generation's fields, and every close finishes. Helpers take
one chunk per visit (workgroup workers) or runs of chunks that keep the
fields while the generation stays (wavefront workers)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("runs", [1, 8])
def test_job_protocol_model(tmp_path, runs):
    exe = str(tmp_path / "job_model")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe,
                    os.path.join(HERE, "job_model", "job_model.cpp")], check=True)
    r = subprocess.run([exe, "3", "12", "3000", str(runs)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
