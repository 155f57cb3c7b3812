"""The help-job ticket protocol of the trade kernel (shared write phases and
giant passes), modelled on the host with std::atomic and many threads that
yield at random points: every chunk of every generation is worked exactly
once with that generation's fields, and every close finishes."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_job_protocol_model(tmp_path):
    exe = str(tmp_path / "job_model")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe,
                    os.path.join(HERE, "job_model", "job_model.cpp")], check=True)
    r = subprocess.run([exe, "3", "12", "3000"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
