"""CPU checks of bench.py's contract that need no GPU: more than one GPU is refused
with a message, the workload list names every form, and the roofline and
oracle-rate arithmetic of the JSON line."""
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_workloads_cover_every_form():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for w in ("c2", "c3", "c4a", "c4b", "c5", "path", "dual", "refreshed", "sparse"):
        assert w in r.stdout


def test_roofline_and_oracle_rate_arithmetic(monkeypatch):
    # achieved = algorithmic bytes / average launch duration, frac = achieved / 8 TB/s;
    # the launch count and total time come from the library's event timings
    import importlib
    import torch
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)

    class FakeLib:
        def rs_profile_enable(self, on=True):
            pass

        def rs_profile_read(self):
            return 10, 0.5                    # 10 launches, 0.5 ms in all

    calls = []
    roof = bench.gradient_roofline(FakeLib(), lambda: calls.append(1), 268_697_600,
                                   "k_grad_partial", "test")
    assert calls == [1]
    assert roof["avg_launch_us"] == 50.0 and roof["launches"] == 10
    assert roof["achieved"] == round(268_697_600 / 50e-6 / 1e9, 1)
    assert roof["peak"] == 8000.0 and roof["unit"] == "GB/s" and roof["bound"] == "hbm"
    assert roof["frac"] == round(roof["achieved"] / 8000.0, 4)
    rate = bench.oracle_rate([lambda: time.sleep(0.01)], "sleep", budget_s=0.05)
    assert rate["kind"] == "oracle" and rate["unit"] == "solves/s" and rate["cores"] >= 1
    assert 0 < rate["value"] <= 100
