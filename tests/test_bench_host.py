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


def test_headline_certificate_maps_every_solution(monkeypatch):
    """c5_certify judges each distinct (nu^2, x) once and hands every timed solve its
    own bound, the same as the oracle's certificate called directly."""
    import importlib
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    from oracle import ridge
    from oracle.certify import StreamedCertificate
    rng = np.random.default_rng(4)
    n, d = 500, 24
    A = rng.standard_normal((n, d)).astype(np.float32) / np.sqrt(n)
    b = rng.standard_normal(n).astype(np.float32)
    A64, b64 = A.astype(np.float64), b.astype(np.float64)
    nus = [1e-2, 1e-4, 1e-2, 1e-4, 1e-2]
    xs = [ridge.solve_svd(A64, b64, nu) for nu in (1e-2, 1e-4)]
    far = rng.standard_normal(d)
    X = np.stack([xs[0], xs[1], xs[0], xs[1], far], axis=1)
    got, nuniq, k = bench.c5_certify(torch.from_numpy(A), torch.from_numpy(b), X, nus, rows=64,
                                     k=d)
    assert nuniq == 3 and k == d and len(got) == 5
    assert got[0] == got[2] and got[1] == got[3]
    C = StreamedCertificate(d, np.stack([xs[0], xs[1], far], axis=1), k=d)
    C.add(A, b)
    want = C.bounds(np.array([1e-2, 1e-4, 1e-2]))
    for g, w in zip((got[0], got[1], got[4]), want):
        np.testing.assert_allclose(g, w, rtol=1e-9, atol=1e-25)
    assert got[0][2] < 1e-12 and got[4][2] > 1e-3


def test_recorded_traffic_needs_the_current_kernel_source(tmp_path):
    """Counter summaries count only while the kernel sources are the ones they were
    taken with; every kernel section of a summary is read."""
    import hashlib
    import importlib
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summ = tmp_path / "t.txt"
    summ.write_text("# header: not data\nkernel_source_sha256: " + sha + "\nkernel: a<1>\n"
                    "traffic_bytes_per_launch: 10.5\nkernel: b<2, 3>\n"
                    "traffic_bytes_per_launch: 20\n")
    assert bench.recorded_traffic_all(str(summ), [str(src)]) == {"a<1>": 10.5, "b<2, 3>": 20.0}
    assert bench.recorded_traffic(str(summ), [str(src)]) == 10.5
    src.write_text("kernel source, changed\n")
    assert bench.recorded_traffic_all(str(summ), [str(src)]) is None


def test_every_error_field_gets_its_square_root():
    import importlib
    import math
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    line = {"rel_pred_err": {"0.01": 1e-8, "0.0001": 4e-10}, "modes": {
        "a": {"worst_rel_pred_err": 2.5e-9, "x": 1}, "b": {"rel_pred_err_bound": 1e-10}},
        "rel_pred_err_bound_sqrt": {"0.01": 1e-4}, "rel_pred_err_bound": {"0.01": 1e-8}}
    out = bench.with_error_roots(line)
    assert out["rel_pred_err_sqrt"] == {"0.01": 1e-4, "0.0001": 2e-5}
    assert math.isclose(out["modes"]["a"]["worst_rel_pred_err_sqrt"], 5e-5)
    assert math.isclose(out["modes"]["b"]["rel_pred_err_bound_sqrt"], 1e-5)
    assert out["rel_pred_err_bound_sqrt"] == {"0.01": 1e-4}    # kept as given
