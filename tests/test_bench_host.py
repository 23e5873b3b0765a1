"""Host-side logic of bench.py (CPU): the traffic lines it reads from the committed counter
summary, and the run-to-epsilon loop of the time-to-epsilon protocol."""
import hashlib
import os
import types

import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_measured_traffic_reads_and_checks_the_source(tmp_path, monkeypatch):
    bench = _bench()
    src = os.path.join(ROOT, "paper_2602_09527_amd", "csrc", "backproject.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    f = tmp_path / "traffic.txt"
    f.write_text("# header\n"
                 f"traffic: class=backproject_subset source=backproject.hip fetch_kib=100.0 fetch_factor=2.0 "
                 f"write_kib=50.0 write_factor=1.0 source_sha256={sha}\n"
                 "traffic: class=project_subset source=backproject.hip fetch_kib=1.0 fetch_factor=2.0 "
                 "write_kib=1.0 write_factor=1.0 source_sha256=0000\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    # HBM bytes = 2 x FETCH_SIZE + 1 x WRITE_SIZE, in KiB
    assert bench.measured_traffic("backproject_subset") == (2.0 * 100.0 + 50.0) * 1024.0
    assert bench.measured_traffic("project_subset") is None      # source changed since
    assert bench.measured_traffic("backproject_full") is None    # no line for it
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("backproject_subset") is None


def test_run_to_eps_counts_passes_to_each_threshold():
    bench = _bench()
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    xstar = torch.ones(4, dtype=torch.float64)
    ref = {"xstar": xstar, "n2": float((xstar * xstar).sum())}
    # squared relative error 0.5 x 10^-k after the k-th step: below 1e-3 from the 3rd pass, below
    # 1e-5 from the 5th, where the loop stops
    state = {"k": 0}

    def step():
        state["k"] += 1

    def current():
        return xstar * (1.0 + (0.5 * 10.0 ** (-state["k"])) ** 0.5)
    rec = bench.run_to_eps(fake_torch, step, current, ref, passes=10)
    assert rec["passes_to_1e-3"] == 3 and rec["passes_to_1e-5"] == 5 and rec["passes"] == 5
    assert abs(rec["final_sq_rel_err"] - 5e-6) < 1e-12
    state["k"] = 0
    rec = bench.run_to_eps(fake_torch, step, current, ref, passes=2)
    assert rec["passes_to_1e-3"] is None and rec["passes_to_1e-5"] is None and rec["passes"] == 2
