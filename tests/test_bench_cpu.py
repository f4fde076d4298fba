"""CPU checks of the benchmark's host-side pieces (no GPU): the oracle baseline
record (threaded run, one-thread run, host description) on small workloads of
each dimensionality, and the error summary."""
import numpy as np
import pytest

import workloads as wl


@pytest.mark.parametrize("name", ["heat1d_65536", "jacobi2d_8192", "star3d_512"])
def test_cpu_baseline_record(name, monkeypatch):
    import bench
    w = wl.config(name)
    # a small grid of the same dimensionality keeps this test quick
    small = tuple(min(n, 64) for n in w.dims)
    monkeypatch.setattr(w, "dims", small, raising=False)
    monkeypatch.setattr(w, "grid", lambda: wl.uniform(3, "grid", int(np.prod(small))).reshape(small), raising=False)
    rec, a0, steps, ref = bench.cpu_baseline(w, budget_s=0.05)
    assert rec["value"] > 0 and rec["cores"] >= 1 and rec["kind"] == "oracle"
    assert 1 <= steps <= 64 and ref.shape == small and a0.shape == small
    one = rec["one_thread"]
    assert one["value"] > 0 and one["parallel_speedup"] > 0
    host = rec["host"]
    assert isinstance(host["cpu_model"], str) and host["usable_cpus"] >= 1


def test_error_summary():
    import bench
    ref = np.array([1.0, -2.0, 4.0])
    e = bench._errors(ref + np.array([0.0, 1e-3, 0.0]), ref)
    assert abs(e["max_abs"] - 1e-3) < 1e-15
    assert abs(e["max_abs_rel"] - 1e-3 / 4.0) < 1e-15
    assert abs(e["rel_l2"] - 1e-3 / np.linalg.norm(ref)) < 1e-15
