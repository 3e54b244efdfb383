"""Host-side checks of bench.py's bookkeeping (no GPU): the HBM traffic
figure is reported only for a measured launch shape and the kernel sources
the counters were taken on, and the refusal of more than one GPU."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def shape(chunk, k, wpc, persistent=1):
    return {"chunk": chunk, "waves_per_block": k, "waves_per_cu": wpc, "persistent": persistent}


def test_traffic_table_is_consistent(bench):
    t = bench.TRAFFIC
    assert t["fetch_scale"] > 0 and t["write_scale"] > 0
    for (chunk, k, wpc, persistent), (fetch, write) in t["kib"].items():
        assert chunk % 64 == 0 and k in (1, 2, 4, 8) and persistent in (0, 1)
        assert (wpc == 0) == (persistent == 0)
        assert fetch > 0 and write > 0


def test_traffic_only_for_measured_shapes_and_sources(bench, monkeypatch):
    t = bench.TRAFFIC
    (chunk, k, wpc, persistent), (fetch, write) = next(iter(t["kib"].items()))
    s = shape(chunk, k, wpc if persistent else 20, persistent)
    if bench.sources_sha1(t["sources"]) == t["sha1"]:
        got = bench.measured_traffic(s)
        assert got == pytest.approx(1024.0 * (fetch * t["fetch_scale"] + write * t["write_scale"]))
    # a shape nobody measured
    assert bench.measured_traffic(shape(64, 1, 7)) is None
    # sources that no longer hash to the recorded SHA-1
    monkeypatch.setitem(t, "sha1", "0" * 40)
    assert bench.measured_traffic(s) is None


def test_grid_launches_ignore_waves_per_cu(bench):
    t = bench.TRAFFIC
    grid = [key for key in t["kib"] if key[3] == 0]
    if not grid or bench.sources_sha1(t["sources"]) != t["sha1"]:
        pytest.skip("no measured one-workgroup-per-item shape for these sources")
    chunk, k, _, _ = grid[0]
    a = bench.measured_traffic(shape(chunk, k, 20, 0))
    b = bench.measured_traffic(shape(chunk, k, 32, 0))
    assert a is not None and a == b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
