"""Host-side logic that needs no GPU: accuracy metrics of the learned mode
and the benchmark's profile bookkeeping."""
import os

import numpy as np

from paper_2006_03372_amd import learned

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_accuracy_metrics():
    exact = np.array([0, 2, 4, 10, 10])
    approx = np.array([0, 2, 5, 8, 10])
    a = learned.accuracy(exact, approx)
    assert a["exact_fraction"] == 3 / 5
    assert a["mae"] == (0 + 0 + 1 + 2 + 0) / 5
    # precision over vertices with exact core > 0: 1 - mean(|c - c^| / c)
    assert np.isclose(a["precision"], 1 - np.mean([0 / 2, 1 / 4, 2 / 10, 0 / 10]))
    assert learned.accuracy(np.zeros(3), np.ones(3))["precision"] == 1.0


def test_profile_traffic_follows_source_hash(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "p.md"
    prof.write_text("    traffic_bytes_per_launch: 123\n    source_sha256: " + bench.level_source_hash() + "\n")
    assert bench.profiled_traffic(str(prof)) == 123.0
    prof.write_text("    traffic_bytes_per_launch: 123\n    source_sha256: 00\n")
    assert bench.profiled_traffic(str(prof)) is None
    assert bench.profiled_traffic(str(tmp_path / "absent.md")) is None


def test_level_byte_counts():
    """Compulsory and modeled bytes of a pull launch on a small graph, by hand:
    path 0-1-2 plus an isolated vertex 3 (rows 0..2 non-isolated, 4 arcs)."""
    import bench
    from paper_2006_03372_amd import synth
    g = synth.from_edges(4, [0, 1], [1, 2])
    comp, model = bench.level_bytes(g, 2)
    rows, arcs, W = 3, 4, 2
    assert comp == rows * (4 + 8 + 8 * W) + arcs * 4 + rows * 8 * W
    assert model == rows * (4 + 8 + 8 * W) + arcs * (4 + 8 * W)


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
