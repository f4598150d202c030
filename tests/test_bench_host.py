"""Host-side logic of bench.py: the one-GPU contract and the counter figures it reads from
profiles/ only while they belong to the current kernel and planner sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_values_need_matching_sources(tmp_path, monkeypatch):
    import bench
    (tmp_path / "profiles").mkdir()
    summ = tmp_path / "profiles" / "summary.md"
    summ.write_text("# counters\n\n- gemm1_traffic_bytes_per_launch: 1.5e+12\n- note: text\n"
                    "- sources sha256: `abc123`\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_digest", lambda: "abc123")
    assert bench.counter_values("summary.md") == {"gemm1_traffic_bytes_per_launch": 1.5e12}
    monkeypatch.setattr(bench, "sources_digest", lambda: "changed")
    assert bench.counter_values("summary.md") == {}
    assert bench.counter_values("missing.md") == {}


def test_sources_digest_covers_the_kernel_sources():
    import bench
    d = bench.sources_digest()
    assert len(d) == 64
    for name in bench.TRAFFIC_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_1908_07628_amd", "csrc", name))
