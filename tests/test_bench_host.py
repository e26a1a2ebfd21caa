"""Host logic of bench.py (no GPU): the one-GPU contract, the staleness rule of the HBM
traffic summary, and the workload table."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    import bench as b
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_traffic_only_for_the_sources_it_was_taken_on(bench, tmp_path, monkeypatch):
    """The counter summary gives bytes per launch only while its recorded source digest
    matches the kernel sources; otherwise (or without the file) the bench reports null."""
    digest = bench.kernel_source_digest()
    f = tmp_path / "traffic.txt"
    f.write_text("# a comment: with a colon\nbwd_bytes_per_launch: 123456\n"
                 f"source_sha256: {digest}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("bwd") == 123456.0
    assert bench.measured_traffic("fwd") is None  # no such line
    f.write_text("bwd_bytes_per_launch: 123456\nsource_sha256: " + "0" * 64 + "\n")
    assert bench.measured_traffic("bwd") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("bwd") is None


def test_source_digest_covers_the_kernel_sources(bench):
    names = {os.path.basename(f) for f in bench.KERNEL_SOURCES}
    assert {"kernels.hip", "spdhg.hip", "geom.hpp"} <= names
    assert all(os.path.exists(f) for f in bench.KERNEL_SOURCES)
    d = bench.kernel_source_digest()
    assert len(d) == 64 and bench.kernel_source_digest() == d


def test_workload_table(bench):
    assert bench.WORKLOADS["mmr-tv21"]["m"] == 21  # the default (headline) workload
    for name, wl in bench.WORKLOADS.items():
        for key in ("m", "prior", "counts", "alpha", "alpha1", "prior_bpv", "label"):
            assert key in wl, (name, key)
        assert wl["prior"] in ("tv", "tgv", "dtv")
        assert wl["m"] >= 1 and wl["counts"] > 0 and wl["prior_bpv"] > 0
        assert wl.get("geometry") in (None, "span1", "scanner")
