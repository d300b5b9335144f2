"""Host-side checks of bench.py's contract (no GPU): one GPU only, and the
measured-traffic figures are reported only for the kernel sources and grid
they were taken with."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_entries_name_existing_sources():
    for kernel, t in bench.TRAFFIC.items():
        for f in t["sources"]:
            assert os.path.exists(os.path.join(ROOT, "paper_1806_06623_amd", "csrc", f)), (kernel, f)
        assert len(bench._kernel_source_digest(t["sources"])) == 16


def test_traffic_is_withheld_off_its_grid_or_kernel():
    for kernel, t in bench.TRAFFIC.items():
        nr, nth, nphi = t["grid"]
        assert bench.measured_traffic(kernel, nr + 1, nth, nphi) is None
    assert bench.measured_traffic("no::such_kernel", 550, 128, 256) is None


def test_traffic_is_withheld_when_the_sources_change(monkeypatch):
    kernel = next(iter(bench.TRAFFIC))
    t = dict(bench.TRAFFIC[kernel], source_digest="0000000000000000")
    monkeypatch.setitem(bench.TRAFFIC, kernel, t)
    assert bench.measured_traffic(kernel, *t["grid"]) is None
