"""Host-side parts of bench.py's contract that need no GPU: more than one GPU
is refused with a message, and the HBM-traffic figure is reported only for
the kernel sources it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_figure_tied_to_the_measured_sources(monkeypatch):
    import bench
    t = dict(bench.TRAFFIC)
    t["sources_sha1"] = bench.kernel_sources_sha1()
    monkeypatch.setattr(bench, "TRAFFIC", t)
    assert bench.measured_traffic(t["kernel"], t["launches_per_estimate"]) == t["bytes_per_launch"]
    # another kernel, another launch count or changed sources: no figure
    assert bench.measured_traffic(t["kernel"], t["launches_per_estimate"] + 1) is None
    assert bench.measured_traffic("large_kernel", t["launches_per_estimate"]) is None
    monkeypatch.setitem(t, "sources_sha1", "0" * 40)
    assert bench.measured_traffic(t["kernel"], t["launches_per_estimate"]) is None


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "k.hip"
    src.write_text("int f() {\n  return 1;  // one\n}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ("k.hip",))
    a = bench.kernel_sources_sha1()
    src.write_text("// a comment\nint f() {\n  return 1;  // uno\n}\n")
    assert bench.kernel_sources_sha1() == a
    src.write_text("int f() {\n  return 2;\n}\n")
    assert bench.kernel_sources_sha1() != a
