"""Host-side parts of bench.py's contract that need no GPU: more than one GPU
is refused with a message, and the counter figures (HBM traffic, VALU busy)
are reported only for the kernel sources they were measured on."""
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


def test_counter_figures_tied_to_the_measured_sources(monkeypatch):
    import bench
    t = dict(bench.COUNTERS)
    t["sources_sha1"] = bench.kernel_sources_sha1()
    monkeypatch.setattr(bench, "COUNTERS", t)
    assert bench.measured_counters(t["kernel"], t["launches_per_estimate"]) is t
    # another kernel, another launch count or changed sources: no figure
    assert bench.measured_counters(t["kernel"], t["launches_per_estimate"] + 1) is None
    assert bench.measured_counters("large_kernel", t["launches_per_estimate"]) is None
    monkeypatch.setitem(t, "sources_sha1", "0" * 40)
    assert bench.measured_counters(t["kernel"], t["launches_per_estimate"]) is None


def test_source_hash_covers_only_the_tiny_sampler(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "k.hip"
    head = "int f() { return 1; }\n"
    src.write_text(head + bench.TINY_REGION_END + " { a(); }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ("k.hip",))
    a = bench.kernel_sources_sha1()
    src.write_text(head + bench.TINY_REGION_END + " { b(); }\n")
    assert bench.kernel_sources_sha1() == a
    src.write_text("int f() { return 2; }\n" + bench.TINY_REGION_END + " { a(); }\n")
    assert bench.kernel_sources_sha1() != a


def test_roofline_constants():
    import bench
    # 10 rounds x (2 wide products + 2 three-input xors); a coin adds a compare
    assert bench.PHILOX_OPS == 40 and bench.OPS_PER_COIN == 11
    assert abs(bench.ALU_PEAK_TOPS - 39.3216) < 1e-9


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
