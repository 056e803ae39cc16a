"""The CPU oracle, and the host side of the HIP library, built with
AddressSanitizer and UndefinedBehaviorSanitizer.  For the oracle:
a C driver (tests/sanitize/oracle_driver.c) calls every oracle entry point,
the skip-sampled Stage 1 and the error paths included, on small generated
graphs.  Any out-of-bounds access, use after free, leak, signed overflow or
misaligned access aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    cmd = [cc, "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "oi_oracle.c"),
           "-o", exe, "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "sanitizer" in (b.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "oracle driver ok" in r.stdout, (r.returncode, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]


def test_host_library_validation_under_asan_ubsan(tmp_path):
    """The library's host code (oi_api.cpp) rebuilt with AddressSanitizer and
    UndefinedBehaviorSanitizer on the host side only, linked with the built
    kernel object, and driven through its validation paths (malformed
    graphs, null handles, out-of-range arguments) by
    tests/sanitize/host_driver.c; needs no GPU."""
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    kobj = os.path.join(ROOT, "paper_1704_04794_amd", "csrc", "_build", "iicp_kernels.hip.o")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not available")
    if not os.path.exists(kobj):
        pytest.skip("kernel object not built (run __graft_entry__.build())")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1704_04794_amd", "csrc")]
    api = str(tmp_path / "oi_api.o")
    drv = str(tmp_path / "host_driver.o")
    exe = str(tmp_path / "host_san")
    steps = [
        [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *inc,
         "-c", os.path.join(ROOT, "paper_1704_04794_amd", "csrc", "oi_api.cpp"), "-o", api],
        [clang, "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", *inc,
         "-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.c"), "-o", drv],
        [clang + "++", "-fsanitize=address,undefined", drv, api, kobj, "-L/opt/rocm/lib", "-lamdhip64",
         "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
    ]
    for cmd in steps:
        b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert b.returncode == 0, (cmd[0], b.stderr[-2000:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "host driver ok" in r.stdout, (r.returncode, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
