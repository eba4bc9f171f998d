"""The C-ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds a host-only copy of the library (no device code, sanitizers on the
host pass only) and a small driver (`abi_sanitize.cpp`) that calls every
entry point with bad arguments, the plans at extreme sizes, and the store
reader and streamer on missing, truncated and corrupted files.  Needs no GPU:
calls that would reach the device report an error instead.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
def test_host_code_under_sanitizers(tmp_path):
    lib = tmp_path / "liblod_san.so"
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_0811_2055_amd", "csrc", "*.hip")))
    # the device code is compiled as for the product (the library must link
    # whole); only the host pass is instrumented.  One process per source.
    base = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
            *SAN, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_0811_2055_amd", "csrc")]
    objs, procs = [], []
    for src in srcs:
        obj = tmp_path / (os.path.basename(src) + ".o")
        objs.append(str(obj))
        procs.append(subprocess.Popen([*base, "-c", src, "-o", str(obj)], stdout=subprocess.PIPE,
                                      stderr=subprocess.PIPE, text=True))
    for pr in procs:
        _, err = pr.communicate()
        assert pr.returncode == 0, err[-4000:]
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, *objs, "-o", str(lib)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = tmp_path / "abi_sanitize"
    cmd = [CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_sanitize.cpp"),
           "-L", str(tmp_path), "-llod_san", "-L", "/opt/rocm/lib", "-lamdhip64",
           f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    scratch = tmp_path / "files"
    scratch.mkdir()
    env = dict(os.environ)
    # the HIP runtime keeps allocations alive until exit: leak reports would be its own
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([str(exe), str(scratch)], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "all checks passed" in r.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]
    shutil.rmtree(scratch, ignore_errors=True)
