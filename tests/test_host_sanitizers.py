"""The library's host code (api.hip, server.hip) built with g++ against a host-only stand-in
for the HIP runtime and stub kernel launchers (tests/hoststub), under the thread sanitizer
and under the address + undefined-behaviour sanitizers, and driven concurrently: a serving
engine with 12 sparse workers and 2 batched lanes under a small device budget (so worker
workspaces are released and regrown between requests), 4 submitting threads, and 3 threads
that create and destroy their own streams and solver handles and solve on them.  Streams
are worker threads, device memory is host memory and a free waits for every stream, as in
the HIP runtime; so a data race between threads, a host read of results before the stream
is synchronised, an access past an allocation, a use after free or a leak fails the run.
CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STUB = os.path.join(ROOT, "tests", "hoststub")
SOURCES = [os.path.join(ROOT, "paper_cs_0408029_amd", "csrc", f) for f in ("api.hip", "server.hip")]
STUBS = [os.path.join(STUB, f) for f in ("stub_runtime.cpp", "stub_kernels.cpp", "drive.cpp")]

pytestmark = pytest.mark.slow


@pytest.mark.parametrize("sanitize", ["thread", "address,undefined"])
def test_host_code_is_clean_under_sanitizers(tmp_path, sanitize):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path / "drive"
    cmd = [gxx, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-omit-frame-pointer", "-pthread",
           "-x", "c++", "-I", STUB, "-I", os.path.join(ROOT, "include"), *SOURCES, "-x", "none", *STUBS,
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    report = res.stdout + res.stderr
    assert "Sanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert res.returncode == 0, report[-4000:]
    assert "completed 144 requests, 0 failures" in res.stdout
