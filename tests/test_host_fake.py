"""The library's host runtime (kn_runtime.cpp) under the address and
undefined-behaviour sanitizers, on the CPU.

It is built with g++ against a host-only stand-in for the HIP runtime
(tests/host_fake/): device memory is host memory with a table of live
allocations that every kernel-launcher stub checks its buffers against, and
streams are synchronous.  The driver creates and packs scenes at several grid
and MLP sizes in every precision, checks argument validation, renders frames,
runs point queries, shared-scene worlds and the serving loop, and checks that a look-back overrun
of the cell scan (raised by the stub when KN_FAKE_SCAN_ERR is set) fails the
call, every request in flight, and poisons the context.  LeakSanitizer runs at
exit.  No GPU is used."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = os.path.join(ROOT, "tests", "host_fake")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("hostfake") / "kn_hostfake")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I" + FAKE, "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2206_10885_amd", "csrc"),
           os.path.join(ROOT, "paper_2206_10885_amd", "csrc", "kn_runtime.cpp"),
           os.path.join(FAKE, "fake_hip.cpp"), os.path.join(FAKE, "driver.cpp"), "-o", exe, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


@pytest.mark.parametrize("case", ["scenes", "validation", "render", "render_scan_err", "query_scan_err", "noalloc",
                                  "grid_eikonal", "world", "render_early", "serve_release",
                                  "serve", "serve_scan_err"])
def test_host_runtime_under_sanitizers(driver, case):
    env = dict(os.environ)
    env.pop("KN_FAKE_SCAN_ERR", None)
    if case.endswith("scan_err"):
        env["KN_FAKE_SCAN_ERR"] = "1"
    if case == "render_early":
        env["KN_FAKE_ROUND_CHUNKS"] = "1"
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    res = subprocess.run([driver, case], capture_output=True, text=True, env=env, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "FAIL" not in out and "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
