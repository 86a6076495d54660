"""The C-ABI library loads and exports every function include/kn.h declares
(CPU only: no call touches a device)."""
from __future__ import annotations

import os
import re
import subprocess
import sys

import pytest

from paper_2206_10885_amd import kn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kn.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared()
    for n in ("kn_scene_create", "kn_render", "kn_serve_submit", "kn_serve_poll"):
        assert n in names
    assert sorted(kn.EXPORTS) == names, "binding and header disagree"


@pytest.mark.skipif(not os.path.exists(kn.LIB_PATH), reason="libkn.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", kn.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    L = kn.lib()
    for n in declared():
        assert getattr(L, n) is not None
    assert L.kn_last_error() == b""


@pytest.mark.skipif(not os.path.exists(kn.LIB_PATH), reason="libkn.so not built")
def test_null_arguments_are_rejected_without_a_device():
    L = kn.lib()
    assert L.kn_ctx_create(0, 0, None) == -1
    assert b"out" in L.kn_last_error()
    assert L.kn_ctx_destroy(None) == -1
    assert L.kn_render(None, 0, None, None, None) == -1


_MAPS_PROBE = r"""
import ctypes, sys
sys.path.insert(0, {root!r})
order = {order!r}
if order == "binding":
    from paper_2206_10885_amd import kn
    L = kn.lib()
else:
    L = ctypes.CDLL({lib!r})
    L.kn_last_error.restype = ctypes.c_char_p
    import torch  # noqa: F401
paths = set()
for line in open("/proc/self/maps"):
    parts = line.split()
    if len(parts) >= 6 and parts[5].rsplit("/", 1)[-1].startswith("libamdhip64.so"):
        paths.add(parts[5])
h = ctypes.c_void_p()
st = L.kn_ctx_create(0, 0, ctypes.byref(h))
print(len(paths), st, L.kn_last_error().decode())
"""


@pytest.mark.skipif(not os.path.exists(kn.LIB_PATH), reason="libkn.so not built")
@pytest.mark.parametrize("order", ["binding", "library first"])
def test_one_hip_runtime_per_process(order):
    """Loading libkn.so before torch maps two HIP runtimes (torch's wheel ships
    its own under another file name): device pointers and streams of one are
    invalid in the other, which crashed such a process inside the library.
    The binding imports torch first, so the library binds to torch's runtime;
    a process that still has two is refused by kn_ctx_create before any HIP
    call.  CPU only: no device is touched."""
    code = _MAPS_PROBE.format(root=ROOT, order=order, lib=kn.LIB_PATH)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr
    n, st, msg = out.stdout.strip().split(" ", 2)
    if order == "binding":
        assert n == "1", out.stdout
        assert "HIP runtimes are loaded" not in msg
    else:
        assert n == "2", out.stdout
        assert int(st) == -5 and "2 HIP runtimes are loaded" in msg, out.stdout
