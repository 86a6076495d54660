"""The C-ABI library loads and exports every function include/kn.h declares
(CPU only: no call touches a device)."""
from __future__ import annotations

import os
import re
import subprocess

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
