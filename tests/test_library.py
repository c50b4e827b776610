"""The C-ABI library builds for gfx950, loads, and exports every symbol include/sko.h declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2503_16717_amd", "libsko.so")
HEADER = os.path.join(ROOT, "include", "sko.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sko_[a-z_]+)\s*\(", text)))


def test_header_declares_boundary():
    names = declared_functions()
    for want in ("sko_create", "sko_destroy", "sko_strerror", "sko_orth_block", "sko_orth_blocks",
                 "sko_gmres", "sko_gmres_batched"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsko.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sko_[a-z_]+)\b", out))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsko.so not built")
def test_library_is_gfx950_code_object():
    # the embedded offload bundle names its target triple
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsko.so not built")
def test_binding_strerror_without_gpu():
    from paper_2503_16717_amd import binding as B
    assert B.strerror(B.SKO_OK) == "success"
    assert "breakdown" in B.strerror(B.SKO_EBREAKDOWN)
    assert set(B.EXPORTED) == set(declared_functions())
