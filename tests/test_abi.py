"""The C-ABI library loads and exports every entry point that
include/fmoxtb.h declares (no compute calls: this runs without a GPU)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmoxtb.h")
LIB = os.path.join(ROOT, "paper_2606_28022_amd", "libfmoxtb.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fx_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("fx_params_load", "fx_ctx_create", "fx_set_system", "fx_build_lists", "fx_run",
              "fx_get_energies", "fx_get_gradient", "fx_eigh_batched"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fx_[a-z_]+)\b", out))
    assert set(declared()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_header():
    from paper_2606_28022_amd import binding
    assert sorted(binding.EXPORTS) == declared()
