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


def test_struct_layouts_match_binding(tmp_path):
    """sizeof and field offsets of the ABI structs, compiled from the header
    with the host C compiler, equal those of the ctypes mirrors."""
    from paper_2606_28022_amd import binding as B
    structs = {"fx_options": B.fx_options, "fx_counts": B.fx_counts, "fx_result": B.fx_result,
               "fx_kernel_stat": B.fx_kernel_stat}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fmoxtb.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            parts = line.split()
            got[(parts[0], parts[1])] = int(parts[2])
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
