"""The C-ABI library loads and exports every entry point include/ladmm.h declares.

CPU only: no compute call is made (there may be no GPU here).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ladmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ladmm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ladmm_create_case", "ladmm_solve_batch", "ladmm_batch_create",
                     "ladmm_batch_run", "ladmm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2509_08602_amd import ladmm
    path = ladmm.LIB_PATH
    if not os.path.exists(path):
        pytest.fail("libladmm.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # every symbol the binding uses is declared in the header
    assert set(ladmm._SIGS) <= set(declared_functions())


STRUCTS = {  # C struct name -> binding class name
    "ladmm_group": "_Group", "ladmm_weights": "_Weights", "ladmm_opts": "_Opts",
    "ladmm_result": "_Result", "ladmm_case_desc": "_CaseDesc", "ladmm_pass2_desc": "_Pass2",
    "ladmm_server_opts": "_ServerOpts", "ladmm_server_stats": "_ServerStats",
}


def test_binding_struct_layouts_match_header(tmp_path):
    """Size and field offsets of every C struct, as gcc lays out the header,
    equal those of the binding's ctypes structures."""
    import shutil
    import subprocess
    from paper_2509_08602_amd import ladmm
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ladmm.h"', "int main(void) {"]
    for cname, pname in STRUCTS.items():
        cls = getattr(ladmm, pname)
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for cname, pname in STRUCTS.items():
        cls = getattr(ladmm, pname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_mask_packing():
    import numpy as np
    from paper_2509_08602_amd import ladmm
    from synth.cases import pack_bits
    rng = np.random.default_rng(0)
    m = rng.random((3, 150)) < 0.3
    assert np.array_equal(ladmm._mask_words(m, 150), pack_bits(m))
