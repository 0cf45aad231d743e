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


def test_binding_struct_layouts_match_header():
    """Sizes of the C structs as the binding lays them out (x86-64 SysV ABI)."""
    from paper_2509_08602_amd import ladmm
    assert ctypes.sizeof(ladmm._Group) == 24
    assert ctypes.sizeof(ladmm._Weights) == 32
    assert ctypes.sizeof(ladmm._Opts) == 56
    assert ctypes.sizeof(ladmm._Result) == 72
    assert ctypes.sizeof(ladmm._CaseDesc) == 88


def test_mask_packing():
    import numpy as np
    from paper_2509_08602_amd import ladmm
    from synth.cases import pack_bits
    rng = np.random.default_rng(0)
    m = rng.random((3, 150)) < 0.3
    assert np.array_equal(ladmm._mask_words(m, 150), pack_bits(m))
