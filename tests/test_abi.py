"""The C-ABI library loads and exports every function include/lbm.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(lb_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ["lb_init", "lb_set_boundary", "lb_step", "lb_couple_chain", "lb_read_fields"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0809_4958_amd import build as b
    if not os.path.exists(b.LIB):
        if not os.path.exists(b.HIPCC):
            pytest.skip("hipcc not available to build liblbm.so")
        b.build()
    lib = ctypes.CDLL(b.LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", b.LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lb_[a-z_]+)", out))
    assert set(declared_functions()) <= exported


def test_python_binding_names_match_header():
    from paper_0809_4958_amd import lbm
    assert set(lbm.EXPORTS) == set(declared_functions())


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_0809_4958_amd import lbm
    with pytest.raises(ImportError):
        lbm._lib_saved = lbm._lib
        lbm._lib = None
        try:
            lbm.load(str(tmp_path / "missing.so"))
        finally:
            lbm._lib = lbm._lib_saved
