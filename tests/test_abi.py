"""The C-ABI library loads and exports every function include/lbm.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="lbm.h", prefix="lb_"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(" + prefix + r"[a-z_]+)\s*\(", txt))
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
    declared = declared_functions() + declared_functions("lbnet.h", "lbn_")
    for n in declared:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", b.LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lbn?_[a-z_]+)", out))
    assert set(declared) <= exported


def test_python_binding_names_match_header():
    from paper_0809_4958_amd import lbm, lbnet
    assert set(lbm.EXPORTS) == set(declared_functions())
    assert set(lbnet.EXPORTS) == set(declared_functions("lbnet.h", "lbn_"))


def test_network_header_constants_match_binding():
    from paper_0809_4958_amd import lbnet
    txt = open(os.path.join(ROOT, "include", "lbnet.h")).read()
    assert int(re.search(r"#define LBN_PARAM_COUNT (\d+)", txt).group(1)) == lbnet.PARAM_COUNT
    assert int(re.search(r"#define LBN_IMG (\d+)", txt).group(1)) == lbnet.IMG
    assert lbnet.PARAM_COUNT == lbnet.HIDDEN * lbnet.IN_CH * 9 + lbnet.HIDDEN + \
        lbnet.HIDDEN * lbnet.HIDDEN * 9 + lbnet.HIDDEN + lbnet.OUT_CH * lbnet.HIDDEN * 9 + lbnet.OUT_CH


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_0809_4958_amd import lbm
    with pytest.raises(ImportError):
        lbm._lib_saved = lbm._lib
        lbm._lib = None
        try:
            lbm.load(str(tmp_path / "missing.so"))
        finally:
            lbm._lib = lbm._lib_saved
