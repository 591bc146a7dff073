"""The C-ABI library loads and exports every function the header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ambddc.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ambddc_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_surface():
    from paper_1301_0191_amd._lib import EXPORTED
    assert sorted(EXPORTED) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_1301_0191_amd._lib import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("libambddc.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_refuses_missing_library(tmp_path):
    from paper_1301_0191_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved


def test_default_options_without_gpu():
    from paper_1301_0191_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libambddc.so not built")
    lib = _lib.load()
    opt = _lib.Options()
    lib.ambddc_default_options(ctypes.byref(opt))
    assert opt.tau == 10.0 and opt.nev_max == 10 and opt.lobpcg_block == 16
    assert opt.precision == 0
