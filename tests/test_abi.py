"""The C-ABI library loads and exports every symbol that include/chem.h
declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chem.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chem_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2405_05974_amd import chem
    if not os.path.exists(chem.LIB_PATH):
        from paper_2405_05974_amd import build
        build.build()
    return chem.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("chem_mech_load", "chem_integrate", "chem_rates"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2405_05974_amd import chem
    names = declared_functions()
    assert set(names) == set(chem.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name


def test_null_handle_errors_without_device(lib):
    from paper_2405_05974_amd import chem
    assert lib.chem_set_option(None, chem.OPT_Q_MAX, 3.0) == chem.CHEM_ERR_ARG
    assert b"NULL" in lib.chem_last_error()
    assert lib.chem_integrate(None, 1, None, None, 1.0, 1.0, 1.0, 1.0, None) == chem.CHEM_ERR_ARG
    assert lib.chem_mech_load_str(None, ctypes.byref(ctypes.c_void_p())) == chem.CHEM_ERR_ARG
    assert lib.chem_mech_load(b"/nonexistent/file", ctypes.byref(ctypes.c_void_p())) == chem.CHEM_ERR_ARG
    lib.chem_mech_free(None)


def test_package_import_does_not_load_oracle():
    import importlib
    import sys
    for mod in list(sys.modules):
        if mod == "oracle" or mod.startswith("oracle."):
            del sys.modules[mod]
    import paper_2405_05974_amd.chem as chem
    importlib.reload(chem)
    assert "oracle" not in sys.modules
    src = open(os.path.join(ROOT, "paper_2405_05974_amd", "chem.py")).read()
    assert "oracle" not in src.replace("oracle.", "")   # the product path never names the oracle
