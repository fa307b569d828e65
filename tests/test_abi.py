"""The C-ABI library loads and exports every entry point include/sdm.h declares
(no GPU needed: nothing is called except the version query)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(sdm_\w+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def libsdm():
    import paper_2101_06318_amd as sdm
    if not os.path.exists(sdm.LIB_PATH):
        from paper_2101_06318_amd import build
        build.build()
    return sdm.lib()


def test_every_declared_symbol_exported(libsdm):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(libsdm, n)]
    assert not missing, missing


def test_binding_covers_header(libsdm):
    import paper_2101_06318_amd as sdm
    assert _declared() == set(sdm.SIGNATURES), _declared() ^ set(sdm.SIGNATURES)


def test_abi_version(libsdm):
    assert libsdm.sdm_abi_version() == 3


def test_invalid_arguments_rejected_without_gpu(libsdm):
    # argument validation happens on the host before any device call
    h = ctypes.c_void_p()
    assert libsdm.sdm_create(ctypes.byref(h), 0, 1, 1) == -1
    assert b"n_sd_max" in libsdm.sdm_last_error()
    assert libsdm.sdm_create(None, 10, 1, 1) == -1
    assert libsdm.sdm_urand(None, None, 4, None, 0, None) == -1


def test_no_oracle_in_product_path():
    """The library and its binding never import or link the oracle."""
    pkg = os.path.join(ROOT, "paper_2101_06318_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "sdmo_" not in txt, f
