"""CPU checks of the C ABI boundary: the built library loads and exports every
function declared in include/gakco.h (no compute call needs a GPU here), and
the Python binding fails loudly when the library is missing."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gakco.h")
LIB = os.path.join(ROOT, "paper_1704_07468_amd", "libgakco.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(gakco_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1704_07468_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["gakco_gram", "gakco_rows", "gakco_gram_batch", "gakco_resident_create", "gakco_server_submit",
                 "gakco_extract", "gakco_mask_groups", "gakco_autotune"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_entry_points(lib):
    lib.gakco_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.gakco_version()
    lib.gakco_count_gmers.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    lens = (ctypes.c_int32 * 4)(10, 3, 0, 7)
    T = ctypes.c_int64()
    assert lib.gakco_count_gmers(lens, 4, 4, ctypes.byref(T)) == 0
    assert T.value == 7 + 0 + 0 + 4
    bad = (ctypes.c_int32 * 1)(-1)
    assert lib.gakco_count_gmers(bad, 1, 4, ctypes.byref(T)) == -1
    lib.gakco_last_error.restype = ctypes.c_char_p
    assert b"negative" in lib.gakco_last_error()
    lib.gakco_profile_phases.restype = ctypes.c_int32
    assert lib.gakco_profile_phases() >= 10


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1704_07468_amd import gakco
    monkeypatch.setattr(gakco, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gakco, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        gakco.lib()


def test_product_does_not_import_the_oracle():
    """The product path never imports, links or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1704_07468_amd")
    pat = re.compile(r"(^\s*(from|import)\s+oracle\b)|liboracle|gakco_oracle", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not pat.search(src), f
