"""The C-ABI library loads and exports every function include/tg.h declares
(no GPU calls), and the Python binding names them all."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tg.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(tg_[a-z_]+)\s*\(", src, flags=re.M)))


def _lib():
    from paper_2405_14866_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libtg.so not built")
    return _native


def test_header_declares_the_boundary():
    names = declared()
    for need in ("tg_project", "tg_bin_sort", "tg_render_fwd", "tg_render_bwd"):
        assert need in names


def test_library_exports_every_declared_symbol():
    N = _lib()
    lib = ctypes.CDLL(N.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    N = _lib()
    assert sorted(N.EXPORTS) == declared()
    for n in declared():
        assert callable(getattr(N, n, None)) or n == "tg_status_string", n


def test_status_strings():
    N = _lib()
    assert N.status_string(N.TG_ERR_CAPACITY) == "key capacity of the frame exceeded"
    assert N.status_string(N.TG_OK) == "ok"
    assert N.status_string(12345) == "unknown status"


def test_product_does_not_reach_the_oracle():
    """The package never imports, loads or links the oracle."""
    pkg = os.path.join(ROOT, "paper_2405_14866_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f
                assert "tgo_" not in txt and "libtgo" not in txt, f
