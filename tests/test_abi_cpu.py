"""CPU-only checks of the boundary: the libraries load, every entry point
declared in the headers is exported, and argument validation that happens
before any device work behaves as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:hx_status|void|double|int|const char\s*\*)\s*"
                          r"(hx\w+)\s*\(", text, flags=re.M))


@pytest.fixture(scope="module")
def libhx():
    from paper_2503_10855_amd.build import LIB, build
    if not os.path.exists(LIB):
        build()
    return ctypes.CDLL(LIB)


def test_header_entry_points_are_exported(libhx):
    names = declared("include/hx.h")
    assert {"hx_pipeline_create", "hx_edge_detect", "hx_edge_detect_batched",
            "hx_serve_submit", "hx_serve_poll", "hx_autotune"} <= names
    for n in sorted(names):
        assert hasattr(libhx, n), n


def test_oracle_entry_points_are_exported(oracle_mod):
    names = declared("oracle/hxo.h")
    assert len(names) >= 8
    for n in sorted(names):
        assert hasattr(oracle_mod.lib(), n), n


def test_binding_names_match_header():
    from paper_2503_10855_amd import hx
    assert set(hx._SIGS) == declared("include/hx.h")


def test_status_strings(libhx):
    libhx.hx_status_str.restype = ctypes.c_char_p
    assert libhx.hx_status_str(0) == b"HX_OK"
    assert libhx.hx_status_str(6) == b"HX_E_PENDING"


@pytest.mark.parametrize("field,value", [("ksize", 4), ("ksize", 17), ("sigma", -1.0),
                                         ("thresh_frac", 1.5), ("max_images", -2)])
def test_create_rejects_bad_params_before_device(field, value):
    from paper_2503_10855_amd import hx
    p = hx.Params(5, 1.0, 0.1, 0, 0, 0, 0, 1 << 20, 16)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    lib = hx.raw()
    assert lib.hx_pipeline_create(ctypes.byref(p), 0, ctypes.byref(h)) == hx.HX_E_INVALID
    assert not h.value
    assert lib.hx_last_error()


def test_product_has_no_cpu_fallback():
    """The package never imports the oracle; the binding refuses to load
    without libhx.so."""
    pkg = os.path.join(ROOT, "paper_2503_10855_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in src and "from oracle" not in src, f
