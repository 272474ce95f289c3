"""The C ABI: the library builds, loads, and exports every declared entry point.

CPU only: nothing here launches GPU work.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fresnel_hip.h")


def _ensure_built():
    from paper_2010_05978_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_2010_05978_amd import build
        build.build()
    return _binding.LIB_PATH


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fh_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("fh_create", "fh_destroy", "fh_set_stream", "fh_quad_radial", "fh_quad_starshade",
                 "fh_field_grid", "fh_field_points", "fh_field_grid_batch", "fh_field_grid_vjp",
                 "fh_starshade_vjp", "fh_autotune_grid"):
        assert must in names


def test_library_exports_every_declared_symbol():
    path = _ensure_built()
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fh_[a-z0-9_]+)", out))
    assert set(_declared()) <= exported


def test_binding_covers_every_declared_symbol():
    from paper_2010_05978_amd import _binding
    assert set(_declared()) == set(_binding.EXPORTED)
    for n in _declared():
        assert hasattr(_binding, n), n


def test_status_strings():
    _ensure_built()
    from paper_2010_05978_amd import _binding as b
    assert b.fh_status_string(b.FH_OK) == "FH_OK"
    assert b.fh_status_string(b.FH_ERR_ODD_GRID) == "FH_ERR_ODD_GRID"
    assert b.fh_status_string(b.FH_ERR_NONPOSITIVE_LZ) == "FH_ERR_NONPOSITIVE_LZ"


def test_library_is_gfx950_code_object():
    path = _ensure_built()
    data = open(path, "rb").read()
    assert b"gfx950" in data


def test_options_struct_layout():
    from paper_2010_05978_amd import fh_options
    # double, int32, double, int32, int32, int32 with natural alignment
    assert ctypes.sizeof(fh_options) == 40
