"""The C-ABI library loads and exports every entry point include/stml.h
declares (no compute call: runs without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_2001_06613_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    with open(os.path.join(ROOT, "include", "stml.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(stml_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _header_functions() == sorted(binding.SIGNATURES)


def test_library_exports_every_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libstml.so not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_workspace_sizing_and_option_checks():
    lib = binding.load()
    o = binding.default_opts(n_spatial=4, n_temporal=3)
    ext = (ctypes.c_int * 2)(256, 256)
    nb = lib.stml_workspace_bytes(ctypes.byref(o), 64, ext)
    # pyramid + Y + Z per level and seven solver vectors at the finest level
    finest = 64 * 2 * 256 * 256 * 4
    assert nb > 7 * finest
    assert lib.stml_workspace_bytes(ctypes.byref(o), 0, ext) == 0
    assert lib.stml_workspace_bytes(ctypes.byref(o), 300, ext) == 0
    bad = binding.default_opts(dim=4)
    assert lib.stml_workspace_bytes(ctypes.byref(bad), 8, ext) == 0
    ctx = ctypes.c_void_p()
    # workspace too small -> ENOMEM, before any device call
    rc = lib.stml_create(ctypes.byref(o), 64, ext, None,
                         ctypes.c_void_p(256), 16, ctypes.byref(ctx))
    assert rc == binding.STML_ENOMEM and not ctx.value


def test_default_opts_values():
    o = binding.default_opts()
    assert (o.dim, o.n_spatial, o.n_temporal, o.regulariser) == (2, 2, 2, 0)
    assert o.beta == 1e-5 and o.ls_max == 10 and o.parity_mode == 0
