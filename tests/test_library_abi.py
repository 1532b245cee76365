"""CPU checks of the C-ABI library: it loads and exports every declared symbol.

No compute call is made (no GPU here); the header is parsed for the
declared entry points and each must be exported by libsph.so.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("sph_create", "sph_init", "sph_step", "sph_reduce", "sph_destroy", "sph_pool_admit",
              "sph_pool_step", "sph_pool_poll", "sph_bytes_required"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2512_09904_amd import sph
    if not os.path.exists(sph.LIB_PATH):
        pytest.fail("libsph.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(sph.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(sph.EXPORTS) == declared_symbols()


def test_error_strings_and_arg_checks_without_gpu():
    """Host-side validation answers before any device work."""
    from paper_2512_09904_amd import cases, sph
    L = sph.lib()
    assert L.sph_error_string(sph.SPH_ERR_BUDGET).decode().startswith("no free slot")
    c = cases.tank_c1()
    P = sph.params_struct(c.params)
    assert L.sph_bytes_required(ctypes.byref(P), c.nf, c.ns) > c.nf * 1000
    bad = sph.params_struct(c.params, h_over_dp=2.5)
    assert L.sph_bytes_required(ctypes.byref(bad), c.nf, c.ns) == 0
    h = ctypes.c_void_p()
    rc = L.sph_create(ctypes.byref(bad), None, None, ctypes.byref(h))
    assert rc == sph.SPH_ERR_ARG
    assert "h_over_dp" in L.sph_last_error().decode()
    huge = sph.params_struct(c.params, grid_hi=(10.0, 0.1, 0.1))
    assert L.sph_create(ctypes.byref(huge), None, None, ctypes.byref(h)) == sph.SPH_ERR_ARG


def test_an_allocator_is_required_without_gpu():
    """The library allocates device memory only through the caller's
    allocator: creating a solver or a pool without one is an argument error,
    answered before any HIP call."""
    from paper_2512_09904_amd import cases, sph
    L = sph.lib()
    c = cases.tank_c1()
    P = sph.params_struct(c.params)
    h = ctypes.c_void_p()
    assert L.sph_create(ctypes.byref(P), None, None, ctypes.byref(h)) == sph.SPH_ERR_ARG
    assert "allocator" in L.sph_last_error().decode()
    assert not h.value
    assert L.sph_pool_create(ctypes.c_size_t(1 << 30), 4, 0, None, None, ctypes.byref(h)) == sph.SPH_ERR_ARG
    assert not h.value
