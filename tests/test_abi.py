"""The C-ABI library loads and exports every symbol declared in include/pmc.h
(no compute calls: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmc.h")
LIB = os.path.join(ROOT, "paper_2308_11759_amd", "libpmc.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_documented_calls():
    syms = declared_symbols()
    for name in ("pmc_compress", "pmc_retrieve", "pmc_refine", "pmc_select_k", "pmc_range",
                 "pmc_store_serialize", "pmc_store_deserialize"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_declared_symbol():
    from paper_2308_11759_amd import pmc
    assert sorted(pmc.SIGNATURES) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_calls():
    """Calls that need no device: size queries and argument rejection."""
    from paper_2308_11759_amd import pmc
    lib = pmc.load()
    f = pmc.Field(nx=64, ny=64, nz=64, dtype=pmc.F64)
    ws, cap = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.pmc_compress_sizes(ctypes.byref(f), 4, ctypes.byref(ws), ctypes.byref(cap)) == pmc.OK
    nchunks = (16 * 16 * 16 + 15) // 16
    assert cap.value >= 64 + 4 * nchunks + 4 * nchunks * ((16 * (2 + 64 * 64) + 31) // 32)
    assert ws.value >= 64 ** 3 * 8
    bad = pmc.Field(nx=0, ny=4, nz=4, dtype=pmc.F32)
    assert lib.pmc_compress_sizes(ctypes.byref(bad), 4, ctypes.byref(ws), ctypes.byref(cap)) == pmc.E_ARG
    assert lib.pmc_compress_sizes(ctypes.byref(f), 0, ctypes.byref(ws), ctypes.byref(cap)) == pmc.E_ARG
    assert lib.pmc_compress_sizes(ctypes.byref(f), 33, ctypes.byref(ws), ctypes.byref(cap)) == pmc.E_ARG
    assert lib.pmc_decode_ws_bytes() >= 4
    need = ctypes.c_size_t()
    assert lib.pmc_store_device_bytes(b"junk" * 20, 80, ctypes.byref(need)) == pmc.E_CORRUPT
