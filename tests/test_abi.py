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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_blob_validation_uses_checked_arithmetic():
    """pmc_store_device_bytes validates a serialised store on the host (no
    device needed): a valid blob of oracle streams passes; sizes chosen so
    that an unchecked sum would wrap around 2^64 are rejected."""
    import struct

    import numpy as np

    from helpers import align256, oracle_run, store_blob
    from paper_2308_11759_amd import inputs, pmc
    lib = pmc.load()
    x = inputs.spectral_field((8, 12, 20), seed=9, dtype=np.float32)
    taus = [2.0 ** -3, 2.0 ** -7]
    comps, meta, _ = oracle_run(x, taus)
    blob = store_blob(x.shape, x.dtype, comps, meta)
    need = ctypes.c_size_t()

    def check(b):
        return lib.pmc_store_device_bytes(bytes(b), len(b), ctypes.byref(need))

    assert check(blob) == pmc.OK
    nblocks = 2 * 3 * 5
    region = align256(len(comps[0])) + len(comps[1])
    assert need.value == 2 * align256(4 * nblocks) + align256(region) + 512
    # a component size that makes the running region sum wrap
    bad = bytearray(blob)
    struct.pack_into("<Q", bad, 48 + 16, (1 << 64) - 64)
    assert check(bad) == pmc.E_CORRUPT
    # a payload word count whose byte size (4 w) wraps to the true one
    off = align256(48 + 64 * 2)
    words = struct.unpack_from("<Q", blob, off + 56)[0]
    bad = bytearray(blob)
    struct.pack_into("<Q", bad, off + 56, words + (1 << 62))
    assert check(bad) == pmc.E_CORRUPT
    # extents whose value count overflows 64 bits
    bad = bytearray(blob)
    struct.pack_into("<QQQ", bad, 16, 1 << 40, 1 << 40, 1 << 40)
    assert check(bad) == pmc.E_CORRUPT
    # tolerances not strictly decreasing
    bad = bytearray(blob)
    struct.pack_into("<d", bad, 48 + 64, taus[0])
    assert check(bad) == pmc.E_CORRUPT
    # a blob cut inside the last stream (its trailing padding is not needed)
    end = align256(48 + 64 * 2) + region
    assert check(blob[:end]) == pmc.OK
    assert check(blob[:end - 4]) == pmc.E_CORRUPT


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_field_size_limits():
    from paper_2308_11759_amd import pmc
    lib = pmc.load()
    ws, cap = ctypes.c_size_t(), ctypes.c_size_t()
    big = pmc.Field(nx=1 << 20, ny=1 << 20, nz=1, dtype=pmc.F32)  # 2^40 values
    assert lib.pmc_compress_sizes(ctypes.byref(big), 2, ctypes.byref(ws), ctypes.byref(cap)) == pmc.E_ARG
    wrap = pmc.Field(nx=1 << 40, ny=1 << 40, nz=1 << 40, dtype=pmc.F32)
    assert lib.pmc_compress_sizes(ctypes.byref(wrap), 2, ctypes.byref(ws), ctypes.byref(cap)) == pmc.E_ARG
    thin = pmc.Field(nx=1, ny=1, nz=1 << 35, dtype=pmc.F32)  # 2^33 blocks of one valid sample each
    assert lib.pmc_compress_sizes(ctypes.byref(thin), 2, ctypes.byref(ws), ctypes.byref(cap)) == pmc.E_ARG
    ok = pmc.Field(nx=1024, ny=1024, nz=1024, dtype=pmc.F32)
    assert lib.pmc_compress_sizes(ctypes.byref(ok), 12, ctypes.byref(ws), ctypes.byref(cap)) == pmc.OK
