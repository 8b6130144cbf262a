"""Shared test helpers (no codec arithmetic here)."""
import struct

import numpy as np

from oracle import driver


def align256(v):
    return (v + 255) & ~255


def store_blob(x_shape, dtype, comps, meta, codec=0):
    """Serialised-store blob (layout of pmc_store_serialize) around streams
    produced by the CPU oracle, so the GPU decoder can be checked on streams
    its own encoder did not write."""
    n = len(comps)
    nz, ny, nx = x_shape
    code = 1 if np.dtype(dtype) == np.float32 else 2
    head = struct.pack("<IIII", 0x53434D50, 1, n, codec) + struct.pack("<QQQii", nx, ny, nz, code, 0)
    for c, m in zip(comps, meta):
        head += struct.pack("<ddQQQQQQ", m["tau"], m["linf"], len(c), m.get("nempty", 0), m.get("ncoded", 0),
                            m.get("nraw", 0), m.get("nesc", 0), m.get("nmiss", 0))
    blob = bytearray(head + b"\0" * (align256(len(head)) - len(head)))
    region = bytearray()
    for c in comps:
        region += b"\0" * (align256(len(region)) - len(region))
        region += bytes(c)
    region += b"\0" * (align256(len(region)) - len(region))
    return bytes(blob + region)


def oracle_run(x, taus, codec=None):
    comps, meta = driver.compress(x, taus, codec)
    recon = [driver.reconstruct(comps, k, x.shape, x.dtype, codec) for k in range(1, len(comps) + 1)]
    return comps, meta, recon


def chunk_payloads(stream):
    """Split a stream (uint8 array) into per-chunk payload word arrays."""
    s = np.asarray(stream, dtype=np.uint8)
    nchunks = int(s[48:56].view(np.uint64)[0])
    words = int(s[56:64].view(np.uint64)[0])
    index = s[64:64 + 4 * nchunks].view(np.uint32).astype(np.int64)
    payload = s[64 + 4 * nchunks:].view(np.uint32)
    assert payload.size == words
    ends = list(index[1:]) + [words]
    return [payload[index[c]:ends[c]] for c in range(nchunks)]
