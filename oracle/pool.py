"""The serial oracle run over independent z-slabs of a field on a thread pool
(TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use it).

Alg. 1 is block-local: a block's residual, code, acceptance and partial sums
depend only on its own samples (blocks of 4^d values that decode
independently, Sec. 6.1).  So a field cut into z-slabs whose blocks form
whole chunks can be compressed slab by slab with the unchanged serial
driver, and the slabs' streams joined chunk by chunk give exactly the serial
run's stream: same chunk payloads, chunk offsets shifted by the payload words
of the slabs before.  The C oracle releases the GIL during its calls, so
slabs run in parallel on threads.

Nothing here computes any part of the method: it cuts, schedules and joins.
"""
import math
import os
import struct
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import driver

HEADER_BYTES = 64
CHUNK_BLOCKS = 16


def slab_planes(shape, min_planes=4):
    """Smallest z-thickness (a multiple of 4 planes, at least min_planes) whose
    blocks form whole chunks: 4 t planes hold t * nbx * nby blocks."""
    nz, ny, nx = shape
    per = ((nx + 3) // 4) * ((ny + 3) // 4)
    t = CHUNK_BLOCKS // math.gcd(per, CHUNK_BLOCKS)
    planes = 4 * t
    while planes < min_planes:
        planes += 4 * t
    return planes


def slabs(shape, planes):
    """(z0, z1) of each slab; the last one may be thinner (it ends the field)."""
    nz = shape[0]
    return [(z0, min(nz, z0 + planes)) for z0 in range(0, nz, planes)]


def run_slab(x, taus, z0, z1):
    """The serial oracle on x[z0:z1]: its components, metadata and every
    partial sum x~_1..x~_n (Alg. 2 continued one component at a time)."""
    xs = np.ascontiguousarray(x[z0:z1])
    comps, meta = driver.compress(xs, taus)
    recon = []
    xt = np.zeros_like(xs)
    for k in range(1, len(comps) + 1):
        xt = driver.refine(xt, comps, k - 1, k)
        recon.append(xt)
    return comps, meta, recon


def map_slabs(x, taus, planes=None, workers=None, fn=None):
    """Run the oracle on every slab on `workers` threads (default: all host
    cores); yields (z0, z1, comps, meta, recon) in slab order, or fn's result
    on those when fn is given (so a caller can keep only what it checks)."""
    planes = planes or slab_planes(x.shape)
    workers = workers or os.cpu_count() or 1
    todo = slabs(x.shape, planes)

    def job(zz):
        r = run_slab(x, taus, zz[0], zz[1])
        return fn(zz[0], zz[1], *r) if fn else (zz[0], zz[1]) + r

    with ThreadPoolExecutor(max_workers=workers) as ex:
        for r in ex.map(job, todo):
            yield r


def join_streams(shape, dtype, slab_streams):
    """One component's stream of the whole field from its slabs' streams (in
    z order): the header with the field's extents, chunk count and payload
    words; the chunk index with each slab's offsets shifted by the payload
    words before it; the payloads one after another."""
    nz, ny, nx = shape
    index, payload, words = [], [], 0
    tau_bits = minexp = None
    for s in slab_streams:
        s = np.asarray(s, dtype=np.uint8)
        nch = int(s[48:56].view(np.uint64)[0])
        w = int(s[56:64].view(np.uint64)[0])
        tb = bytes(s[32:40])
        me = bytes(s[40:44])
        assert tau_bits in (None, tb) and minexp in (None, me)
        tau_bits, minexp = tb, me
        index.append(s[64:64 + 4 * nch].view(np.uint32).astype(np.uint64) + words)
        payload.append(s[64 + 4 * nch:64 + 4 * nch + 4 * w])
        words += w
    first = np.asarray(slab_streams[0], dtype=np.uint8)
    nchunks = sum(len(i) for i in index)
    head = bytes(first[0:8]) + struct.pack("<QQQ", nx, ny, nz) + tau_bits + minexp + bytes(first[44:48])
    head += struct.pack("<QQ", nchunks, words)
    assert len(head) == HEADER_BYTES
    idx = np.concatenate(index)
    assert idx.max(initial=0) < 2 ** 32
    return np.concatenate([np.frombuffer(head, dtype=np.uint8), idx.astype(np.uint32).view(np.uint8)] + payload)


def compress(x, taus, planes=None, workers=None):
    """The whole-field result of the serial oracle (streams, metadata with the
    measured error over the whole field, partial sums), computed slab-parallel."""
    parts = list(map_slabs(x, taus, planes, workers))
    n = len(taus)
    comps = [join_streams(x.shape, x.dtype, [p[2][i] for p in parts]) for i in range(n)]
    meta = []
    for i in range(n):
        m = {"tau": float(taus[i])}
        for key in ("nempty", "ncoded", "nraw", "nesc", "nmiss"):
            m[key] = sum(int(p[3][i][key]) for p in parts)
        m["linf"] = max(p[3][i]["linf"] for p in parts)
        meta.append(m)
    recon = [np.concatenate([p[4][k] for p in parts], axis=0) for k in range(n)]
    return comps, meta, recon
