"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (pmc_compress + fused pmc_retrieve): the 512^3 float32 spectral field,
8 components, tau_i = 2^-3i, and its 256^3 float64 variant; the largest
fields, 1024^3 float32 (12 components) and 768^3 float64 (10 components) with
tau_i = 2^-2i and white noise.

Whole-field parity (512^3 float32, 256^3 float64): the unchanged serial
oracle runs over every 4-plane z-slab of the field on a thread pool
(oracle/pool.py; Alg. 1 is block-local, and a 4-plane slab of these fields
is a whole number of chunks), and every chunk's words of every component and
every sample of every x~_k must equal the GPU's; the measured errors of the
whole field (the largest over the slabs) must equal the store's.

Sampled parity (1024^3, 768^3): every chunk of 16 blocks depends only on its
own samples, so the oracle compresses the 4 x 4 x 64 sub-box of a sampled
chunk on its own, and its single chunk must equal the GPU stream's chunk word
for word, for every component, and the GPU's x~_k on that sub-box the
oracle's.  Properties that hold at any size (Eq. (1) for every k, measured
error equal to the stored metadata) are checked on the whole field on the
device."""
import os
import sys
import time

import numpy as np
import pytest

from oracle import driver, pool
from paper_2308_11759_amd import inputs

from helpers import chunk_payloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def stream_chunk(stream, c):
    """Payload words of chunk c of a device stream, found through its chunk
    index: only the header, two index entries and the chunk's own words are
    copied to the host."""
    head = stream[:64].cpu().numpy()
    nchunks = int(head[48:56].view(np.uint64)[0])
    words = int(head[56:64].view(np.uint64)[0])
    idx = stream[64 + 4 * c:64 + 4 * min(c + 2, nchunks)].cpu().numpy().view(np.uint32)
    start = int(idx[0])
    end = int(idx[1]) if c + 1 < nchunks else words
    base = 64 + 4 * nchunks
    return stream[base + 4 * start:base + 4 * end].cpu().numpy().view(np.uint32)


def run_case(shape, dtype, seed, taus, samples, noise=0.0, codec=0):
    import torch
    from paper_2308_11759_amd import pmc
    n = len(taus)
    say("full-size case %s %s seed %d, %d components, codec %d" % (shape, np.dtype(dtype).name, seed, n, codec))
    x = inputs.spectral_field(shape, seed=seed, dtype=dtype, noise_rel=noise)
    say("  field generated")
    ctx = pmc.Context(0)
    ctx.set_option(pmc.OPT_CODEC, codec)
    oc = driver.PredictionCodec() if codec == 1 else None
    xd = torch.from_numpy(x).to("cuda:0")
    store = ctx.compress(xd, taus)
    assert store.codec == codec
    nz, ny, nx = shape
    nbx, nby = nx // 4, ny // 4
    assert nbx % 16 == 0  # each chunk is 16 blocks of one block row
    chunks_per_row = nbx // 16
    nchunks = chunks_per_row * nby * (nz // 4)
    rng = np.random.default_rng(seed)
    picks = sorted(set(int(c) for c in rng.integers(0, nchunks, size=samples)) | {0, nchunks - 1})
    boxes = {}
    for c in picks:
        bx0 = 16 * (c % chunks_per_row)
        by = (c // chunks_per_row) % nby
        bz = c // (chunks_per_row * nby)
        sl = (slice(4 * bz, 4 * bz + 4), slice(4 * by, 4 * by + 4), slice(4 * bx0, 4 * bx0 + 64))
        sub = np.ascontiguousarray(x[sl])
        comps, meta = driver.compress(sub, taus, oc)
        for i in range(n):
            want = chunk_payloads(comps[i])[0]
            assert np.array_equal(stream_chunk(store.stream(i), c), want), (c, i)
            assert meta[i]["linf"] <= store.info[i]["linf"]
        boxes[c] = (sl, sub, comps)
    say("  %d sampled chunks: streams bit-exact for every component" % len(picks))
    out = torch.empty_like(xd)
    slab = max(4, (1 << 27) // (ny * nx))  # float64 temporaries of at most 1 GiB
    for k in range(1, n + 1):
        ctx.retrieve(store, k, out=out)
        for c, (sl, sub, comps) in boxes.items():
            got = out[sl].cpu().numpy()
            assert np.array_equal(got, driver.reconstruct(comps, k, sub.shape, sub.dtype, oc)), (c, k)
        # Eq. (1) and the stored measured error, on the whole field
        err = 0.0
        for z0 in range(0, nz, slab):
            d = (xd[z0:z0 + slab].double() - out[z0:z0 + slab].double()).abs().max()
            err = max(err, float(d))
        assert err <= taus[k - 1]
        assert err == store.info[k - 1]["linf"]
    say("  x~_k bit-exact on the sampled chunks, Eq. (1) holds for k = 1..%d" % n)
    torch.cuda.synchronize()


def host_chunks(stream):
    """(chunk start offsets, payload words) of a stream copied to the host."""
    s = stream.cpu().numpy()
    nchunks = int(s[48:56].view(np.uint64)[0])
    words = int(s[56:64].view(np.uint64)[0])
    index = s[64:64 + 4 * nchunks].view(np.uint32).astype(np.int64)
    payload = s[64 + 4 * nchunks:64 + 4 * nchunks + 4 * words].view(np.uint32)
    return np.append(index, words), payload


def run_whole_field(shape, dtype, seed, taus):
    import torch
    from paper_2308_11759_amd import pmc
    n = len(taus)
    say("whole-field case %s %s seed %d, %d components" % (shape, np.dtype(dtype).name, seed, n))
    x = inputs.spectral_field(shape, seed=seed, dtype=dtype)
    ctx = pmc.Context(0)
    ctx.set_option(pmc.OPT_SYNC_CHECK, 1)
    xd = torch.from_numpy(x).to("cuda:0")
    store = ctx.compress(xd, taus)
    gpu = [host_chunks(store.stream(i)) for i in range(n)]
    outs = [ctx.retrieve(store, k) for k in range(1, n + 1)]  # x~_1..x~_n stay on the device
    torch.cuda.synchronize()
    nz, ny, nx = shape
    per_plane4 = ((nx + 3) // 4) * ((ny + 3) // 4)
    planes = pool.slab_planes(shape)
    assert planes == 4
    workers = min(16, os.cpu_count() or 1)
    say("  GPU store done; oracle on %d slabs of %d planes, %d threads" % (nz // planes, planes, workers))
    linf = [0.0] * n
    t0 = time.time()
    nslab = 0
    for z0, z1, comps, meta, recon in pool.map_slabs(x, taus, planes, workers):
        c0 = (z0 // 4) * per_plane4 // 16
        for i in range(n):
            index, payload = gpu[i]
            for j, want in enumerate(chunk_payloads(comps[i])):
                c = c0 + j
                assert np.array_equal(payload[index[c]:index[c + 1]], want), (z0, i, c)
            linf[i] = max(linf[i], meta[i]["linf"])
        for k in range(n):
            assert np.array_equal(outs[k][z0:z1].cpu().numpy(), recon[k]), (z0, k + 1)
        nslab += 1
        if nslab % 16 == 0:
            say("  %d slabs match (%.0f s)" % (nslab, time.time() - t0))
    for i in range(n):
        assert linf[i] == store.info[i]["linf"] <= taus[i]
        # Eq. (1) and the stored measured error, on the device as well
        err = float((xd.double() - outs[i].double()).abs().max())
        assert err == linf[i]
    say("  every chunk of every component and every x~_k sample equal the oracle's (%.0f s)" % (time.time() - t0))
    torch.cuda.synchronize()


def test_bulk_512_f32():
    run_whole_field((512, 512, 512), np.float32, 1, [2.0 ** (-3 * i) for i in range(1, 9)])


def test_bulk_256_f64():
    run_whole_field((256, 256, 256), np.float64, 2, [2.0 ** (-3 * i) for i in range(1, 9)])


def test_bulk_512_f32_prediction_codec():
    """The second codec at the bulk size in the benchmark's launch
    configuration: sampled chunks against the oracle's codec 1, Eq. (1) and
    the measured errors on the whole field."""
    run_case((512, 512, 512), np.float32, 1, [2.0 ** (-3 * i) for i in range(1, 9)], samples=24, codec=1)


def test_largest_1024_f32():
    """4 GiB float32 field with white noise at 1e-4 of the range, 12
    components, tau_i = 2^-2i: the later components lie below the noise floor
    and are nearly incompressible."""
    run_case((1024, 1024, 1024), np.float32, 3, [2.0 ** (-2 * i) for i in range(1, 13)], samples=16, noise=1e-4)


def test_largest_768_f64():
    run_case((768, 768, 768), np.float64, 4, [2.0 ** (-2 * i) for i in range(1, 11)], samples=16, noise=1e-4)
