"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (pmc_compress + fused pmc_retrieve): the 512^3 float32 spectral field,
8 components, tau_i = 2^-3i, and its 256^3 float64 variant; the largest
fields, 1024^3 float32 (12 components) and 768^3 float64 (10 components) with
tau_i = 2^-2i and white noise.

The oracle cannot compress 512^3 in seconds, but every chunk of 16 blocks
depends only on its own samples: the oracle compresses the 4 x 4 x 64 sub-box
of a sampled chunk on its own, and its single chunk must equal the GPU
stream's chunk word for word, for every component; the GPU's x~_k on that
sub-box must equal the oracle's.  Properties that hold at any size (Eq. (1)
for every k, measured error equal to the stored metadata) are checked on the
whole field on the device."""
import sys

import numpy as np
import pytest

from oracle import driver
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


def run_case(shape, dtype, seed, taus, samples, noise=0.0):
    import torch
    from paper_2308_11759_amd import pmc
    n = len(taus)
    say("full-size case %s %s seed %d, %d components" % (shape, np.dtype(dtype).name, seed, n))
    x = inputs.spectral_field(shape, seed=seed, dtype=dtype, noise_rel=noise)
    say("  field generated")
    ctx = pmc.Context(0)
    xd = torch.from_numpy(x).to("cuda:0")
    store = ctx.compress(xd, taus)
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
        comps, meta = driver.compress(sub, taus)
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
            assert np.array_equal(got, driver.reconstruct(comps, k, sub.shape, sub.dtype)), (c, k)
        # Eq. (1) and the stored measured error, on the whole field
        err = 0.0
        for z0 in range(0, nz, slab):
            d = (xd[z0:z0 + slab].double() - out[z0:z0 + slab].double()).abs().max()
            err = max(err, float(d))
        assert err <= taus[k - 1]
        assert err == store.info[k - 1]["linf"]
    say("  x~_k bit-exact on the sampled chunks, Eq. (1) holds for k = 1..%d" % n)
    torch.cuda.synchronize()


def test_bulk_512_f32():
    run_case((512, 512, 512), np.float32, 1, [2.0 ** (-3 * i) for i in range(1, 9)], samples=24)


def test_bulk_256_f64():
    run_case((256, 256, 256), np.float64, 2, [2.0 ** (-3 * i) for i in range(1, 9)], samples=24)


def test_largest_1024_f32():
    """4 GiB float32 field with white noise at 1e-4 of the range, 12
    components, tau_i = 2^-2i: the later components lie below the noise floor
    and are nearly incompressible."""
    run_case((1024, 1024, 1024), np.float32, 3, [2.0 ** (-2 * i) for i in range(1, 13)], samples=16, noise=1e-4)


def test_largest_768_f64():
    run_case((768, 768, 768), np.float64, 4, [2.0 ** (-2 * i) for i in range(1, 11)], samples=16, noise=1e-4)
