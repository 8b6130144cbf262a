"""Parity at the benchmark's full size, in the launch configuration bench.py
times (pmc_compress + fused pmc_retrieve on the 512^3 float32 spectral field,
8 components, tau_i = 2^-3i; and the 256^3 float64 variant).

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


def run_case(shape, dtype, seed, n, samples):
    import torch
    from paper_2308_11759_amd import pmc
    say("full-size case %s %s seed %d" % (shape, np.dtype(dtype).name, seed))
    x = inputs.spectral_field(shape, seed=seed, dtype=dtype)
    taus = [2.0 ** (-3 * (i + 1)) for i in range(n)]
    ctx = pmc.Context(0)
    xd = torch.from_numpy(x).to("cuda:0")
    store = ctx.compress(xd, taus)
    nz, ny, nx = shape
    nbx, nby = nx // 4, ny // 4
    chunks_per_row = nbx // 16
    streams = [chunk_payloads(store.stream(i).cpu().numpy()) for i in range(n)]
    nchunks = len(streams[0])
    rng = np.random.default_rng(seed)
    picks = sorted(set(int(c) for c in rng.integers(0, nchunks, size=samples)) | {0, nchunks - 1})
    outs = [ctx.retrieve(store, k).cpu().numpy() for k in range(1, n + 1)]
    for c in picks:
        bx0 = 16 * (c % chunks_per_row)
        by = (c // chunks_per_row) % nby
        bz = c // (chunks_per_row * nby)
        sub = np.ascontiguousarray(x[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx0:4 * bx0 + 64])
        comps, meta = driver.compress(sub, taus)
        for i in range(n):
            want = chunk_payloads(comps[i])[0]
            assert np.array_equal(streams[i][c], want), (c, i)
            assert meta[i]["linf"] <= store.info[i]["linf"]
        for k in range(1, n + 1):
            got = outs[k - 1][4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx0:4 * bx0 + 64]
            assert np.array_equal(got, driver.reconstruct(comps, k, sub.shape, sub.dtype)), (c, k)
    # Eq. (1) and the stored measured errors, on the whole field
    for k in range(1, n + 1):
        out = torch.from_numpy(outs[k - 1]).to("cuda:0")
        err = float((xd.double() - out.double()).abs().max())
        assert err <= taus[k - 1]
        assert err == store.info[k - 1]["linf"]
    say("  %d sampled chunks bit-exact, Eq. (1) holds for k = 1..%d" % (len(picks), n))
    torch.cuda.synchronize()


def test_bulk_512_f32():
    run_case((512, 512, 512), np.float32, 1, 8, samples=24)


def test_bulk_256_f64():
    run_case((256, 256, 256), np.float64, 2, 8, samples=24)
