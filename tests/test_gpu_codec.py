"""The second codec (prediction and uniform quantisation, codec 1) behind the
same multi-component driver (Sec. 6.2: any error-bounded compressor), on the
GPU through the C-ABI: selected with PMC_OPT_CODEC, recorded in every stream
header and in the store, and carried unchanged through retrieval, refinement,
region retrieval, serialisation and the server.

Every case compares the GPU streams byte for byte with the oracle's codec 1
(oracle/pmc_oracle.c) and every x~_k bit for bit with the oracle's Alg. 2,
and checks Eq. (1) for every component."""
import sys

import numpy as np
import pytest

from oracle import driver
from paper_2308_11759_amd import inputs

from helpers import oracle_run, store_blob

pytestmark = pytest.mark.gpu

PRED = driver.PredictionCodec()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2308_11759_amd import pmc
    c = pmc.Context(0)
    c.set_option(pmc.OPT_SYNC_CHECK, 1)
    c.set_option(pmc.OPT_CODEC, pmc.CODEC_PREDICTION)
    yield c
    torch.cuda.synchronize()


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def check(ctx, x, taus, label):
    say("codec 1 case %s shape=%s dtype=%s n=%d" % (label, x.shape, x.dtype, len(taus)))
    comps, meta, recon = oracle_run(x, taus, PRED)
    store = ctx.compress(to_dev(x), taus)
    assert store.codec == 1
    for i in range(len(taus)):
        got = store.stream(i).cpu().numpy()
        assert int(got[5]) == 1  # the header names the codec
        assert got.size == comps[i].size, (label, i, got.size, comps[i].size)
        if not np.array_equal(got, comps[i]):
            bad = np.nonzero(got != comps[i])[0]
            raise AssertionError("%s: stream %d differs at %d bytes, first %d" % (label, i, bad.size, bad[0]))
        assert store.info[i]["linf"] == meta[i]["linf"] <= taus[i], (label, i)
        for key in ("nempty", "ncoded", "nraw", "nesc", "nmiss"):
            assert store.info[i][key] == meta[i][key], (label, i, key)
    for k in range(1, len(taus) + 1):
        out = ctx.retrieve(store, k).cpu().numpy()
        assert np.array_equal(out, recon[k - 1]), (label, k)
    return store, comps, meta, recon


def test_small_blobs_f64(ctx):
    x = inputs.blobs_field(64, seed=0)
    r = float(x.max() - x.min())
    check(ctx, x, [r * 10.0 ** -(i + 1) for i in range(4)], "blobs64")


def test_ragged_spectral_f32(ctx):
    x = inputs.spectral_field((29, 22, 37), seed=11, dtype=np.float32)
    check(ctx, x, [2.0 ** (-3 * (i + 1)) for i in range(8)], "ragged32")


def test_ragged_spectral_f64(ctx):
    x = inputs.spectral_field((13, 41, 18), seed=12, dtype=np.float64)
    check(ctx, x, [2.0 * 4.0 ** -(i + 1) for i in range(6)], "ragged64")


def test_full_field_kernel_f32_and_f64(ctx):
    """Extents that are multiples of 4 take the encoder and decoder
    instantiations without edge paths."""
    for dt in (np.float32, np.float64):
        x = inputs.spectral_field((16, 24, 64), seed=13, dtype=dt)
        check(ctx, x, [2.0 ** (-3 * (i + 1)) for i in range(6)], "full-%s" % np.dtype(dt).name)


def test_tiny_zero_constant(ctx):
    for dt in (np.float32, np.float64):
        for shape in ((1, 1, 1), (3, 1, 5), (4, 4, 4)):
            x = inputs.spectral_field((4, 4, 6), seed=3, dtype=dt)[: shape[0], : shape[1], : shape[2]].copy()
            check(ctx, x, [0.5, 0.01, 1e-4], "tiny%s" % (shape,))
        check(ctx, np.zeros((8, 8, 12), dtype=dt), [1.0, 0.1], "zeros")
        check(ctx, np.full((8, 9, 12), 3.25, dtype=dt), [1.0, 0.1, 1e-3], "const")


def test_escalation_raw_and_lossless(ctx):
    """Tolerances near the float32 spacing force escalated bins, and one
    below every difference forces exact blocks (x~_n == x, Sec. 5.1.3)."""
    x = inputs.spectral_field((12, 16, 20), seed=5, dtype=np.float32)
    store, comps, meta, recon = check(ctx, x, [2.0 ** -8, 2.0 ** -24, 2.0 ** -150], "lossless")
    assert np.array_equal(recon[2], x)
    rng = np.random.default_rng(22)
    w = (rng.normal(size=(8, 8, 16)) * 10.0 ** rng.integers(-6, 3, size=(8, 8, 16))).astype(np.float32)
    store, comps, meta, recon = check(ctx, w, [10.0, 1e-3, 1e-6, 1e-9], "wide")
    assert sum(m["nesc"] for m in meta) + sum(m["nraw"] for m in meta) > 0


def test_retrieval_paths_agree(ctx):
    """Fused and literal Alg. 2, incremental refinement and region retrieval
    give the same x~_k with codec 1."""
    import torch
    from paper_2308_11759_amd import pmc
    x = inputs.spectral_field((21, 30, 45), seed=14, dtype=np.float32)
    taus = [2.0 ** (-3 * (i + 1)) for i in range(5)]
    store, comps, meta, recon = check(ctx, x, taus, "paths")
    ctx.set_option(pmc.OPT_FUSED_DECODE, 0)
    try:
        for k in range(1, 6):
            assert np.array_equal(ctx.retrieve(store, k).cpu().numpy(), recon[k - 1])
    finally:
        ctx.set_option(pmc.OPT_FUSED_DECODE, 1)
    xt = ctx.retrieve(store, 1)
    for k in range(2, 6):
        ctx.refine(store, k - 1, k, xt)
        assert np.array_equal(xt.cpu().numpy(), recon[k - 1])
    lo, hi = (5, 3, 2), (40, 27, 19)  # x, y, z
    box = ctx.retrieve_box(store, 4, lo, hi).cpu().numpy()
    assert np.array_equal(box, recon[3][lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])
    torch.cuda.synchronize()


def test_serialisation_and_oracle_streams(ctx):
    """A codec-1 store survives serialisation, and the GPU decodes streams
    the oracle wrote (a blob of oracle streams with codec 1 in its header)."""
    x = inputs.spectral_field((11, 19, 26), seed=15, dtype=np.float64)
    taus = [0.1, 0.01, 1e-3, 1e-4]
    store, comps, meta, recon = check(ctx, x, taus, "serial")
    again = ctx.deserialize(store.serialize())
    assert again.codec == 1
    for k in range(1, 5):
        assert np.array_equal(ctx.retrieve(again, k).cpu().numpy(), recon[k - 1])
    blob = store_blob(x.shape, x.dtype, comps, meta, codec=1)
    theirs = ctx.deserialize(blob)
    assert theirs.codec == 1
    for k in range(1, 5):
        assert np.array_equal(ctx.retrieve(theirs, k).cpu().numpy(), recon[k - 1])
    # a blob whose codec disagrees with its stream headers is refused
    from paper_2308_11759_amd import pmc
    with pytest.raises(pmc.PmcError) as ei:
        ctx.deserialize(store_blob(x.shape, x.dtype, comps, meta, codec=0))
    assert ei.value.status == pmc.E_CORRUPT


def test_served_mix_of_codecs():
    """The server decodes stores of both codecs in one step (one launch per
    element type and codec); every answer equals the oracle's x~_k."""
    import time

    import torch
    from paper_2308_11759_amd import pmc
    ctx = pmc.Context(0)
    ctx.set_option(pmc.OPT_SYNC_CHECK, 1)
    fields, stores, taus, refs = [], [], [], []
    for i, (shape, dt) in enumerate((((12, 14, 20), np.float32), ((17, 9, 23), np.float64),
                                     ((20, 20, 20), np.float32), ((9, 13, 8), np.float64))):
        x = inputs.spectral_field(shape, seed=600 + i, dtype=dt)
        r = float(x.max() - x.min())
        t = [r * 10.0 ** (-(j + 1) / 2.0) for j in range(5)]
        codec = i % 2 if i < 2 else 1 - i % 2
        ctx.set_option(pmc.OPT_CODEC, codec)
        st = ctx.compress(to_dev(x), t)
        assert st.codec == codec
        oc = PRED if codec == 1 else None
        comps, _ = driver.compress(x, t, oc)
        refs.append([driver.reconstruct(comps, k, x.shape, x.dtype, oc) for k in range(1, 6)])
        stores.append(st)
        taus.append(t)
    ctx.set_option(pmc.OPT_CODEC, 0)
    srv = pmc.Server(ctx, arena_bytes=64 << 20, max_batch=16)
    fids = [srv.add(s) for s in stores]
    rng = np.random.default_rng(5)
    tickets = []
    for q in range(80):
        f = int(rng.integers(0, 4))
        k = int(rng.integers(1, 6))
        tickets.append((srv.submit(fids[f], taus[f][k - 1]), f, k))
    t0 = time.time()
    for t, f, k in tickets:
        while True:
            done, st, _ = srv.poll(t)
            if done:
                break
            assert time.time() - t0 < 60.0
            time.sleep(0.0005)
        assert st == pmc.OK
        view, kk, _ = srv.result(t, f)
        assert kk == k
        assert np.array_equal(view.cpu().numpy(), refs[f][k - 1]), (f, k)
        srv.release(t)
    srv.close()
    torch.cuda.synchronize()


def test_tolerance_range_and_batches_refused(ctx):
    from paper_2308_11759_amd import pmc
    x = to_dev(np.ones((4, 4, 4), dtype=np.float64))
    with pytest.raises(pmc.PmcError) as ei:
        ctx.compress(x, [1e-300])
    assert ei.value.status == pmc.E_ARG
    with pytest.raises(pmc.PmcError) as ei:
        ctx.batch([((4, 4, 4), x.dtype)], [[0.1]])
    assert ei.value.status == pmc.E_ARG
