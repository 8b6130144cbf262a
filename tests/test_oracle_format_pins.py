"""Pins of the oracle's readings of the block format (format version 1).

The paper treats the compressor as a black box (Sec. 4) and fixes only the
driver; the codec's layout is this build's reading of a zfp-style
fixed-accuracy codec (one exponent per block, Sec. 4.4; blocks of 4^d values
that decode independently, Sec. 6.1; the acceptance rule that makes Eq. (1)
of Sec. 4.3 exact).  The kernels and the oracle were written together, so
byte parity between them cannot catch a misreading they share; these tests
pin each reading to something worked out by hand (tests/golden/, with the
derivation in each file) or to exact arithmetic:

  inverse transform order (z, y, x)    inverse_single_coefficient.txt
  minexp = floor(log2 tau)              exact rationals; tau = 3 * 2^-11 block
  chunk index in 32-bit words           two_chunk_stream.txt (17 blocks)
  coded before empty                    coded_within_tolerance.txt
  raw payload = residual bits           forced-raw block with x~ != 0
  edge replication of partial blocks    partial_block_stream.txt
"""
import math
import os
import struct
from fractions import Fraction

import numpy as np

from oracle import lib as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    g = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(None, 1)
            g.setdefault(k, []).append(v)
    return g


def _one(g, k):
    return g[k][0]


def _bits_of(buf, nbits):
    return "".join(str((int(buf[i >> 3]) >> (i & 7)) & 1) for i in range(nbits))


def _pack_bits(bits):
    """LSB-first bit string -> little-endian bytes (whole 32-bit words)."""
    nwords = (len(bits) + 31) // 32
    out = bytearray(4 * nwords)
    for i, b in enumerate(bits):
        if b == "1":
            out[i >> 3] |= 1 << (i & 7)
    return bytes(out)


def _header(g, tau):
    dims = [int(t) for t in _one(g, "dims").split()]
    h = struct.pack("<IHBB", int(_one(g, "magic"), 16), int(_one(g, "version")), int(_one(g, "dtype")),
                    int(_one(g, "d")))
    h += struct.pack("<QQQ", *dims)
    h += struct.pack("<d", tau)
    h += struct.pack("<iI", int(_one(g, "minexp")), int(_one(g, "chunk_blocks")))
    h += struct.pack("<QQ", int(_one(g, "nchunks")), int(_one(g, "payload_words")))
    return h


CONST_BLOCK = "1000000000101101000000000000000000000000000000000"  # constant_block.txt


# ------------------------------------------------------------ inverse order
def test_inverse_transform_single_coefficient_golden():
    g = _golden("inverse_single_coefficient.txt")
    P = int(_one(g, "P"))
    idx, c = (int(t) for t in _one(g, "coefficient").split())
    q = np.zeros(64, dtype=np.int64)
    q[idx] = c
    want_rows = [[int(t) for t in r.split()] for r in g["row"]]
    got = orc.inv_xform(q, 3, P).reshape(4, 4, 4)  # [lz][ly][lx]
    for lz in range(4):
        assert got[lz].tolist() == want_rows


def test_inverse_transform_3d_round_trip_bound():
    """Forward then inverse over random blocks: each 1-D inverse undoes its
    forward step to within 4 (the dropped parity bits, doubled back), and an
    error entering a later inverse pass is scaled by at most the row sum of
    |M^-1|, 15/4, where M is the 1/16 basis matrix.  The passes run z, y, x
    after x, y, z, so the round trip is off by at most about
    4 + 15/4 * (4 + 15/4 * 4) = 75.25 per value; the observed maximum is far
    lower."""
    rng = np.random.default_rng(22)
    Minv = np.linalg.inv(np.array([[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]]) / 16.0)
    row = float(np.max(np.sum(np.abs(Minv), axis=1)))
    assert row == 3.75
    bound = 4 + row * (4 + row * 4)
    worst = 0
    for P, lim in ((32, 1 << 28), (64, 1 << 60)):
        for _ in range(400):
            q = rng.integers(-lim, lim, size=64).astype(np.int64)
            back = orc.inv_xform(orc.fwd_xform(q, 3, P), 3, P)
            worst = max(worst, int(np.max(np.abs(back - q))))
    assert worst <= bound


# ------------------------------------------------------------ minexp
def _floor_log2_exact(tau):
    """floor(log2 tau) of a positive double by exact rational comparison."""
    t = Fraction(tau)
    e = t.numerator.bit_length() - t.denominator.bit_length()
    while Fraction(2) ** e > t:
        e -= 1
    while Fraction(2) ** (e + 1) <= t:
        e += 1
    return e


def test_minexp_is_floor_log2_exact():
    rng = np.random.default_rng(23)
    taus = [3 * 2.0 ** -11, 0.1, 1e-5, 0.75, 1.5, 1.0, 2.0 ** -30, 5e-324, 2.5e-310, 1e-320, 1.7e308,
            math.nextafter(1.0, 0.0), math.nextafter(0.5, 1.0)]
    taus += [float(m) * 2.0 ** int(e) for m, e in zip(rng.uniform(1.0, 2.0, 500), rng.integers(-1070, 1020, 500))]
    taus += [float(v) for v in rng.uniform(0, 1, 200) * 2.0 ** -1040]  # subnormal
    for tau in taus:
        if tau > 0:
            assert orc.minexp(tau) == _floor_log2_exact(tau), tau


def test_block_at_tau_not_a_power_of_two():
    """tau = 3 * 2^-11 lies between 2^-10 and 2^-9: floor(log2 tau) = -10, the
    same minexp as tau = 2^-10, so the constant block of constant_block.txt
    codes to the same 49 bits with 19 planes (a ceiling would give 18)."""
    tau = 3 * 2.0 ** -11
    x = np.ones(64)
    r = orc.encode_one_block(x, x, np.zeros(64), tau, np.float32, 3)
    assert r["mode"] == orc.CODED and r["p"] == 19
    assert _bits_of(r["buf"], r["nbits"]) == CONST_BLOCK
    y, _ = orc.encode(np.ones((4, 4, 4), np.float32), np.ones((4, 4, 4), np.float32),
                      np.zeros((4, 4, 4), np.float32), tau)
    assert struct.unpack_from("<d", bytes(y), 32)[0] == tau
    assert struct.unpack_from("<i", bytes(y), 40)[0] == -10


# ------------------------------------------------------------ chunk index
def test_two_chunk_stream_golden():
    g = _golden("two_chunk_stream.txt")
    tau = 2.0 ** int(_one(g, "tau_log2"))
    nblk = [int(t) for t in _one(g, "chunk_blocks_bits").split()]
    cw = [int(t) for t in _one(g, "chunk_words").split()]
    payload = b""
    for c in range(2):
        bits = CONST_BLOCK * nblk[c]
        chunk = _pack_bits(bits)
        assert len(chunk) == 4 * cw[c]
        payload += chunk
    assert struct.unpack_from("<I", payload, 0)[0] == int(_one(g, "first_word"), 16)
    index = [int(t) for t in _one(g, "index").split()]
    assert index == [0, cw[0]]
    want = _header(g, tau) + struct.pack("<II", *index) + payload
    assert len(want) == int(_one(g, "total_bytes"))
    x = np.ones((4, 4, 68), dtype=np.float32)
    y, st = orc.encode(x, x, np.zeros_like(x), tau)
    assert bytes(y) == want
    assert np.all(orc.decode(y, x.shape, x.dtype) == 1.0)


# ------------------------------------------------------------ coded before empty
def test_coded_preferred_over_empty_golden():
    g = _golden("coded_within_tolerance.txt")
    x = np.full(64, float(_one(g, "x")))
    xt = np.full(64, float(_one(g, "xt")))
    tau = float(_one(g, "tau"))
    e = (x.astype(np.float32) - xt.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(x - xt)) <= tau  # already within tau before coding
    r = orc.encode_one_block(e, x, xt, tau, np.float32, 3)
    assert r["mode"] == orc.CODED and r["p"] == int(_one(g, "p"))
    assert _bits_of(r["buf"], r["nbits"]) == _one(g, "bits")
    assert np.all(r["xi"] == 0.25) and r["err"] == 0.0


# ------------------------------------------------------------ raw payload
def _wide_block(rng, dt):
    """64 values whose exponents spread over 40 binades (120 for float64):
    quantised on one block exponent, the smallest lose their low bits at
    every plane count, so a tolerance below every difference forces raw."""
    k = rng.integers(0, 41, size=64).astype(np.float64)
    m = rng.integers(0, 1 << 23, size=64)
    s = rng.choice([-1.0, 1.0], size=64)
    scale = 1.0 if dt == np.float32 else 3.0
    x = (s * (1.0 + m * 2.0 ** -23) * 2.0 ** (-scale * k)).astype(dt)
    xt = (x.astype(np.float64) * (1.0 + 2.0 ** -10)).astype(dt)  # x~ != 0, within a factor 2 of x
    return x, xt


def test_raw_block_stores_the_residual_bits():
    """A raw block's payload is the residual e = x - x~_{i-1} (computed in the
    field's type), not x: its 64 values follow the two header bits as IEEE
    words, and x~_{i-1} + e reproduces x exactly (Sterbenz: x~ is within a
    factor 2 of x, so e is exact)."""
    rng = np.random.default_rng(24)
    for dt, P, utype in ((np.float32, 32, np.uint32), (np.float64, 64, np.uint64)):
        for _ in range(5):
            x, xt = _wide_block(rng, dt)
            e = x - xt  # IEEE subtraction in the field's type (numpy)
            tau = 2.0 ** -200 if dt == np.float32 else 2.0 ** -1070
            r = orc.encode_one_block(e.astype(np.float64), x.astype(np.float64), xt.astype(np.float64), tau, dt, 3)
            assert r["mode"] == orc.RAW and not r["miss"]
            assert r["nbits"] == 2 + 64 * P
            bits = _bits_of(r["buf"], r["nbits"])
            assert bits[:2] == "11"
            words = [int(bits[2 + P * l: 2 + P * (l + 1)][::-1], 2) for l in range(64)]
            assert words == [int(w) for w in e.view(utype)]
            assert not np.array_equal(e, x)
            assert np.array_equal(xt + r["xi"].astype(dt), x)
            m, dec, used = orc.decode_one_block(r["buf"], r["nbits"], tau, dt, 3)
            assert m == orc.RAW and np.array_equal(dec, e.astype(np.float64))


# ------------------------------------------------------------ edge replication
def test_partial_block_stream_golden():
    g = _golden("partial_block_stream.txt")
    tau = 2.0 ** int(_one(g, "tau_log2"))
    assert _one(g, "block0") == CONST_BLOCK
    payload = _pack_bits(_one(g, "block0") + _one(g, "block1"))
    assert len(payload) == 4 * int(_one(g, "payload_words"))
    want = _header(g, tau) + struct.pack("<I", int(_one(g, "index"))) + payload
    assert len(want) == int(_one(g, "total_bytes"))
    x = np.ones((4, 4, 5), dtype=np.float32)
    x[:, :, 4] = 0.5
    y, st = orc.encode(x, x, np.zeros_like(x), tau)
    assert bytes(y) == want
    assert np.array_equal(orc.decode(y, x.shape, x.dtype), x)
