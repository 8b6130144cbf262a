"""Pins of the oracle's second codec, prediction and uniform quantisation
(codec 1; the driver's compressor agnosticism, Sec. 6.2; prediction-based
compressors, Sec. 5).  Each check is a textbook definition (zigzag, the
Lorenzo predictor's eight-term formula, running sums by numpy), an exact
rational bound, a hand-derived block (tests/golden/prediction_codec_blocks.txt)
or an invariant of the driver (Eq. (1) of Sec. 4.3, monotone error, Alg. 2
reproducing the encoder's partial sums), never the oracle against itself."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import driver
from oracle import lib as orc
from paper_2308_11759_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bits_of(buf, nbits):
    return "".join(str((int(buf[i >> 3]) >> (i & 7)) & 1) for i in range(nbits))


def test_zigzag_definition_exhaustive_int16():
    for P in (32, 64):
        seen = set()
        for r in range(-(1 << 15), 1 << 15):
            z = orc.zigzag(r, P)
            assert z == (2 * r if r >= 0 else -2 * r - 1)
            assert orc.unzigzag(z, P) == r
            seen.add(z)
        assert seen == set(range(1 << 16))  # a bijection onto 0 .. 2^16 - 1


def test_zigzag_wide_values():
    rng = np.random.default_rng(31)
    for P, lim in ((32, 1 << 30), (64, 1 << 62)):
        for r in rng.integers(-lim, lim, size=2000):
            r = int(r)
            z = orc.zigzag(r, P)
            assert z == (2 * r if r >= 0 else -2 * r - 1)
            assert orc.unzigzag(z, P) == r


def _lorenzo_textbook(q):
    """The 3-D Lorenzo prediction error from its eight-term definition,
    samples outside the block taken as 0."""
    q = np.asarray(q, dtype=np.int64).reshape(4, 4, 4)  # [z][y][x]

    def at(z, y, x):
        return int(q[z, y, x]) if z >= 0 and y >= 0 and x >= 0 else 0

    r = np.zeros((4, 4, 4), dtype=object)
    for z in range(4):
        for y in range(4):
            for x in range(4):
                pred = (at(z, y, x - 1) + at(z, y - 1, x) + at(z - 1, y, x) - at(z, y - 1, x - 1)
                        - at(z - 1, y, x - 1) - at(z - 1, y - 1, x) + at(z - 1, y - 1, x - 1))
                r[z, y, x] = at(z, y, x) - pred
    return r.ravel()


def test_lorenzo_is_the_eight_term_predictor():
    rng = np.random.default_rng(32)
    for P, lim in ((32, 1 << 20), (64, 1 << 40)):
        for _ in range(200):
            q = rng.integers(-lim, lim, size=64)
            assert [int(v) for v in orc.lorenzo_fwd(q, 3, P)] == list(_lorenzo_textbook(q))


def test_lorenzo_inverse_is_running_sums():
    rng = np.random.default_rng(33)
    for _ in range(200):
        r = rng.integers(-(1 << 20), 1 << 20, size=64)
        want = np.cumsum(np.cumsum(np.cumsum(r.reshape(4, 4, 4), axis=0), axis=1), axis=2).ravel()
        assert np.array_equal(orc.lorenzo_inv(r, 3, 64), want)
        assert np.array_equal(orc.lorenzo_fwd(orc.lorenzo_inv(r, 3, 64), 3, 64), r)


def test_lorenzo_round_trip_wraps_in_p_bits():
    """Prediction errors of integers up to 2^(P-2) may leave the P-bit range;
    in wrapping arithmetic the running sums still return the integers."""
    rng = np.random.default_rng(34)
    for P, lim in ((32, 1 << 30), (64, 1 << 62)):
        for _ in range(200):
            q = rng.integers(-lim, lim, size=64)
            assert np.array_equal(orc.lorenzo_inv(orc.lorenzo_fwd(q, 3, P), 3, P), q)


def test_lorenzo_predicts_linear_functions_exactly():
    """q = a + b x + c y + d z: the prediction error vanishes wherever all
    three predecessors lie inside the block (x, y, z >= 1)."""
    rng = np.random.default_rng(35)
    z, y, x = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
    for _ in range(50):
        a, b, c, d = (int(v) for v in rng.integers(-1000, 1000, size=4))
        q = (a + b * x + c * y + d * z).ravel()
        r = orc.lorenzo_fwd(q, 3, 32).reshape(4, 4, 4)
        assert np.all(r[1:, 1:, 1:] == 0)
        assert r[0, 0, 0] == a


@pytest.mark.parametrize("case", ["ramp", "constant", "escalation"])
def test_prediction_codec_golden_blocks(case):
    g = {}
    for line in open(os.path.join(GOLDEN, "prediction_codec_blocks.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            name, rest = line.split(None, 1)
            g[name] = rest.split("->")[1].split()
    delta, pred, w, nbits, prefix = g[case]
    if case == "ramp":
        x = (np.arange(64) % 4) / 8.0
        xt, tau = np.zeros(64), 2.0 ** -4
    elif case == "constant":
        x, xt, tau = np.full(64, 0.25), np.zeros(64), 2.0 ** -4
    else:
        x, xt, tau = np.full(64, 1.0 + 2.0 ** -23), np.ones(64), 3 * 2.0 ** -25
    e = (x.astype(np.float32) - xt.astype(np.float32)).astype(np.float64)
    r = orc.encode_one_block_pq(e, x, xt, tau, np.float32, 3)
    assert r["mode"] == orc.CODED and r["delta"] == int(delta) and r["nbits"] == int(nbits)
    bits = _bits_of(r["buf"], r["nbits"])
    assert bits.startswith(prefix)
    assert bits[len("10") + int(delta) + 1] == pred
    assert int(bits[len("10") + int(delta) + 2:][:6][::-1], 2) == int(w)
    if case == "ramp":
        vals = bits[-128:]
        z = [int(vals[2 * l:2 * l + 2][::-1], 2) for l in range(64)]
        assert z == [2 if l in (1, 2, 3) else 0 for l in range(64)]
    elif case == "constant":
        assert bits[-192:] == "001" * 64
    else:
        assert bits[-128:] == "01" * 64
    assert r["err"] == 0.0 and np.array_equal(np.float32(xt) + np.float32(r["xi"]), np.float32(x))
    m, dec, used = orc.decode_one_block_pq(r["buf"], r["nbits"], tau, np.float32, 3)
    assert m == orc.CODED and used == r["nbits"] and np.array_equal(dec, r["xi"])


def test_quantisation_is_a_nearest_integer():
    """q is an integer next to e / h (exact rationals): |e / h - q| <= 1/2
    up to the one rounding of the product e * (1/h)."""
    rng = np.random.default_rng(36)
    for dt in (np.float32, np.float64):
        for _ in range(300):
            tau = float(rng.uniform(0.5, 2.0)) * 2.0 ** int(rng.integers(-30, 5))
            e = (rng.uniform(-1, 1, size=64) * tau * 2.0 ** int(rng.integers(0, 6))).astype(dt).astype(np.float64)
            x = e.copy()
            r = orc.encode_one_block_pq(e, x, np.zeros(64), tau, dt, 3)
            if r["mode"] != orc.CODED:
                continue
            h = Fraction(2.0 * tau) / 2 ** r["delta"]
            dec = r["xi"]
            for l in range(64):
                if dt == np.float64:  # the value is q * h rounded once; q is recovered exactly here
                    q = Fraction(dec[l]) / h
                    assert abs(Fraction(e[l]) / h - round(q)) <= Fraction(1, 2) + Fraction(1, 1 << 40)
            assert np.max(np.abs(dec - e)) <= tau


def _all_625():
    vals = [-2, -1, 0, 1, 2]
    for a in vals:
        for b in vals:
            for c in vals:
                for d in vals:
                    yield [a, b, c, d]


def test_brute_force_1d_blocks_prediction_codec():
    """All 625 blocks of {0, +-1, +-2} * 2^s with random previous
    approximations: the tolerance holds (or the block stays empty within it),
    the error never grows, and the decoder reproduces the encoder's
    component exactly."""
    rng = np.random.default_rng(37)
    for dt in (np.float32, np.float64):
        for s in (-3, 10):
            for tau_rel in (0.5, 1e-2, 1e-5):
                for pat in _all_625():
                    x = np.array(pat, dtype=np.float64) * 2.0 ** s
                    xt = x + rng.normal(size=4) * 2.0 ** s
                    x = x.astype(dt).astype(np.float64)
                    xt = xt.astype(dt).astype(np.float64)
                    e = (x.astype(dt) - xt.astype(dt)).astype(np.float64)
                    tau = tau_rel * 2.0 ** s
                    r = orc.encode_one_block_pq(e, x, xt, tau, dt, 1)
                    assert not r["miss"]
                    before = np.max(np.abs(x - xt))
                    after = np.max(np.abs(x - (xt.astype(dt) + r["xi"].astype(dt)).astype(np.float64)))
                    assert after <= tau or (r["mode"] == orc.EMPTY and before <= tau)
                    assert after <= before
                    m, dec, used = orc.decode_one_block_pq(r["buf"], r["nbits"], tau, dt, 1)
                    assert m == r["mode"] and used == r["nbits"]
                    assert np.array_equal(dec, r["xi"])


def test_driver_with_prediction_codec():
    """Alg. 1 / Alg. 2 with the second codec: Eq. (1) for every component,
    non-increasing error, Alg. 2 at k reproduces the encoder's x~_k, the
    codec's own accepted block errors equal the measured ones, and the
    stream header names codec 1."""
    cases = [(inputs.blobs_field(24, seed=0), 10.0, 4),
             (inputs.spectral_field((20, 24, 36), seed=1, dtype=np.float32), 8.0, 6),
             (inputs.spectral_field((9, 13, 30), seed=2, dtype=np.float64), 4.0, 6)]
    for x, ratio, n in cases:
        r = float(x.max() - x.min())
        taus = [r * ratio ** -(i + 1) for i in range(n)]
        comps, meta = driver.compress(x, taus, driver.PredictionCodec())
        prev = math.inf
        for i, m in enumerate(meta):
            assert m["linf"] <= taus[i] and m["linf"] <= prev and m["nmiss"] == 0
            assert m["encoder_linf"] == m["linf"]
            assert int(comps[i][5]) == 1 and int(comps[i][4]) == 1
            prev = m["linf"]
        for k in range(1, n + 1):
            xt = driver.reconstruct(comps, k, x.shape, x.dtype, driver.PredictionCodec())
            assert driver.measured_error(x, xt) == meta[k - 1]["linf"]


def test_prediction_codec_lossless_limit():
    """Sec. 5.1.3 with the second codec: a last tolerance below every float32
    difference forces x~_n == x."""
    x = inputs.spectral_field((12, 16, 20), seed=5, dtype=np.float32)
    taus = [2.0 ** -8, 2.0 ** -32, 2.0 ** -150]
    comps, meta = driver.compress(x, taus, driver.PredictionCodec())
    xt = driver.reconstruct(comps, 3, x.shape, x.dtype, driver.PredictionCodec())
    assert np.array_equal(xt, x)
