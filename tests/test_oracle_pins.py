"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each check is a textbook
definition, a closed form, a hand-derived encoding (tests/golden/), an exact
rational computation, or an invariant the paper states (Eq. (1) of Sec. 4.3,
the left-to-right partial sums of Sec. 3 and Alg. 2, the lossless limit of
Sec. 5.1.3, the scalar expansion of Sec. 3).
"""
import math
import os
import struct
from fractions import Fraction

import numpy as np
import pytest

from oracle import lib as orc
from oracle import driver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# the basis matrix of the zfp paper's decorrelating transform (times 16)
M16 = np.array([[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]], dtype=np.float64)


# ---------------------------------------------------------------- negabinary
def test_negabinary_is_base_minus_two_exhaustive_int16():
    """u = (q + M) ^ M must be the base(-2) digit string of q."""
    for P in (32, 64):
        for q in range(-(1 << 15), 1 << 15):
            u = orc.to_negabinary(q, P)
            val = sum(((u >> k) & 1) * (-2) ** k for k in range(P))
            assert val == q
            assert orc.from_negabinary(u, P) == q


def test_negabinary_random_wide():
    rng = np.random.default_rng(3)
    for P, lo, hi in ((32, -(1 << 30), 1 << 30), (64, -(1 << 62), 1 << 62)):
        for q in rng.integers(lo, hi, size=2000):
            q = int(q)
            u = orc.to_negabinary(q, P)
            assert sum(((u >> k) & 1) * (-2) ** k for k in range(P)) == q
            assert orc.from_negabinary(u, P) == q


# ---------------------------------------------------------------- transform
def test_lift_constant_gives_single_dc():
    for c in (0, 1, -1, 12345, -(1 << 29), (1 << 29) - 1):
        for P in (32, 64):
            assert list(orc.fwd_lift4([c, c, c, c], P)) == [c, 0, 0, 0]


def test_lift_ramp_gives_dc_and_first_order_only():
    """A ramp a, a+s, a+2s, a+3s with even s maps to DC = a + 3s/2 and c1 = -s,
    which is the matrix row (5, 1, -1, -5)/16 applied exactly."""
    for a in (0, 7, -100, 1 << 20):
        for s in (2, 4, -6, 1000):
            v = [a, a + s, a + 2 * s, a + 3 * s]
            c = orc.fwd_lift4(v, 32)
            assert c[0] == a + 3 * s // 2
            assert c[1] == -s
            assert c[2] == 0 and c[3] == 0
            exact = M16 @ np.array(v, dtype=np.float64) / 16.0
            assert c[1] == exact[1]


def test_lift_matches_basis_matrix_within_rounding():
    """Each of the three halving steps drops at most 1/2; propagating those
    through the lifting steps bounds |lift(v) - M v| by 9/4 per output."""
    rng = np.random.default_rng(5)
    for P, lim in ((32, 1 << 29), (64, 1 << 61)):
        for _ in range(3000):
            v = [int(t) for t in rng.integers(-lim, lim, size=4)]
            c = orc.fwd_lift4(v, P)
            exact = [sum(Fraction(int(M16[r, t]), 16) * v[t] for t in range(4)) for r in range(4)]
            for r in range(4):
                assert abs(Fraction(int(c[r])) - exact[r]) <= Fraction(9, 4)


def test_inverse_lift_undoes_forward_up_to_dropped_parity():
    rng = np.random.default_rng(6)
    Minv = np.linalg.inv(M16 / 16.0)
    for _ in range(3000):
        v = [int(t) for t in rng.integers(-(1 << 29), 1 << 29, size=4)]
        c = orc.fwd_lift4(v, 32)
        back = orc.inv_lift4(c, 32)
        assert max(abs(int(back[t]) - v[t]) for t in range(4)) <= 4
        # the inverse applies M^-1 up to its own rounding
        approx = Minv @ np.array(c, dtype=np.float64)
        assert np.max(np.abs(approx - back)) <= 8.0


def test_3d_transform_constant_and_ramp():
    for P in (32, 64):
        q = np.full(64, 1 << 20, dtype=np.int64)
        c = orc.fwd_xform(q, 3, P)
        assert c[0] == 1 << 20 and np.count_nonzero(c) == 1
        # ramp along x with slope 4: only (0,0,0) and (1,0,0) survive
        lx = np.arange(64) % 4
        q = (1000 + 4 * lx).astype(np.int64)
        c = orc.fwd_xform(q, 3, P)
        nz = set(np.nonzero(c)[0].tolist())
        assert nz == {0, 1}
        assert c[1] == -4
        # ramp along z: only (0,0,0) and (0,0,1) = index 16
        lz = np.arange(64) // 16
        q = (-500 + 8 * lz).astype(np.int64)
        c = orc.fwd_xform(q, 3, P)
        assert set(np.nonzero(c)[0].tolist()) == {0, 16}
        assert c[16] == -8


def test_3d_transform_matches_kronecker_matrix():
    """The separable x, y, z passes apply M (x) M (x) M up to rounding."""
    rng = np.random.default_rng(8)
    M = M16 / 16.0
    K = np.kron(np.kron(M, M), M)  # acts on index lz*16 + ly*4 + lx
    for _ in range(200):
        q = rng.integers(-(1 << 28), 1 << 28, size=64).astype(np.int64)
        c = orc.fwd_xform(q, 3, 32)
        exact = K @ q.astype(np.float64)
        assert np.max(np.abs(c - exact)) <= 8.0


# ---------------------------------------------------------------- ordering
def test_permutation_is_sequency_order():
    for d in (1, 2, 3):
        p = orc.perm(d)
        B = 4 ** d
        assert sorted(p.tolist()) == list(range(B))
        keys = [sum((int(l) >> (2 * a)) & 3 for a in range(d)) for l in p]
        assert keys == sorted(keys)
        for r in range(1, B):
            if keys[r] == keys[r - 1]:
                assert p[r] > p[r - 1]
    p3 = orc.perm(3)
    assert p3[0] == 0 and sorted(p3[1:4].tolist()) == [1, 4, 16]
    assert p3[-1] == 63


# ---------------------------------------------------------------- quantiser
def test_value_exponent_is_frexp_convention():
    rng = np.random.default_rng(9)
    for dt, bias in ((np.float32, 127), (np.float64, 1023)):
        vals = list(rng.normal(size=200).astype(dt)) + [dt(0.0), dt(1.0), dt(-0.75)]
        tiny = np.finfo(dt).tiny
        vals += [dt(tiny), dt(tiny / 4), dt(np.finfo(dt).max)]
        for v in vals:
            v = float(v)
            want = 2 - bias if v == 0.0 else max(math.frexp(v)[1], 2 - bias)
            assert orc.value_expo(v, dt) == want


def test_quantize_is_exact_truncation():
    rng = np.random.default_rng(10)
    for dt, P in ((np.float32, 32), (np.float64, 64)):
        for _ in range(2000):
            v = float(dt(rng.normal() * 2.0 ** rng.integers(-20, 20)))
            emax = max(math.frexp(v)[1], -100) + int(rng.integers(0, 3))
            q = orc.quantize(v, emax, dt)
            exact = Fraction(v) * Fraction(2) ** (P - 2 - emax)
            assert q == int(exact)  # int() truncates toward zero
            assert abs(q) < 2 ** (P - 2)


def test_dequantize_rounds_once_to_nearest_even():
    rng = np.random.default_rng(11)
    for _ in range(3000):
        q = int(rng.integers(-(1 << 31), 1 << 31))
        emax = int(rng.integers(-140, 120))
        got = orc.dequantize(q, emax, np.float32)
        exact = float(Fraction(q) * Fraction(2) ** (emax - 30))  # exact in double
        assert got == float(np.float32(exact))
    for _ in range(3000):
        q = int(rng.integers(-(1 << 63), (1 << 63) - 1))
        emax = int(rng.choice([int(rng.integers(-1021, -1000)), int(rng.integers(-50, 50))]))
        got = orc.dequantize(q, emax, np.float64)
        exact = Fraction(q) * Fraction(2) ** (emax - 62)
        assert got == float(exact)  # Fraction -> float is correctly rounded


# ---------------------------------------------------------------- plane coder
def _read_plane_golden():
    cases = []
    for line in open(os.path.join(GOLDEN, "plane_coder.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        lhs, bits = line.split("->")
        parts = lhs.split()
        B, P, p = int(parts[1]), int(parts[2]), int(parts[3])
        u = [int(h, 16) for h in parts[4:4 + B]]
        cases.append((parts[0], B, P, p, u, bits.strip()))
    return cases


def _bits_of(buf, nbits):
    return "".join(str((int(buf[i >> 3]) >> (i & 7)) & 1) for i in range(nbits))


@pytest.mark.parametrize("case", _read_plane_golden(), ids=lambda c: c[0])
def test_plane_coder_golden(case):
    name, B, P, p, u, bits = case
    buf, nbits = orc.encode_planes(np.array(u, dtype=np.uint64), P, p)
    assert _bits_of(buf, nbits) == bits
    dec, used = orc.decode_planes(buf, nbits, B, P, p)
    assert used == nbits
    keep = ~((1 << (P - p)) - 1) & ((1 << 64) - 1)
    assert [int(t) for t in dec] == [t & keep for t in u]


def closed_form_plane_bits(u, B, P, p):
    """Bit count derived in closed form: per plane, n verbatim bits; then if
    n < B and m ones lie at positions >= n with the highest at h, m group bits,
    the h - n + 1 scanned bits minus an implied last bit, plus a final negative
    group bit when h < B - 1; with no such ones, one negative group bit."""
    n, total = 0, 0
    for k in range(P - 1, P - p - 1, -1):
        word = sum(((int(u[j]) >> k) & 1) << j for j in range(B))
        total += n
        if n < B:
            hi = word >> n
            if hi == 0:
                total += 1
            else:
                m = bin(hi).count("1")
                h = hi.bit_length() - 1 + n
                total += m + (h - n + 1) - (1 if h == B - 1 else 0) + (1 if h < B - 1 else 0)
                n = h + 1
    return total


def test_plane_coder_lossless_and_closed_form_count():
    rng = np.random.default_rng(12)
    for B in (4, 16, 64):
        for P in (32, 64):
            for trial in range(40):
                density = rng.uniform(0.0, 1.0)
                u = [int(rng.integers(0, 1 << 62)) if rng.random() < density else 0 for _ in range(B)]
                u = [t & ((1 << P) - 1) for t in u]
                if P == 64 and trial % 3 == 0:
                    u = [t | (1 << 63) if rng.random() < 0.3 else t for t in u]
                for p in (1, 5, P):
                    buf, nbits = orc.encode_planes(np.array(u, dtype=np.uint64), P, p)
                    assert nbits == closed_form_plane_bits(u, B, P, p)
                    dec, used = orc.decode_planes(buf, nbits, B, P, p)
                    assert used == nbits
                    keep = ((1 << P) - 1) & ~((1 << (P - p)) - 1)
                    assert [int(t) for t in dec] == [t & keep for t in u]


# ---------------------------------------------------------------- block codec
def test_empty_block_is_one_bit():
    z = np.zeros(64)
    r = orc.encode_one_block(z, z, z, 1e-3, np.float32, 3)
    assert r["nbits"] == 1 and r["mode"] == orc.EMPTY and r["buf"][0] == 0


def test_constant_block_golden():
    g = {}
    for line in open(os.path.join(GOLDEN, "constant_block.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(None, 1)
            g[k] = v
    tau = 2.0 ** int(g["tau_log2"])
    x = np.full(64, float(g["value"]))
    r = orc.encode_one_block(x, x, np.zeros(64), tau, np.float32, 3)
    assert r["mode"] == orc.CODED and r["p"] == int(g["p"])
    assert _bits_of(r["buf"], r["nbits"]) == g["bits"]
    assert np.all(r["xi"] == 1.0) and r["err"] == 0.0


def test_constant_stream_golden():
    g = {}
    for line in open(os.path.join(GOLDEN, "constant_stream.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(None, 1)
            g[k] = v
    tau = 2.0 ** int(g["tau_log2"])
    dims = [int(t) for t in g["dims"].split()]
    want = struct.pack("<IHBB", int(g["magic"], 16), int(g["version"]), int(g["dtype"]), int(g["d"]))
    want += struct.pack("<QQQ", *dims)
    want += struct.pack("<d", tau)
    want += struct.pack("<iI", int(g["minexp"]), int(g["chunk_blocks"]))
    want += struct.pack("<QQ", int(g["nchunks"]), int(g["payload_words"]))
    want += struct.pack("<I", int(g["index"]))
    want += bytes.fromhex(g["payload_hex"])
    assert len(want) == int(g["total_bytes"])
    x = np.ones((4, 4, 4), dtype=np.float32)
    y, st = orc.encode(x, x, np.zeros_like(x), tau)
    assert bytes(y) == want
    assert np.all(orc.decode(y, x.shape, x.dtype) == 1.0)


def _all_625():
    vals = [-2, -1, 0, 1, 2]
    for a in vals:
        for b in vals:
            for c in vals:
                for d in vals:
                    yield [a, b, c, d]


def test_brute_force_1d_blocks():
    """All 625 blocks with values {0, +-1, +-2} * 2^s, several tau and previous
    approximations: the tolerance holds, the error never grows, the encoder's
    component equals the decoder's, and the chosen plane count is the smallest
    accepted one (checked by trying every smaller count through the oracle's
    own block decoder)."""
    rng = np.random.default_rng(13)
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
                    r = orc.encode_one_block(e, x, xt, tau, dt, 1)
                    assert not r["miss"]
                    before = np.max(np.abs(x - xt))
                    after = np.max(np.abs(x - (xt.astype(dt) + r["xi"].astype(dt)).astype(np.float64)))
                    assert after <= tau or (r["mode"] == orc.EMPTY and before <= tau)
                    assert after <= before
                    m, dec, used = orc.decode_one_block(r["buf"], r["nbits"], tau, dt, 1)
                    assert m == r["mode"] and used == r["nbits"]
                    assert np.array_equal(dec, r["xi"])
                    if r["mode"] == orc.CODED:
                        nz, emax, u = orc.block_coeffs(e, dt, 1)
                        P = 32 if dt == np.float32 else 64
                        p0 = min(max(emax - orc.minexp(tau) + 4, 0), P)
                        for p in range(max(p0, 1), r["p"]):
                            ut = u & np.uint64(((1 << 64) - 1) & ~((1 << (P - p)) - 1))
                            v = orc.block_values(ut, emax, dt, 1)
                            ea = np.max(np.abs(x - (xt.astype(dt) + v.astype(dt)).astype(np.float64)))
                            assert not (ea <= tau and ea <= before)


def test_random_blocks_2d_3d_edge_content():
    """Seeded random, spike, constant, subnormal and large-exponent blocks."""
    rng = np.random.default_rng(14)
    for dt in (np.float32, np.float64):
        fi = np.finfo(dt)
        for d in (2, 3):
            B = 4 ** d
            kinds = ["normal", "spike", "const", "subnormal", "huge", "mixed"]
            for kind in kinds:
                for t in range(12):
                    if kind == "normal":
                        x = rng.normal(size=B)
                    elif kind == "spike":
                        x = np.zeros(B)
                        x[rng.integers(0, B)] = rng.normal() * 100
                    elif kind == "const":
                        x = np.full(B, rng.normal())
                    elif kind == "subnormal":
                        x = rng.normal(size=B) * float(fi.tiny) * 0.01
                    elif kind == "huge":
                        x = rng.uniform(-1.0, 1.0, size=B) * float(fi.max) * 0.5
                    else:
                        x = rng.normal(size=B) * 10.0 ** rng.integers(-30, 30, size=B)
                    x = x.astype(dt).astype(np.float64)
                    xt = np.zeros(B)
                    e = x.copy()
                    scale = max(float(np.max(np.abs(x))), float(fi.tiny))
                    for tau in (scale * 0.1, scale * 1e-4, scale * 2.0 ** -30):
                        if not tau > 0:
                            continue
                        r = orc.encode_one_block(e, x, xt, tau, dt, d)
                        assert not r["miss"], (kind, d, dt, tau)
                        m, dec, used = orc.decode_one_block(r["buf"], r["nbits"], tau, dt, d)
                        assert m == r["mode"] and used == r["nbits"]
                        assert np.array_equal(dec, r["xi"])


def test_raw_block_round_trip_exact():
    """Tolerance below every representable error forces RAW (or exact coded)."""
    rng = np.random.default_rng(15)
    x = rng.normal(size=64).astype(np.float32).astype(np.float64)
    r = orc.encode_one_block(x, x, np.zeros(64), 2.0 ** -200, np.float32, 3)
    assert r["err"] == 0.0
    assert np.array_equal(r["xi"], x)
    assert r["mode"] == orc.RAW and r["nbits"] == 2 + 64 * 32


# ---------------------------------------------------------------- driver
def _small_fields():
    from paper_2308_11759_amd import inputs
    x0 = inputs.blobs_field(32, seed=0)
    x1 = inputs.spectral_field((20, 24, 36), seed=1, dtype=np.float32)
    x2 = inputs.spectral_field((9, 13, 30), seed=2, dtype=np.float64)
    return [(x0, 10.0, 4), (x1, 2.0 ** 3, 8), (x2, 4.0, 6)]


def test_driver_bound_monotone_and_partial_sums():
    """Eq. (1): ||x - x~_i|| <= tau_i for every component; the error never
    grows; Alg. 2 at k reproduces the encoder's x~_k bit for bit; refining
    from k to k' equals rebuilding at k'."""
    for x, ratio, n in _small_fields():
        rng_ = float(x.max() - x.min())
        taus = [rng_ * ratio ** -(i + 1) for i in range(n)]
        comps, meta = driver.compress(x, taus)
        prev = math.inf
        for i, m in enumerate(meta):
            assert m["linf"] <= taus[i]
            assert m["linf"] <= prev
            assert m["nmiss"] == 0
            # the encoder's decode-for-verify and the decoder agree: the
            # largest block error the encoder accepted is the measured error
            # of the decoded x~_i
            assert m["encoder_linf"] == m["linf"]
            prev = m["linf"]
        xt_prev = np.zeros_like(x)
        for k in range(1, n + 1):
            xt = driver.reconstruct(comps, k, x.shape, x.dtype)
            assert driver.measured_error(x, xt) == meta[k - 1]["linf"]
            assert np.array_equal(driver.refine(xt_prev, comps, k - 1, k), xt)
            xt_prev = xt


def test_first_component_is_a_single_component_run():
    """Alg. 1 starts from x~_0 = 0, so the first component of any store is
    the one-component compression of x at tau_1, whatever follows it; and a
    one-component store's reconstruction is D(C(x, tau)) with error <= tau."""
    for x, ratio, n in _small_fields():
        rng_ = float(x.max() - x.min())
        taus = [rng_ * ratio ** -(i + 1) for i in range(n)]
        comps, meta = driver.compress(x, taus)
        one, meta1 = driver.compress(x, taus[:1])
        assert np.array_equal(one[0], comps[0])
        assert meta1[0]["linf"] == meta[0]["linf"] <= taus[0]
        other, _ = driver.compress(x, [taus[0], taus[0] / 3.0])
        assert np.array_equal(other[0], comps[0])


def test_cast_f32_codec_non_overlapping_pair():
    """Sec. 3: with fl = round-to-float32, x = a + b with a, b float32 and
    |b| < ulp(a)/2 (held exactly by the double x) splits into x_1 = a,
    x_2 = b, x_3 = 0."""
    rng = np.random.default_rng(16)
    a = rng.normal(size=1000).astype(np.float32)
    ulp = np.spacing(np.abs(a)).astype(np.float64)
    # |b| in [2^-5, 0.49] ulp(a): a + b then spans at most 51 bits, so the
    # double x holds it exactly
    mag = rng.uniform(2.0 ** -5, 0.49, size=1000) * rng.choice([-1.0, 1.0], size=1000)
    b = (mag * ulp).astype(np.float32)
    x = a.astype(np.float64) + b.astype(np.float64)
    comps, meta = driver.compress(x, [1.0, 0.5, 0.25], driver.CastF32Codec())
    assert np.array_equal(comps[0], a)
    assert np.array_equal(comps[1], b)
    assert np.all(comps[2] == 0)


def test_cast_f32_codec_three_components_are_lossless():
    """A double has 53 significand bits; three float32 components carry
    24 + 24 + 24 and each residual is exact, so x~_3 == x (normal range)."""
    rng = np.random.default_rng(17)
    x = rng.normal(size=5000) * 2.0 ** rng.integers(-40, 40, size=5000)
    comps, meta = driver.compress(x, [1.0, 0.5, 0.25], driver.CastF32Codec())
    xt = driver.reconstruct(comps, 3, x.shape, x.dtype, driver.CastF32Codec())
    assert np.array_equal(xt, x)
    xt2 = driver.reconstruct(comps, 2, x.shape, x.dtype, driver.CastF32Codec())
    assert np.all(np.abs(x - xt2) <= np.abs(x) * 2.0 ** -47)
    assert meta[2]["linf"] == 0.0


def test_cast_f32_codec_exact_range():
    """The expansion's limits: exact for 2^-97 <= |x| < 2^128 (x's last bit,
    2^(e-52), is still a float32 subnormal step at e = -97), not below, where
    the third component loses bits."""
    rng = np.random.default_rng(18)
    m = rng.uniform(1.0, 2.0, size=2000) * rng.choice([-1.0, 1.0], size=2000)
    for e, exact in ((-97, True), (0, True), (127, True), (-100, False)):
        x = m * 2.0 ** e
        comps, _ = driver.compress(x, [1.0, 0.5, 0.25], driver.CastF32Codec())
        xt = driver.reconstruct(comps, 3, x.shape, x.dtype, driver.CastF32Codec())
        assert bool(np.array_equal(xt, x)) == exact, e


def test_lossless_limit_block_codec():
    """Sec. 5.1.3: enough components reach zero error.  With tau_n below the
    smallest nonzero float32 difference, Eq. (1) forces x~_n == x."""
    from paper_2308_11759_amd import inputs
    x = inputs.spectral_field((12, 16, 20), seed=5, dtype=np.float32)
    taus = [2.0 ** (-16 * (i + 1)) for i in range(10)]
    comps, meta = driver.compress(x, taus)
    xt = driver.reconstruct(comps, len(comps), x.shape, x.dtype)
    assert np.array_equal(xt, x)


def test_select_k_prescribed_and_measured():
    meta = [dict(tau=1.0, linf=0.3), dict(tau=0.1, linf=0.02), dict(tau=0.01, linf=0.004)]
    assert driver.select_k(meta, 0.5) == 2
    assert driver.select_k(meta, 0.5, use_measured=True) == 1
    assert driver.select_k(meta, 0.001) is None
    assert driver.select_k(meta, 0.01) == 3


def test_corrupt_streams_rejected():
    from paper_2308_11759_amd import inputs
    x = inputs.spectral_field((8, 12, 16), seed=6, dtype=np.float32)
    y, _ = orc.encode(x, x, np.zeros_like(x), 1e-3)
    assert orc.decode_rc(y[:-4], x.shape, x.dtype)[0] == orc.E_CORRUPT
    bad = y.copy()
    bad[0] ^= 1
    assert orc.decode_rc(bad, x.shape, x.dtype)[0] == orc.E_CORRUPT
    bad = y.copy()
    bad[40] ^= 1  # minexp no longer matches tau
    assert orc.decode_rc(bad, x.shape, x.dtype)[0] == orc.E_CORRUPT
    rng = np.random.default_rng(7)
    for _ in range(50):  # random payload flips never read out of bounds
        bad = y.copy()
        pos = int(rng.integers(64, y.size))
        bad[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        rc, _ = orc.decode_rc(bad, x.shape, x.dtype)
        assert rc in (orc.OK, orc.E_CORRUPT)


def test_accuracy_gain_closed_forms():
    """Sec. 5.1.1: gain = log2(sigma / rmse) - rate, pinned by fields whose
    standard deviation and error are known exactly."""
    # the digits 0..9 repeated: variance (10^2 - 1) / 12; a constant offset c
    # as the error: rmse = |c|
    x = np.tile(np.arange(10, dtype=np.float64), 7)
    for c, rate in ((0.25, 3.0), (-2.0, 0.5)):
        sigma, rmse, gain = driver.accuracy_gain(x, x + c, rate)
        assert sigma == pytest.approx(math.sqrt(99.0 / 12.0), rel=1e-15)
        assert rmse == abs(c)
        assert gain == pytest.approx(math.log2(math.sqrt(99.0 / 12.0) / abs(c)) - rate, rel=1e-15)
    # alternating +-1 and x~ = 1.5 x: sigma = 1, rmse = 1/2, gain = 1 - rate
    a = np.tile([1.0, -1.0], 32)
    assert driver.accuracy_gain(a, 1.5 * a, 2.0) == (1.0, 0.5, -1.0)
    # a lossless reconstruction has infinite gain
    assert driver.accuracy_gain(a, a, 5.0)[2] == math.inf


def test_accuracy_gain_invariants():
    """Scaling data and error by a power of two leaves the gain unchanged, and
    halving the error raises it by exactly one bit."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=4096)
    e = rng.normal(scale=1e-3, size=4096)
    g0 = driver.accuracy_gain(x, x + e, 1.5)[2]
    g1 = driver.accuracy_gain(8.0 * x, 8.0 * (x + e), 1.5)[2]
    assert g1 == pytest.approx(g0, abs=1e-12)
    s0, r0, _ = driver.accuracy_gain(x, x - e, 0.0)
    s1, r1, _ = driver.accuracy_gain(x, x - e / 2, 0.0)
    assert math.log2(s1 / r1) - math.log2(s0 / r0) == pytest.approx(1.0, abs=1e-12)
