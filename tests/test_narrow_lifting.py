"""The identity behind the decoders' narrow inverse-transform routes (CPU).

When every coefficient of a block is a multiple of 2^(H+6), where H is half
the integer width, the inverse lifting of the whole words (wrapping integer
arithmetic, arithmetic right shifts) equals the lifting of their high halves
alone, shifted back: every word it forms is a multiple of 2^H, sums,
differences and doublings act on the high halves modulo 2^H, and each of the
at most six halvings along a chain meets an even high half.  The float32
decoder uses H = 16 (coded planes in the top ten bit positions: multiples of
2^22), the float64 decoder H = 32 (top 26 positions: multiples of 2^38).

The lifting here is written from the basis the oracle pins (rows (1/16)
[4,4,4,4], [5,1,-1,-5], [-4,4,4,-4], [-2,6,-6,2]): an independent numpy
restatement with the three passes in z, y, x order.  The test checks the
identity on random blocks across the whole range (values that wrap
included), and that it fails for some block once the coefficients are only
multiples of 2^(H+5): the six halvings need the full margin."""
import numpy as np


def lift_inv(a, b, c, d, half):
    w = b + half(d)
    t1 = d + half(w)
    t0 = 2 * w - t1
    s1 = c + a
    s0 = a - c
    return t0 + s0, t1 + s1, s1 - t1, s0 - t0


def inverse3(q, half):
    """q: (..., 64) in block order l = x + 4 y + 16 z; z, then y, then x"""
    q = q.copy()
    for l in range(16):
        idx = [l, l + 16, l + 32, l + 48]
        q[..., idx[0]], q[..., idx[1]], q[..., idx[2]], q[..., idx[3]] = lift_inv(
            q[..., idx[0]], q[..., idx[1]], q[..., idx[2]], q[..., idx[3]], half)
    for l in range(16):
        b = 16 * (l >> 2) + (l & 3)
        idx = [b, b + 4, b + 8, b + 12]
        q[..., idx[0]], q[..., idx[1]], q[..., idx[2]], q[..., idx[3]] = lift_inv(
            q[..., idx[0]], q[..., idx[1]], q[..., idx[2]], q[..., idx[3]], half)
    for r in range(16):
        idx = [4 * r, 4 * r + 1, 4 * r + 2, 4 * r + 3]
        q[..., idx[0]], q[..., idx[1]], q[..., idx[2]], q[..., idx[3]] = lift_inv(
            q[..., idx[0]], q[..., idx[1]], q[..., idx[2]], q[..., idx[3]], half)
    return q


def run(wide, narrow, hbits, zero_bits, nblocks, seed):
    rng = np.random.default_rng(seed)
    bits = 8 * np.dtype(wide).itemsize
    # random high parts over the whole range, so that sums wrap
    top = rng.integers(-(1 << (bits - 1 - zero_bits)), 1 << (bits - 1 - zero_bits), size=(nblocks, 64),
                       dtype=np.int64)
    c = (top.astype(wide) << wide(zero_bits)).astype(wide)  # multiples of 2^zero_bits
    with np.errstate(over="ignore"):
        full = inverse3(c, lambda v: v >> wide(1))
        hi = (c >> wide(hbits)).astype(narrow)  # the high halves (low halves are zero)
        part = inverse3(hi, lambda v: v >> narrow(1))
    back = (part.astype(wide) << wide(hbits)).astype(wide)
    return full, back


def test_float32_route_identity():
    full, back = run(np.int32, np.int16, 16, 22, 20000, 1)
    assert np.array_equal(full, back)


def test_float64_route_identity():
    full, back = run(np.int64, np.int32, 32, 38, 20000, 2)
    assert np.array_equal(full, back)


def test_margin_is_needed():
    """With one bit less (multiples of 2^21, resp. 2^37) some block differs."""
    full, back = run(np.int32, np.int16, 16, 21, 20000, 3)
    assert not np.array_equal(full, back)
    full, back = run(np.int64, np.int32, 32, 37, 20000, 4)
    assert not np.array_equal(full, back)
