"""Multi-component driver of the oracle (test infrastructure only).

Alg. 1 (Sec. 4.1) builds components y_i = C(x - x~_{i-1}, tau_i), decodes each
one straight away (x_i = D(y_i)) and adds it to the running approximation
x~_i = x~_{i-1} + x_i in the precision of x, left to right (Sec. 3, last
paragraph).  Alg. 2 (Sec. 4.2) rebuilds x~_m as the same left-to-right sum of
the first m decoded components; adding further components continues the
refinement without any decoder state.  Per-component metadata holds the
prescribed tau_i and the measured error max|x - x~_i| (Sec. 4.3, last
paragraph), evaluated in float64.

Codecs plug in through ``encode(e, tau, x, xt) -> (y, stats)`` and
``decode(y, shape, dtype) -> x_i``: the block-transform codec and the
prediction codec of the C oracle, and the scalar cast-to-float32
"compressor" of Sec. 3, which turns Alg. 1 into the classical
multi-component floating-point expansion.
"""
import math

import numpy as np

from . import lib


class BlockCodec:
    """The zfp-style fixed-accuracy block codec of pmc_oracle.c."""

    name = "block"

    def encode(self, e, tau, x, xt):
        return lib.encode(e, x, xt, tau)

    def decode(self, y, shape, dtype):
        return lib.decode(y, shape, dtype)


class PredictionCodec:
    """The prediction-and-quantisation codec (codec 1) of pmc_oracle.c: a
    second error-bounded compressor behind the same driver (Sec. 6.2)."""

    name = "prediction"

    def encode(self, e, tau, x, xt):
        return lib.encode(e, x, xt, tau, codec=1)

    def decode(self, y, shape, dtype):
        return lib.decode(y, shape, dtype)


class CastF32Codec:
    """fl[.] of Sec. 3: round to the nearest float32 (tau is ignored)."""

    name = "cast_f32"

    def encode(self, e, tau, x, xt):
        return np.asarray(e, dtype=np.float64).astype(np.float32), {}

    def decode(self, y, shape, dtype):
        return np.asarray(y, dtype=np.float32).astype(dtype).reshape(shape)


def measured_error(x, xt):
    """max |x - x~| evaluated in float64 (Sec. 4.3)."""
    if x.size == 0:
        return 0.0
    return float(np.max(np.abs(x.astype(np.float64) - xt.astype(np.float64))))


def accuracy_gain(x, xt, rate):
    """Sec. 5.1.1: gain = log2(sigma / rmse) - rate, sigma the standard deviation
    of x, rmse the root-mean-square of x - x~, rate in bits per value; all in
    float64.  Returns (sigma, rmse, gain)."""
    xd = np.asarray(x, dtype=np.float64)
    ed = xd - np.asarray(xt, dtype=np.float64)
    sigma = math.sqrt(float(np.mean((xd - np.mean(xd)) ** 2)))
    rmse = math.sqrt(float(np.mean(ed ** 2)))
    with np.errstate(divide="ignore"):
        gain = float(np.log2(np.float64(sigma) / np.float64(rmse))) - rate
    return sigma, rmse, gain


def compress(x, taus, codec=None):
    """Alg. 1.  Returns (components y_1..y_n, per-component stats with tau and linf)."""
    codec = codec or BlockCodec()
    taus = [float(t) for t in taus]
    if len(taus) < 1:
        raise ValueError("need at least one component")
    for a, b in zip(taus, taus[1:]):
        if not a > b:
            raise ValueError("tolerances must be strictly decreasing")
    xt = np.zeros_like(x)                       # x~ starts at zero
    comps, meta = [], []
    for tau in taus:                            # one component per tolerance
        e = x - xt                              # residual (field precision, RNE)
        y, st = codec.encode(e, tau, x, xt)     # compress it under tau
        xi = codec.decode(y, x.shape, x.dtype)  # decode the new component
        xt = xt + xi                            # partial-sum update (left-to-right sum)
        m = dict(st)
        m["tau"] = tau
        if "linf" in st:
            m["encoder_linf"] = st["linf"]      # the codec's own largest accepted block error
        m["linf"] = measured_error(x, xt)
        comps.append(y)
        meta.append(m)
    return comps, meta


def reconstruct(comps, m, shape, dtype, codec=None):
    """Alg. 2: x~_m = (...((0 + x_1) + x_2) ...) + x_m."""
    codec = codec or BlockCodec()
    if not 0 <= m <= len(comps):
        raise ValueError("m out of range")
    xt = np.zeros(shape, dtype=dtype)
    for i in range(m):
        xt = xt + codec.decode(comps[i], shape, dtype)
    return xt


def refine(xt, comps, k_from, k_to, codec=None):
    """Continue Alg. 2 from x~_{k_from} to x~_{k_to} (no decoder state kept)."""
    codec = codec or BlockCodec()
    for i in range(k_from, k_to):
        xt = xt + codec.decode(comps[i], xt.shape, xt.dtype)
    return xt


def select_k(meta, tol, use_measured=False):
    """Smallest k whose prescribed tau_k (or measured error) is <= tol (Sec. 6.2).

    Returns None when no component reaches tol."""
    for i, m in enumerate(meta):
        v = m["linf"] if use_measured else m["tau"]
        if v <= tol:
            return i + 1
    return None
