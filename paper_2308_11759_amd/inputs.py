"""Seeded synthetic input fields (shared by the tests, the benchmark and the oracle).

This module only draws inputs; it holds none of the codec's arithmetic and
imports nothing else from the package.  The paper evaluates on SDRBench
fields (Sec. 5, Table 1: Miranda, S3D, S3D JICF in float64; Nyx, QMCPACK, SCALE
in float32), which are not available here; these generators stand in for them
with the same shapes and precisions and with smoothness on both sides of the
paper's per-axis autocorrelation split (Sec. 5.1.1, last paragraph: below 0.79
for Nyx, above 0.95 for the others).

All arrays are numpy, C order, shape (nz, ny, nx) with x fastest.
"""
import hashlib
import math

import numpy as np


def blobs_field(n=64, seed=0, dtype=np.float64):
    """Sum of 16 Gaussian blobs + 3 sinusoids + N(0, 1e-3^2) noise on an n^3 grid.

    Blob amplitude U[-1, 1], width sigma U[2, 10] cells, centre U[0, n)^3,
    profile exp(-r^2 / (2 sigma^2)); sinusoid a sin(2 pi k.r / n + phi) with
    a ~ U[-0.5, 0.5], integer k in [-4, 4]^3 \\ {0}, phi ~ U[0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z, y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                          np.arange(n, dtype=np.float64), indexing="ij")
    f = np.zeros((n, n, n), dtype=np.float64)
    for _ in range(16):
        amp = rng.uniform(-1.0, 1.0)
        sigma = rng.uniform(2.0, 10.0)
        cx, cy, cz = rng.uniform(0.0, n, size=3)
        r2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
        f += amp * np.exp(-r2 / (2.0 * sigma * sigma))
    for _ in range(3):
        a = rng.uniform(-0.5, 0.5)
        while True:
            k = rng.integers(-4, 5, size=3)
            if np.any(k != 0):
                break
        phi = rng.uniform(0.0, 2.0 * math.pi)
        f += a * np.sin(2.0 * math.pi * (k[0] * x + k[1] * y + k[2] * z) / n + phi)
    f += rng.normal(0.0, 1e-3, size=f.shape)
    return f.astype(dtype)


def spectral_field(shape, seed=1, dtype=np.float32, noise_rel=0.0):
    """Random-phase isotropic field with shell spectrum E(k) ~ k^(-5/3).

    rfft-layout amplitude |k|^(-11/6), DC = 0, phases uniform in [0, 2 pi),
    inverse FFT in float64, affine map onto exactly [-1, 1], then optional
    N(0, (noise_rel * range)^2) white noise (range = 2), then the cast."""
    shape = tuple(int(s) for s in shape)
    rng = np.random.Generator(np.random.PCG64(seed))
    nz, ny, nx = shape
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    k2 = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (-11.0 / 12.0), 0.0)
    del k2
    phase = rng.uniform(0.0, 2.0 * math.pi, size=amp.shape)
    spec = amp * np.exp(1j * phase)
    del amp, phase
    try:
        import scipy.fft as sfft
        f = sfft.irfftn(spec, s=shape, workers=-1)
    except ImportError:  # pragma: no cover
        f = np.fft.irfftn(spec, s=shape)
    del spec
    lo, hi = float(f.min()), float(f.max())
    f = (f - lo) * (2.0 / (hi - lo)) - 1.0
    np.clip(f, -1.0, 1.0, out=f)
    if noise_rel > 0.0:
        f += rng.normal(0.0, noise_rel * 2.0, size=f.shape)
    return f.astype(dtype)


def batched_shapes(count=256, base_seed=100, lo=16, hi=256):
    """(shape, is_float32) of the batched workload's fields."""
    out = []
    for f in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + f))
        dims = [log_uniform_int(rng, lo, hi) for _ in range(3)]
        out.append((tuple(reversed(dims)), f % 2 == 0))
    return out


def served_shapes(count=64, base_seed=200, lo=64, hi=384):
    out = []
    for f in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + f))
        n = log_uniform_int(rng, lo, hi)
        out.append(((n, n, n), f % 2 == 0))
    return out


def log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batched_fields(count=256, base_seed=100, lo=16, hi=256, max_edge=None):
    """Fields of the batched workload: per-axis edge log-uniform in [lo, hi]
    (non-multiples of 4 allowed), even index -> float32, odd -> float64,
    spectral generator with seed base_seed + f."""
    out = []
    for f in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + f))
        dims = [log_uniform_int(rng, lo, hi) for _ in range(3)]
        if max_edge is not None:
            dims = [min(d, max_edge) for d in dims]
        dt = np.float32 if f % 2 == 0 else np.float64
        out.append(spectral_field(tuple(dims), seed=base_seed + f, dtype=dt))
    return out


def served_fields(count=64, base_seed=200, lo=64, hi=384, max_edge=None):
    """Store of the served workload: cubic, edge log-uniform in [lo, hi],
    dtype alternating float32 / float64, spectral generator."""
    out = []
    for f in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + f))
        n = log_uniform_int(rng, lo, hi)
        if max_edge is not None:
            n = min(n, max_edge)
        dt = np.float32 if f % 2 == 0 else np.float64
        out.append(spectral_field((n, n, n), seed=base_seed + f, dtype=dt))
    return out


def query_trace(nfields, rate_qps, nqueries, seed=7, tol_lo=1e-5, tol_hi=1e-1):
    """Open-loop Poisson arrivals: (arrival_s, field, relative tolerance) tuples;
    the relative tolerance is log-uniform in [tol_lo, tol_hi] (times the range)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_qps, size=nqueries)
    t = np.cumsum(gaps)
    fields = rng.integers(0, nfields, size=nqueries)
    rel = np.exp(rng.uniform(math.log(tol_lo), math.log(tol_hi), size=nqueries))
    return [(float(t[i]), int(fields[i]), float(rel[i])) for i in range(nqueries)]


def lag1_autocorrelation(f):
    """Per-axis lag-1 autocorrelation (x, y, z), to place a field against the
    paper's smooth (> 0.95) / rough (< 0.79) split."""
    g = f.astype(np.float64)
    g -= float(np.mean(g))
    var = float(np.mean(g * g))
    out = []
    for axis in (2, 1, 0):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, g.shape[axis] - 1)
        hi[axis] = slice(1, g.shape[axis])
        out.append(float(np.mean(g[tuple(lo)] * g[tuple(hi)])) / var if var > 0 else 1.0)
    return out


def sha256(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
