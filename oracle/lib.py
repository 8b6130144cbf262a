"""ctypes loader for the C oracle (test infrastructure only).

Every function here marshals arguments; the arithmetic lives in pmc_oracle.c.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F32, F64 = 1, 2
EMPTY, CODED, RAW = 0, 1, 2
OK, E_ARG, E_NOMEM, E_CORRUPT = 0, -1, -3, -4
CHUNK_BLOCKS = 16
HEADER_BYTES = 64


class Field(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("d", ctypes.c_int), ("dims", ctypes.c_uint64 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("nempty", ctypes.c_uint64),
        ("ncoded", ctypes.c_uint64),
        ("nraw", ctypes.c_uint64),
        ("nesc", ctypes.c_uint64),
        ("nmiss", ctypes.c_uint64),
        ("linf", ctypes.c_double),
        ("bits", ctypes.c_uint64),
    ]


def build(force=False):
    """Compile pmc_oracle.c with gcc (plain C11, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall",
             "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    u8p, u64p, dp, ip = P(ctypes.c_uint8), P(ctypes.c_uint64), P(ctypes.c_double), P(ctypes.c_int)
    i64p = P(ctypes.c_int64)
    vp = ctypes.c_void_p
    lib.orc_minexp.argtypes = [ctypes.c_double]
    lib.orc_minexp.restype = ctypes.c_int
    lib.orc_fwd_lift4.argtypes = [i64p, ctypes.c_int]
    lib.orc_inv_lift4.argtypes = [i64p, ctypes.c_int]
    lib.orc_fwd_xform.argtypes = [i64p, ctypes.c_int, ctypes.c_int]
    lib.orc_inv_xform.argtypes = [i64p, ctypes.c_int, ctypes.c_int]
    lib.orc_perm.argtypes = [ctypes.c_int, ip]
    lib.orc_to_negabinary.argtypes = [ctypes.c_int64, ctypes.c_int]
    lib.orc_to_negabinary.restype = ctypes.c_uint64
    lib.orc_from_negabinary.argtypes = [ctypes.c_uint64, ctypes.c_int]
    lib.orc_from_negabinary.restype = ctypes.c_int64
    lib.orc_encode_planes.argtypes = [u64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_uint64]
    lib.orc_encode_planes.restype = ctypes.c_uint64
    lib.orc_decode_planes.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p]
    lib.orc_decode_planes.restype = ctypes.c_uint64
    lib.orc_block_coeffs.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip, u64p]
    lib.orc_block_coeffs.restype = ctypes.c_int
    lib.orc_block_values.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p, dp]
    lib.orc_quantize.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.orc_quantize.restype = ctypes.c_int64
    lib.orc_dequantize.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int]
    lib.orc_dequantize.restype = ctypes.c_double
    lib.orc_value_expo.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.orc_value_expo.restype = ctypes.c_int
    lib.orc_stream_cap.argtypes = [P(Field)]
    lib.orc_stream_cap.restype = ctypes.c_uint64
    lib.orc_encode.argtypes = [P(Field), vp, vp, vp, ctypes.c_double, u8p, ctypes.c_uint64, u64p, P(Stats)]
    lib.orc_encode.restype = ctypes.c_int
    lib.orc_encode_codec.argtypes = [P(Field), ctypes.c_int, vp, vp, vp, ctypes.c_double, u8p, ctypes.c_uint64,
                                     u64p, P(Stats)]
    lib.orc_encode_codec.restype = ctypes.c_int
    lib.orc_lorenzo_fwd.argtypes = [i64p, ctypes.c_int, ctypes.c_int]
    lib.orc_lorenzo_inv.argtypes = [i64p, ctypes.c_int, ctypes.c_int]
    lib.orc_zigzag.argtypes = [ctypes.c_int64, ctypes.c_int]
    lib.orc_zigzag.restype = ctypes.c_uint64
    lib.orc_unzigzag.argtypes = [ctypes.c_uint64, ctypes.c_int]
    lib.orc_unzigzag.restype = ctypes.c_int64
    lib.orc_encode_one_block_pq.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double, u8p,
                                            ctypes.c_uint64, u64p, ip, ip, dp, dp]
    lib.orc_encode_one_block_pq.restype = ctypes.c_int
    lib.orc_decode_one_block_pq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, u8p, ctypes.c_uint64,
                                            dp, u64p]
    lib.orc_decode_one_block_pq.restype = ctypes.c_int
    lib.orc_stream_info.argtypes = [u8p, ctypes.c_uint64, P(Field), dp, u64p, u64p]
    lib.orc_stream_info.restype = ctypes.c_int
    lib.orc_decode.argtypes = [u8p, ctypes.c_uint64, P(Field), vp]
    lib.orc_decode.restype = ctypes.c_int
    lib.orc_encode_one_block.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double, u8p,
                                         ctypes.c_uint64, u64p, ip, ip, dp, dp]
    lib.orc_encode_one_block.restype = ctypes.c_int
    lib.orc_decode_one_block.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, u8p, ctypes.c_uint64,
                                         dp, u64p]
    lib.orc_decode_one_block.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def dtype_code(dt):
    dt = np.dtype(dt)
    if dt == np.float32:
        return F32
    if dt == np.float64:
        return F64
    raise ValueError("unsupported dtype %s" % dt)


def make_field(shape, dtype):
    """numpy shape (nz, ny, nx) / (ny, nx) / (nx,) -> Field with x fastest."""
    f = Field()
    f.dtype = dtype_code(dtype)
    f.d = len(shape)
    dims = list(reversed(shape)) + [1] * (3 - len(shape))
    for a in range(3):
        f.dims[a] = int(dims[a])
    return f


# ---- thin wrappers --------------------------------------------------------
def minexp(tau):
    return load().orc_minexp(float(tau))


def fwd_lift4(v, P):
    a = np.array(v, dtype=np.int64)
    load().orc_fwd_lift4(_ptr(a, ctypes.c_int64), P)
    return a


def inv_lift4(v, P):
    a = np.array(v, dtype=np.int64)
    load().orc_inv_lift4(_ptr(a, ctypes.c_int64), P)
    return a


def fwd_xform(q, d, P):
    a = np.array(q, dtype=np.int64).copy()
    load().orc_fwd_xform(_ptr(a, ctypes.c_int64), d, P)
    return a


def inv_xform(q, d, P):
    a = np.array(q, dtype=np.int64).copy()
    load().orc_inv_xform(_ptr(a, ctypes.c_int64), d, P)
    return a


def perm(d):
    a = np.zeros(4 ** d, dtype=np.int32)
    load().orc_perm(d, _ptr(a, ctypes.c_int))
    return a


def to_negabinary(q, P):
    return load().orc_to_negabinary(int(q), P)


def from_negabinary(u, P):
    return load().orc_from_negabinary(int(u), P)


def quantize(e, emax, dtype):
    return load().orc_quantize(float(e), int(emax), dtype_code(dtype))


def dequantize(q, emax, dtype):
    return load().orc_dequantize(int(q), int(emax), dtype_code(dtype))


def value_expo(v, dtype):
    return load().orc_value_expo(float(v), dtype_code(dtype))


def encode_planes(u, P, p):
    u = np.ascontiguousarray(u, dtype=np.uint64)
    cap = 4096
    buf = np.zeros(cap, dtype=np.uint8)
    nbits = load().orc_encode_planes(_ptr(u, ctypes.c_uint64), len(u), P, p, _ptr(buf, ctypes.c_uint8), cap)
    return buf, int(nbits)


def decode_planes(buf, nbits, B, P, p):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    u = np.zeros(B, dtype=np.uint64)
    used = load().orc_decode_planes(_ptr(buf, ctypes.c_uint8), nbits, B, P, p, _ptr(u, ctypes.c_uint64))
    return u, used


def block_coeffs(e, dtype, d):
    e = np.ascontiguousarray(e, dtype=np.float64)
    em = ctypes.c_int(0)
    u = np.zeros(4 ** d, dtype=np.uint64)
    nz = load().orc_block_coeffs(dtype_code(dtype), d, _ptr(e, ctypes.c_double), ctypes.byref(em),
                                 _ptr(u, ctypes.c_uint64))
    return bool(nz), em.value, u


def block_values(u, emax, dtype, d):
    u = np.ascontiguousarray(u, dtype=np.uint64)
    out = np.zeros(4 ** d, dtype=np.float64)
    load().orc_block_values(dtype_code(dtype), d, emax, _ptr(u, ctypes.c_uint64), _ptr(out, ctypes.c_double))
    return out


def encode_one_block(e, x, xt, tau, dtype, d):
    """Encode one whole block; returns dict(bits, nbits, mode, p, err, xi, miss)."""
    B = 4 ** d
    e = np.ascontiguousarray(e, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    assert e.size == B and x.size == B and xt.size == B
    cap = 1200
    buf = np.zeros(cap, dtype=np.uint8)
    nbits = ctypes.c_uint64(0)
    mode, p = ctypes.c_int(0), ctypes.c_int(0)
    err = ctypes.c_double(0)
    xi = np.zeros(B, dtype=np.float64)
    rc = load().orc_encode_one_block(dtype_code(dtype), d, _ptr(e, ctypes.c_double), _ptr(x, ctypes.c_double),
                                     _ptr(xt, ctypes.c_double), float(tau), _ptr(buf, ctypes.c_uint8), cap,
                                     ctypes.byref(nbits), ctypes.byref(mode), ctypes.byref(p), ctypes.byref(err),
                                     _ptr(xi, ctypes.c_double))
    assert rc in (0, 1), rc
    return dict(buf=buf, nbits=nbits.value, mode=mode.value, p=p.value, err=err.value, xi=xi, miss=rc == 1)


def decode_one_block(buf, nbits, tau, dtype, d):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    out = np.zeros(4 ** d, dtype=np.float64)
    used = ctypes.c_uint64(0)
    m = load().orc_decode_one_block(dtype_code(dtype), d, float(tau), _ptr(buf, ctypes.c_uint8), nbits,
                                    _ptr(out, ctypes.c_double), ctypes.byref(used))
    return m, out, used.value


def lorenzo_fwd(q, d, P):
    a = np.array(q, dtype=np.int64).copy()
    load().orc_lorenzo_fwd(_ptr(a, ctypes.c_int64), d, P)
    return a


def lorenzo_inv(r, d, P):
    a = np.array(r, dtype=np.int64).copy()
    load().orc_lorenzo_inv(_ptr(a, ctypes.c_int64), d, P)
    return a


def zigzag(r, P):
    return load().orc_zigzag(int(r), P)


def unzigzag(z, P):
    return load().orc_unzigzag(int(z), P)


def encode_one_block_pq(e, x, xt, tau, dtype, d):
    """Codec 1 on one whole block; returns dict(buf, nbits, mode, delta, err, xi, miss)."""
    B = 4 ** d
    e = np.ascontiguousarray(e, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    assert e.size == B and x.size == B and xt.size == B
    cap = 1200
    buf = np.zeros(cap, dtype=np.uint8)
    nbits = ctypes.c_uint64(0)
    mode, delta = ctypes.c_int(0), ctypes.c_int(0)
    err = ctypes.c_double(0)
    xi = np.zeros(B, dtype=np.float64)
    rc = load().orc_encode_one_block_pq(dtype_code(dtype), d, _ptr(e, ctypes.c_double), _ptr(x, ctypes.c_double),
                                        _ptr(xt, ctypes.c_double), float(tau), _ptr(buf, ctypes.c_uint8), cap,
                                        ctypes.byref(nbits), ctypes.byref(mode), ctypes.byref(delta),
                                        ctypes.byref(err), _ptr(xi, ctypes.c_double))
    assert rc in (0, 1), rc
    return dict(buf=buf, nbits=nbits.value, mode=mode.value, delta=delta.value, err=err.value, xi=xi,
                miss=rc == 1)


def decode_one_block_pq(buf, nbits, tau, dtype, d):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    out = np.zeros(4 ** d, dtype=np.float64)
    used = ctypes.c_uint64(0)
    m = load().orc_decode_one_block_pq(dtype_code(dtype), d, float(tau), _ptr(buf, ctypes.c_uint8), nbits,
                                       _ptr(out, ctypes.c_double), ctypes.byref(used))
    return m, out, used.value


def stream_cap(shape, dtype):
    f = make_field(shape, dtype)
    return int(load().orc_stream_cap(ctypes.byref(f)))


def encode(e, x, xt, tau, codec=0):
    """y = C(e, tau) for one component; e = x - xt already computed (the residual step of Alg. 1).
    codec 0: the block-transform codec; 1: prediction and quantisation.

    Returns (stream bytes as np.uint8 array, stats dict)."""
    assert e.dtype == x.dtype == xt.dtype and e.shape == x.shape == xt.shape
    e = np.ascontiguousarray(e)
    x = np.ascontiguousarray(x)
    xt = np.ascontiguousarray(xt)
    f = make_field(x.shape, x.dtype)
    cap = int(load().orc_stream_cap(ctypes.byref(f)))
    out = np.zeros(cap, dtype=np.uint8)
    nbytes = ctypes.c_uint64(0)
    st = Stats()
    rc = load().orc_encode_codec(ctypes.byref(f), int(codec), e.ctypes.data, x.ctypes.data, xt.ctypes.data,
                                 float(tau), _ptr(out, ctypes.c_uint8), cap, ctypes.byref(nbytes), ctypes.byref(st))
    if rc != OK:
        raise RuntimeError("oracle encode failed: %d" % rc)
    stats = {k: getattr(st, k) for k, _ in Stats._fields_}
    return out[: nbytes.value].copy(), stats


def stream_info(stream):
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    f = Field()
    tau = ctypes.c_double(0)
    nch, words = ctypes.c_uint64(0), ctypes.c_uint64(0)
    rc = load().orc_stream_info(_ptr(stream, ctypes.c_uint8), stream.size, ctypes.byref(f), ctypes.byref(tau),
                                ctypes.byref(nch), ctypes.byref(words))
    if rc != OK:
        return rc, None
    shape = tuple(int(f.dims[a]) for a in reversed(range(f.d)))
    return OK, dict(dtype=np.float32 if f.dtype == F32 else np.float64, shape=shape, tau=tau.value,
                    nchunks=nch.value, words=words.value)


def decode(stream, shape, dtype):
    """x_i = D(y_i) as a dense field (the decode step of Alg. 2).  Raises on a corrupt stream."""
    rc, out = decode_rc(stream, shape, dtype)
    if rc != OK:
        raise RuntimeError("oracle decode failed: %d" % rc)
    return out


def decode_rc(stream, shape, dtype):
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    f = make_field(shape, dtype)
    out = np.zeros(shape, dtype=dtype)
    rc = load().orc_decode(_ptr(stream, ctypes.c_uint8), stream.size, ctypes.byref(f), out.ctypes.data)
    return rc, out
