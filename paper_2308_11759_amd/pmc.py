"""Python binding of the C-ABI in include/pmc.h (ctypes; argument marshalling only).

PyTorch provides device memory and the HIP stream; every step of compression
and retrieval runs in the HIP kernels of libpmc.so.  There is no CPU fallback:
importing this module without the built library raises.

Names follow the paper (Magri & Lindstrom): ``compress`` is Alg. 1 (Sec. 4.1),
``retrieve`` is Alg. 2 (Sec. 4.2), ``refine`` continues Alg. 2 from a cached
partial sum, ``select_k`` picks the component count for a tolerance from the
per-component metadata (Sec. 6.2).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmc.so")

OK, E_ARG, E_NONFINITE, E_NOMEM, E_CORRUPT, E_UNREACHABLE, E_BOUND, E_DEVICE = 0, -1, -2, -3, -4, -5, -6, -7
E_CANCELLED = -8
F32, F64 = 1, 2
OPT_FUSED_DECODE, OPT_SYNC_CHECK, OPT_PROFILE, OPT_CODEC = 1, 2, 3, 4
CODEC_TRANSFORM, CODEC_PREDICTION = 0, 1
_NAMES = {0: "OK", -1: "E_ARG", -2: "E_NONFINITE", -3: "E_NOMEM", -4: "E_CORRUPT", -5: "E_UNREACHABLE",
          -6: "E_BOUND", -7: "E_DEVICE", -8: "E_CANCELLED"}


class PmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(status, "?"), status, msg))
        self.status = status


class Field(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint64), ("ny", ctypes.c_uint64), ("nz", ctypes.c_uint64),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "hits", "partial", "misses", "steps",
                                                "batched_queries", "max_queue", "cache_entries", "cache_bytes",
                                                "arena_peak", "pending", "running", "cancelled")]


_lib = None

# every exported symbol of include/pmc.h with (restype, argtypes)
_vp, _sz, _u64, _dbl, _int = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
_P = ctypes.POINTER
SIGNATURES = {
    "pmc_ctx_create": (_int, [_int, _vp, _P(_vp)]),
    "pmc_ctx_destroy": (None, [_vp]),
    "pmc_last_error": (ctypes.c_char_p, [_vp]),
    "pmc_ctx_set_option": (_int, [_vp, _int, _int]),
    "pmc_range": (_int, [_vp, _P(Field), _vp, _vp, _sz, _P(_dbl), _P(_dbl), _P(_u64)]),
    "pmc_stats_ws_bytes": (_sz, []),
    "pmc_retrieve_box": (_int, [_vp, _vp, _int, _P(_u64), _P(_u64), _vp, _vp, _sz]),
    "pmc_cast_compress": (_int, [_vp, _P(Field), _vp, _int, _vp, _vp, _sz, _P(_dbl)]),
    "pmc_cast_retrieve": (_int, [_vp, _P(Field), _vp, _int, _vp]),
    "pmc_accuracy_gain": (_int, [_vp, _P(Field), _vp, _vp, _dbl, _vp, _sz, _P(_dbl)]),
    "pmc_compress_sizes": (_int, [_P(Field), _int, _P(_sz), _P(_sz)]),
    "pmc_compress": (_int, [_vp, _P(Field), _vp, _int, _P(_dbl), _vp, _sz, _vp, _sz, _P(_vp)]),
    "pmc_compress_static": (_int, [_vp, _P(Field), _vp, _int, _P(_dbl), _vp, _sz, _P(_vp)]),
    "pmc_store_info": (_int, [_vp, _P(_int), _P(_dbl), _P(_dbl), _P(_u64), _P(_u64), _P(_u64)]),
    "pmc_store_counts": (_int, [_vp, _int, _P(_u64)]),
    "pmc_store_decode_route": (_int, [_vp, _int, _P(_int)]),
    "pmc_store_codec": (_int, [_vp, _P(_int)]),
    "pmc_store_span": (_int, [_vp, _int, _P(_u64), _P(_int)]),
    "pmc_store_field": (_int, [_vp, _P(Field)]),
    "pmc_store_stream": (_int, [_vp, _int, _P(_vp), _P(_u64)]),
    "pmc_select_k": (_int, [_vp, _dbl, _int, _P(_int)]),
    "pmc_decode_ws_bytes": (_sz, []),
    "pmc_retrieve": (_int, [_vp, _vp, _int, _vp, _vp, _sz]),
    "pmc_refine": (_int, [_vp, _vp, _int, _int, _vp, _vp, _sz]),
    "pmc_store_serialize": (_int, [_vp, _vp, _vp, _sz, _P(_sz)]),
    "pmc_store_device_bytes": (_int, [_vp, _sz, _P(_sz)]),
    "pmc_store_deserialize": (_int, [_vp, _vp, _sz, _vp, _sz, _P(_vp)]),
    "pmc_store_free": (None, [_vp]),
    "pmc_prof_read": (_int, [_vp, _P(ProfEntry), _int, _P(_int), _int]),
    "pmc_batch_plan": (_int, [_vp, _int, _P(Field), _P(_int), _P(_P(_dbl)), _P(_vp)]),
    "pmc_batch_sizes": (_int, [_vp, _P(_sz), _P(_sz)]),
    "pmc_batch_schedule": (_int, [_vp, _int, _int]),
    "pmc_batch_get_schedule": (_int, [_vp, _P(_int), _P(_int)]),
    "pmc_batch_compress": (_int, [_vp, _P(_vp), _vp, _sz, _vp, _sz, _P(_vp)]),
    "pmc_batch_tune": (_int, [_vp, _P(_vp), _vp, _sz, _vp, _sz, _P(ctypes.c_float)]),
    "pmc_batch_order_name": (ctypes.c_char_p, [_int]),
    "pmc_batch_free": (None, [_vp]),
    "pmc_server_create": (_int, [_vp, _sz, _vp, _sz, _int, _P(_vp)]),
    "pmc_server_add": (_int, [_vp, _vp, _P(_int)]),
    "pmc_server_submit": (_int, [_vp, _int, _dbl, _vp, _P(_u64)]),
    "pmc_clock": (_dbl, []),
    "pmc_server_submit_at": (_int, [_vp, _int, _dbl, _vp, _dbl, _P(_u64)]),
    "pmc_server_poll": (_int, [_vp, _u64, _P(_int), _P(_int), _P(_dbl)]),
    "pmc_server_result": (_int, [_vp, _u64, _P(_vp), _P(_int), _P(_int)]),
    "pmc_server_release": (_int, [_vp, _u64]),
    "pmc_server_cancel": (_int, [_vp, _u64]),
    "pmc_server_get_stats": (_int, [_vp, _P(ServerStats)]),
    "pmc_server_destroy": (None, [_vp]),
}


def load(path=LIB_PATH):
    """Load libpmc.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libpmc.so not built (run __graft_entry__.build()): %s" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dtype_code(dt):
    if dt == torch.float32:
        return F32
    if dt == torch.float64:
        return F64
    raise TypeError("fields must be float32 or float64, got %s" % dt)


def field_of(t):
    """Field descriptor of a contiguous tensor with shape (nz, ny, nx), (ny, nx) or (nx,)."""
    if not t.is_contiguous():
        raise ValueError("field tensor must be contiguous")
    shape = list(t.shape)
    if not 1 <= len(shape) <= 3:
        raise ValueError("fields are 1-D to 3-D")
    dims = list(reversed(shape)) + [1] * (3 - len(shape))
    f = Field()
    f.nx, f.ny, f.nz = dims
    f.dtype = _dtype_code(t.dtype)
    return f


def _torch_dtype(code):
    return torch.float32 if code == F32 else torch.float64


class Context:
    """A pmc_ctx bound to a device and a HIP stream (default: torch's current)."""

    def __init__(self, device=0, stream=None):
        self.lib = load()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self.device.index or 0
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.pmc_ctx_create(idx, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), ctx=None)
        self.handle = h
        self._ws = None
        self._dec_ws = torch.empty(int(self.lib.pmc_decode_ws_bytes()), dtype=torch.uint8, device=self.device)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pmc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ctx="self"):
        if st != OK:
            msg = ""
            if ctx == "self" and getattr(self, "handle", None):
                msg = (self.lib.pmc_last_error(self.handle) or b"").decode()
            raise PmcError(st, msg)

    def set_option(self, option, value):
        self._check(self.lib.pmc_ctx_set_option(self.handle, option, int(value)))

    def prof_read(self, reset=True):
        """{kernel name: (launches, total ms)} from the library's HIP events."""
        cap = 64
        arr = (ProfEntry * cap)()
        n = ctypes.c_int()
        self._check(self.lib.pmc_prof_read(self.handle, arr, cap, ctypes.byref(n), int(bool(reset))))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].ms)) for i in range(min(n.value, cap))}

    def _workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def range(self, x):
        """(min, max, non-finite count) of a device field."""
        f = field_of(x)
        ws = self._workspace(256)
        lo, hi, bad = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
        self._check(self.lib.pmc_range(self.handle, ctypes.byref(f), ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(lo),
                                       ctypes.byref(hi), ctypes.byref(bad)))
        return lo.value, hi.value, bad.value

    def accuracy_gain(self, x, xt, rate):
        """Sec. 5.1.1: (sigma, rmse, gain) with gain = log2(sigma / rmse) - rate."""
        f = field_of(x)
        if field_of(xt).dtype != f.dtype or tuple(xt.shape) != tuple(x.shape):
            raise ValueError("x and xt must have the same shape and dtype")
        ws = self._workspace(self.lib.pmc_stats_ws_bytes())
        out = (ctypes.c_double * 3)()
        self._check(self.lib.pmc_accuracy_gain(self.handle, ctypes.byref(f), ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(xt.data_ptr()), float(rate),
                                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), out))
        return out[0], out[1], out[2]

    def cast_compress(self, x, n):
        """Sec. 3's float32-cast compressor: (components as an (n,) + x.shape
        float32 tensor, measured errors max |x - x~_i|)."""
        f = field_of(x)
        comps = torch.empty((int(n),) + tuple(x.shape), dtype=torch.float32, device=self.device)
        ws = self._workspace(256)
        linf = (ctypes.c_double * int(n))()
        self._check(self.lib.pmc_cast_compress(self.handle, ctypes.byref(f), ctypes.c_void_p(x.data_ptr()), int(n),
                                               ctypes.c_void_p(comps.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                               ws.numel(), linf))
        return comps, list(linf)

    def cast_retrieve(self, comps, k, out):
        """x~_k of the float32-cast compressor into out (the field's shape and type)."""
        f = field_of(out)
        if comps.dtype != torch.float32 or tuple(comps.shape[1:]) != tuple(out.shape) or not comps.is_contiguous():
            raise ValueError("comps must be a contiguous float32 (n,) + out.shape tensor")
        if not 0 <= int(k) <= comps.shape[0]:
            raise ValueError("k out of range")
        self._check(self.lib.pmc_cast_retrieve(self.handle, ctypes.byref(f), ctypes.c_void_p(comps.data_ptr()),
                                               int(k), ctypes.c_void_p(out.data_ptr())))
        return out

    def compress_sizes(self, x, n):
        f = field_of(x)
        ws, cap = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.lib.pmc_compress_sizes(ctypes.byref(f), int(n), ctypes.byref(ws), ctypes.byref(cap)))
        return ws.value, cap.value

    def compress(self, x, taus, streams=None, allow_bound_miss=False):
        """Alg. 1: compress a device field into len(taus) components.

        With allow_bound_miss a PMC_E_BOUND result still returns the store
        (flagged ``bound_missed``); otherwise every error raises PmcError."""
        taus = [float(t) for t in taus]
        n = len(taus)
        f = field_of(x)
        ws_bytes, cap1 = self.compress_sizes(x, n)
        ws = self._workspace(ws_bytes)
        if streams is None:
            streams = torch.empty(cap1 * n, dtype=torch.uint8, device=self.device)
        tau_arr = (ctypes.c_double * n)(*taus)
        h = ctypes.c_void_p()
        st = self.lib.pmc_compress(self.handle, ctypes.byref(f), ctypes.c_void_p(x.data_ptr()), n, tau_arr,
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(streams.data_ptr()),
                                   streams.numel(), ctypes.byref(h))
        if st == E_BOUND and allow_bound_miss and h.value:
            store = Store(self, h, streams)
            store.bound_missed = True
            return store
        if st != OK:
            if h.value:
                self.lib.pmc_store_free(h)
            self._check(st)
        return Store(self, h, streams)

    STATIC_WS_BYTES = 64 << 20  # PMC_STATIC_WS_BYTES

    def compress_static(self, x, taus, streams=None):
        """Alg. 1 without any workspace allocation: the library's static
        per-GPU workspace (fields whose workspace fits STATIC_WS_BYTES).  With
        `streams` given, no device memory is allocated at all."""
        taus = [float(t) for t in taus]
        n = len(taus)
        f = field_of(x)
        if streams is None:
            streams = torch.empty(self.compress_sizes(x, n)[1] * n, dtype=torch.uint8, device=self.device)
        tau_arr = (ctypes.c_double * n)(*taus)
        h = ctypes.c_void_p()
        st = self.lib.pmc_compress_static(self.handle, ctypes.byref(f), ctypes.c_void_p(x.data_ptr()), n, tau_arr,
                                          ctypes.c_void_p(streams.data_ptr()), streams.numel(), ctypes.byref(h))
        if st != OK:
            if h.value:
                self.lib.pmc_store_free(h)
            self._check(st)
        return Store(self, h, streams)

    def retrieve(self, store, k, out=None):
        """Alg. 2: x~_k = sum of the first k decoded components (left to right)."""
        if out is None:
            out = torch.empty(store.shape, dtype=store.dtype, device=self.device)
        self._check(self.lib.pmc_retrieve(self.handle, store.handle, int(k), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(self._dec_ws.data_ptr()), self._dec_ws.numel()))
        return out

    def retrieve_box(self, store, k, lo, hi, out=None):
        """x~_k on the box lo <= (x, y, z) < hi only (Sec. 6.1); returns a
        (z, y, x)-shaped tensor of the box."""
        lo = [int(v) for v in lo]
        hi = [int(v) for v in hi]
        shape = (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])
        if out is None:
            out = torch.empty(shape, dtype=store.dtype, device=self.device)
        elif out.dtype != store.dtype or out.numel() != shape[0] * shape[1] * shape[2] or not out.is_contiguous():
            raise ValueError("out must be a contiguous %s tensor of %s values" % (store.dtype, shape))
        self._check(self.lib.pmc_retrieve_box(self.handle, store.handle, int(k), (ctypes.c_uint64 * 3)(*lo),
                                              (ctypes.c_uint64 * 3)(*hi), ctypes.c_void_p(out.data_ptr()),
                                              ctypes.c_void_p(self._dec_ws.data_ptr()), self._dec_ws.numel()))
        return out

    def refine(self, store, k_from, k_to, xt):
        """Add components k_from+1..k_to to x~_{k_from} in place."""
        self._check(self.lib.pmc_refine(self.handle, store.handle, int(k_from), int(k_to),
                                        ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(self._dec_ws.data_ptr()),
                                        self._dec_ws.numel()))
        return xt

    def batch(self, shapes_dtypes, taus):
        """Plan a batch: shapes_dtypes = [(shape, torch dtype)], taus = [[tau...]]."""
        return Batch(self, shapes_dtypes, taus)

    def deserialize(self, blob, streams=None):
        """Rebuild a store from bytes written by Store.serialize (or any valid blob)."""
        blob = bytes(blob)
        need = ctypes.c_size_t()
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.pmc_store_device_bytes(buf, len(blob), ctypes.byref(need)), ctx=None)
        if streams is None:
            streams = torch.empty(max(need.value, 256), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.pmc_store_deserialize(self.handle, buf, len(blob), ctypes.c_void_p(streams.data_ptr()),
                                                   streams.numel(), ctypes.byref(h)))
        return Store(self, h, streams)


class Batch:
    """Many fields compressed together (one captured HIP graph per call)."""

    def __init__(self, ctx, shapes_dtypes, taus):
        self.ctx = ctx
        self.lib = ctx.lib
        nf = len(shapes_dtypes)
        assert len(taus) == nf
        self.fields = (Field * nf)()
        for i, (shape, dt) in enumerate(shapes_dtypes):
            dims = list(reversed(list(shape))) + [1] * (3 - len(shape))
            self.fields[i].nx, self.fields[i].ny, self.fields[i].nz = dims
            self.fields[i].dtype = _dtype_code(dt)
        self.shapes = [tuple(s) for s, _ in shapes_dtypes]
        self.n = (ctypes.c_int * nf)(*[len(t) for t in taus])
        self._tau_arrays = [(ctypes.c_double * len(t))(*[float(v) for v in t]) for t in taus]
        tau_ptrs = (_P(_dbl) * nf)(*[ctypes.cast(a, _P(_dbl)) for a in self._tau_arrays])
        h = ctypes.c_void_p()
        ctx._check(self.lib.pmc_batch_plan(ctx.handle, nf, self.fields, self.n, tau_ptrs, ctypes.byref(h)))
        self.handle = h
        ws, st = ctypes.c_size_t(), ctypes.c_size_t()
        self.lib.pmc_batch_sizes(h, ctypes.byref(ws), ctypes.byref(st))
        self.ws = torch.empty(max(ws.value, 256), dtype=torch.uint8, device=ctx.device)
        self.streams = torch.empty(max(st.value, 256), dtype=torch.uint8, device=ctx.device)
        self.nf = nf

    def _ptrs(self, xs):
        assert len(xs) == self.nf
        for i, x in enumerate(xs):
            f = field_of(x)
            g = self.fields[i]
            if (f.nx, f.ny, f.nz, f.dtype) != (g.nx, g.ny, g.nz, g.dtype):
                raise ValueError("field %d does not match the plan" % i)
        return (_vp * self.nf)(*[x.data_ptr() for x in xs])

    def schedule(self, grid_mult=None, order=None):
        gm, od = ctypes.c_int(), ctypes.c_int()
        self.lib.pmc_batch_get_schedule(self.handle, ctypes.byref(gm), ctypes.byref(od))
        if grid_mult is not None or order is not None:
            gm.value = gm.value if grid_mult is None else grid_mult
            od.value = od.value if order is None else order
            self.ctx._check(self.lib.pmc_batch_schedule(self.handle, gm.value, od.value))
        return gm.value, od.value

    def tune(self, xs):
        ms = ctypes.c_float()
        self.ctx._check(self.lib.pmc_batch_tune(self.handle, self._ptrs(xs), ctypes.c_void_p(self.ws.data_ptr()),
                                                self.ws.numel(), ctypes.c_void_p(self.streams.data_ptr()),
                                                self.streams.numel(), ctypes.byref(ms)))
        return self.schedule() + (ms.value,)

    def compress(self, xs, streams=None):
        """Returns one Store per field; their streams share one device buffer
        (a fresh one per call unless `streams` is given)."""
        if streams is None:
            streams = torch.empty_like(self.streams)
        outs = (_vp * self.nf)()
        st = self.lib.pmc_batch_compress(self.handle, self._ptrs(xs), ctypes.c_void_p(self.ws.data_ptr()),
                                         self.ws.numel(), ctypes.c_void_p(streams.data_ptr()), streams.numel(),
                                         outs)
        if st != OK:
            for o in outs:
                if o:
                    self.lib.pmc_store_free(ctypes.c_void_p(o))
            self.ctx._check(st)
        return [Store(self.ctx, ctypes.c_void_p(o), streams) for o in outs]

    def free(self):
        if getattr(self, "handle", None):
            self.lib.pmc_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Progressive-retrieval server with a device-resident partial-sum cache
    and continuous batching (request loop on a library thread)."""

    def __init__(self, ctx, arena_bytes, budget_bytes=None, max_batch=64):
        self.ctx = ctx
        self.lib = ctx.lib
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=ctx.device)
        budget = int(budget_bytes if budget_bytes is not None else arena_bytes)
        h = ctypes.c_void_p()
        ctx._check(self.lib.pmc_server_create(ctx.handle, budget, ctypes.c_void_p(self.arena.data_ptr()),
                                              self.arena.numel(), int(max_batch), ctypes.byref(h)))
        self.handle = h
        self.stores = []
        self._outs = {}  # ticket -> caller output tensor of a query not yet done

    def add(self, store):
        fid = ctypes.c_int()
        self.ctx._check(self.lib.pmc_server_add(self.handle, store.handle, ctypes.byref(fid)))
        self.stores.append(store)
        return fid.value

    def submit(self, field, tol, out=None, arrival=None):
        """Queue "field at tolerance tol"; returns a ticket.  With `out` (a
        device tensor of the field's shape and type) the result is written
        there: the server keeps a reference to `out` until poll() reports the
        query done or release() is called, so the caching allocator cannot
        hand its memory to another tensor while the server still writes it.
        `arrival` (seconds on clock()) is the time the latency counts from,
        e.g. a trace's scheduled arrival; default: now."""
        t = ctypes.c_uint64()
        ptr = ctypes.c_void_p(out.data_ptr()) if out is not None else None
        self.ctx._check(self.lib.pmc_server_submit_at(self.handle, int(field), float(tol), ptr,
                                                      float(arrival or 0.0), ctypes.byref(t)))
        if out is not None:
            self._outs[t.value] = out
        return t.value

    def poll(self, ticket):
        """(done, status, latency_s)"""
        d, st, lat = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self.ctx._check(self.lib.pmc_server_poll(self.handle, int(ticket), ctypes.byref(d), ctypes.byref(st),
                                                 ctypes.byref(lat)))
        if d.value:
            self._outs.pop(int(ticket), None)
        return bool(d.value), st.value, lat.value

    def result(self, ticket, field):
        """(x~_k as a device tensor view, k, source); valid until release()."""
        p, k, src = ctypes.c_void_p(), ctypes.c_int(), ctypes.c_int()
        self.ctx._check(self.lib.pmc_server_result(self.handle, int(ticket), ctypes.byref(p), ctypes.byref(k),
                                                   ctypes.byref(src)))
        st = self.stores[field]
        nbytes = int(np_prod(st.shape)) * (4 if st.dtype == torch.float32 else 8)
        off = p.value - self.arena.data_ptr()
        if 0 <= off < self.arena.numel():
            view = self.arena[off:off + nbytes].view(st.dtype).view(st.shape)
        else:
            view = None  # caller-owned output
        return view, k.value, src.value

    def release(self, ticket):
        self.ctx._check(self.lib.pmc_server_release(self.handle, int(ticket)))
        self._outs.pop(int(ticket), None)

    def cancel(self, ticket):
        """Cancel a query: a waiting one never runs; a running one finishes on
        the device and its result is dropped when its step ends.  poll() then
        reports it done with status E_CANCELLED (the caller's `out` stays
        referenced until then)."""
        self.ctx._check(self.lib.pmc_server_cancel(self.handle, int(ticket)))

    def stats(self):
        s = ServerStats()
        self.lib.pmc_server_get_stats(self.handle, ctypes.byref(s))
        return {n: getattr(s, n) for n, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pmc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def clock():
    """Seconds on the library's monotonic clock (server latencies use it)."""
    return load().pmc_clock()


def np_prod(shape):
    p = 1
    for v in shape:
        p *= int(v)
    return p


class Store:
    """Handle of a pmc_store plus the device buffer that holds its streams."""

    def __init__(self, ctx, handle, streams):
        self.ctx = ctx
        self.lib = ctx.lib
        self.handle = handle
        self.streams = streams  # keeps the caller-owned stream memory alive
        f = Field()
        ctx._check(self.lib.pmc_store_field(handle, ctypes.byref(f)))
        self.field = f
        shape = [f.nz, f.ny, f.nx]
        self.shape = tuple(int(s) for s in shape)
        self.dtype = _torch_dtype(f.dtype)
        self.bound_missed = False
        self._info_cache = None  # per-component metadata, read on first use

    @property
    def info(self):
        """Per-component metadata (a list of dicts), read from the library on
        first use (a batch returns many stores; most callers read few)."""
        if self._info_cache is None:
            self._info_cache = self._info()
        return self._info_cache

    @property
    def codec(self):
        c = ctypes.c_int()
        self.ctx._check(self.lib.pmc_store_codec(self.handle, ctypes.byref(c)))
        return c.value

    def _info(self):
        n = ctypes.c_int()
        self.lib.pmc_store_info(self.handle, ctypes.byref(n), None, None, None, None, None)
        k = n.value
        tau, linf = (ctypes.c_double * k)(), (ctypes.c_double * k)()
        by, raw, esc = (ctypes.c_uint64 * k)(), (ctypes.c_uint64 * k)(), (ctypes.c_uint64 * k)()
        self.lib.pmc_store_info(self.handle, ctypes.byref(n), tau, linf, by, raw, esc)
        out = []
        for i in range(k):
            c = (ctypes.c_uint64 * 5)()
            self.lib.pmc_store_counts(self.handle, i, c)
            span, staged = ctypes.c_uint64(), ctypes.c_int()
            self.lib.pmc_store_span(self.handle, i, ctypes.byref(span), ctypes.byref(staged))
            hh = ctypes.c_int()
            self.lib.pmc_store_decode_route(self.handle, i, ctypes.byref(hh))
            out.append(dict(tau=tau[i], linf=linf[i], bytes=by[i], nempty=c[0], ncoded=c[1], nraw=c[2],
                            nesc=c[3], nmiss=c[4], max_span=span.value, staged=bool(staged.value),
                            high_half=bool(hh.value)))
        return out

    @property
    def n(self):
        return len(self.info)

    def select_k(self, tol, use_measured=False):
        k = ctypes.c_int()
        st = self.lib.pmc_select_k(self.handle, float(tol), int(bool(use_measured)), ctypes.byref(k))
        if st == E_UNREACHABLE:
            return None
        self.ctx._check(st)
        return k.value

    def stream(self, i):
        """Bytes of component i's stream as a uint8 device tensor view."""
        p, nb = ctypes.c_void_p(), ctypes.c_uint64()
        self.ctx._check(self.lib.pmc_store_stream(self.handle, int(i), ctypes.byref(p), ctypes.byref(nb)))
        off = p.value - self.streams.data_ptr()
        return self.streams[off:off + nb.value]

    def serialize(self):
        used = ctypes.c_size_t()
        self.ctx._check(self.lib.pmc_store_serialize(self.ctx.handle, self.handle, None, 0, ctypes.byref(used)))
        buf = ctypes.create_string_buffer(used.value)
        self.ctx._check(self.lib.pmc_store_serialize(self.ctx.handle, self.handle, buf, used.value,
                                                     ctypes.byref(used)))
        return buf.raw[:used.value]

    def free(self):
        if getattr(self, "handle", None):
            self.lib.pmc_store_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
