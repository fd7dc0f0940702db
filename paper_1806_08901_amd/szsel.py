"""Thin ctypes binding of libszsel.so (the C ABI of include/szsel.h).

Argument marshalling only: every step of the estimator runs in the HIP
kernels.  PyTorch supplies device memory (``tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  There is no CPU fallback: if
the library is not built or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libszsel.so")

F32, F64 = 0, 1
EB_ABS, EB_REL = 0, 1
OP_SZ, OP_ZFP, OP_SELECT, OP_FIXED_EB = 0, 1, 2, 3
FLAG_CONSTANT, FLAG_NONFINITE, FLAG_ZERO_MSE = 1, 2, 4
FLAG_EB_EXCEEDS, FLAG_NO_BLOCKS, FLAG_BAD_EB, FLAG_NO_HUFFMAN = 8, 16, 32, 64
FLAG_EC_SAMPLED, FLAG_FAILED = 128, 256
OPT_SZ_OFFSET, OPT_PROFILE, OPT_AUTOTUNE, OPT_BATCH_GRAPH = 1, 2, 3, 4
OPT_SZ_WGS, OPT_ZFP_CHUNK, OPT_RANGE_WGS, OPT_BATCH_GROUPS, OPT_HUFFMAN = 5, 6, 7, 8, 9
OPT_EC_SAMPLING, OPT_BATCH_SHARE, OPT_RANGE_GRID, OPT_BATCH_LANES = 10, 11, 12, 13
NBINS = 65536


class SzselError(RuntimeError):
    pass


class Result(C.Structure):
    _fields_ = [
        ("flags", C.c_uint32), ("choice", C.c_int32),
        ("vmin", C.c_double), ("vmax", C.c_double), ("vr", C.c_double), ("eb_abs", C.c_double),
        ("minexp", C.c_int32), ("pad0", C.c_int32),
        ("zfp_bitrate", C.c_double), ("zfp_mse", C.c_double), ("zfp_psnr", C.c_double),
        ("zfp_nsb_mean", C.c_double), ("zfp_maxerr", C.c_double), ("zfp_sse", C.c_double),
        ("zfp_bits", C.c_uint64), ("zfp_values", C.c_uint64), ("zfp_blocks", C.c_uint64),
        ("zfp_nsb_total", C.c_uint64),
        ("sz_delta", C.c_double), ("sz_inv_delta", C.c_double), ("sz_eb", C.c_double),
        ("sz_entropy", C.c_double), ("sz_bitrate", C.c_double),
        ("sz_psnr_model", C.c_double), ("sz_psnr_measured", C.c_double), ("sz_mse", C.c_double),
        ("sz_maxerr", C.c_double), ("sz_sse", C.c_double),
        ("sz_values", C.c_uint64), ("sz_unpredictable", C.c_uint64),
        ("chosen_eb", C.c_double),
        ("sz_huffman_bits", C.c_uint64), ("sz_huffman_bitrate", C.c_double),
        ("zfp_ec_points", C.c_uint64), ("zfp_ec_nsb2", C.c_uint64),
    ]


class Request(C.Structure):
    _fields_ = [
        ("field", C.c_void_p), ("dims", C.c_int64 * 3), ("ndims", C.c_int32), ("dtype", C.c_int32),
        ("eb", C.c_double), ("eb_mode", C.c_int32), ("op", C.c_int32), ("stride", C.c_int32 * 3),
        ("pad0", C.c_int32),
    ]


class Debug(C.Structure):
    _fields_ = [("codes", C.c_void_p), ("zfp_bits", C.c_void_p), ("zfp_sse", C.c_void_p),
                ("zfp_emax", C.c_void_p), ("sz_sse", C.c_void_p), ("hist", C.c_void_p)]


class Compressed(C.Structure):
    _fields_ = [("bits", C.c_uint64), ("values", C.c_uint64), ("blocks", C.c_uint64),
                ("bitrate", C.c_double), ("sse", C.c_double), ("mse", C.c_double), ("psnr", C.c_double),
                ("maxerr", C.c_double), ("vr", C.c_double), ("eb_abs", C.c_double),
                ("unpredictable", C.c_uint64), ("symbols", C.c_uint64), ("code_bits", C.c_uint64),
                ("code_entropy", C.c_double), ("flags", C.c_uint32), ("pad", C.c_int32)]


RESULT_KEYS = [name for name, _ in Result._fields_ if name != "pad0"]
_SINGLE = ("szsel_estimate_sz", "szsel_estimate_zfp", "szsel_select", "szsel_select_fixed_eb")
EXPORTS = _SINGLE + ("szsel_create", "szsel_destroy", "szsel_select_batch", "szsel_last_error",
                     "szsel_stride_for_rate", "szsel_set_option", "szsel_set_debug",
                     "szsel_profile_read", "szsel_profile_read_split", "szsel_server_create", "szsel_server_destroy",
                     "szsel_server_reserve", "szsel_server_cancel", "szsel_server_submit",
                     "szsel_server_progress", "szsel_server_status", "szsel_server_stats",
                     "szsel_server_last_error", "szsel_zfp_stream_bytes", "szsel_zfp_compress",
                     "szsel_sz_compress", "szsel_select_noalloc")

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libszsel.so and declares its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SzselError("libszsel.so is not built (run __graft_entry__.build()); "
                         "there is no CPU fallback")
    L = C.CDLL(path)
    P, I64P, I32P = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)
    L.szsel_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_size_t]
    L.szsel_destroy.argtypes = [P]
    L.szsel_destroy.restype = None
    for name in _SINGLE:
        getattr(L, name).argtypes = [P, P, I64P, C.c_int, C.c_int, C.c_double, C.c_int, I32P,
                                     C.POINTER(Result), P]
    L.szsel_select_noalloc.argtypes = [P, P, I64P, C.c_int, C.c_int, C.c_double, C.c_int, I32P,
                                       C.POINTER(Result), P]
    L.szsel_select_batch.argtypes = [P, C.POINTER(Request), C.c_int, C.POINTER(Result), P]
    L.szsel_last_error.argtypes = [P]
    L.szsel_last_error.restype = C.c_char_p
    L.szsel_stride_for_rate.argtypes = [C.c_double, C.c_int, I64P, I32P]
    L.szsel_set_option.argtypes = [P, C.c_int, C.c_double]
    L.szsel_set_debug.argtypes = [P, C.POINTER(Debug)]
    L.szsel_profile_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    L.szsel_profile_read_split.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    L.szsel_server_create.argtypes = [C.POINTER(C.c_void_p), P, P, C.c_size_t, C.c_int, C.c_size_t]
    L.szsel_server_destroy.argtypes = [P]
    L.szsel_server_destroy.restype = None
    L.szsel_server_reserve.argtypes = [P, C.c_size_t, C.POINTER(C.c_void_p), C.POINTER(C.c_uint64)]
    L.szsel_server_cancel.argtypes = [P, C.c_uint64]
    L.szsel_server_submit.argtypes = [P, C.c_uint64, C.POINTER(Request), C.c_int, C.POINTER(Result), P]
    L.szsel_server_progress.argtypes = [P, C.c_int]
    L.szsel_server_status.argtypes = [P, C.c_uint64, C.POINTER(C.c_double)]
    L.szsel_server_stats.argtypes = [P, C.POINTER(C.c_uint64)]
    L.szsel_server_last_error.argtypes = [P]
    L.szsel_server_last_error.restype = C.c_char_p
    L.szsel_zfp_stream_bytes.argtypes = [I64P, C.c_int, C.c_int]
    L.szsel_zfp_stream_bytes.restype = C.c_size_t
    L.szsel_zfp_compress.argtypes = [P, P, I64P, C.c_int, C.c_int, C.c_double, P, C.c_size_t, P,
                                     C.POINTER(Compressed), P]
    L.szsel_sz_compress.argtypes = [P, P, I64P, C.c_int, C.c_int, C.c_double, P, P,
                                    C.POINTER(Compressed), P]
    _lib = L
    return L


def stride_for_rate(r_sp: float, shape) -> tuple:
    L = load_library()
    nd = len(shape)
    dims = (C.c_int64 * nd)(*shape)
    out = (C.c_int32 * nd)()
    rc = L.szsel_stride_for_rate(float(r_sp), nd, dims, out)
    if rc != 0:
        raise SzselError("szsel_stride_for_rate rejected r_sp=%r shape=%r" % (r_sp, shape))
    return tuple(out)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise SzselError("fields are float32 or float64, got %s" % t.dtype)


def _as_dict(r: Result) -> dict:
    return {k: getattr(r, k) for k in RESULT_KEYS}


class Context:
    """One szsel context on one HIP device (not thread-safe)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        if not torch.cuda.is_available():
            raise SzselError("no HIP device available; the estimator runs only on the GPU")
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.szsel_create(C.byref(h), device, budget_bytes)
        if rc != 0:
            raise SzselError("szsel_create failed with %d" % rc)
        self.h = h
        self._pinned = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.szsel_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers -----------------------------------------------------------
    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.szsel_last_error(self.h).decode()
            raise SzselError("%s failed (%d): %s" % (what, rc, msg))

    def _results(self, n: int):
        """Pinned host buffer for n results (reused)."""
        buf = self._pinned.get(n)
        if buf is None:
            t = torch.empty(n * C.sizeof(Result), dtype=torch.uint8, pin_memory=True)
            buf = (t, (Result * n).from_address(t.data_ptr()))
            self._pinned[n] = buf
        return buf[1]

    @staticmethod
    def _stream(stream):
        s = stream if stream is not None else torch.cuda.current_stream()
        return s, C.c_void_p(s.cuda_stream)

    def set_option(self, option: int, value: float):
        self._check(self.lib.szsel_set_option(self.h, option, float(value)), "szsel_set_option")

    PHASES = ("range", "zfp", "sz", "ovf", "ent")

    def profile_read(self):
        """Per-phase GPU milliseconds and call counts since the last read:
        {"range": (ms, n), "zfp": ..., "sz": ..., "ovf": ..., "ent": ...}."""
        ms = (C.c_double * 5)()
        n = (C.c_uint64 * 5)()
        self._check(self.lib.szsel_profile_read(self.h, ms, n), "szsel_profile_read")
        return {k: (ms[i], n[i]) for i, k in enumerate(self.PHASES)}

    def profile_read_split(self):
        """As profile_read, split by field dtype: {("range", "f32"): (ms, n), ...}."""
        ms = (C.c_double * 10)()
        n = (C.c_uint64 * 10)()
        self._check(self.lib.szsel_profile_read_split(self.h, ms, n), "szsel_profile_read_split")
        return {(k, dt): (ms[2 * i + d], n[2 * i + d]) for i, k in enumerate(self.PHASES)
                for d, dt in enumerate(("f32", "f64"))}

    def set_debug(self, dbg: dict | None):
        """Arms per-sample dumps for the next single call.  ``dbg`` maps the
        names of szsel_debug to device tensors."""
        if dbg is None:
            self._check(self.lib.szsel_set_debug(self.h, None), "szsel_set_debug")
            return
        d = Debug(*[dbg[k].data_ptr() if dbg.get(k) is not None else None
                    for k, _ in Debug._fields_])
        self._check(self.lib.szsel_set_debug(self.h, C.byref(d)), "szsel_set_debug")

    # -- single requests ---------------------------------------------------
    def run(self, op: int, field: torch.Tensor, eb: float, eb_mode: int = EB_REL, stride=None,
            stream=None, sync: bool = True):
        if not field.is_cuda or not field.is_contiguous():
            raise SzselError("field must be a contiguous device tensor")
        nd = field.dim()
        dims = (C.c_int64 * nd)(*field.shape)
        st = None if stride is None else (C.c_int32 * nd)(*stride)
        out = self._results(1)
        s, sp = self._stream(stream)
        fn = getattr(self.lib, _SINGLE[op])
        self._check(fn(self.h, C.c_void_p(field.data_ptr()), dims, nd, _dtype_code(field),
                       float(eb), eb_mode, st, out, sp), _SINGLE[op])
        if not sync:
            return out
        s.synchronize()
        return _as_dict(out[0])

    def estimate_sz(self, field, eb, eb_mode=EB_REL, stride=None, stream=None):
        return self.run(OP_SZ, field, eb, eb_mode, stride, stream)

    def estimate_zfp(self, field, eb, eb_mode=EB_REL, stride=None, stream=None):
        return self.run(OP_ZFP, field, eb, eb_mode, stride, stream)

    def select(self, field, eb, eb_mode=EB_REL, stride=None, stream=None):
        return self.run(OP_SELECT, field, eb, eb_mode, stride, stream)

    def select_fixed_eb(self, field, eb, eb_mode=EB_REL, stride=None, stream=None):
        return self.run(OP_FIXED_EB, field, eb, eb_mode, stride, stream)

    def select_noalloc(self, field: torch.Tensor, eb: float, eb_mode: int = EB_REL, stride=None,
                       stream=None, sync: bool = True):
        """szsel_select_noalloc: Algorithm 1 with the workspace in the
        library's static device array (allocates nothing; calls that may
        overlap on the device race)."""
        if not field.is_cuda or not field.is_contiguous():
            raise SzselError("field must be a contiguous device tensor")
        nd = field.dim()
        dims = (C.c_int64 * nd)(*field.shape)
        st = None if stride is None else (C.c_int32 * nd)(*stride)
        out = self._results(1)
        s, sp = self._stream(stream)
        self._check(self.lib.szsel_select_noalloc(self.h, C.c_void_p(field.data_ptr()), dims, nd,
                                                  _dtype_code(field), float(eb), eb_mode, st, out, sp),
                    "szsel_select_noalloc")
        if not sync:
            return out
        s.synchronize()
        return _as_dict(out[0])

    # -- Step 4: compression of the whole field -----------------------------
    def zfp_compress(self, field: torch.Tensor, eb_abs: float, decoded: bool = True, stream=None):
        """ZFP fixed-accuracy compression of the whole field at eb_abs.
        Returns (result dict, stream words as an int64 device tensor of
        ceil(bits / 64) words, decompressed field or None)."""
        if not field.is_cuda or not field.is_contiguous():
            raise SzselError("field must be a contiguous device tensor")
        nd = field.dim()
        dims = (C.c_int64 * nd)(*field.shape)
        nbytes = self.lib.szsel_zfp_stream_bytes(dims, nd, _dtype_code(field))
        if nbytes == 0:
            raise SzselError("szsel_zfp_stream_bytes rejected the shape")
        buf = torch.empty(nbytes // 8, dtype=torch.int64, device=field.device)
        dec = torch.empty_like(field) if decoded else None
        out = Compressed()
        s, sp = self._stream(stream)
        self._check(self.lib.szsel_zfp_compress(self.h, C.c_void_p(field.data_ptr()), dims, nd,
                                                _dtype_code(field), float(eb_abs),
                                                C.c_void_p(buf.data_ptr()), nbytes,
                                                C.c_void_p(dec.data_ptr()) if dec is not None else None,
                                                C.byref(out), sp), "szsel_zfp_compress")
        res = {name: getattr(out, name) for name, _ in Compressed._fields_ if name != "pad"}
        return res, buf[: (res["bits"] + 63) // 64], dec

    def sz_compress(self, field: torch.Tensor, eb_abs: float, decoded: bool = True, symbols: bool = False,
                    stream=None):
        """SZ compression of the whole field at eb_abs (quantize first, then
        the integer Lorenzo predictor).  Returns (result dict, symbols as an
        int16 device tensor or None, decompressed field or None)."""
        if not field.is_cuda or not field.is_contiguous():
            raise SzselError("field must be a contiguous device tensor")
        nd = field.dim()
        dims = (C.c_int64 * nd)(*field.shape)
        dec = torch.empty_like(field) if decoded else None
        sym = torch.empty(field.shape, dtype=torch.int16, device=field.device) if symbols else None
        out = Compressed()
        s, sp = self._stream(stream)
        self._check(self.lib.szsel_sz_compress(self.h, C.c_void_p(field.data_ptr()), dims, nd,
                                               _dtype_code(field), float(eb_abs),
                                               C.c_void_p(sym.data_ptr()) if sym is not None else None,
                                               C.c_void_p(dec.data_ptr()) if dec is not None else None,
                                               C.byref(out), sp), "szsel_sz_compress")
        res = {name: getattr(out, name) for name, _ in Compressed._fields_ if name != "pad"}
        return res, sym, dec

    # -- batches -----------------------------------------------------------
    def make_requests(self, items):
        """items: iterable of (tensor, eb, eb_mode, stride, op)."""
        items = list(items)
        reqs = (Request * len(items))()
        for q, (t, eb, mode, stride, op) in zip(reqs, items):
            if not t.is_cuda or not t.is_contiguous():
                raise SzselError("fields must be contiguous device tensors")
            q.field = t.data_ptr()
            for k, n in enumerate(t.shape):
                q.dims[k] = n
            q.ndims = t.dim()
            q.dtype = _dtype_code(t)
            q.eb = float(eb)
            q.eb_mode = mode
            q.op = op
            for k in range(t.dim()):
                q.stride[k] = 1 if stride is None else int(stride[k])
        return reqs

    def result_buffer(self, n: int):
        """A pinned array of n Result for asynchronous calls."""
        t = torch.empty(max(1, n) * C.sizeof(Result), dtype=torch.uint8, pin_memory=True)
        out = (Result * n).from_address(t.data_ptr())
        out._owner = t
        return out

    def select_batch(self, items, stream=None, sync: bool = True, reqs=None, out=None):
        """Runs the requests as one batch.  With sync=False the call returns
        `out` (or a fresh pinned array of Result), filled once the stream
        reaches it."""
        if reqs is None:
            reqs = self.make_requests(items)
        n = len(reqs)
        if out is not None:
            pass
        elif sync:
            out = self._results(n)
        else:
            out = self.result_buffer(n)
        s, sp = self._stream(stream)
        self._check(self.lib.szsel_select_batch(self.h, reqs, n, out, sp), "szsel_select_batch")
        if not sync:
            return out
        s.synchronize()
        return [_as_dict(out[i]) for i in range(n)]


class Server:
    """Continuous-batching serving engine (szsel_server_*): snapshots are
    admitted by reserving their bytes in `pool` (a device uint8 tensor the
    caller owns), written there by the producer, then submitted.

    With ctx=None only the admission calls work (bookkeeping, no device):
    pass pool_bytes and no pool."""

    STATS = ("batches", "batched_requests", "snapshots_done", "waiting_requests", "busy_lanes",
             "pool_reserved", "pool_bytes", "largest_free")

    def __init__(self, ctx=None, pool=None, lanes: int = 4, lane_workspace_bytes: int = 0,
                 pool_bytes: int = None):
        self.lib = load_library()
        self.ctx = ctx
        self.pool = pool
        base = pool.data_ptr() if pool is not None else 0
        nbytes = pool.numel() * pool.element_size() if pool is not None else int(pool_bytes or 0)
        self.base = base
        h = C.c_void_p()
        rc = self.lib.szsel_server_create(C.byref(h), ctx.h if ctx is not None else None,
                                          C.c_void_p(base) if base else None, nbytes,
                                          lanes if ctx is not None else 0, lane_workspace_bytes)
        if rc != 0:
            raise SzselError("szsel_server_create failed with %d" % rc)
        self.h = h
        self._outs = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.szsel_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self):
        return self.lib.szsel_server_last_error(self.h).decode()

    def reserve(self, nbytes: int):
        """(offset in the pool, ticket), or None while the pool lacks room."""
        p = C.c_void_p()
        t = C.c_uint64()
        rc = self.lib.szsel_server_reserve(self.h, int(nbytes), C.byref(p), C.byref(t))
        if rc == -5:  # SZSEL_EBUSY
            return None
        if rc != 0:
            raise SzselError("szsel_server_reserve failed (%d): %s" % (rc, self._err()))
        return (p.value or 0) - self.base, t.value

    def cancel(self, ticket: int):
        rc = self.lib.szsel_server_cancel(self.h, ticket)
        if rc != 0:
            raise SzselError("szsel_server_cancel failed (%d): %s" % (rc, self._err()))

    def submit(self, ticket: int, items, stream=None):
        reqs = self.ctx.make_requests(items)
        n = len(reqs)
        out = (Result * n)()
        self._outs[ticket] = out
        sp = C.c_void_p(stream.cuda_stream) if stream is not None else None
        rc = self.lib.szsel_server_submit(self.h, ticket, reqs, n, out, sp)
        if rc != 0:
            raise SzselError("szsel_server_submit failed (%d): %s" % (rc, self._err()))

    def progress(self, wait: bool = False) -> int:
        rc = self.lib.szsel_server_progress(self.h, 1 if wait else 0)
        if rc < 0:
            raise SzselError("szsel_server_progress failed (%d): %s" % (rc, self._err()))
        return rc

    def status(self, ticket: int):
        """None while the snapshot runs; else (results, submit-to-done ms)."""
        lat = C.c_double()
        rc = self.lib.szsel_server_status(self.h, ticket, C.byref(lat))
        if rc < 0:
            raise SzselError("szsel_server_status failed (%d): %s" % (rc, self._err()))
        if rc == 0:
            return None
        out = self._outs.pop(ticket)
        return [_as_dict(out[i]) for i in range(len(out))], lat.value

    def stats(self) -> dict:
        v = (C.c_uint64 * 8)()
        self.lib.szsel_server_stats(self.h, v)
        return {k: int(v[i]) for i, k in enumerate(self.STATS)}
