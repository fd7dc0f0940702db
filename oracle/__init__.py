"""ctypes front end of the plain CPU oracle (``szsel_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The product package never imports it.

The oracle follows arXiv:1806.08901 (Algorithm 1 with Sections 4 and 5) step by
step in FP64; the conventions the paper leaves open are stated in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "szsel_oracle.c")
_LIB = os.path.join(_HERE, "libszsel_oracle.so")

OP_SZ, OP_ZFP, OP_SELECT, OP_FIXED_EB = 0, 1, 2, 3
EB_ABS, EB_REL = 0, 1
F32, F64 = 0, 1
FLAG_CONSTANT, FLAG_NONFINITE, FLAG_ZERO_MSE = 1, 2, 4
FLAG_EB_EXCEEDS, FLAG_NO_BLOCKS, FLAG_BAD_EB = 8, 16, 32
FLAG_EC_SAMPLED = 128
NBINS = 65536


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


class Step4(C.Structure):
    _fields_ = [
        ("bits", C.c_uint64), ("values", C.c_uint64), ("blocks", C.c_uint64),
        ("bitrate", C.c_double), ("sse", C.c_double), ("mse", C.c_double), ("psnr", C.c_double),
        ("maxerr", C.c_double), ("vr", C.c_double), ("eb_abs", C.c_double),
        ("unpredictable", C.c_uint64), ("symbols", C.c_uint64), ("code_bits", C.c_uint64),
        ("code_entropy", C.c_double),
    ]


class Dump(C.Structure):
    _fields_ = [
        ("codes", C.c_void_p), ("zfp_bits", C.c_void_p), ("zfp_sse", C.c_void_p),
        ("zfp_emax", C.c_void_p), ("sz_sse", C.c_void_p), ("hist", C.c_void_p),
        ("ec_nsb2", C.c_void_p), ("ec_err", C.c_void_p),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P, I64P, I32P = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        L.orc_run.argtypes = [C.c_int, P, I64P, C.c_int, C.c_int, C.c_double, C.c_int, I32P,
                              C.c_double, C.c_int, C.c_int, C.c_int, C.POINTER(Result), C.POINTER(Dump)]
        L.orc_zfp_compress.argtypes = [P, I64P, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_uint8),
                                       C.c_int64, C.POINTER(C.c_double), C.POINTER(Step4)]
        L.orc_sz_compress.argtypes = [P, I64P, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_uint32),
                                      C.POINTER(C.c_uint16), C.POINTER(C.c_double), C.POINTER(Step4)]
        L.orc_zfp_num_blocks.argtypes = [I64P, C.c_int]
        L.orc_zfp_num_blocks.restype = C.c_int64
        L.orc_ec_gain.argtypes = [C.c_int, C.c_int]
        L.orc_ec_gain.restype = C.c_double
        L.orc_ec_default_points.argtypes = [C.c_int]
        L.orc_ec_positions.argtypes = [C.c_int, C.c_int, I32P]
        L.orc_zfp_block_ec.argtypes = [C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]
        L.orc_range.argtypes = [P, C.c_int64, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_num_sampled_blocks.argtypes = [I64P, C.c_int, I32P]
        L.orc_num_sampled_blocks.restype = C.c_int64
        L.orc_sampled_block_origin.argtypes = [I64P, C.c_int, I32P, C.c_int64, I64P]
        L.orc_frexp_exponent.argtypes = [C.c_double]
        L.orc_floor_log2.argtypes = [C.c_double]
        L.orc_precision.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        for f in ("orc_fwd_lift", "orc_inv_lift"):
            getattr(L, f).argtypes = [I64P, C.c_ssize_t, C.c_int]
        for f in ("orc_fwd_xform", "orc_inv_xform"):
            getattr(L, f).argtypes = [I64P, C.c_int, C.c_int]
        L.orc_reorder_table.argtypes = [C.c_int, I32P]
        L.orc_to_negabinary.argtypes = [C.c_int64, C.c_int]
        L.orc_to_negabinary.restype = C.c_uint64
        L.orc_from_negabinary.argtypes = [C.c_uint64, C.c_int]
        L.orc_from_negabinary.restype = C.c_int64
        L.orc_encode_planes.argtypes = [C.POINTER(C.c_uint64), C.c_int, C.c_int, C.c_int,
                                        C.POINTER(C.c_uint8), C.c_int64]
        L.orc_encode_planes.restype = C.c_int64
        L.orc_zfp_block.argtypes = [C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_uint64), C.POINTER(C.c_int32)]
        L.orc_zfp_block.restype = C.c_uint32
        L.orc_lorenzo.argtypes = [P, I64P, C.c_int, C.c_int, I64P]
        L.orc_lorenzo.restype = C.c_double
        L.orc_tree_sum.argtypes = [C.POINTER(C.c_double), C.c_int64]
        L.orc_tree_sum.restype = C.c_double
        L.orc_entropy.argtypes = [C.POINTER(C.c_uint32), C.c_int64, C.c_uint64]
        L.orc_entropy.restype = C.c_double
        L.orc_huffman_bits.argtypes = [C.POINTER(C.c_uint32), C.c_int64]
        L.orc_huffman_bits.restype = C.c_uint64
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float32:
        return F32
    if a.dtype == np.float64:
        return F64
    raise TypeError("oracle fields are float32 or float64, got %s" % a.dtype)


def result_dict(r: Result) -> dict:
    return {name: getattr(r, name) for name, _ in Result._fields_ if name != "pad0"}


def run(op: int, field: np.ndarray, eb: float, eb_mode: int = EB_REL, stride=None,
        sz_offset: float = 0.5, dump: bool = False, huffman: int = 0, ec_points: int = 0,
        ec_weight: int = 0):
    """Run the estimator on a C-order numpy field.  Returns (result dict, dump dict|None).

    ec_points: 0 = exact ZFP estimate; 1 = the paper's point sub-sampling
    (3/9/16 points per 1/2/3-D block); r >= 2 = r points per block.
    ec_weight: 1 = weight each sub-sampled squared error by its coefficient's
    data-domain gain under the inverse transform."""
    field = np.ascontiguousarray(field)
    nd = field.ndim
    dims = np.array(field.shape, dtype=np.int64)
    st = np.array(stride if stride is not None else [1] * nd, dtype=np.int32)
    if st.shape != (nd,):
        raise ValueError("stride needs one entry per axis")
    out = Result()
    dp = None
    arrays = None
    if dump:
        nblk = num_sampled_blocks(field.shape, st)
        size = 4 ** nd
        arrays = {
            "codes": np.zeros(nblk * size, np.uint16),
            "zfp_bits": np.zeros(nblk, np.uint32),
            "zfp_sse": np.zeros(nblk, np.float64),
            "zfp_emax": np.zeros(nblk, np.int32),
            "sz_sse": np.zeros(nblk, np.float64),
            "hist": np.zeros(NBINS, np.uint32),
            "ec_nsb2": np.zeros(nblk, np.uint32),
            "ec_err": np.zeros(nblk * ec_slots(nd, ec_points), np.float64),
        }
        dp = Dump(*[arrays[k].ctypes.data for k, _ in Dump._fields_])
    rc = lib().orc_run(op, field.ctypes.data, _ptr(dims, C.c_int64), nd, _dtype_code(field),
                       float(eb), eb_mode, _ptr(st, C.c_int32), float(sz_offset), int(huffman),
                       int(ec_points), int(ec_weight), C.byref(out),
                       C.byref(dp) if dp is not None else None)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return result_dict(out), arrays


def select(field, eb, eb_mode=EB_REL, stride=None, sz_offset=0.5, dump=False, huffman=0, ec_points=0,
           ec_weight=0):
    return run(OP_SELECT, field, eb, eb_mode, stride, sz_offset, dump, huffman, ec_points, ec_weight)


def ec_points_per_block(nd: int, ec_points: int) -> int:
    """Sub-sampled points per block for an ec_points argument (0: none)."""
    return int(lib().orc_ec_default_points(nd)) if ec_points == 1 else int(ec_points)


def ec_slots(nd: int, ec_points: int) -> int:
    """Dump slots per block: the points rounded up to a power of two (1 when off)."""
    r = ec_points_per_block(nd, ec_points)
    R = 1
    while R < r:
        R *= 2
    return R


def ec_positions(size: int, r: int):
    pos = np.zeros(r, np.int32)
    lib().orc_ec_positions(size, r, pos.ctypes.data_as(C.POINTER(C.c_int32)))
    return pos


def zfp_block_ec(x, nd: int, dtype: int, minexp: int, r: int):
    """(twice the interpolated significant bits, significant bits of the r
    points, scaled errors in R slots, their gains, emax) of one block."""
    xb = np.ascontiguousarray(x, dtype=np.float64)
    R = 1
    while R < r:
        R *= 2
    err = np.zeros(R, np.float64)
    gain = np.zeros(R, np.float64)
    twice, pts, emax = C.c_uint64(), C.c_uint64(), C.c_int32()
    lib().orc_zfp_block_ec(xb.ctypes.data_as(C.POINTER(C.c_double)), nd, dtype, minexp, r,
                           C.byref(twice), C.byref(pts), err.ctypes.data_as(C.POINTER(C.c_double)),
                           gain.ctypes.data_as(C.POINTER(C.c_double)), C.byref(emax))
    return int(twice.value), int(pts.value), err, gain, int(emax.value)


def ec_gain(i: int, nd: int) -> float:
    return float(lib().orc_ec_gain(i, nd))


def huffman_bits(hist) -> int:
    """Total bits of an optimal prefix code for the symbol counts `hist`."""
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    return int(lib().orc_huffman_bits(h.ctypes.data_as(C.POINTER(C.c_uint32)), h.size))


# ---- pieces for the pin tests ----

def value_range(field: np.ndarray):
    field = np.ascontiguousarray(field)
    lo, hi = C.c_double(), C.c_double()
    bad = lib().orc_range(field.ctypes.data, field.size, _dtype_code(field), C.byref(lo), C.byref(hi))
    return bool(bad), lo.value, hi.value


def num_sampled_blocks(shape, stride) -> int:
    d = np.array(shape, np.int64)
    s = np.array(stride, np.int32)
    return int(lib().orc_num_sampled_blocks(_ptr(d, C.c_int64), len(shape), _ptr(s, C.c_int32)))


def sampled_block_origin(shape, stride, j):
    d = np.array(shape, np.int64)
    s = np.array(stride, np.int32)
    o = np.zeros(len(shape), np.int64)
    lib().orc_sampled_block_origin(_ptr(d, C.c_int64), len(shape), _ptr(s, C.c_int32), j,
                                   _ptr(o, C.c_int64))
    return tuple(int(v) for v in o)


def frexp_exponent(m: float) -> int:
    return lib().orc_frexp_exponent(m)


def floor_log2(t: float) -> int:
    return lib().orc_floor_log2(t)


def precision(emax, minexp, nd, W) -> int:
    return lib().orc_precision(emax, minexp, nd, W)


def fwd_lift(v, W=32):
    a = np.array(v, np.int64)
    lib().orc_fwd_lift(_ptr(a, C.c_int64), 1, W)
    return a


def inv_lift(v, W=32):
    a = np.array(v, np.int64)
    lib().orc_inv_lift(_ptr(a, C.c_int64), 1, W)
    return a


def fwd_xform(c, nd, W=32):
    a = np.array(c, np.int64).reshape(-1).copy()
    lib().orc_fwd_xform(_ptr(a, C.c_int64), nd, W)
    return a


def inv_xform(c, nd, W=32):
    a = np.array(c, np.int64).reshape(-1).copy()
    lib().orc_inv_xform(_ptr(a, C.c_int64), nd, W)
    return a


def reorder_table(nd):
    p = np.zeros(4 ** nd, np.int32)
    lib().orc_reorder_table(nd, _ptr(p, C.c_int32))
    return p


def to_negabinary(c: int, W=32) -> int:
    return int(lib().orc_to_negabinary(int(c), W))


def from_negabinary(u: int, W=32) -> int:
    return int(lib().orc_from_negabinary(int(u), W))


def encode_planes(u, W, prec, want_bits=False):
    a = np.array(u, np.uint64)
    if want_bits:
        cap = 64 * (2 * len(a) + 2)
        bits = np.zeros(cap, np.uint8)
        n = lib().orc_encode_planes(_ptr(a, C.c_uint64), len(a), W, prec, _ptr(bits, C.c_uint8), cap)
        return int(n), bits[:n].copy()
    return int(lib().orc_encode_planes(_ptr(a, C.c_uint64), len(a), W, prec, None, 0))


def zfp_block(x, nd, dtype, minexp):
    xv = np.array(x, np.float64).reshape(-1)
    xh = np.zeros_like(xv)
    sse, nsb, emax = C.c_double(), C.c_uint64(), C.c_int32()
    bits = lib().orc_zfp_block(_ptr(xv, C.c_double), nd, dtype, minexp, _ptr(xh, C.c_double),
                               C.byref(sse), C.byref(nsb), C.byref(emax))
    return int(bits), xh, sse.value, int(nsb.value), int(emax.value)


def lorenzo(field: np.ndarray, p):
    field = np.ascontiguousarray(field)
    d = np.array(field.shape, np.int64)
    pp = np.array(p, np.int64)
    return lib().orc_lorenzo(field.ctypes.data, _ptr(d, C.c_int64), field.ndim, _dtype_code(field),
                             _ptr(pp, C.c_int64))


def tree_sum(a) -> float:
    v = np.ascontiguousarray(a, np.float64)
    return lib().orc_tree_sum(_ptr(v, C.c_double), len(v))


def entropy(hist, n=None) -> float:
    h = np.ascontiguousarray(hist, np.uint32)
    if n is None:
        n = int(h.sum())
    return lib().orc_entropy(_ptr(h, C.c_uint32), len(h), n)


def zfp_compress(field: np.ndarray, eb_abs: float):
    """Step 4, ZFP: (result dict, stream as little-endian uint64 words,
    decompressed field as float64)."""
    field = np.ascontiguousarray(field)
    dims = np.array(field.shape, dtype=np.int64)
    out = Step4()
    L = lib()
    rc = L.orc_zfp_compress(field.ctypes.data, _ptr(dims, C.c_int64), field.ndim, _dtype_code(field),
                            float(eb_abs), None, 0, None, C.byref(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    nbits = int(out.bits)
    bits = np.zeros(max(nbits, 1), np.uint8)
    dec = np.zeros(field.size, np.float64)
    rc = L.orc_zfp_compress(field.ctypes.data, _ptr(dims, C.c_int64), field.ndim, _dtype_code(field),
                            float(eb_abs), _ptr(bits, C.c_uint8), nbits, _ptr(dec, C.c_double),
                            C.byref(out))
    if rc != 0:
        raise ValueError("oracle compression failed (%d)" % rc)
    nwords = (nbits + 63) // 64
    packed = np.zeros(nwords * 8, np.uint8)
    pb = np.packbits(bits[:nbits], bitorder="little")
    packed[:pb.size] = pb
    res = {name: getattr(out, name) for name, _ in Step4._fields_}
    return res, packed.view("<u8"), dec.reshape(field.shape)


def zfp_num_blocks(shape) -> int:
    d = np.array(shape, np.int64)
    return int(lib().orc_zfp_num_blocks(_ptr(d, C.c_int64), len(shape)))


def sz_compress(field: np.ndarray, eb_abs: float):
    """Step 4, SZ: (result dict, 65536 symbol counts, symbol of every value,
    decompressed field as float64)."""
    field = np.ascontiguousarray(field)
    dims = np.array(field.shape, dtype=np.int64)
    out = Step4()
    hist = np.zeros(NBINS, np.uint32)
    syms = np.zeros(field.size, np.uint16)
    dec = np.zeros(field.size, np.float64)
    rc = lib().orc_sz_compress(field.ctypes.data, _ptr(dims, C.c_int64), field.ndim, _dtype_code(field),
                               float(eb_abs), _ptr(hist, C.c_uint32), _ptr(syms, C.c_uint16),
                               _ptr(dec, C.c_double), C.byref(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    res = {name: getattr(out, name) for name, _ in Step4._fields_}
    return res, hist, syms.reshape(field.shape), dec.reshape(field.shape)
