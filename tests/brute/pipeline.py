"""The estimator for one request, in plain Python (see the package docstring).

Integer work uses Python's unbounded integers reduced modulo 2^W; real work
uses Python floats (IEEE binary64, round to nearest, no fused operations),
with values of binary32 fields rounded through numpy.float32.  Every
floating-point sum is the adjacent-pair tree over the sequence padded with
zeros to a power of two.
"""
from __future__ import annotations

import heapq
import itertools
import math

import numpy as np

OP_SZ, OP_ZFP, OP_SELECT, OP_FIXED_EB = 0, 1, 2, 3
EB_ABS, EB_REL = 0, 1
FLAG_CONSTANT, FLAG_NONFINITE, FLAG_ZERO_MSE = 1, 2, 4
FLAG_EB_EXCEEDS, FLAG_NO_BLOCKS, FLAG_BAD_EB = 8, 16, 32


def pair_tree(values):
    """Adjacent-pair tree: level l+1 element i = element 2i + element 2i+1."""
    v = [float(a) for a in values]
    if not v:
        return 0.0
    n = 1
    while n < len(v):
        n *= 2
    v += [0.0] * (n - len(v))
    while len(v) > 1:
        v = [v[2 * i] + v[2 * i + 1] for i in range(len(v) // 2)]
    return v[0]


class Width:
    """Two's complement words of W bits."""

    def __init__(self, W):
        self.W = W
        self.mod = 1 << W
        self.nb = int("10" * (W // 2), 2)  # ...1010: the negabinary mask

    def s(self, v):
        """v as a signed W-bit integer."""
        v %= self.mod
        return v - self.mod if v >> (self.W - 1) else v

    def to_nb(self, c):
        return ((c + self.nb) ^ self.nb) % self.mod

    def from_nb(self, u):
        return self.s((u ^ self.nb) - self.nb)


# ---------------------------------------------------------------------------
# ZFP side
# ---------------------------------------------------------------------------

def lift_forward(w, x):
    """The 4-point lift: halves of sums and differences of the outer and the
    inner pair, then of those, then two shears between the last outputs."""
    a, b, c, d = x
    outer_mean = w.s(a + d) >> 1
    outer_diff = w.s(a - outer_mean)
    inner_mean = w.s(b + c) >> 1
    inner_diff = w.s(b - inner_mean)
    y0 = w.s(outer_mean + inner_mean) >> 1
    y2 = w.s(inner_mean - y0)
    m = w.s(outer_diff + inner_diff) >> 1
    r = w.s(outer_diff - m)
    y3 = w.s((m >> 1) - r)
    y1 = w.s(m - (y3 >> 1))
    return [y0, y1, y2, y3]


def lift_inverse(w, y):
    y0, y1, y2, y3 = y
    m = w.s(y1 + (y3 >> 1))
    r = w.s((m >> 1) - y3)
    outer_diff = w.s(m + r)
    inner_diff = w.s(m - r)
    inner_mean = w.s(y0 + y2)
    outer_mean = w.s(y0 - y2)
    return [w.s(outer_mean + outer_diff), w.s(inner_mean + inner_diff),
            w.s(inner_mean - inner_diff), w.s(outer_mean - outer_diff)]


def lines(nd, axis):
    """In-block index lists of the 4-point lines along `axis` (0 = the
    fastest axis), in-block index = sum over axes of f_a 4^a."""
    step = 4 ** axis
    for i in range(4 ** nd):
        if (i // step) % 4 == 0:
            yield [i + k * step for k in range(4)]


def transform(w, c, nd, inverse=False):
    c = list(c)
    axes = range(nd - 1, -1, -1) if inverse else range(nd)
    for a in axes:
        for idx in lines(nd, a):
            out = (lift_inverse if inverse else lift_forward)(w, [c[i] for i in idx])
            for i, v in zip(idx, out):
                c[i] = v
    return c


def coding_order(nd):
    """In-block indices in coding order: total sequency, then the sum of
    squared frequencies, then the frequencies from the slowest axis down."""
    def key(i):
        f = [(i >> (2 * a)) & 3 for a in range(nd)]  # f[0]: fastest axis
        return (sum(f), sum(v * v for v in f)) + tuple(reversed(f))
    return sorted(range(4 ** nd), key=key)


def group_test_bits(u, W, planes):
    """Bits of the group-testing coder for planes W-1 .. W-planes."""
    size = len(u)
    known = 0      # values found significant so far (a prefix)
    total = 0
    for k in range(W - 1, W - 1 - planes, -1):
        bit = [(v >> k) & 1 for v in u]
        total += known  # their bits, verbatim
        at = known
        while at < size:
            total += 1  # "is there a 1 at or after `at`?"
            if 1 not in bit[at:]:
                break
            while at < size - 1 and bit[at] == 0:
                total += 1
                at += 1
            if at < size - 1:
                total += 1  # the 1 itself (implied at the last position)
            at += 1
            known = at
    return total


def frexp_e(m):
    return math.frexp(m)[1]


def bfp_integer(x, e, P):
    """trunc(x 2^(P - e)) from the exact value of x."""
    if x == 0.0:
        return 0
    mant, ex = math.frexp(abs(x))
    M = int(mant * (1 << 53))  # |x| = M 2^(ex - 53) exactly
    shift = ex - 53 + P - e
    mag = M << shift if shift >= 0 else M >> (-shift)
    return -mag if x < 0 else mag


def round_to(v, f32):
    return float(np.float32(v)) if f32 else v


def zfp_block(xs, nd, f32, minexp):
    """(bits, decoded values, significant bits) of one block."""
    W = 32 if f32 else 64
    P, E = W - 2, (8 if f32 else 11)
    size = 4 ** nd
    big = max(abs(v) for v in xs)
    if big == 0.0:
        return 1, [0.0] * size, 0
    e = frexp_e(big)
    planes = min(W, max(0, e - minexp + 2 * (nd + 1)))
    if planes == 0:
        return 1, [0.0] * size, 0
    w = Width(W)
    coef = transform(w, [bfp_integer(v, e, P) for v in xs], nd)
    order = coding_order(nd)
    u = [w.to_nb(coef[i]) for i in order]
    bits = 1 + E + group_test_bits(u, W, planes)
    low = W - planes
    sig = sum(max(0, v.bit_length() - low) for v in u)
    kept = [(v >> low) << low for v in u]
    back = [0] * size
    for r, i in enumerate(order):
        back[i] = w.from_nb(kept[r])
    back = transform(w, back, nd, inverse=True)
    dec = [round_to(math.ldexp(float(v), e - P), f32) for v in back]
    return bits, dec, sig


# ---------------------------------------------------------------------------
# SZ side
# ---------------------------------------------------------------------------

def lorenzo_terms(nd):
    """Axis subsets in the predictor's order: single axes slowest first, then
    pairs in lexicographic order, then all three (axis 0 = slowest)."""
    out = []
    for k in range(1, nd + 1):
        out += list(itertools.combinations(range(nd), k))
    return out


def lorenzo(field, p):
    """Prediction of point p from its original neighbours p - e_S (0 outside
    the field), sum over subsets S of (-1)^(|S|+1) X[p - e_S]."""
    acc = None
    for S in lorenzo_terms(field.ndim):
        q = tuple(c - 1 if a in S else c for a, c in enumerate(p))
        v = 0.0 if min(q) < 0 else float(field[q])
        if acc is None:
            acc = v
        elif len(S) % 2:
            acc = acc + v
        else:
            acc = acc - v
    return acc


def quantize(xv, pred, delta, inv, half, f32):
    """(code, squared error, |error|); code 0 = unpredictable."""
    d = xv - pred
    t = abs(d) * inv + 0.5
    if not t < 32768.0:
        return 0, 0.0, 0.0
    q = math.floor(t)
    if d < 0.0:
        q = -q
    rec = round_to(pred + float(q) * delta, f32)
    err = xv - rec
    if abs(err) > half:
        return 0, 0.0, 0.0
    return q + 32768, err * err, abs(err)


def huffman_cost(hist):
    h = [int(v) for v in hist if v]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

def sampled_blocks(shape, stride):
    """Origins of the sampled full 4^d blocks in row-major block order."""
    axes = [range(0, n // 4, s) for n, s in zip(shape, stride)]
    return [tuple(4 * b for b in idx) for idx in itertools.product(*axes)]


def block_points(origin):
    return list(itertools.product(*[range(o, o + 4) for o in origin]))


def psnr(vr, mse):
    return 20.0 * math.log10(vr) - 10.0 * math.log10(mse) if mse > 0.0 else math.inf


def run(op, field, eb, eb_mode=EB_REL, stride=None, sz_offset=0.5, huffman=0):
    """The estimator on a numpy field; a dict with the oracle's result keys."""
    f32 = field.dtype == np.float32
    W = 32 if f32 else 64
    nd = field.ndim
    stride = tuple(stride) if stride is not None else (1,) * nd
    keys = ("flags choice vmin vmax vr eb_abs minexp zfp_bitrate zfp_mse zfp_psnr zfp_nsb_mean "
            "zfp_maxerr zfp_sse zfp_bits zfp_values zfp_blocks zfp_nsb_total sz_delta sz_inv_delta "
            "sz_eb sz_entropy sz_bitrate sz_psnr_model sz_psnr_measured sz_mse sz_maxerr sz_sse "
            "sz_values sz_unpredictable chosen_eb sz_huffman_bits sz_huffman_bitrate zfp_ec_points "
            "zfp_ec_nsb2").split()
    r = {k: 0 for k in keys}
    selecting = op in (OP_SELECT, OP_FIXED_EB)
    r["choice"] = -1
    vals = [float(v) for v in field.reshape(-1)]
    if any(not math.isfinite(v) for v in vals):
        r["flags"] = FLAG_NONFINITE
        return r
    lo, hi = min(vals), max(vals)
    r["vmin"], r["vmax"] = lo, hi
    vr = hi - lo
    r["vr"] = vr
    eb_abs = eb * vr if eb_mode == EB_REL else eb
    r["eb_abs"] = eb_abs
    if vr == 0.0 or not (eb_abs > 0.0 and math.isfinite(eb_abs)) or not sampled_blocks(field.shape, stride):
        r["flags"] = (FLAG_CONSTANT if vr == 0.0 else
                      FLAG_BAD_EB if not (eb_abs > 0.0 and math.isfinite(eb_abs)) else FLAG_NO_BLOCKS)
        if selecting:
            r["choice"] = 0
        return r
    origins = sampled_blocks(field.shape, stride)
    npts = len(origins) * 4 ** nd
    minexp = frexp_e(eb_abs) - 1
    r["minexp"] = minexp

    br_zfp, mse_zfp = 0.0, 0.0
    if op != OP_SZ:
        bits = sig = 0
        sq, worst = [], 0.0
        for o in origins:
            xs = [float(field[p]) for p in block_points(o)]
            b, dec, s = zfp_block(xs, nd, f32, minexp)
            bits += b
            sig += s
            for xv, xh in zip(xs, dec):
                e = xv - xh
                sq.append(e * e)
                worst = max(worst, abs(e))
        sse = pair_tree(sq)
        mse_zfp = sse / npts
        br_zfp = bits / npts
        r.update(zfp_sse=sse, zfp_mse=mse_zfp, zfp_bits=bits, zfp_values=npts, zfp_blocks=len(origins),
                 zfp_nsb_total=sig, zfp_nsb_mean=sig / npts, zfp_bitrate=br_zfp, zfp_maxerr=worst,
                 zfp_psnr=psnr(vr, mse_zfp))

    if op != OP_ZFP:
        delta = 2.0 * eb_abs
        if op == OP_SELECT:
            if mse_zfp > 0.0:
                delta = math.sqrt(12.0 * mse_zfp)
            else:
                r["flags"] |= FLAG_ZERO_MSE
        inv = 1.0 / delta
        half = 0.5 * delta
        hist = [0] * 65536
        sq, worst, unpred = [], 0.0, 0
        for o in origins:
            for p in block_points(o):
                code, e2, ae = quantize(float(field[p]), lorenzo(field, p), delta, inv, half, f32)
                hist[code] += 1
                unpred += code == 0
                sq.append(e2)
                worst = max(worst, ae)
        sse = pair_tree(sq)
        ent = math.log2(npts) - pair_tree([h * math.log2(h) if h else 0.0 for h in hist]) / npts
        br = ent + sz_offset
        br = br + (unpred * W) / npts
        r.update(sz_delta=delta, sz_inv_delta=inv, sz_eb=half, sz_entropy=ent, sz_bitrate=br, sz_sse=sse,
                 sz_mse=sse / npts, sz_maxerr=worst, sz_values=npts, sz_unpredictable=unpred,
                 sz_psnr_model=20.0 * math.log10(vr / delta) + 10.0 * math.log10(12.0),
                 sz_psnr_measured=psnr(vr, sse / npts))
        br_sel = br
        if huffman:
            hb = huffman_cost(hist)
            hbr = hb / npts
            hbr = hbr + (unpred * W) / npts
            r.update(sz_huffman_bits=hb, sz_huffman_bitrate=hbr)
            if huffman == 2:
                br_sel = hbr
        if selecting:
            r["choice"] = 0 if br_sel < br_zfp else 1
            r["chosen_eb"] = half if r["choice"] == 0 else eb_abs
            if half > eb_abs:
                r["flags"] |= FLAG_EB_EXCEEDS
    return r
