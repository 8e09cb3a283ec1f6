"""Format parser and exact error-bound checker used by the tests.

Neither the oracle nor the HIP library is used here: the stream is parsed from
its documented byte layout with numpy, and every bound is checked against the
user's bound as an exact rational (fractions.Fraction), using float64 only
where it is provably decisive.
"""
import struct
from fractions import Fraction

import numpy as np

MAGIC = 0x3151434C
CHUNK = 1024
SENT = -(1 << 31)


def align16(v):
    return (v + 15) // 16 * 16


def layout(n, s):
    C = (n + CHUNK - 1) // CHUNK
    ct = align16(64 + 4 * n)
    out = align16(ct + 8 * C)
    return C, ct, out


def parse(stream, dtype):
    """Split a stream (bytes / uint8 array) into its parts."""
    b = np.asarray(stream, dtype=np.uint8).tobytes() if not isinstance(stream, bytes) else stream
    dtype = np.dtype(dtype)
    s = dtype.itemsize
    ut = np.uint32 if s == 4 else np.uint64
    magic, ver, dt, q, l2c, n, k, eb = struct.unpack_from("<IBBBBQQd", b, 0)
    stepb, boundb, aux0b, aux1b = struct.unpack_from("<QQQQ", b, 32)
    C, ct, out = layout(n, s)

    def tv(bits):
        return np.array([bits], dtype=ut).view(dtype)[0]
    hdr = dict(magic=magic, version=ver, dtype=dt, q=q, log2chunk=l2c, n=n, k=k, eb=eb,
               step=tv(stepb), bound=tv(boundb), aux0=tv(aux0b), aux1=tv(aux1b),
               step_hi=stepb >> (8 * s) if s == 4 else 0,
               bound_hi=boundb >> (8 * s) if s == 4 else 0)
    codes = np.frombuffer(b, dtype=np.int32, count=n, offset=64)
    chunks = np.frombuffer(b, dtype=np.uint64, count=C, offset=ct)
    outl = np.frombuffer(b, dtype=ut, count=k, offset=out) if k else np.zeros(0, ut)
    pads = b[64 + 4 * n: ct] + b[ct + 8 * C: out]
    return dict(hdr=hdr, codes=codes, chunks=chunks, outliers_bits=outl, pad=pads,
                size=len(b), expected_size=out + s * k)


def bits(x):
    x = np.asarray(x)
    return x.view(np.uint32 if x.dtype.itemsize == 4 else np.uint64)


def is_special(x):
    """NaN, +-INF or denormal (nonzero with zero exponent field)."""
    x = np.asarray(x)
    f32 = x.dtype == np.float32
    u = bits(x)
    mb = 23 if f32 else 52
    emask = 0xFF if f32 else 0x7FF
    E = (u >> mb) & emask
    F = u & ((1 << mb) - 1)
    return (E == emask) | ((E == 0) & (F != 0))


def _exact_abs_ok(a, b, bound):
    return abs(Fraction(float(a)) - Fraction(float(b))) <= bound


def abs_violations(x, xd, bound):
    """Indices where a finite, non-special x is reconstructed with
    |x - x'| > bound (bound given as a Python float or Fraction, exact).
    Special values must be bit-identical (reported separately)."""
    x = np.asarray(x)
    xd = np.asarray(xd)
    bound = Fraction(bound)
    spec = is_special(x)
    bad_special = np.flatnonzero(spec & (bits(x) != bits(xd)))
    fin = ~spec
    with np.errstate(all="ignore"):
        d = np.abs(x.astype(np.float64) - xd.astype(np.float64))
    bf = float(bound)
    # float64 subtraction has relative error <= 2^-53: decisive away from bf
    sure_ok = d <= bf * (1 - 2.0 ** -50)
    sure_bad = d > bf * (1 + 2.0 ** -50)
    unsure = np.flatnonzero(fin & ~sure_ok & ~sure_bad)
    bad = list(np.flatnonzero(fin & sure_bad & np.isfinite(d)))
    bad += list(np.flatnonzero(fin & ~np.isfinite(d)))
    for i in unsure:
        if not _exact_abs_ok(x[i], xd[i], bound):
            bad.append(i)
    return np.array(sorted(set(int(i) for i in bad)), dtype=np.int64), bad_special


def rel_violations(x, xd, eb):
    """Indices where x' does not have x's sign or lies outside
    [|x|/(1+eb), |x|(1+eb)] (section 2.1.2, second form; implies the first).
    Zeros and special values must be bit-identical."""
    x = np.asarray(x)
    xd = np.asarray(xd)
    e = Fraction(eb)
    spec = is_special(x) | (x == 0)
    bad_special = np.flatnonzero(spec & (bits(x) != bits(xd)))
    fin = ~spec
    sx = np.signbit(x)
    sd = np.signbit(xd)
    with np.errstate(all="ignore"):
        a = np.abs(x.astype(np.float64))
        ad = np.abs(xd.astype(np.float64))
        hi = a * (1.0 + eb)
        lo = a / (1.0 + eb)
        m = 2.0 ** -48
        # decisive only where the float64 products are finite and normal
        safe = np.isfinite(hi) & (lo > 1e-300)
        sure_ok = safe & (ad <= hi * (1 - m)) & (ad >= lo * (1 + m))
        sure_bad = ((safe & ((ad > hi * (1 + m)) | (ad < lo * (1 - m))))
                    | ~np.isfinite(ad) | (sx != sd) | (xd == 0))
    bad = list(np.flatnonzero(fin & sure_bad))
    for i in np.flatnonzero(fin & ~sure_ok & ~sure_bad):
        A = abs(Fraction(float(x[i])))
        D = abs(Fraction(float(xd[i])))
        if not (D <= A * (1 + e) and D * (1 + e) >= A):
            bad.append(int(i))
    return np.array(sorted(set(int(i) for i in bad)), dtype=np.int64), bad_special


def finite_range(x):
    """(lo, hi) over finite values with -0 read as +0 (textbook min/max)."""
    x = np.asarray(x)
    f = x[np.isfinite(x)]
    if f.size == 0:
        return None
    return float(f.min()) + 0.0, float(f.max()) + 0.0


def check_structure(st, x, dtype):
    """Format invariants that hold for any correct encoder: sentinel codes
    are exactly the outliers, outliers are the input's raw bits in input
    order, the chunk table counts the outliers before each chunk, sizes and
    padding are as documented.  Returns a list of failure strings."""
    fails = []
    x = np.asarray(x)
    h = st["hdr"]
    n = x.size
    if h["magic"] != MAGIC or h["version"] != 1 or h["log2chunk"] != 10:
        fails.append("header magic/version/log2chunk")
    if h["n"] != n:
        fails.append("header n")
    if h["step_hi"] or h["bound_hi"]:
        fails.append("float32 header fields not zero-extended")
    codes = st["codes"]
    sent = np.flatnonzero(codes == SENT)
    if h["k"] != sent.size:
        fails.append(f"n_outliers {h['k']} != sentinel count {sent.size}")
    elif not np.array_equal(st["outliers_bits"], bits(x)[sent]):
        fails.append("outlier list is not the input bits in input order")
    C = (n + CHUNK - 1) // CHUNK
    cum = np.concatenate([[0], np.cumsum(codes == SENT)])
    want = cum[np.arange(C) * CHUNK].astype(np.uint64)
    if not np.array_equal(st["chunks"], want):
        fails.append("chunk table is not the outlier count before each chunk")
    if any(st["pad"]):
        fails.append("padding bytes not zero")
    if st["size"] != st["expected_size"]:
        fails.append(f"stream size {st['size']} != layout size {st['expected_size']}")
    valid = codes[codes != SENT]
    if h["q"] == 1:
        b = valid >> 1
    else:
        b = valid
    if valid.size and (b.max() >= (1 << 30) or b.min() <= -(1 << 30)):
        fails.append("a bin lies outside -(2^30-1) .. 2^30-1")
    return fails
