"""Pins of the CPU oracle: checks against what the paper and the mathematics
fix, never against the oracle's own formulas retyped.

Each pin takes a loaded oracle library (so the same pins can be run against
deliberately broken builds of the oracle, see test_oracle_mutants.py) and
raises AssertionError on failure.

Sources of truth used here:
  * closed forms of the section 3.2 approximations (tests/golden/mitchell.txt)
    and Mitchell's textbook error bounds for log2 / 2^y;
  * the error-bound definitions of section 2.1, checked as exact rationals;
  * the special-value policy of sections 2.2 / 3.1 (NaN, INF, denormals kept
    bit-exact) and the bin-range rule of section 3.3;
  * textbook stable compaction (np.flatnonzero, cumulative counts) for the
    outlier list and chunk table;
  * textbook finite min / max for the NOA range;
  * brute force: when the exact nearest bin is unambiguous and well inside
    the bound, the encoder must take it (the method is not allowed to be
    vacuously lossless).
"""
import math
import os
from fractions import Fraction

import numpy as np

import oracle as O
import synth
from streamcheck import (SENT, abs_violations, check_structure, finite_range,
                         is_special, parse, rel_violations, bits)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mitchell.txt")

# Mitchell's maximum error of log2(x) - approx(x) over one octave:
# max_m log2(1+m) - m at m = 1/ln2 - 1.
MITCHELL_LOG_MAX = math.log2(1 / math.log(2)) - (1 / math.log(2) - 1)  # 0.0860713...
# and of the antilog (1+f) / 2^f at the same f.
MITCHELL_EXP_MAX = (1 / math.log(2)) / 2 ** (1 / math.log(2) - 1)       # 1.0615...


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _random_normals(dtype, n, seed, lo_exp=None, hi_exp=None):
    """Random positive normal floats with uniformly random bit patterns in a
    range of exponent fields."""
    rng = _rng(seed)
    if np.dtype(dtype) == np.float32:
        lo_exp = 1 if lo_exp is None else lo_exp
        hi_exp = 254 if hi_exp is None else hi_exp
        e = rng.integers(lo_exp, hi_exp + 1, n, dtype=np.uint32)
        f = rng.integers(0, 1 << 23, n, dtype=np.uint32)
        return ((e << np.uint32(23)) | f).view(np.float32)
    lo_exp = 1 if lo_exp is None else lo_exp
    hi_exp = 2046 if hi_exp is None else hi_exp
    e = rng.integers(lo_exp, hi_exp + 1, n, dtype=np.uint64)
    f = rng.integers(0, 1 << 52, n, dtype=np.uint64)
    return ((e << np.uint64(52)) | f).view(np.float64)


# ------------------------------------------------------------ section 3.2 ---
def load_golden():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        dt, op, a, b = line.split()
        rows.append((np.float32 if dt == "f32" else np.float64, op, float(a), float(b)))
    return rows


def pin_mitchell_golden(L):
    for dt, op, a, b in load_golden():
        fn = O.log2approx if op == "log2" else O.pow2approx
        got = fn(np.array([a], dtype=dt), L=L)[0]
        assert got == dt(b) and np.signbit(got) == np.signbit(dt(b)), (dt, op, a, b, got)


def pin_mitchell_powers_of_two(L):
    for dt, lo, hi in ((np.float32, -126, 127), (np.float64, -1022, 1023)):
        k = np.arange(lo, hi + 1)
        x = np.ldexp(np.ones(k.size), k).astype(dt)
        assert np.array_equal(O.log2approx(x, L=L), k.astype(dt))
        assert np.array_equal(O.pow2approx(k.astype(dt), L=L), x)


def pin_mitchell_log2_error(L):
    """0 <= log2(x) - approx(x) <= Mitchell's 0.0861, up to the rounding of
    the final float add (at most half an ulp of |approx| <= 2^-16 here)."""
    for dt, slack in ((np.float32, 2.0 ** -16), (np.float64, 2.0 ** -42)):
        x = _random_normals(dt, 200000, 11)
        lg = O.log2approx(x, L=L).astype(np.float64)
        d = np.log2(x.astype(np.float64)) - lg
        assert d.min() >= -slack, (dt, d.min())
        assert d.max() <= MITCHELL_LOG_MAX + slack, (dt, d.max())
        # inside [1,2) the approximation is exactly x - 1 (no rounding)
        y = _random_normals(dt, 10000, 12, *((127, 127) if dt == np.float32 else (1023, 1023)))
        assert np.array_equal(O.log2approx(y, L=L), y - dt(1))


def pin_mitchell_log2_monotone(L):
    for dt in (np.float32, np.float64):
        x = np.sort(_random_normals(dt, 200000, 13))
        lg = O.log2approx(x, L=L)
        assert np.all(np.diff(lg.astype(np.float64)) >= 0)


def pin_mitchell_pow2_error(L):
    """1 <= approx(y) / 2^y <= Mitchell's 1.0615, up to the rounding of
    y + bias (|y| <= 120 here, so at most 2^-17 in y)."""
    rng = _rng(14)
    for dt, yl in ((np.float32, 120.0), (np.float64, 1000.0)):
        y = rng.uniform(-yl, yl, 200000).astype(dt)
        p = O.pow2approx(y, L=L).astype(np.float64)
        ratio = p / np.exp2(y.astype(np.float64))
        slack = 2.0 ** -16 if dt == np.float32 else 2.0 ** -40
        assert ratio.min() >= 1 - slack, (dt, ratio.min())
        assert ratio.max() <= MITCHELL_EXP_MAX + slack, (dt, ratio.max())


# ------------------------------------------------------------ parameters ----
def _next_up(v):
    return np.nextafter(v, type(v)(np.inf))


def pin_params_abs(L):
    for dt in (np.float32, np.float64):
        for eb in (1e-1, 1e-3, 1e-4, 1e-6, 3.3e-7, 0.5, 1e-30):
            p = O.params("abs", dt, eb, L=L)
            e = p["bound"]
            # largest float of the type not above eb
            assert Fraction(float(e)) <= Fraction(eb) < Fraction(float(_next_up(e))), (dt, eb)
            assert Fraction(float(p["step"])) == 2 * Fraction(float(e))
            # 1/step correctly rounded
            inv = Fraction(float(p["inv"]))
            exact = 1 / Fraction(float(p["step"]))
            lo = Fraction(float(np.nextafter(p["inv"], dt(0))))
            hi = Fraction(float(_next_up(p["inv"])))
            assert abs(inv - exact) <= min(abs(lo - exact), abs(hi - exact)), (dt, eb)


def pin_params_rel(L):
    for dt in (np.float32, np.float64):
        for eb in (0.5, 1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 0.999, 3e-7):
            p = O.params("rel", dt, eb, L=L)
            eh, el = p["bound"], p["aux0"]
            E = Fraction(eb)
            assert Fraction(float(eh)) <= E < Fraction(float(_next_up(eh))), (dt, eb)
            Q = E / (1 + E)
            assert Fraction(float(el)) <= Q < Fraction(float(_next_up(el))), (dt, eb)
            # lambda = approx-log2 of (1 + eh): for an argument in [1,2) that
            # is exactly (1 + eh) - 1, the sum rounded to the type
            one_plus = dt(1) + eh
            assert p["lambda"] == one_plus - dt(1), (dt, eb)
            assert Fraction(float(p["step"])) == 2 * Fraction(float(p["lambda"]))


def pin_params_noa(L):
    rng = _rng(21)
    for dt in (np.float32, np.float64):
        for trial in range(300):
            n = int(rng.integers(1, 50))
            scale = 10.0 ** rng.uniform(-30, 30)
            x = (rng.standard_normal(n) * scale + rng.standard_normal() * scale * 3).astype(dt)
            eb = float(10.0 ** rng.uniform(-7, -0.5))
            p = O.params("noa", dt, eb, x=x, L=L)
            lo, hi = finite_range(x)
            assert p["aux0"] == dt(lo) and p["aux1"] == dt(hi)
            R = Fraction(hi) - Fraction(lo)
            ebr = Fraction(float(p["bound"]))
            if R == 0:
                assert p["degenerate"]
                continue
            assert not p["degenerate"]
            assert 0 < ebr <= Fraction(eb) * R, (dt, eb, lo, hi)
            # not more than a few ulps conservative
            assert ebr >= Fraction(eb) * R * (1 - Fraction(8, 2 ** (24 if dt == np.float32 else 53)))
            assert Fraction(float(p["step"])) == 2 * ebr
        # range ignores NaN / INF, counts denormals and zeros, -0 reads as +0
        x = np.array([np.nan, -np.inf, np.inf, 3.0, -0.0, 5.0], dtype=dt)
        p = O.params("noa", dt, 0.1, x=x, L=L)
        assert p["aux0"] == 0 and not np.signbit(p["aux0"]) and p["aux1"] == 5.0
        p = O.params("noa", dt, 0.1, x=np.array([np.nan, np.inf], dtype=dt), L=L)
        assert p["degenerate"]
        p = O.params("noa", dt, 0.1, x=np.array([2.5, 2.5], dtype=dt), L=L)
        assert p["degenerate"]


def pin_arg_errors(L):
    x = np.ones(4, np.float32)
    for q, eb in (("abs", 0.0), ("abs", -1e-3), ("abs", float("nan")), ("abs", float("inf")),
                  ("rel", 1.0), ("rel", 2.0), ("noa", 0.0)):
        try:
            O.quantize(q, x, eb, L=L)
        except O.OracleError as e:
            assert e.status == O.ERR_ARG
        else:
            raise AssertionError(f"accepted {q} eb={eb}")


# ---------------------------------------------------------------- streams ---
def _config0_like(dt, n, seed, eb):
    x = synth.sines_1d(n, seed, dtype=dt)
    x, _, _ = synth.inject_specials(x, max(19, n // 1000), seed + 100, eb)
    return x


def _cases():
    """(dtype, q, eb, x) encode cases spanning specials, ragged sizes and
    bin borders."""
    out = []
    for dt in (np.float32, np.float64):
        for q, eb in (("abs", 1e-3), ("noa", 1e-4), ("rel", 1e-2), ("rel", 1e-3)):
            n = 3 * 1024 + 517
            if q == "noa":
                # specials that keep the field's range (its bins are real),
                # border values at the field's own eb * R
                x = synth.with_specials(synth.sines_1d(n, 5, dtype=dt), "noa",
                                        max(19, n // 1000), 105, eb)
                lo, hi = synth.finite_range(x)
                adv = synth.adversarial_noa(4000, synth.noa_half_bin(x, eb), lo, hi, 8, dt)
                x = np.concatenate([x, adv]).astype(dt)
                out.append((dt, q, eb, x))
                continue
            x = _config0_like(dt, n, 5, eb)
            if q == "rel":
                x = synth.rel_variant(x.astype(np.float64), 6, dtype=dt)
                x, _, _ = synth.inject_specials(x, 40, 7, eb)
                adv = synth.adversarial_rel(4000, eb, 8, dt)
            else:
                adv = synth.adversarial_abs(4000, eb, 8, dt)
            x = np.concatenate([x, adv]).astype(dt)
            out.append((dt, q, eb, x))
    return out


def _encode_decode(L, q, x, eb):
    st = O.quantize(q, x, eb, L=L)
    xd = O.dequantize(st, x.dtype, x.size, L=L)
    return st, xd


def pin_structure(L):
    for dt, q, eb, x in _cases():
        st, _ = _encode_decode(L, q, x, eb)
        P = parse(st, dt)
        f = check_structure(P, x, dt)
        assert not f, (dt, q, eb, f)
        h = P["hdr"]
        assert h["dtype"] == (0 if dt == np.float32 else 1)
        assert h["q"] == {"abs": 0, "rel": 1, "noa": 2}[q]
        assert h["eb"] == eb


def pin_bounds(L):
    for dt, q, eb, x in _cases():
        st, xd = _encode_decode(L, q, x, eb)
        if q == "rel":
            bad, bad_sp = rel_violations(x, xd, eb)
        else:
            if q == "abs":
                bound = Fraction(eb)
            else:
                lo, hi = finite_range(x)
                bound = Fraction(eb) * (Fraction(hi) - Fraction(lo))
            bad, bad_sp = abs_violations(x, xd, bound)
        assert bad.size == 0, (dt, q, eb, bad[:5], x[bad[:5]], xd[bad[:5]])
        assert bad_sp.size == 0, (dt, q, eb, bad_sp[:5])


def pin_specials(L):
    """NaN (quiet and signalling, with payloads), INF and denormals are kept
    bit-exact in every quantizer; REL keeps zeros too; ABS/NOA decode +-0 to
    +0 (bin 0)."""
    for dt in (np.float32, np.float64):
        base = synth.sines_1d(2048, 3, dtype=dt)
        x, pos, names = synth.inject_specials(base, 600, 4, 1e-3)
        for q in ("abs", "rel", "noa"):
            st, xd = _encode_decode(L, q, x, 1e-3)
            codes = parse(st, dt)["codes"]
            sp = is_special(x)
            assert np.all(codes[sp] == SENT), (dt, q)
            assert np.array_equal(bits(xd)[sp], bits(x)[sp]), (dt, q)
            zeros = (x == 0) & ~sp
            if q == "rel":
                assert np.all(codes[zeros] == SENT)
                assert np.array_equal(bits(xd)[zeros], bits(x)[zeros])
            else:
                assert np.all(codes[zeros] == 0), (dt, q)
                assert np.all(bits(xd)[zeros] == 0), (dt, q)


def pin_abs_nearest_bin(L):
    """Brute force: where x / (2e) is within 0.3 of an integer j with
    |j| < 2^20 (float32) / 2^40 (float64), the rounding errors of the
    method cannot move the bin or break the bound, so the encoder must emit
    code j (no spurious lossless fallback).  Same for NOA with ebR."""
    rng = _rng(31)
    for dt, jmax in ((np.float32, 2 ** 20), (np.float64, 2 ** 40)):
        for q in ("abs", "noa"):
            eb = 1e-3
            x = (rng.standard_normal(20000) * 50).astype(dt)
            x[:50] = dt(0.0)
            st = O.quantize(q, x, eb, L=L)
            P = parse(st, dt)
            e = Fraction(float(P["hdr"]["bound"]))
            two_e = 2 * e
            codes = P["codes"]
            checked = 0
            for i in range(x.size):
                t = Fraction(float(x[i])) / two_e
                j = round(t)
                if abs(t - j) < Fraction(3, 10) and abs(j) < jmax:
                    assert codes[i] == j, (dt, q, x[i], j, codes[i])
                    checked += 1
            assert checked > x.size // 2


def _mitchell_log2_exact(a, dt):
    """Exact rational Mitchell log2 of a positive normal float: e + m."""
    u = int(np.array([a], dtype=dt).view(np.uint32 if dt == np.float32 else np.uint64)[0])
    mb, bias = (23, 127) if dt == np.float32 else (52, 1023)
    E = (u >> mb) & (0xFF if dt == np.float32 else 0x7FF)
    F = u & ((1 << mb) - 1)
    return Fraction(int(E) - bias) + Fraction(F, 1 << mb)


def pin_rel_nearest_bin(L):
    """Brute force for REL: with L* the exact Mitchell log2 of |x| and
    step = 2 lambda, if L*/step is within 0.3 of an integer j, the bin is j
    and the reconstruction is within 0.61 lambda (< the bound) relative, so
    the encoder must emit code (j << 1) | sign."""
    rng = _rng(32)
    for dt, eb in ((np.float32, 1e-3), (np.float32, 1e-2), (np.float64, 1e-4)):
        mag = np.power(10.0, rng.uniform(-30, 30, 20000))
        x = (mag * np.where(rng.integers(0, 2, mag.size) == 1, -1.0, 1.0)).astype(dt)
        st = O.quantize("rel", x, eb, L=L)
        P = parse(st, dt)
        step = Fraction(float(P["hdr"]["step"]))
        codes = P["codes"]
        checked = 0
        for i in range(x.size):
            Ls = _mitchell_log2_exact(abs(x[i]), dt)
            t = Ls / step
            j = round(t)
            if abs(t - j) < Fraction(3, 10):
                want = (j << 1) | int(np.signbit(x[i]))
                assert codes[i] == want, (dt, eb, x[i], j, codes[i])
                checked += 1
        assert checked > x.size // 2


def pin_bin_range(L):
    """Section 3.3: bins at or beyond +-2^30 (including where the float bin
    would convert to INT_MIN) are stored losslessly; bins just inside are
    quantized."""
    for dt in (np.float32, np.float64):
        eb = 0.5  # step 1: the bin is rint(x)
        v = [2.0 ** 30, -(2.0 ** 30), 2.0 ** 31, -(2.0 ** 31), 2.0 ** 31 + 2 ** 8,
             -(2.0 ** 31) - 2 ** 8, 2.0 ** 32, float(np.finfo(dt).max), -float(np.finfo(dt).max),
             2.0 ** 30 - 64, -(2.0 ** 30) + 64]
        x = np.array(v, dtype=dt)
        st, xd = _encode_decode(L, "abs", x, eb)
        codes = parse(st, dt)["codes"]
        assert np.all(codes[:9] == SENT), (dt, codes)
        assert codes[9] == 2 ** 30 - 64 and codes[10] == -(2 ** 30) + 64, (dt, codes)
        assert np.array_equal(bits(xd), bits(x))


def pin_roundtrip_sizes(L):
    """Empty and ragged inputs: n = 0 gives a header-only 64-byte stream;
    every n decodes within bound and has the documented layout."""
    for dt in (np.float32, np.float64):
        st = O.quantize("abs", np.zeros(0, dt), 1e-3, L=L)
        assert st.size == 64
        assert O.dequantize(st, dt, 0, L=L).size == 0
        for n in (1, 3, 1023, 1024, 1025, 4097):
            x = synth.sines_1d(n, 9, dtype=dt)
            for q in ("abs", "noa"):
                st, xd = _encode_decode(L, q, x, 1e-3)
                assert not check_structure(parse(st, dt), x, dt)
                bound = Fraction(1e-3)
                if q == "noa":
                    lo, hi = finite_range(x)
                    bound *= Fraction(hi) - Fraction(lo)
                bad, _ = abs_violations(x, xd, bound)
                assert bad.size == 0


def pin_stream_errors(L):
    x = synth.sines_1d(5000, 10, dtype=np.float32)
    st = O.quantize("abs", x, 1e-3, L=L)

    def rejects(s, dt=np.float32, n=x.size):
        try:
            O.dequantize(s, dt, n, L=L)
        except O.OracleError as e:
            return e.status == O.ERR_STREAM
        return False
    assert not rejects(st)
    bad = st.copy(); bad[0] ^= 1
    assert rejects(bad)                      # magic
    assert rejects(st, n=x.size - 1)         # n mismatch
    assert rejects(st, dt=np.float64)        # dtype mismatch
    assert rejects(st[:63])                  # truncated header
    y = x.copy(); y[100] = np.nan; y[3000] = np.inf
    st2 = O.quantize("abs", y, 1e-3, L=L)
    assert rejects(st2[:-1])                 # truncated outliers
    P = parse(st2, np.float32)
    ct = 64 + 4 * y.size
    ct = (ct + 15) // 16 * 16
    bad = st2.copy(); bad[ct + 8 * 2] ^= 1   # chunk table entry 2
    assert rejects(bad)
    assert P["hdr"]["k"] == parse(st, np.float32)["hdr"]["k"] + 2


def pin_noa_degenerate(L):
    for dt in (np.float32, np.float64):
        x = np.full(3000, 7.25, dt)
        x[5] = np.nan
        st, xd = _encode_decode(L, "noa", x, 1e-2)
        P = parse(st, dt)
        assert np.all(P["codes"] == SENT)
        assert np.array_equal(bits(xd), bits(x))
        assert P["hdr"]["step"] == 0 and P["hdr"]["bound"] == 0


def pin_inline_format(L):
    """The in-line layout (section 3.1, the paper's own) carries the same
    decisions as the pinned separate-list layout: a word is the value's code
    (sign-extended) where that code is not the sentinel, else the value's raw
    bits with its flag set; unused bits and padding are zero; it decodes to
    the same values."""
    for dt, q, eb, x in _cases():
        st = O.quantize(q, x, eb, L=L)
        P = parse(st, dt)
        il = O.quantize_inline(q, x, eb, L=L)
        s = np.dtype(dt).itemsize
        n = x.size
        hdr = np.frombuffer(il[:64].tobytes(), dtype=np.uint8)
        assert bytes(hdr[:4]) == b"LCQI" and hdr[4] == 1 and hdr[7] == 0
        assert np.array_equal(hdr[32:64], np.frombuffer(st[32:64].tobytes(), np.uint8))
        words = np.frombuffer(il.tobytes(), dtype=np.int32 if s == 4 else np.int64, count=n, offset=64)
        fl = (64 + s * n + 15) // 16 * 16
        flags = np.unpackbits(np.frombuffer(il.tobytes(), np.uint8, count=(n + 7) // 8, offset=fl),
                              bitorder="little")
        raw = P["codes"] == SENT
        assert np.array_equal(flags[:n].astype(bool), raw)
        assert not flags[n:].any()
        assert np.array_equal(words[~raw], P["codes"][~raw].astype(words.dtype))
        assert np.array_equal(words[raw].view(bits(x).dtype), bits(x)[raw])
        assert il.size == fl + (n + 7) // 8 and not il[64 + s * n: fl].any()
        dec = O.dequantize_inline(il, dt, n, L=L)
        assert np.array_equal(bits(dec), bits(O.dequantize(st, dt, n, L=L)))


# ------------------------------------------------- section 6 ablations ---
def pin_ablation_abs_unchecked(L):
    """ABS without the double-check: specials stay lossless, every finite
    normal whose bin is in range gets the nearest-bin code rint(x * inv)
    (replayed with numpy's IEEE operations of the field type), codes agree
    with the protected stream wherever that one has a code, and on bin-border
    inputs some codes decode outside the bound -- exactly at values the
    protected stream stores raw (the check is what the guarantee rests on)."""
    for dt in (np.float32, np.float64):
        eb = 1e-3
        x = np.concatenate([_config0_like(dt, 3000, 41, eb),
                            synth.adversarial_abs(6000, eb, 42, dt)]).astype(dt)
        st_u = O.quantize("abs_unchecked", x, eb, L=L)
        st_p = O.quantize("abs", x, eb, L=L)
        Pu, Pp = parse(st_u, dt), parse(st_p, dt)
        assert Pu["hdr"]["q"] == 3 and not check_structure(Pu, x, dt)
        assert Pu["hdr"]["step"] == Pp["hdr"]["step"] and Pu["hdr"]["bound"] == Pp["hdr"]["bound"]
        inv = O.params("abs", dt, eb, L=L)["inv"]
        sp = is_special(x)
        with np.errstate(all="ignore"):
            qf = np.rint(x * inv)
        inr = ~sp & (qf > -(2.0 ** 30)) & (qf < 2.0 ** 30)
        cu, cp = Pu["codes"], Pp["codes"]
        assert np.all(cu[~inr] == SENT), dt
        assert np.array_equal(cu[inr].astype(np.int64), qf[inr].astype(np.int64)), dt
        assert np.array_equal(cu[cp != SENT], cp[cp != SENT]), dt
        xd = O.dequantize(st_u, dt, x.size, L=L)
        bad, bad_sp = abs_violations(x, xd, Fraction(eb))
        assert bad.size > 0 and bad_sp.size == 0, (dt, bad.size)
        assert np.all(cp[bad] == SENT), dt


def pin_ablation_rel_libm(L):
    """REL with the C library's log2 / exp2: same eh / el, lambda =
    log2(1 (+) eh) (within an ulp of the exact value, wider than the
    approximation's (1 + eh) - 1 since 1/ln 2 > 1), the double-check still
    bounds every decoded value exactly, and exact powers of two -- whose
    log2 is an integer in any library -- get the bin rint(k * inv) unless
    they are stored raw."""
    for dt in (np.float32, np.float64):
        for eb in (1e-2, 1e-3):
            pm = O.params("rel", dt, eb, L=L)
            pl = O.params("rel_libm", dt, eb, L=L)
            assert pl["bound"] == pm["bound"] and pl["aux0"] == pm["aux0"], (dt, eb)
            lam = pl["lambda"]
            exact = math.log2(float(dt(1) + pm["bound"]))  # log2 of 1 (+) eh, the type's sum
            assert abs(Fraction(float(lam)) - Fraction(exact)) <= Fraction(float(np.spacing(lam))), (dt, eb)
            assert lam > pm["lambda"], (dt, eb)
            assert Fraction(float(pl["step"])) == 2 * Fraction(float(lam))
            x = synth.rel_variant(np.nan_to_num(_config0_like(dt, 3000, 51, eb).astype(np.float64)),
                                  52, dtype=dt)
            x, _, _ = synth.inject_specials(x, 60, 53, eb)
            x = np.concatenate([x, synth.adversarial_rel(4000, eb, 54, dt)]).astype(dt)
            st = O.quantize("rel_libm", x, eb, L=L)
            P = parse(st, dt)
            assert P["hdr"]["q"] == 4 and not check_structure(P, x, dt), (dt, eb)
            xd = O.dequantize(st, dt, x.size, L=L)
            bad, bad_sp = rel_violations(x, xd, eb)
            assert bad.size == 0 and bad_sp.size == 0, (dt, eb)
            k = np.arange(-100, 101)
            sgn = (k % 2 == 0)
            a = (np.ldexp(1.0, k) * np.where(sgn, -1.0, 1.0)).astype(dt)
            codes = parse(O.quantize("rel_libm", a, eb, L=L), dt)["codes"]
            qf = np.rint(k.astype(dt) * pl["inv"])
            want = (qf.astype(np.int64) * 2 + sgn.astype(np.int64)).astype(np.int32)
            coded = codes != SENT
            assert coded.mean() > 0.9 and np.array_equal(codes[coded], want[coded]), (dt, eb)


# --------------------------------------------------- lossless packing ---
def _lcq1_by_hand(codes, dtype=np.float32, outliers=()):
    """An LCQ1 stream assembled field by field from its layout (ABS header
    words zero apart from magic / version / dtype / n / k)."""
    codes = np.asarray(codes, dtype=np.int32)
    n = codes.size
    s = np.dtype(dtype).itemsize
    C = (n + 1023) // 1024
    ct = (64 + 4 * n + 15) // 16 * 16
    out = (ct + 8 * C + 15) // 16 * 16
    k = len(outliers)
    b = np.zeros(out + s * k, dtype=np.uint8)
    b[0:4] = np.frombuffer(b"LCQ1", dtype=np.uint8)
    b[4], b[5], b[6], b[7] = 1, (0 if s == 4 else 1), 0, 10
    b[8:16] = np.array([n], dtype=np.uint64).view(np.uint8)
    b[16:24] = np.array([k], dtype=np.uint64).view(np.uint8)
    b[64: 64 + 4 * n] = codes.view(np.uint8)
    sent = codes == np.iinfo(np.int32).min
    before = np.concatenate([[0], np.cumsum(sent)])[::1024][:C]
    b[ct: ct + 8 * C] = before.astype(np.uint64).view(np.uint8)
    if k:
        b[out:] = np.asarray(outliers, dtype=np.uint32 if s == 4 else np.uint64).view(np.uint8)
    return b


def pin_pack_golden(L):
    """Codes 0, 1, 2, 3 by hand: plain zigzag 0, 2, 4, 6 needs 3 bits, deltas
    0, 1, 1, 1 -> zigzag 0, 2, 2, 2 need 2: delta mode, w = 2, and the bits
    00 01 01 01 (value j at bits 2j..2j+1, least significant first) make the
    single byte 0b10101000."""
    st = _lcq1_by_hand([0, 1, 2, 3])
    want = np.zeros(128, dtype=np.uint8)
    want[:64] = st[:64]
    want[0:4] = np.frombuffer(b"LCQP", dtype=np.uint8)
    # [64,72) chunk table entry 0 = 0; [80,88) record offset 0; [88,96) payload 32
    want[88] = 32
    want[96], want[97], want[98] = 2, 1, 0
    want[112] = 0xA8
    got = O.pack(st, np.float32, 4, L=L)
    assert np.array_equal(got, want), (got, want)
    assert np.array_equal(O.unpack(got, np.float32, 4, L=L), st)


def _zz(v):
    v = np.asarray(v, dtype=np.int64) & 0xFFFFFFFF
    s = v.astype(np.uint32).view(np.int32).astype(np.int64)
    return ((s << 1) ^ (s >> 31)) & 0xFFFFFFFF


def _bitlen(v):
    return int(v).bit_length()


def pin_pack_roundtrip_and_widths(L):
    """unpack(pack(s)) == s byte for byte for quantizer streams of every kind
    and size; each record's width is the bit length of the largest zigzag
    value of the mode it names, that mode is the narrower one (plain on a
    tie), and the outlier bitmap is present exactly for chunks with
    outliers."""
    rng = _rng(61)
    streams = []
    for dt in (np.float32, np.float64):
        for n in (0, 1, 5, 1023, 1024, 1025, 3 * 1024 + 77):
            x = synth.sines_1d(max(n, 1), 62 + n, dtype=dt)[:n]
            if n:
                x, _, _ = synth.inject_specials(x, max(1, n // 300), 63, 1e-3)
            for q in ("abs", "rel", "noa"):
                y = x if q != "rel" else synth.rel_variant(np.nan_to_num(x.astype(np.float64)), 64, dtype=dt)
                streams.append((dt, y.size, O.quantize(q, y, 1e-3, L=L)))
        base = synth.sines_1d(2500, 65, dtype=dt)
        allsp, _, _ = synth.inject_specials(base, 2500, 66, 1e-3)
        streams.append((dt, 2500, O.quantize("abs", allsp, 1e-3, L=L)))
    # codes that use all 32 bits and wrap in delta mode
    big = rng.integers(-(2 ** 31) + 1, 2 ** 31, 3000).astype(np.int32)
    big[::97] = np.iinfo(np.int32).min
    streams.append((np.float32, 3000, _lcq1_by_hand(big, outliers=np.arange(np.count_nonzero(big == np.iinfo(np.int32).min)))))
    for dt, n, st in streams:
        pk = O.pack(st, dt, n, L=L)
        assert np.array_equal(O.unpack(pk, dt, n, L=L), st), (dt, n)
        codes = parse(st, dt)["codes"].astype(np.int64)
        C = (n + 1023) // 1024
        ot = (64 + 8 * C + 15) // 16 * 16
        pl = (ot + 8 * (C + 1) + 15) // 16 * 16
        offs = pk[ot: ot + 8 * (C + 1)].view(np.uint64).astype(np.int64)
        for c in range(C):
            cc = codes[c * 1024: (c + 1) * 1024]
            sent = cc == np.iinfo(np.int32).min
            cv = np.where(sent, 0, cc)
            wp = _bitlen(_zz(cv).max())
            wd = _bitlen(_zz(cv - np.concatenate([[0], cv[:-1]])).max())
            r = pl + offs[c]
            w, mode, hb = int(pk[r]), int(pk[r + 1]), int(pk[r + 2])
            assert (w, mode) == ((wd, 1) if wd < wp else (wp, 0)), (dt, n, c, w, mode, wp, wd)
            assert hb == int(sent.any())
            size = 16 + 128 * hb + (cc.size * w + 7) // 8
            assert offs[c + 1] - offs[c] == (size + 15) // 16 * 16


def pin_pack_errors(L):
    st = O.quantize("abs", synth.sines_1d(3000, 67, dtype=np.float32), 1e-3, L=L)
    pk = O.pack(st, np.float32, 3000, L=L)
    C = 3
    ot = (64 + 8 * C + 15) // 16 * 16
    pl = (ot + 8 * (C + 1) + 15) // 16 * 16
    for name, off, val in (("magic", 0, 0x58), ("n", 8, 0x01), ("width", pl, 40),
                           ("offset", ot + 8, 0xFF)):
        bad = pk.copy()
        bad[off] = val if name != "n" else bad[off] ^ val
        try:
            O.unpack(bad, np.float32, 3000, L=L)
        except O.OracleError as e:
            assert e.status == O.ERR_STREAM, name
        else:
            raise AssertionError(f"accepted corrupted {name}")
    try:
        O.unpack(pk[:-1], np.float32, 3000, L=L)
    except O.OracleError as e:
        assert e.status == O.ERR_STREAM
    else:
        raise AssertionError("accepted truncated stream")


PINS = [pin_mitchell_golden, pin_mitchell_powers_of_two, pin_mitchell_log2_error,
        pin_mitchell_log2_monotone, pin_mitchell_pow2_error, pin_params_abs,
        pin_params_rel, pin_params_noa, pin_arg_errors, pin_structure, pin_bounds,
        pin_specials, pin_abs_nearest_bin, pin_rel_nearest_bin, pin_bin_range,
        pin_roundtrip_sizes, pin_stream_errors, pin_noa_degenerate, pin_inline_format,
        pin_ablation_abs_unchecked, pin_ablation_rel_libm, pin_pack_golden,
        pin_pack_roundtrip_and_widths, pin_pack_errors]
