"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

These stand in for the SDRBench single-precision suites the paper measures on
(section 5, Table 2), which are not available here, and for the paper's
generated special-value inputs (section 5).  Nothing in this module performs
the quantizers' arithmetic: it only draws numbers.  All draws use numpy's
PCG64 generator with an explicit seed, are computed in float64 and cast to the
field type with round-to-nearest-even.

Workloads:
  sines_1d        1-D sum of 8 sines plus N(0, 0.01) noise (2^20 float32)
  grf_3d          3-D Gaussian random field, power spectrum k^-3, unit variance
  rel_variant     sign * 10^(-30 + 60 Phi(g)) of a field g, 1 % exact zeros
  inject_specials NaN (quiet, signalling with payload), +-INF, +-0, denormals,
                  values next to half-bin borders, values whose bin overflows
  adversarial_abs values at (2k+1) e and one ulp either side (ABS/NOA borders)
  adversarial_rel values at Mitchell-antilog bin borders and one ulp either side

NOA's bound scales with the range of the field's finite values (section
2.1.3), so a NOA input gets a special-value mix that leaves that range
alone: no finite value outside the base field's [min, max] (no bin-overflow
values, no +-FLT_MAX), and its half-bin neighbours and bin-border values are
aimed at eps * R of the base field (R = max - min, computed here in float64
from the data; the quantizer's own rounded bound lies within a few ulps of
it).  `with_specials(x, q, ...)` picks the right mix for a quantizer.
"""
import math

import numpy as np

__all__ = ["sines_1d", "grf_3d", "rel_variant", "inject_specials", "n_specials",
           "adversarial_abs", "adversarial_rel", "special_classes", "finite_range",
           "noa_half_bin", "with_specials", "adversarial_noa"]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def sines_1d(n=1 << 20, seed=0, dtype=np.float32):
    """x[i] = sum_k A_k sin(2 pi f_k i / n + phi_k) + N(0, 0.01)."""
    rng = _rng(seed)
    amp = rng.uniform(0.1, 10.0, 8)
    freq = np.exp(rng.uniform(0.0, math.log(max(n / 16.0, 1.0)), 8))
    phase = rng.uniform(0.0, 2 * math.pi, 8)
    t = np.arange(n, dtype=np.float64) / n
    x = np.zeros(n, dtype=np.float64)
    for a, f, p in zip(amp, freq, phase):
        x += a * np.sin(2 * math.pi * f * t + p)
    x += rng.normal(0.0, 0.01, n)
    return x.astype(dtype)


def grf_3d(N, seed, dtype=np.float32, workers=None):
    """Gaussian random field on an N^3 grid with power spectrum ~ |k|^-3
    (amplitude |k|^-3/2, zero mean mode), normalised to mean 0, variance 1.
    Returns a flat array of N^3 values (C order)."""
    import scipy.fft as sfft
    if workers is None:
        import os
        workers = max(1, min(16, os.cpu_count() or 1))
    rng = _rng(seed)
    w = rng.standard_normal((N, N, N))
    spec = sfft.rfftn(w, workers=workers)
    del w
    k0 = np.fft.fftfreq(N) * N
    k2 = np.fft.rfftfreq(N) * N
    kk = (k0[:, None, None] ** 2 + k0[None, :, None] ** 2)
    # multiply plane by plane to bound memory
    for i in range(N):
        mag = np.sqrt(kk[i] + k2[None, :] ** 2)
        with np.errstate(divide="ignore"):
            amp = np.where(mag > 0, mag ** -1.5, 0.0)
        spec[i] *= amp
    g = sfft.irfftn(spec, s=(N, N, N), workers=workers).reshape(-1)
    del spec
    g -= g.mean()
    g /= g.std()
    return g.astype(dtype)


def rel_variant(g, seed, dtype=None, zero_frac=0.01):
    """Lognormal-magnitude variant for REL: x = s * 10^(-30 + 60 Phi(g)) with
    i.i.d. random signs s and zero_frac of positions set to exactly +0, so
    log10|x| ~ U(-30, 30) while the field stays spatially smooth."""
    from scipy.special import ndtr
    dtype = dtype or g.dtype
    rng = _rng(seed)
    u = ndtr(np.asarray(g, dtype=np.float64))
    x = np.power(10.0, -30.0 + 60.0 * u)
    sign = rng.integers(0, 2, x.size, dtype=np.int8)
    x[sign == 1] *= -1.0
    nz = int(round(zero_frac * x.size))
    if nz:
        x[rng.choice(x.size, nz, replace=False)] = 0.0
    return x.astype(dtype)


def plain_step_inputs(N=512, eb=1e-3, seed=1, rel_seed=11, frac=1e-4):
    """The single-field workload: an N^3 float32 Gaussian random field with a
    fraction `frac` of special values (for ABS), the same field with the
    same fraction of range-preserving specials aimed at eb * R (for NOA),
    and its lognormal-magnitude variant (for REL) with `frac` specials.
    Returns (x_abs, x_noa, x_rel)."""
    g = grf_3d(N, seed, dtype=np.float64)
    base = g.astype(np.float32)
    nsp = n_specials(base.size, frac)
    x, _, _ = inject_specials(base, nsp, seed + 1000, eb)
    xn = plain_noa_field(base, eb, seed, frac)
    del base
    xr = rel_variant(g, rel_seed, dtype=np.float32)
    del g
    xr, _, _ = inject_specials(xr, nsp, rel_seed + 1000, eb)
    return x, xn, xr


def plain_noa_field(base, eb, seed=1, frac=1e-4):
    """The NOA field of the single-field workload for bound eb: the base
    grid (float32 GRF of `seed`, no specials) with `frac` range-keeping
    specials, half-bin neighbours at eb * R."""
    return with_specials(base, "noa", n_specials(base.size, frac), seed + 2000, eb)


def f64_grid_inputs(N=384, abs_eb=1e-6, rel_eb=1e-4, seed=2, rel_seed=12, frac=1e-4,
                    adversarial=1 << 20, adv_seed=22, noa_eb=None):
    """The float64 single-field workload: an N^3 Gaussian random field with
    a fraction `frac` of special values and the `adversarial` contiguous
    values from n/2 on replaced by ABS bin-border values for abs_eb; the
    same field with range-preserving specials and NOA bin-border values
    (aimed at noa_eb * R of the base field, noa_eb defaulting to abs_eb) in
    the same place; the REL variant likewise with REL bin-border values for
    rel_eb.  Returns (x_abs, x_noa, x_rel)."""
    noa_eb = abs_eb if noa_eb is None else noa_eb
    g = grf_3d(N, seed, dtype=np.float64)
    nsp = n_specials(g.size, frac)
    x, _, _ = inject_specials(g, nsp, seed + 1000, abs_eb)
    half = noa_half_bin(g, noa_eb)
    lo, hi = finite_range(g)
    xn = with_specials(g, "noa", nsp, seed + 2000, noa_eb)
    xr = rel_variant(g, rel_seed, dtype=np.float64)
    del g
    xr, _, _ = inject_specials(xr, nsp, rel_seed + 1000, rel_eb)
    if adversarial:
        h = x.size // 2
        x[h: h + adversarial] = adversarial_abs(adversarial, abs_eb, adv_seed, np.float64)
        xn[h: h + adversarial] = adversarial_noa(adversarial, half, lo, hi, adv_seed + 2,
                                                 np.float64)
        xr[h: h + adversarial] = adversarial_rel(adversarial, rel_eb, adv_seed + 1, np.float64)
    return x, xn, xr


def n_specials(n, frac):
    return int(round(n * frac))


def special_classes(dtype, in_range=False):
    """Class names injected round-robin.  in_range: only classes that never
    put a finite value outside the field's range (no bin overflow, no
    +-max); see inject_specials."""
    out = ["qnan+", "qnan-", "snan", "inf+", "inf-", "zero+", "zero-",
           "den_min+", "den_min-", "den_max+", "den_max-", "den_rand+", "den_rand-",
           "half_prev", "half_at", "half_next"]
    return out if in_range else out + ["overflow", "fmax+", "fmax-"]


def finite_range(x):
    """Smallest and largest finite value of x as Python floats (-0 counts as
    +0); (inf, -inf) when x has none."""
    x = np.asarray(x)
    f = x[np.isfinite(x)]
    if f.size == 0:
        return float("inf"), float("-inf")
    lo, hi = float(f.min()), float(f.max())
    return (0.0 if lo == 0 else lo), (0.0 if hi == 0 else hi)


def noa_half_bin(x, eps):
    """eps * (max - min) of x's finite values, in float64: the NOA bin
    half-width that bin-border inputs aim at (0 when the range is empty)."""
    lo, hi = finite_range(x)
    return eps * (hi - lo) if hi > lo else 0.0


def with_specials(x, q, count, seed, eb):
    """x with `count` special values for quantizer q: the full mix for ABS /
    REL (half-bin neighbours at eb); for NOA the range-preserving mix with
    half-bin neighbours at eb * R of x."""
    if q == "noa":
        lo, hi = finite_range(x)
        out, _, _ = inject_specials(x, count, seed, noa_half_bin(x, eb), in_range=(lo, hi))
        return out
    out, _, _ = inject_specials(x, count, seed, eb)
    return out


def _bits_view(dtype):
    return np.uint32 if np.dtype(dtype) == np.float32 else np.uint64


def _special_value(cls, dtype, rng, eb, in_range=None):
    dtype = np.dtype(dtype)
    f32 = dtype == np.float32
    ut = _bits_view(dtype)
    mbits = 23 if f32 else 52
    ebits = 8 if f32 else 11
    expmask = ((1 << ebits) - 1) << mbits
    sign = 1 << (mbits + ebits)
    fmax = np.finfo(dtype).max

    def from_bits(b):
        return np.array([b], dtype=ut).view(dtype)[0]
    if cls in ("qnan+", "qnan-"):
        b = expmask | (1 << (mbits - 1)) | int(rng.integers(0, 1 << 8))
        return from_bits(b | (sign if cls == "qnan-" else 0))
    if cls == "snan":  # quiet bit clear, non-zero payload
        return from_bits(expmask | int(rng.integers(1, 1 << (mbits - 1))))
    if cls == "inf+":
        return dtype.type(np.inf)
    if cls == "inf-":
        return dtype.type(-np.inf)
    if cls == "zero+":
        return dtype.type(0.0)
    if cls == "zero-":
        return dtype.type(-0.0)
    if cls.startswith("den_"):
        s = sign if cls.endswith("-") else 0
        if cls.startswith("den_min"):
            return from_bits(1 | s)
        if cls.startswith("den_max"):
            return from_bits(((1 << mbits) - 1) | s)
        return from_bits(int(rng.integers(1, 1 << mbits)) | s)
    if cls.startswith("half_"):
        if in_range is None:
            k = int(rng.integers(-10000, 10001))
        else:
            # (2k+1) eb strictly inside the range, one ulp either side too
            lo, hi = in_range
            kmin = max(-10000, math.ceil((lo / eb - 1) / 2) + 1) if eb > 0 else 0
            kmax = min(10000, math.floor((hi / eb - 1) / 2) - 1) if eb > 0 else -1
            if kmin > kmax:  # no bin border inside the range
                return from_bits(expmask | (1 << (mbits - 1)))
            k = int(rng.integers(kmin, kmax + 1))
        v = dtype.type((2 * k + 1) * eb)
        if cls == "half_prev":
            return np.nextafter(v, dtype.type(-np.inf))
        if cls == "half_next":
            return np.nextafter(v, dtype.type(np.inf))
        return v
    if cls == "overflow":  # |x| / (2 eb) beyond the 2^30 bin range
        lo = math.log(min(2.0 ** 31 * eb, float(fmax) / 2))
        hi = math.log(float(fmax))
        v = math.exp(rng.uniform(lo, hi))
        return dtype.type(v if rng.integers(0, 2) else -v)
    if cls == "fmax+":
        return dtype.type(fmax)
    if cls == "fmax-":
        return dtype.type(-fmax)
    raise ValueError(cls)


def inject_specials(x, count, seed, eb, in_range=None):
    """Replace `count` positions of x (chosen without replacement) by special
    values; the classes are assigned round-robin over the sorted positions.
    in_range = (lo, hi): keep every finite value inside [lo, hi] (the NOA
    mix): no overflow / +-max classes, half-bin neighbours at (2k+1) eb
    strictly inside, and zeros / denormals replaced by quiet NaNs when 0
    lies outside [lo, hi].  Returns (x_copy, positions, class_names)."""
    x = np.array(x, copy=True)
    rng = _rng(seed)
    count = min(count, x.size)
    pos = np.sort(rng.choice(x.size, count, replace=False)) if count else np.zeros(0, np.int64)
    classes = special_classes(x.dtype, in_range is not None)
    zero_ok = in_range is None or (in_range[0] <= 0.0 <= in_range[1])
    names = []
    for j, p in enumerate(pos):
        c = classes[j % len(classes)]
        if not zero_ok and (c.startswith("zero") or c.startswith("den_")):
            c = "qnan+"
        x[p] = _special_value(c, x.dtype, rng, eb, in_range)
        names.append(c)
    return x, pos, names


def adversarial_abs(m, eb, seed, dtype):
    """m values at (2k + 1) * eb (an ABS/NOA bin border for bound eb) and one
    ulp below / above, k ~ U{-2^20, 2^20}."""
    rng = _rng(seed)
    dtype = np.dtype(dtype)
    k = rng.integers(-(1 << 20), (1 << 20) + 1, m)
    sgn = np.where(rng.integers(0, 2, m) == 1, 1.0, -1.0)
    v = (2.0 * k + sgn) * eb
    v = v.astype(dtype)
    j = rng.integers(-1, 2, m)
    v = np.where(j < 0, np.nextafter(v, dtype.type(-np.inf)), v)
    v = np.where(j > 0, np.nextafter(v, dtype.type(np.inf)), v)
    return v.astype(dtype)


def adversarial_noa(m, half, lo, hi, seed, dtype):
    """m values at (2k + 1) * half and one ulp below / above, with k drawn so
    that every value lies strictly inside [lo, hi] (NOA bin borders of a
    field whose range is [lo, hi] and bin half-width `half`)."""
    rng = _rng(seed)
    dtype = np.dtype(dtype)
    kmin = math.ceil((lo / half - 1) / 2) + 1
    kmax = math.floor((hi / half - 1) / 2) - 1
    k = rng.integers(kmin, kmax + 1, m)
    v = ((2.0 * k + 1.0) * half).astype(dtype)
    j = rng.integers(-1, 2, m)
    v = np.where(j < 0, np.nextafter(v, dtype.type(-np.inf)), v)
    v = np.where(j > 0, np.nextafter(v, dtype.type(np.inf)), v)
    return v.astype(dtype)


def adversarial_rel(m, eb, seed, dtype):
    """m values at the Mitchell antilog of (k +- 1/2) * 2 eb (an approximate
    REL bin border for bound eb) and one ulp either side, random signs."""
    rng = _rng(seed)
    dtype = np.dtype(dtype)
    step = 2.0 * eb
    lim = 100.0 if dtype == np.float32 else 900.0
    k = rng.integers(int(-lim / step), int(lim / step), m)
    y = (k + np.where(rng.integers(0, 2, m) == 1, 0.5, -0.5)) * step
    fl = np.floor(y)
    v = np.ldexp(1.0 + (y - fl), fl.astype(np.int64))
    v = v.astype(dtype)
    j = rng.integers(-1, 2, m)
    v = np.where(j < 0, np.nextafter(v, dtype.type(-np.inf)), v)
    v = np.where(j > 0, np.nextafter(v, dtype.type(np.inf)), v)
    v = np.where(rng.integers(0, 2, m) == 1, -v, v)
    return v.astype(dtype)


def log_uniform_sizes(rng, m, lo_bytes, hi_bytes):
    """m sizes in bytes, log-uniform on [lo_bytes, hi_bytes]."""
    return np.exp(rng.uniform(np.log(lo_bytes), np.log(hi_bytes), m))


def field_specs(m, seed, lo_bytes, hi_bytes, p_f32=0.7, eb_lo=1e-5, eb_hi=1e-1):
    """Per-field (or per-payload) choices of the batched / serving workloads:
    byte size log-uniform on [lo_bytes, hi_bytes], float32 with probability
    p_f32 else float64, quantizer uniform over ABS / REL / NOA, bound
    log-uniform on [eb_lo, eb_hi].  Returns a list of dicts."""
    rng = _rng(seed)
    sizes = log_uniform_sizes(rng, m, lo_bytes, hi_bytes)
    out = []
    for b in sizes:
        f32 = rng.random() < p_f32
        s = 4 if f32 else 8
        out.append(dict(dtype=np.float32 if f32 else np.float64, n=max(1, int(b) // s),
                        q=["abs", "rel", "noa"][int(rng.integers(0, 3))],
                        eb=float(np.exp(rng.uniform(np.log(eb_lo), np.log(eb_hi)))),
                        offset_u=float(rng.random())))
    return out


def field_data(spec, master, rel_master, seed, special_frac=1e-4):
    """A field's values: a contiguous (wrapping) slice of the master field
    (its lognormal variant for REL), cast to the field's dtype, with
    special_frac of the positions replaced by special values (for NOA the
    range-preserving mix aimed at the slice's own eb * R)."""
    src = rel_master if spec["q"] == "rel" else master
    n = spec["n"]
    off = int(spec["offset_u"] * src.size)
    if off + n <= src.size:
        x = src[off: off + n].astype(spec["dtype"])
    else:
        x = np.take(src, np.arange(off, off + n) % src.size).astype(spec["dtype"])
    k = int(round(n * special_frac))
    if k:
        x = with_specials(x, spec["q"], k, seed, spec["eb"])
    return x


def poisson_arrivals(rate_per_s, seconds, seed):
    """Arrival times (ns) of a Poisson process of the given rate."""
    rng = _rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= seconds:
            break
        out.append(int(t * 1e9))
    return np.array(out, dtype=np.int64)
