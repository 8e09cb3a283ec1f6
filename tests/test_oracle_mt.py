"""The oracle's chunk-parallel wrapper gives the single-threaded oracle's
bytes and statuses: every quantizer (and both section 6 ablations), both
dtypes, ragged sizes, special values, runs of chunks full of outliers,
degenerate and huge NOA ranges, thread counts below, at and above the
number of chunks; and the same errors on corrupted streams."""
import numpy as np
import pytest

import oracle as O
import synth

SIZES = [0, 1, 1023, 1024, 1025, 3 * 1024 + 517, 65536 + 13, (1 << 20) + 333]
THREADS = [1, 2, 3, 7, 16, 300]


def _inputs(dt, n, q, seed):
    x = synth.sines_1d(max(n, 1), seed, dtype=dt)[:n]
    if q in ("rel", "rel_libm"):
        x = synth.rel_variant(x.astype(np.float64), seed + 1, dtype=dt)
    if n:
        x = synth.with_specials(x, "noa" if q == "noa" else "abs", max(1, n // 500), seed + 2, 1e-3)
    return x


def _same(q, x, eb, threads):
    a = O.quantize(q, x, eb)
    b = O.quantize_mt(q, x, eb, threads)
    assert a.size == b.size and np.array_equal(a, b), (q, x.dtype, x.size, eb, threads)
    if q in ("abs_unchecked", "rel_libm"):
        return a
    d1 = O.dequantize(a, x.dtype, x.size)
    d2 = O.dequantize_mt(a, x.dtype, x.size, threads)
    u = np.uint32 if x.dtype == np.float32 else np.uint64
    assert np.array_equal(d1.view(u), d2.view(u)), (q, x.dtype, x.size, threads)
    return a


@pytest.mark.parametrize("dt", [np.float32, np.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("q", ["abs", "rel", "noa", "abs_unchecked", "rel_libm"])
def test_mt_same_bytes(dt, q):
    for i, n in enumerate(SIZES):
        x = _inputs(dt, n, q, 500 + i)
        for t in THREADS if n < (1 << 20) else (3, 16):
            _same(q, x, 1e-3, t)


@pytest.mark.parametrize("dt", [np.float32, np.float64], ids=["f32", "f64"])
def test_mt_outlier_runs_and_edges(dt):
    n = 40 * 1024 + 77
    x = synth.sines_1d(n, 520, dtype=dt)
    # runs of chunks where every other value is NaN, across range borders
    x[5000:30000:2] = np.nan
    rng = np.random.default_rng(521)
    bits = rng.integers(0, np.iinfo(np.uint32 if dt == np.float32 else np.uint64).max,
                        6000, dtype=np.uint32 if dt == np.float32 else np.uint64)
    x[33000:39000] = bits.view(dt)
    for q in ("abs", "rel", "noa"):
        for t in (2, 5, 13):
            _same(q, x, 1e-2, t)
    # all special, constant (degenerate NOA), huge NOA range
    allsp, _, _ = synth.inject_specials(synth.sines_1d(9000, 522, dtype=dt), 9000, 523, 1e-3)
    const = np.full(5000, 2.5, dtype=dt)
    huge, _, _ = synth.inject_specials(synth.sines_1d(9000, 524, dtype=dt), 100, 525, 1e-3)
    for y in (allsp, const, huge):
        for q in ("abs", "rel", "noa"):
            _same(q, y, 1e-3, 4)


def test_mt_same_errors_on_corrupt_streams():
    n = 20 * 1024 + 300
    x = _inputs(np.float32, n, "abs", 530)
    x[::97] = np.nan  # an outlier in every chunk
    st = O.quantize("abs", x, 1e-3)
    C = (n + 1023) // 1024
    ct = (64 + 4 * n + 15) // 16 * 16
    cases = []
    for c in (0, 1, 7, 10, C - 1):  # first entries of ranges and inside them
        b = st.copy()
        b[ct + 8 * c] ^= 1
        cases.append(b)
    b = st.copy()
    b[16] ^= 1  # outlier count
    cases.append(b)
    b = st.copy()
    b[64 + 4 * 5: 64 + 4 * 6] = np.frombuffer(np.int32(-(1 << 31)).tobytes(), np.uint8)
    cases.append(b)  # an extra sentinel
    cases.append(st[:-1])  # truncated
    for b in cases:
        errs = []
        for fn in (lambda: O.dequantize(b, np.float32, n),
                   lambda: O.dequantize_mt(b, np.float32, n, 3),
                   lambda: O.dequantize_mt(b, np.float32, n, 16)):
            try:
                fn()
                errs.append(O.OK)
            except O.OracleError as e:
                errs.append(e.status)
        assert errs[0] == errs[1] == errs[2] == O.ERR_STREAM, errs


def test_mt_thread_count():
    assert O.threads_used(5) == 5
    assert O.threads_used(0) >= 1
    assert O.threads_used(10 ** 6) == 256
