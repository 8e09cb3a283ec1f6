"""GPU vs oracle parity: the HIP library's stream and decode must equal the
CPU oracle's byte for byte (integer / byte work: bit-exact), on the same
seeded inputs, across dtypes, quantizers, bounds, tile-spanning sizes with
ragged tails and the edge cases of the method."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce, bits, first_diff, gpu_decode, gpu_roundtrip
from streamcheck import SENT, abs_violations, check_structure, finite_range, parse, rel_violations

pytestmark = pytest.mark.gpu

DTYPES = [np.float32, np.float64]


def _parity(q, x, eb, label=""):
    announce("parity", q, x.dtype, x.size, eb, label)
    st_g, dec_g = gpu_roundtrip(q, x, eb)
    st_o = O.quantize(q, x, eb)
    diff = first_diff(st_g, st_o)
    assert diff is None, f"{label} {q} {x.dtype} n={x.size} eb={eb}: stream {diff}"
    dec_o = O.dequantize(st_o, x.dtype, x.size)
    diff = first_diff(bits(dec_g), bits(dec_o))
    assert diff is None, f"{label} {q} {x.dtype} n={x.size} eb={eb}: decode {diff}"
    return st_g, dec_g


def _field(dt, n, seed, eb, q):
    x = synth.sines_1d(n, seed, dtype=dt)
    if q == "noa":  # specials that keep the range, half-bin values at eb * R
        return synth.with_specials(x, "noa", max(19, n // 1000), seed + 1, eb)
    x, _, _ = synth.inject_specials(x, max(19, n // 1000), seed + 1, eb)
    if q == "rel":
        x = synth.rel_variant(np.nan_to_num(x.astype(np.float64)), seed + 2, dtype=dt)
        x, _, _ = synth.inject_specials(x, max(19, n // 1000), seed + 3, eb)
    return x


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("q,eb", [("abs", 1e-3), ("abs", 1e-6), ("noa", 1e-4),
                                  ("rel", 1e-2), ("rel", 1e-3)])
def test_parity_mixed(dt, q, eb):
    # several tiles plus a ragged tail, specials, bin-border adversarial values
    n = 5 * 4096 + 777
    x = _field(dt, n, 11, eb, q)
    if q == "rel":
        adv = synth.adversarial_rel(3000, eb, 12, dt)
    elif q == "noa":  # bin borders of the field's own range, which they keep
        lo, hi = synth.finite_range(x)
        adv = synth.adversarial_noa(3000, synth.noa_half_bin(x, eb), lo, hi, 12, dt)
    else:
        adv = synth.adversarial_abs(3000, eb, 12, dt)
    x = np.concatenate([x, adv]).astype(dt)
    st, _ = _parity(q, x, eb)
    if q == "noa":
        # a real range: most codes are bins other than 0, and the border
        # values send some through the lossless fallback
        codes = parse(st, dt)["codes"]
        assert np.count_nonzero((codes != 0) & (codes != SENT)) > x.size // 2
        assert parse(st, dt)["hdr"]["k"] > max(19, n // 1000)


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
def test_parity_noa_huge_range_edge(dt):
    """Edge case: finite specials up to +-max stretch NOA's range to the
    whole type, so the bound saturates and nearly every value lands in bin
    0; still the oracle's bytes."""
    n = 5 * 4096 + 777
    x = synth.sines_1d(n, 13, dtype=dt)
    x, _, _ = synth.inject_specials(x, max(19, n // 1000), 14, 1e-4)
    st, _ = _parity("noa", x, 1e-4, "huge range")
    assert parse(st, dt)["hdr"]["bound"] > np.finfo(dt).max / 1e9


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096,
                               4097, 8191, 12289, 65536 + 13])
def test_parity_sizes(dt, n):
    x = synth.sines_1d(max(n, 1), 21, dtype=dt)[:n]
    for q, eb in (("abs", 1e-3), ("noa", 1e-3), ("rel", 1e-3)):
        y = x if q != "rel" else synth.rel_variant(x.astype(np.float64), 22, dtype=dt)
        _parity(q, y, eb, f"n={n}")


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
def test_parity_all_specials(dt):
    base = synth.sines_1d(9000, 31, dtype=dt)
    x, _, _ = synth.inject_specials(base, 9000, 32, 1e-3)  # every value special
    for q in ("abs", "rel", "noa"):
        st, dec = _parity(q, x, 1e-3, "all-specials")
        P = parse(st, dt)
        assert not check_structure(P, x, dt)


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
def test_parity_degenerate_noa(dt):
    x = np.full(10000, 3.5, dt)
    x[17] = np.inf
    st, dec = _parity("noa", x, 1e-2, "constant")
    assert np.all(parse(st, dt)["codes"] == SENT)
    x = np.full(5000, np.nan, dt)
    _parity("noa", x, 1e-2, "no-finite")


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
def test_parity_bin_range(dt):
    # every value's bin near +-2^30 and beyond, and values that need INT_MIN
    rng = np.random.default_rng(41)
    t = rng.uniform(-2.0 ** 31.5, 2.0 ** 31.5, 20000)
    t[:8] = [2.0 ** 30, -(2.0 ** 30), 2.0 ** 31, -(2.0 ** 31), 2.0 ** 30 - 64,
             -(2.0 ** 30) + 64, 2.0 ** 30 + 64, -(2.0 ** 30) - 64]
    x = t.astype(dt)  # eb = 0.5 -> step 1, bin = rint(x)
    _parity("abs", x, 0.5, "bin-range")
    fmax = np.finfo(dt).max
    y = np.array([fmax, -fmax, fmax / 2, -fmax / 3, 1.0, -1.0] * 700, dt)
    for q in ("abs", "noa", "rel"):
        _parity(q, y, 1e-3 if q != "abs" else 1e-30, "huge")


@pytest.mark.parametrize("eb", [1e-1, 1e-3, 1e-5, 1e-7, 0.5, 0.999])
def test_parity_rel_bounds(eb):
    for dt in DTYPES:
        mag = np.power(10.0, np.random.default_rng(51).uniform(-37, 37, 30000))
        x = (mag * np.where(np.arange(mag.size) % 3 == 0, -1, 1)).astype(dt)
        _parity("rel", x, eb, "rel-eb")


def test_decode_oracle_stream_and_errors():
    """The GPU decoder reads oracle-made streams, and rejects broken ones."""
    for dt in DTYPES:
        x = _field(dt, 3 * 4096 + 5, 61, 1e-3, "abs")
        st = O.quantize("abs", x, 1e-3)
        ref = O.dequantize(st, dt, x.size)
        announce("decode-oracle", dt)
        got, status = gpu_decode(st, dt, x.size)
        assert status == 0 and first_diff(bits(got), bits(ref)) is None
        bad = st.copy(); bad[0] ^= 0xFF
        announce("decode-bad-magic", dt)
        _, status = gpu_decode(bad, dt, x.size)
        assert status == 3
        bad = st.copy()
        ct = (64 + 4 * x.size + 15) // 16 * 16
        bad[ct + 8] ^= 0x01  # chunk table entry 1
        announce("decode-bad-chunk", dt)
        _, status = gpu_decode(bad, dt, x.size)
        assert status == 3
        announce("decode-truncated", dt)
        _, status = gpu_decode(st[: st.size - 1], dt, x.size) if parse(st, dt)["hdr"]["k"] else (None, 3)
        assert status == 3
        # a good decode after an error reports OK again
        got, status = gpu_decode(st, dt, x.size)
        assert status == 0


def test_bounds_hold_on_gpu_output():
    """Independent of the oracle: GPU decodes satisfy the bound exactly."""
    for dt in DTYPES:
        for q, eb in (("abs", 1e-4), ("noa", 1e-3), ("rel", 1e-3)):
            x = _field(dt, 2 * 4096 + 99, 71, eb, q)
            announce("bound", q, dt)
            st, dec = gpu_roundtrip(q, x, eb)
            if q == "rel":
                bad, bsp = rel_violations(x, dec, eb)
            else:
                from fractions import Fraction
                bound = Fraction(eb)
                if q == "noa":
                    lo, hi = finite_range(x)
                    bound *= Fraction(hi) - Fraction(lo)
                bad, bsp = abs_violations(x, dec, bound)
            assert bad.size == 0 and bsp.size == 0
            assert not check_structure(parse(st, dt), x, dt)


def test_stream_reuse_and_determinism():
    """Same input twice (buffers and workspace reused) -> identical bytes;
    a smaller call after a larger one is unaffected by leftovers."""
    import torch
    import paper_2407_15037_amd as lcq
    x = _field(np.float32, 7 * 4096 + 3, 81, 1e-3, "abs")
    xt = torch.from_numpy(x).cuda()
    ws = torch.empty(lcq.workspace_bytes("noa", torch.float32, x.size), dtype=torch.uint8, device="cuda")
    out = torch.empty(lcq.max_stream_bytes(torch.float32, x.size), dtype=torch.uint8, device="cuda")
    nb = torch.empty(1, dtype=torch.int64, device="cuda")
    sizes = []
    streams = []
    announce("reuse")
    for xi in (xt, xt, xt[: 4096 + 1]):
        for q in ("abs", "noa", "rel"):
            lcq.quantize(xi, q, 1e-3, out=out[: lcq.max_stream_bytes(torch.float32, xi.numel())],
                         nbytes=nb, ws=ws)
            torch.cuda.synchronize()
            s = int(nb.item())
            sizes.append(s)
            streams.append(out[:s].cpu().numpy().copy())
    for i in range(3):
        assert np.array_equal(streams[i], streams[3 + i])
    xs = x[: 4096 + 1]
    for i, q in enumerate(("abs", "noa", "rel")):
        assert np.array_equal(streams[6 + i], O.quantize(q, xs, 1e-3))


def test_lookback_fallback_same_bytes():
    """With the look-back wait forced to zero polls, every workgroup counts
    unfinished predecessor tiles from their input itself; the stream must not
    change."""
    import paper_2407_15037_amd as lcq
    try:
        lcq.set_lookback_spin(0)
        for dt in DTYPES:
            for q, eb in (("abs", 1e-3), ("noa", 1e-3), ("rel", 1e-2)):
                x = _field(dt, 9 * 4096 + 1234, 91, eb, q)
                _parity(q, x, eb, "spin0")
    finally:
        lcq.set_lookback_spin(4096)


def test_every_launch_variant_same_bytes():
    """All launch-shape variants (tile sizes, loads in flight) produce the
    oracle's bytes, including ragged tails and multi-tile look-backs."""
    import torch
    import paper_2407_15037_amd as lcq
    saved = {tdt: (lcq.tune_get("quantize", tdt), lcq.tune_get("dequantize", tdt))
             for tdt in (torch.float32, torch.float64)}
    try:
        for v in range(lcq.tune_variants()):
            for dt, tdt in ((np.float32, torch.float32), (np.float64, torch.float64)):
                lcq.tune_set("quantize", tdt, v)
                lcq.tune_set("dequantize", tdt, v)
                for q, eb in (("abs", 1e-3), ("noa", 1e-4), ("rel", 1e-3)):
                    x = _field(dt, 11 * 4096 + 2345, 101 + v, eb, q)
                    _parity(q, x, eb, f"variant {v}")
    finally:
        for tdt, (qv, dv) in saved.items():
            lcq.tune_set("quantize", tdt, qv)
            lcq.tune_set("dequantize", tdt, dv)


def test_status_word_ignores_workspace_contents():
    """The decode status word is tagged per call: a workspace whose first
    bytes hold anything (here all ones, the largest possible word) still
    reports OK for a good stream and ERR_STREAM for a broken one, in both
    layouts."""
    import torch
    import paper_2407_15037_amd as lcq
    x = _field(np.float32, 3 * 4096 + 5, 261, 1e-3, "abs")
    st = O.quantize("abs", x, 1e-3)
    sti = O.quantize_inline("abs", x, 1e-3)
    for fill in (0xFF, 0x00, 0x7F):
        for inline in (False, True):
            s = sti if inline else st
            for broken in (False, True):
                b = s.copy()
                if broken:
                    b[0] ^= 0xFF
                announce("status word", hex(fill), "inline" if inline else "list", broken)
                buf = torch.from_numpy(b).cuda()
                ws = torch.full((64,), fill, dtype=torch.uint8, device="cuda")
                if inline:
                    lcq.dequantize_inline(buf, torch.float32, x.size, ws=ws)
                else:
                    lcq.dequantize(buf, torch.float32, x.size, ws=ws)
                assert lcq.stream_status(ws) == (3 if broken else 0)


@pytest.mark.parametrize("q", ["abs", "noa", "rel"])
def test_parity_sines_2_20(q):
    """The small 1-D case at its full size: 2^20 float32 values from the sum
    of 8 sines plus noise, 0.1 % special values (NaN, +-INF, +-0, denormals,
    half-bin neighbours, bins beyond 2^30; for NOA only the classes that keep
    the range), eb = 1e-3; streams and decodes compared whole."""
    n = 1 << 20
    x = synth.sines_1d(n, 1, dtype=np.float32)
    if q == "noa":  # the range-keeping mix, half-bin neighbours at eb * R
        x = synth.with_specials(x, "noa", synth.n_specials(n, 1e-3), 2, 1e-3)
    else:
        x, _, _ = synth.inject_specials(x, synth.n_specials(n, 1e-3), 2, 1e-3)
    if q == "rel":
        x = synth.rel_variant(np.nan_to_num(x.astype(np.float64)), 3, dtype=np.float32)
        x, _, _ = synth.inject_specials(x, synth.n_specials(n, 1e-3), 4, 1e-3)
    _parity(q, x, 1e-3, "sines 2^20")


@pytest.mark.parametrize("q,eb", [("abs", 1e-3), ("abs", 1e-12), ("noa", 1e-6), ("rel", 1e-3),
                                  ("rel", 1e-9)])
def test_parity_random_float64_bit_patterns(q, eb):
    """2^22 float64 values with uniformly random bit patterns (every
    exponent, NaN payloads, INF, denormals, values whose bin leaves the
    range): the float64 counterpart of the exhaustive float32 sweep."""
    rng = np.random.default_rng(int(-np.log10(eb)) * 10 + len(q))
    u = rng.integers(0, np.iinfo(np.uint64).max, 1 << 22, dtype=np.uint64, endpoint=True)
    x = u.view(np.float64)
    _parity(q, x, eb, "random f64 bits")


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("q,eb", [("abs", 1e-3), ("noa", 1e-3), ("rel", 1e-3)])
@pytest.mark.parametrize("nchunks", [40, 300, 1203])
def test_parity_overflow_runs(dt, q, eb, nchunks):
    """Runs of chunks with more outliers than a chunk stages (NaN every other
    value, or random bit patterns) in a smooth field: a run across a group
    boundary, a run of random bits, and a ragged last chunk full of NaNs;
    runs of chunks whose staged rows are longer than one pass-2 copy round
    or sit at the stage cap.
    Such chunks are rescanned by workgroups other than their own group's, at
    offsets found from the pass-1 sums; the stream must still equal the
    oracle's."""
    n = nchunks * 1024 - 333
    x = _field(dt, n, 900 + nchunks, eb, q)
    rng = np.random.default_rng(nchunks)
    a, b = 60 * 1024, min(75 * 1024, n)
    x[a:b:2] = np.nan
    if nchunks > 200:
        ub = np.uint64 if dt == np.float64 else np.uint32
        lo, hi = 200 * 1024, 264 * 1024
        x[lo:hi] = rng.integers(0, np.iinfo(ub).max, hi - lo, dtype=ub, endpoint=True).view(dt)
        # stretches with 114, 128, 256 and 342 outliers per chunk: staged
        # rows copied whole by other pass-2 workgroups, rows at the float32
        # and float64 stage caps (128, 256), and rows over both (rescanned)
        for s0, step in ((90, 9), (100, 8), (120, 4), (140, 3)):
            x[s0 * 1024:(s0 + 10) * 1024:step] = np.nan
    x[(nchunks - 1) * 1024:] = np.nan
    st, _ = _parity(q, x, eb, f"overflow runs {nchunks} chunks")
    k = int(st[16:24].view(np.uint64)[0])
    assert k >= (n - (nchunks - 1) * 1024) + (b - a) // 2, (k, n)
