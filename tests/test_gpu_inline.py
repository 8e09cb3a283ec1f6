"""GPU vs oracle parity for the in-line outlier layout (the paper's own,
section 3.1: one word per value, code or raw bits, plus a flag bitmap).
Stream bytes and decodes must equal the oracle's bit for bit; decodes must
also equal those of the separate-list layout; broken headers are rejected."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce, bits, first_diff

pytestmark = pytest.mark.gpu

DTYPES = [np.float32, np.float64]


def _tdt(dt):
    import torch
    return torch.float32 if np.dtype(dt) == np.float32 else torch.float64


def gpu_inline(q, x, eb):
    import torch
    import paper_2407_15037_amd as lcq
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    st = lcq.quantize_inline(xt, q, eb)
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    dec = lcq.dequantize_inline(st, _tdt(x.dtype), x.size, ws=ws)
    status = lcq.stream_status(ws)
    return st.cpu().numpy(), dec.cpu().numpy(), status


def gpu_inline_decode(st, dt, n):
    import torch
    import paper_2407_15037_amd as lcq
    buf = torch.from_numpy(np.ascontiguousarray(st)).cuda()
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    try:
        out = lcq.dequantize_inline(buf, _tdt(dt), n, ws=ws)
    except lcq.LCQError as e:
        return None, e.status
    return out.cpu().numpy(), lcq.stream_status(ws)


def _parity(q, x, eb, label=""):
    announce("inline parity", q, x.dtype, x.size, eb, label)
    st_g, dec_g, status = gpu_inline(q, x, eb)
    assert status == 0
    st_o = O.quantize_inline(q, x, eb)
    diff = first_diff(st_g, st_o)
    assert diff is None, f"{label} {q} {x.dtype} n={x.size} eb={eb}: stream {diff}"
    dec_o = O.dequantize_inline(st_o, x.dtype, x.size)
    diff = first_diff(bits(dec_g), bits(dec_o))
    assert diff is None, f"{label} {q} {x.dtype} n={x.size} eb={eb}: decode {diff}"
    dec_l = O.dequantize(O.quantize(q, x, eb), x.dtype, x.size)
    assert first_diff(bits(dec_g), bits(dec_l)) is None, "in-line and list layouts decode differently"
    return st_g, dec_g


def _field(dt, n, seed, eb, q):
    x = synth.sines_1d(n, seed, dtype=dt)
    x, _, _ = synth.inject_specials(x, max(19, n // 1000), seed + 1, eb)
    if q == "rel":
        x = synth.rel_variant(np.nan_to_num(x.astype(np.float64)), seed + 2, dtype=dt)
        x, _, _ = synth.inject_specials(x, max(19, n // 1000), seed + 3, eb)
    return x


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("q,eb", [("abs", 1e-3), ("abs", 1e-6), ("noa", 1e-4),
                                  ("rel", 1e-2), ("rel", 1e-3)])
def test_inline_parity_mixed(dt, q, eb):
    n = 5 * 4096 + 777
    x = _field(dt, n, 211, eb, q)
    adv = synth.adversarial_rel(3000, eb, 212, dt) if q == "rel" else synth.adversarial_abs(3000, eb, 212, dt)
    _parity(q, np.concatenate([x, adv]).astype(dt), eb)


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 7, 8, 9, 31, 32, 33, 63, 1023, 2047, 2048, 2049,
                               4095, 4096, 4097, 12289, 65536 + 13])
def test_inline_parity_sizes(dt, n):
    # tiles are 4096 (float32) / 2048 (float64) values; flag words 32 values
    x = synth.sines_1d(max(n, 1), 221, dtype=dt)[:n]
    x = x.copy()
    x[::7] = np.nan  # raw values at every flag-bit position over time
    for q, eb in (("abs", 1e-3), ("noa", 1e-3), ("rel", 1e-3)):
        y = x if q != "rel" else synth.rel_variant(np.nan_to_num(x.astype(np.float64)), 222, dtype=dt)
        if q == "rel" and n:
            y[::5] = np.inf
        _parity(q, y, eb, f"n={n}")


@pytest.mark.parametrize("dt", DTYPES, ids=["f32", "f64"])
def test_inline_all_specials_and_degenerate(dt):
    base = synth.sines_1d(9000, 231, dtype=dt)
    x, _, _ = synth.inject_specials(base, 9000, 232, 1e-3)
    for q in ("abs", "rel", "noa"):
        _parity(q, x, 1e-3, "all-specials")
    c = np.full(10000, 3.5, dt)
    c[17] = np.inf
    st, _ = _parity("noa", c, 1e-2, "constant")
    flags = st[(64 + c.itemsize * c.size + 15) // 16 * 16:]
    assert np.all(np.unpackbits(flags, bitorder="little")[: c.size] == 1)


def test_inline_decode_oracle_stream_and_errors():
    for dt in DTYPES:
        x = _field(dt, 3 * 4096 + 5, 241, 1e-3, "abs")
        st = O.quantize_inline("abs", x, 1e-3)
        ref = O.dequantize_inline(st, dt, x.size)
        announce("inline decode-oracle", dt)
        got, status = gpu_inline_decode(st, dt, x.size)
        assert status == 0 and first_diff(bits(got), bits(ref)) is None
        cases = {"magic": (0, 0xFF), "version": (4, 0x02), "dtype": (5, 0x01),
                 "quantizer": (6, 0x04), "byte7": (7, 0x0A), "n": (8, 0x01)}
        for name, (off, mask) in cases.items():
            bad = st.copy()
            bad[off] ^= mask
            with pytest.raises(O.OracleError) as e:
                O.dequantize_inline(bad, dt, x.size)
            assert e.value.status == O.ERR_STREAM
            announce("inline decode-bad", name, dt)
            _, status = gpu_inline_decode(bad, dt, x.size)
            assert status == 3, name
        announce("inline decode-truncated", dt)
        _, status = gpu_inline_decode(st[:-1], dt, x.size)
        assert status == 3
        got, status = gpu_inline_decode(st, dt, x.size)
        assert status == 0 and first_diff(bits(got), bits(ref)) is None


def test_inline_buffer_reuse():
    """A smaller call into buffers that held a larger stream writes the
    smaller stream exactly (padding and flag tail included)."""
    import torch
    import paper_2407_15037_amd as lcq
    x = _field(np.float32, 7 * 4096 + 3, 251, 1e-3, "abs")
    xt = torch.from_numpy(x).cuda()
    out = torch.full((lcq.inline_stream_bytes(torch.float32, x.size),), 0xAB, dtype=torch.uint8,
                     device="cuda")
    ws = torch.empty(lcq.inline_workspace_bytes("noa"), dtype=torch.uint8, device="cuda")
    announce("inline reuse")
    for m in (x.size, 4096 + 5, 13):
        for q in ("abs", "noa", "rel"):
            nb = lcq.inline_stream_bytes(torch.float32, m)
            st = lcq.quantize_inline(xt[:m], q, 1e-3, out=out[:nb], ws=ws)
            assert np.array_equal(st.cpu().numpy(), O.quantize_inline(q, x[:m], 1e-3)), (m, q)
