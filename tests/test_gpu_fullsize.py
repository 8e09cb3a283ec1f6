"""Parity at the full single-field sizes: the 512^3 float32 GRF (and its
lognormal variant for REL) at every bound of that workload, and the 384^3
float64 GRF with a 2^20-value adversarial bin-border slice (ABS / NOA at
1e-6, REL at 1e-4).  The oracle finishes these in seconds, so whole streams
and decodes are compared -- at eb = 1e-3 under every quantize / dequantize
launch variant the tuner can pick (the benchmark times whichever wins), and
for the in-line layout.

NOA fields carry special values that keep the base field's range (section
2.1.3: the bound scales with it), so their bins are the field's real bins:
each NOA test checks that the stream's bound is the field's eb * R (at most
4 ulps below it: RD(eb), hi - lo and the product are each rounded and then
stepped down once) and that most codes are bins other than 0."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce, bits, first_diff
from streamcheck import SENT, parse

pytestmark = pytest.mark.gpu

EB = 1e-3


@pytest.fixture(scope="module")
def fields():
    x, xn, xr = synth.plain_step_inputs(512, EB)
    return {"abs": x, "noa": xn, "rel": xr}


@pytest.fixture(scope="module")
def grf512():
    """The base grid of the float32 workload (no specials)."""
    return synth.grf_3d(512, 1, dtype=np.float64).astype(np.float32)


def assert_real_noa_range(st, x, eb, min_nonzero):
    """The NOA stream's bound is eb * R of x's finite values (exactly not
    above, at most 4 ulps below) and at least min_nonzero of the codes are
    bins other than 0."""
    P = parse(st, x.dtype)
    lo, hi = synth.finite_range(x)
    exact = Fraction(eb) * (Fraction(hi) - Fraction(lo))
    ebr = P["hdr"]["bound"]
    ulp = Fraction(float(np.spacing(ebr)))
    assert Fraction(float(ebr)) <= exact, (ebr, float(exact))
    assert exact - Fraction(float(ebr)) <= 4 * ulp, (ebr, float(exact))
    codes = P["codes"]
    nz = np.count_nonzero((codes != 0) & (codes != SENT))
    assert nz >= min_nonzero * x.size, (nz, x.size)


@pytest.mark.parametrize("q", ["abs", "noa", "rel"])
def test_fullsize_every_variant(fields, q):
    import torch
    import paper_2407_15037_amd as lcq
    x = fields[q]
    n = x.size
    st_o = O.quantize(q, x, EB)
    dec_o = bits(O.dequantize(st_o, np.float32, n))
    xt = torch.from_numpy(x).cuda()
    out = torch.empty(lcq.max_stream_bytes(torch.float32, n), dtype=torch.uint8, device="cuda")
    nb = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(lcq.workspace_bytes(q, torch.float32, n), dtype=torch.uint8, device="cuda")
    dec = torch.empty(n, dtype=torch.float32, device="cuda")
    saved = (lcq.tune_get("quantize", torch.float32), lcq.tune_get("dequantize", torch.float32))
    try:
        for v in range(lcq.tune_variants()):
            lcq.tune_set("quantize", torch.float32, v)
            lcq.tune_set("dequantize", torch.float32, v)
            announce("fullsize", q, n, "variant", v)
            lcq.quantize(xt, q, EB, out=out, nbytes=nb, ws=ws)
            size = int(nb.item())
            diff = first_diff(out[:size].cpu().numpy(), st_o)
            assert diff is None, f"{q} variant {v}: stream {diff}"
            lcq.dequantize(out, torch.float32, n, stream_bytes=size, out=dec, ws=ws)
            assert lcq.stream_status(ws) == 0
            diff = first_diff(bits(dec.cpu().numpy()), dec_o)
            assert diff is None, f"{q} variant {v}: decode {diff}"
    finally:
        lcq.tune_set("quantize", torch.float32, saved[0])
        lcq.tune_set("dequantize", torch.float32, saved[1])
    if q == "noa":
        assert_real_noa_range(st_o, x, EB, 0.9)


@pytest.mark.parametrize("q", ["abs", "noa", "rel"])
def test_fullsize_inline(fields, q):
    import torch
    import paper_2407_15037_amd as lcq
    x = fields[q]
    announce("fullsize inline", q, x.size)
    st_o = O.quantize_inline(q, x, EB)
    xt = torch.from_numpy(x).cuda()
    st = lcq.quantize_inline(xt, q, EB)
    assert first_diff(st.cpu().numpy(), st_o) is None
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    dec = lcq.dequantize_inline(st, torch.float32, x.size, ws=ws)
    assert lcq.stream_status(ws) == 0
    ref = bits(O.dequantize_inline(st_o, np.float32, x.size))
    assert first_diff(bits(dec.cpu().numpy()), ref) is None


def _compare_default(q, x, eb, label):
    import torch
    import paper_2407_15037_amd as lcq
    announce("fullsize", label, q, x.dtype, x.size, eb)
    st_o = O.quantize(q, x, eb)
    xt = torch.from_numpy(x).cuda()
    buf, nb = lcq.quantize(xt, q, eb)
    size = int(nb.item())
    diff = first_diff(buf[:size].cpu().numpy(), st_o)
    assert diff is None, f"{label} {q} eb={eb}: stream {diff}"
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    dec = lcq.dequantize(buf, xt.dtype, x.size, stream_bytes=size, ws=ws)
    assert lcq.stream_status(ws) == 0
    diff = first_diff(bits(dec.cpu().numpy()), bits(O.dequantize(st_o, x.dtype, x.size)))
    assert diff is None, f"{label} {q} eb={eb}: decode {diff}"
    return st_o


@pytest.mark.parametrize("q,eb", [("abs", 1e-2), ("abs", 1e-4), ("rel", 1e-2)])
def test_fullsize_other_bounds(fields, q, eb):
    _compare_default(q, fields[q], eb, "grf512 f32")


@pytest.mark.parametrize("eb,min_nonzero", [(1e-2, 0.85), (1e-4, 0.99)])
def test_fullsize_noa_other_bounds(grf512, eb, min_nonzero):
    """NOA at the workload's other bounds, each on the base grid with its
    own range-keeping specials (half-bin neighbours at that eb * R)."""
    x = synth.plain_noa_field(grf512, eb)
    st = _compare_default("noa", x, eb, "grf512 f32")
    assert_real_noa_range(st, x, eb, min_nonzero)


def test_fullsize_noa_huge_range_edge(fields):
    """Edge case: the ABS field's specials include +-FLT_MAX, which stretch
    NOA's range to the whole type; the bound saturates and nearly every
    value lands in bin 0, but the bytes are still the oracle's."""
    st = _compare_default("noa", fields["abs"], EB, "grf512 f32 huge range")
    assert parse(st, np.float32)["hdr"]["bound"] > 1e35


@pytest.fixture(scope="module")
def fields64():
    x, xn, xr = synth.f64_grid_inputs()
    return {"abs": x, "noa": xn, "rel": xr}


@pytest.mark.parametrize("q,eb", [("abs", 1e-6), ("noa", 1e-6), ("rel", 1e-4)])
def test_fullsize_f64_grid_with_adversarial_slice(fields64, q, eb):
    x = fields64[q]
    st = _compare_default(q, x, eb, "grf384 f64")
    k = int(st[16:24].view(np.uint64)[0])
    # the bin-border slice sends values through the verify-and-fallback path
    # (ABS and NOA: its values sit at the bin borders of eb, resp. of the
    # field's own eb * R; REL: the lower side) beyond the injected specials
    nsp = synth.n_specials(x.size, 1e-4)
    assert k > nsp + 10000, (q, k, nsp)
    if q == "noa":
        assert_real_noa_range(st, x, eb, 0.99)


def test_fullsize_abs_unchecked_ablation(fields):
    """The section 6 ablation without the double-check is deterministic IEEE
    arithmetic too: its full-size stream and decode equal the oracle's."""
    import torch
    import paper_2407_15037_amd as lcq
    x = fields["abs"]
    announce("fullsize ablation abs_unchecked", x.size)
    st_o = O.quantize("abs_unchecked", x, EB)
    xt = torch.from_numpy(x).cuda()
    buf, nb = lcq.quantize_ablation(xt, "abs_unchecked", EB)
    size = int(nb.item())
    assert first_diff(buf[:size].cpu().numpy(), st_o) is None
    dec = lcq.dequantize_ablation(buf, "abs_unchecked", torch.float32, x.size, stream_bytes=size)
    assert first_diff(bits(dec.cpu().numpy()), bits(O.dequantize(st_o, np.float32, x.size))) is None


@pytest.mark.parametrize("q", ["abs", "noa", "rel"])
def test_fullsize_packing_stage(fields, q):
    """Packed bytes of the full-size streams equal the oracle's, and the
    GPU unpack restores each stream byte for byte."""
    import torch
    import paper_2407_15037_amd as lcq
    x = fields[q]
    announce("fullsize packing", q, x.size)
    st_o = O.quantize(q, x, EB)
    pk_o = O.pack(st_o, np.float32, x.size)
    buf = torch.from_numpy(st_o).cuda()
    pk, pnb = lcq.pack(buf, torch.float32, x.size)
    psize = int(pnb.item())
    assert first_diff(pk[:psize].cpu().numpy(), pk_o) is None
    back, bnb = lcq.unpack(pk, torch.float32, x.size, packed_bytes=psize)
    assert int(bnb.item()) == st_o.size
    assert torch.equal(back[: st_o.size], buf)


@pytest.mark.parametrize("q", ["abs", "noa", "rel"])
def test_fullsize_compress_decompress(fields, q):
    """The fused forms on the full-size fields: compress equals the oracle's
    pack of the oracle's stream, decompress of it equals the oracle's
    decode."""
    import torch
    import paper_2407_15037_amd as lcq
    x = fields[q]
    announce("fullsize compress / decompress", q, x.size)
    st_o = O.quantize_mt(q, x, EB)
    pk_o = O.pack(st_o, np.float32, x.size)
    pk, pnb = lcq.compress(torch.from_numpy(x).cuda(), q, EB)
    psize = int(pnb.item())
    assert first_diff(pk[:psize].cpu().numpy(), pk_o) is None
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    dec = lcq.decompress(pk, torch.float32, x.size, packed_bytes=psize, ws=ws)
    assert lcq.stream_status(ws) == 0
    ref = O.dequantize_mt(st_o, np.float32, x.size)
    assert first_diff(bits(dec.cpu().numpy()), bits(ref)) is None
