"""Lossless packing stage on the GPU: packed bytes equal the oracle's for
the same LCQ1 stream, unpacking restores the stream byte for byte (from the
GPU's and from the oracle's packed bytes), and broken packed streams are
rejected."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce, first_diff

pytestmark = pytest.mark.gpu

DTYPES = [np.float32, np.float64]


def _tdt(dt):
    import torch
    return torch.float32 if np.dtype(dt) == np.float32 else torch.float64


def _gpu_pack(st, dt, n):
    import torch
    import paper_2407_15037_amd as lcq
    buf = torch.from_numpy(np.ascontiguousarray(st)).cuda()
    ws = torch.zeros(lcq.pack_workspace_bytes(_tdt(dt), n), dtype=torch.uint8, device="cuda")
    pk, nb = lcq.pack(buf, _tdt(dt), n, ws=ws)
    status = lcq.stream_status(ws)
    return pk[: int(nb.item())].cpu().numpy(), status


def _gpu_unpack(pk, dt, n):
    import torch
    import paper_2407_15037_amd as lcq
    buf = torch.from_numpy(np.ascontiguousarray(pk)).cuda()
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    try:
        out, nb = lcq.unpack(buf, _tdt(dt), n, ws=ws)
    except lcq.LCQError as e:
        return None, e.status
    status = lcq.stream_status(ws)
    return (out[: int(nb.item())].cpu().numpy() if status == 0 else None), status


def _streams():
    out = []
    for dt in DTYPES:
        for n in (0, 1, 5, 1023, 1024, 1025, 4097, 5 * 4096 + 777):
            x = synth.sines_1d(max(n, 1), 700 + n, dtype=dt)[:n]
            if n:
                x, _, _ = synth.inject_specials(x, max(1, n // 300), 701, 1e-3)
            for q in ("abs", "noa", "rel"):
                y = x if q != "rel" else synth.rel_variant(np.nan_to_num(x.astype(np.float64)), 702, dtype=dt)
                out.append((dt, q, y))
        allsp, _, _ = synth.inject_specials(synth.sines_1d(3000, 703, dtype=dt), 3000, 704, 1e-3)
        out.append((dt, "abs", allsp))
        rough = np.random.default_rng(705).standard_normal(9000).astype(dt) * 1e6
        out.append((dt, "abs", rough))  # wide codes: bit widths up to the mid 20s
    return out


@pytest.mark.parametrize("case", range(len(_streams())))
def test_pack_equals_oracle_and_roundtrips(case):
    dt, q, x = _streams()[case]
    n = x.size
    st = O.quantize(q, x, 1e-3)
    announce("pack", np.dtype(dt).name, q, n)
    pk, status = _gpu_pack(st, dt, n)
    assert status == 0
    pk_o = O.pack(st, dt, n)
    assert first_diff(pk, pk_o) is None
    back, status = _gpu_unpack(pk_o, dt, n)
    assert status == 0 and first_diff(back, st) is None


def test_pack_of_gpu_stream_and_errors():
    import torch
    import paper_2407_15037_amd as lcq
    x, _, _ = synth.plain_step_inputs(64, 1e-3)
    n = x.size
    announce("pack gpu stream", n)
    buf, nb = lcq.quantize(torch.from_numpy(x).cuda(), "abs", 1e-3)
    st = buf[: int(nb.item())].cpu().numpy()
    pk, status = _gpu_pack(st, np.float32, n)
    assert status == 0 and first_diff(pk, O.pack(st, np.float32, n)) is None
    assert pk.size < st.size // 2
    C = (n + 1023) // 1024
    ot = (64 + 8 * C + 15) // 16 * 16
    pl = (ot + 8 * (C + 1) + 15) // 16 * 16
    for name, off, val in (("magic", 0, 0x58), ("width", pl, 40), ("offset", ot + 8, 0xFF),
                           ("payload", ot + 8 * C, 0xFF)):
        bad = pk.copy()
        bad[off] = val
        announce("unpack corrupt", name)
        _, status = _gpu_unpack(bad, np.float32, n)
        assert status == 3, name
    announce("unpack truncated")
    _, status = _gpu_unpack(pk[:-1], np.float32, n)
    assert status == 3
    bad = st.copy()
    bad[0] ^= 0xFF
    announce("pack corrupt input")
    _, status = _gpu_pack(bad, np.float32, n)
    assert status == 3


def test_compress_decompress_pipeline():
    """The one-call forms (lcq_compress, lcq_decompress) on the same fields as
    the two-call pipeline: packed bytes equal the oracle's pack of its own
    stream, and the decode equals the oracle's decode."""
    import torch
    import paper_2407_15037_amd as lcq
    for dt in DTYPES:
        x = synth.sines_1d(50000, 900, dtype=dt)
        x, _, _ = synth.inject_specials(x, 60, 901, 1e-4)
        for q in ("abs", "noa", "rel"):
            y = x if q != "rel" else synth.rel_variant(np.nan_to_num(x.astype(np.float64)), 902, dtype=dt)
            announce("compress pipeline", np.dtype(dt).name, q)
            pk, nb = lcq.compress(torch.from_numpy(y).cuda(), q, 1e-4)
            pk = pk[: int(nb.item())]
            assert first_diff(pk.cpu().numpy(), O.pack(O.quantize(q, y, 1e-4), dt, y.size)) is None
            ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
            dec = lcq.decompress(pk, _tdt(dt), y.size, ws=ws)
            assert lcq.stream_status(ws) == 0
            ref = O.dequantize(O.quantize(q, y, 1e-4), dt, y.size)
            assert np.array_equal(dec.cpu().numpy().view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("q", ["abs", "rel"])
def test_pack_many_groups_equals_oracle(q):
    """2^21 + 333 codes: 513 workgroups of 4 chunks in 65 groups of the
    record-offset scan, a ragged last chunk; packed bytes and the unpacked stream must equal the
    oracle's."""
    n = (1 << 21) + 333
    x = synth.sines_1d(n, 710, dtype=np.float32)
    x, _, _ = synth.inject_specials(x, n // 500, 711, 1e-3)
    if q == "rel":
        x = synth.rel_variant(np.nan_to_num(x.astype(np.float64)), 712, dtype=np.float32)
    st = O.quantize(q, x, 1e-3)
    want = O.pack(st, np.float32, n)
    announce("pack many groups", q)
    got, status = _gpu_pack(st, np.float32, n)
    assert status == 0
    assert first_diff(got, want) is None
    back, status = _gpu_unpack(got, np.float32, n)
    assert status == 0 and first_diff(back, st) is None
