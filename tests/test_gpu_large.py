"""Maximum-size behaviour: a field of more than 2^31 values (64-bit indexing
of values, codes, chunk table and outliers) quantized and dequantized on the
GPU; sampled chunks (including chunks past value 2^31 and the ragged tail)
are checked against the CPU oracle one by one.  ABS parameters do not depend
on the data, so the oracle's encoding of a chunk alone must equal the GPU's
codes for that chunk, its outliers the GPU's outliers from that chunk's
chunk-table entry on."""
import numpy as np
import pytest

import oracle as O
from gpu_util import announce

pytestmark = pytest.mark.gpu

CHUNK = 1024


def test_more_than_2_31_values():
    import torch
    import paper_2407_15037_amd as lcq
    n = (1 << 31) + 4099
    eb = 1e-3
    announce("large field", n)
    # a smooth ramp with a sprinkling of values that must be stored losslessly
    i = torch.arange(n, dtype=torch.int64, device="cuda")
    x = torch.sin(i.to(torch.float32) * 1e-6) * 50.0
    sp = (i % 1000003) == 7
    x[sp] = float("nan")
    x[(i % 999983) == 11] = float("inf")
    del i, sp
    buf, nb = lcq.quantize(x, "abs", eb)
    torch.cuda.synchronize()
    size = int(nb.item())
    hdr = buf[:64].cpu().numpy()
    k = int(hdr[16:24].view(np.uint64)[0])
    assert int(hdr[8:16].view(np.uint64)[0]) == n
    ct = (64 + 4 * n + 15) // 16 * 16
    nchunks = (n + CHUNK - 1) // CHUNK
    oo = (ct + 8 * nchunks + 15) // 16 * 16
    assert size == oo + 4 * k
    codes = buf[64: 64 + 4 * n].view(torch.int32)
    assert int((codes == -(1 << 31)).sum().item()) == k
    dec = lcq.dequantize(buf, torch.float32, n, stream_bytes=size)
    torch.cuda.synchronize()
    table = buf[ct: ct + 8 * nchunks].view(torch.int64)
    outl = buf[oo: oo + 4 * k].view(torch.int32)
    sample = [0, 1, 2097151, 2097152, 2097153, nchunks // 2, nchunks - 2, nchunks - 1]
    for c in sample:
        b, e = c * CHUNK, min((c + 1) * CHUNK, n)
        xs = x[b:e].cpu().numpy()
        st = O.quantize("abs", xs, eb)
        oc = st[64: 64 + 4 * xs.size].view(np.int32)
        assert np.array_equal(codes[b:e].cpu().numpy(), oc), f"codes of chunk {c}"
        ko = int(st[16:24].view(np.uint64)[0])
        base = int(table[c].item())
        got_out = outl[base: base + ko].cpu().numpy()
        oct_ = (64 + 4 * xs.size + 15) // 16 * 16
        ooo = (oct_ + 8 * ((xs.size + CHUNK - 1) // CHUNK) + 15) // 16 * 16
        assert np.array_equal(got_out, st[ooo: ooo + 4 * ko].view(np.int32)), f"outliers of chunk {c}"
        if c + 1 < nchunks:
            assert int(table[c + 1].item()) - base == ko
        od = O.dequantize(st, np.float32, xs.size)
        assert np.array_equal(dec[b:e].cpu().numpy().view(np.uint32), od.view(np.uint32)), f"decode of chunk {c}"


def test_compress_more_than_2_31_values():
    """The fused forms at the same size: header and outlier count as the
    two-call stream's, every sampled chunk's record byte-equal to the
    oracle's record for that chunk alone (a record depends only on its
    chunk's codes), its chunk-table entry equal to the LCQ1 stream's, and
    decompress equal to the oracle's decode of the chunk."""
    import torch
    import paper_2407_15037_amd as lcq
    n = (1 << 31) + 4099
    eb = 1e-3
    announce("large field, compress / decompress", n)
    i = torch.arange(n, dtype=torch.int64, device="cuda")
    x = torch.sin(i.to(torch.float32) * 1e-6) * 50.0
    x[(i % 1000003) == 7] = float("nan")
    x[(i % 999983) == 11] = float("inf")
    del i
    pk, pnb = lcq.compress(x, "abs", eb)
    torch.cuda.synchronize()
    psize = int(pnb.item())
    hdr = pk[:64].cpu().numpy()
    assert int(hdr[8:16].view(np.uint64)[0]) == n
    k = int(hdr[16:24].view(np.uint64)[0])
    nchunks = (n + CHUNK - 1) // CHUNK
    ot = (64 + 8 * nchunks + 15) // 16 * 16
    pl = (ot + 8 * (nchunks + 1) + 15) // 16 * 16
    table = pk[64: 64 + 8 * nchunks].view(torch.int64)
    offs = pk[ot: ot + 8 * (nchunks + 1)].view(torch.int64)
    payload = int(offs[nchunks].item())
    assert psize == (pl + payload + 15) // 16 * 16 + 4 * k
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    dec = lcq.decompress(pk, torch.float32, n, packed_bytes=psize, ws=ws)
    assert lcq.stream_status(ws) == 0
    sample = [0, 1, 2097151, 2097152, 2097153, nchunks // 2, nchunks - 2, nchunks - 1]
    run = 0
    for c in sample:
        b, e = c * CHUNK, min((c + 1) * CHUNK, n)
        xs = x[b:e].cpu().numpy()
        st = O.quantize("abs", xs, eb)
        po = O.pack(st, np.float32, xs.size)
        # the oracle's single-chunk packed stream: one record at its payload offset
        ot1 = (64 + 8 + 15) // 16 * 16
        pl1 = (ot1 + 16 + 15) // 16 * 16
        rsize = int(po[ot1 + 8: ot1 + 16].view(np.uint64)[0])
        off = int(offs[c].item())
        assert int(offs[c + 1].item()) - off == rsize, f"record size of chunk {c}"
        got = pk[pl + off: pl + off + rsize].cpu().numpy()
        assert np.array_equal(got, po[pl1: pl1 + rsize]), f"record of chunk {c}"
        od = O.dequantize(st, np.float32, xs.size)
        assert np.array_equal(dec[b:e].cpu().numpy().view(np.uint32), od.view(np.uint32)), f"decode of chunk {c}"
        if c + 1 < nchunks:
            ko = int(st[16:24].view(np.uint64)[0])
            assert int(table[c + 1].item()) - int(table[c].item()) == ko
        run += 1
    assert run == len(sample)
