"""The plain entry points inside a captured HIP graph: quantize + dequantize
(ABS, NOA, REL; the two-pass kernels, the NOA range pass, the workspace
clears) recorded once with torch.cuda.graph and replayed on new data, with
eager work and synchronisation between replays; every replay must equal the
eager result for the same input, and the oracle's."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce, bits, first_diff

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("q", ["abs", "noa", "rel"])
def test_plain_path_replays_in_a_graph(q):
    import torch
    import paper_2407_15037_amd as lcq
    n = 7 * 4096 + 1234
    eb = 1e-3
    inputs = []
    for seed in range(3):
        x = synth.sines_1d(n, 800 + seed, dtype=np.float32)
        x, _, _ = synth.inject_specials(x, 40, 810 + seed, eb)
        if q == "rel":
            x = synth.rel_variant(np.nan_to_num(x.astype(np.float64)), 820 + seed, dtype=np.float32)
        inputs.append(x)
    xt = torch.from_numpy(inputs[0]).cuda()
    buf = torch.empty(lcq.max_stream_bytes(torch.float32, n), dtype=torch.uint8, device="cuda")
    nb = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(lcq.workspace_bytes(q, torch.float32, n), dtype=torch.uint8, device="cuda")
    dws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    cap = buf.numel()

    def step():
        lcq.quantize(xt, q, eb, out=buf, nbytes=nb, ws=ws)
        lcq.dequantize(buf, torch.float32, n, stream_bytes=cap, out=out, ws=dws)

    announce("graph warm-up", q)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    announce("graph capture", q)
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(2):
        for i, x in enumerate(inputs):
            xt.copy_(torch.from_numpy(x))
            torch.cuda.synchronize()
            announce("graph replay", q, rep, i)
            g.replay()
            torch.cuda.synchronize()
            size = int(nb.item())
            got = buf[:size].cpu().numpy()
            dec = out.cpu().numpy()
            want = O.quantize(q, x, eb)
            assert first_diff(got, want) is None, (q, rep, i)
            assert first_diff(bits(dec), bits(O.dequantize(want, np.float32, n))) is None, (q, rep, i)
            # eager work between replays
            e, enb = lcq.quantize(xt, q, eb)
            torch.cuda.synchronize()
            assert torch.equal(e[: int(enb.item())], buf[:size])
    del g
