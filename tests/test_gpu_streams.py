"""Calls on caller-chosen streams: wrapper temporaries stay valid while the
call's kernels run, and a batch plan without decode buffers refuses to
decode instead of writing through null pointers."""
import ctypes

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce, first_diff

pytestmark = pytest.mark.gpu


def test_side_streams_with_wrapper_buffers():
    """Two quantizes on two side streams, every buffer (stream, size word,
    workspace) allocated by the wrapper and dropped while the kernels may
    still run; meanwhile the current stream allocates and fills memory of the
    same sizes.  Both streams still equal the oracle's bytes."""
    import torch
    import paper_2407_15037_amd as lcq
    n = 3 * (1 << 20) + 4099
    xs = {q: synth.with_specials(synth.sines_1d(n, 301 + i, dtype=np.float32), q, 500, 302 + i, 1e-3)
          for i, q in enumerate(("abs", "noa"))}
    want = {q: O.quantize(q, x, 1e-3) for q, x in xs.items()}
    dx = {q: torch.from_numpy(x).cuda() for q, x in xs.items()}
    streams = {q: torch.cuda.Stream() for q in xs}
    torch.cuda.synchronize()
    for rep in range(3):
        announce("side streams", rep)
        got = {}
        for q in xs:
            st, nb = lcq.quantize(dx[q], q, 1e-3, stream=streams[q])
            got[q] = (st, nb)
        # churn on the current stream: allocations the size of the dropped
        # workspaces, written at once
        junk = [torch.full((lcq.workspace_bytes(q, torch.float32, n),), 0xA5, dtype=torch.uint8,
                           device="cuda") for q in xs]
        for q in xs:
            streams[q].synchronize()
            st, nb = got[q]
            size = int(nb.item())
            diff = first_diff(st[:size].cpu().numpy(), want[q])
            assert diff is None, (q, rep, diff)
        del junk


def test_batch_plan_without_decode_buffers():
    """A plan whose fields have no d_out quantizes normally; its dequantize
    returns LCQ_ERR_ARG and launches nothing."""
    import torch
    import paper_2407_15037_amd as lcq
    from paper_2407_15037_amd import batch as B
    L = lcq.lib()
    xs = [synth.sines_1d(5000 + 1000 * i, 310 + i, dtype=np.float32) for i in range(3)]
    dx = [torch.from_numpy(x).cuda() for x in xs]
    bufs = [torch.empty(lcq.max_stream_bytes(torch.float32, x.size), dtype=torch.uint8,
                        device="cuda") for x in xs]
    nbs = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in xs]
    arr = (B.Field * len(xs))()
    for i, x in enumerate(xs):
        arr[i] = B.Field(lcq.ABS, lcq.F32, 1e-3, dx[i].data_ptr(), x.size, bufs[i].data_ptr(),
                         bufs[i].numel(), nbs[i].data_ptr(), None)
    tune = b"batch=0"
    need = int(L.lcq_batch_workspace_bytes(arr, len(xs), tune))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    plan = ctypes.c_void_p()
    stream = lcq._stream_handle(None)
    announce("batch plan without d_out")
    assert L.lcq_batch_plan_create(arr, len(xs), tune, ws.data_ptr(), need, stream,
                                   ctypes.byref(plan)) == lcq.OK
    try:
        assert L.lcq_batch_quantize(plan, stream) == lcq.OK
        torch.cuda.synchronize()
        for i, x in enumerate(xs):
            size = int(nbs[i].item())
            assert first_diff(bufs[i][:size].cpu().numpy(), O.quantize("abs", x, 1e-3)) is None
        assert L.lcq_batch_dequantize(plan, stream) == lcq.ERR_ARG
        torch.cuda.synchronize()
    finally:
        L.lcq_batch_plan_destroy(plan)
