"""Helpers for the GPU tests: run the HIP library through its C ABI binding
and the CPU oracle on the same host array."""
import sys

import numpy as np


def announce(*what):
    """Name the case before a GPU step (flushed), so a failing run says which."""
    print("[gpu case]", *what, flush=True)


def gpu_roundtrip(q, x, eb, stream=None):
    """Quantize x (numpy) on the GPU, decode it on the GPU.
    Returns (stream bytes as numpy uint8 of the exact size, decoded numpy)."""
    import torch
    import paper_2407_15037_amd as lcq
    tdt = torch.float32 if x.dtype == np.float32 else torch.float64
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    buf, nb = lcq.quantize(xt, q, eb, stream=stream)
    torch.cuda.synchronize()
    size = int(nb.item())
    dec = lcq.dequantize(buf, tdt, x.size, stream_bytes=size, stream=stream)
    torch.cuda.synchronize()
    return buf[:size].cpu().numpy(), dec.cpu().numpy()


def gpu_decode(st, dtype, n):
    """Decode a host stream (numpy uint8) on the GPU; returns (values, status)."""
    import torch
    import paper_2407_15037_amd as lcq
    tdt = torch.float32 if np.dtype(dtype) == np.float32 else torch.float64
    cap = max(st.size, 16)
    buf = torch.zeros(cap + 64, dtype=torch.uint8, device="cuda")
    buf[: st.size] = torch.from_numpy(st).cuda()
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    out = lcq.dequantize(buf, tdt, n, stream_bytes=st.size, ws=ws)
    status = lcq.stream_status(ws)
    return out.cpu().numpy(), status


def bits(a):
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def first_diff(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    if a.size != b.size:
        return f"sizes {a.size} vs {b.size}"
    d = np.flatnonzero(a != b)
    return None if d.size == 0 else f"{d.size} differ, first at {d[0]}: {a[d[0]]} vs {b[d[0]]}"
