"""ctypes binding of lcq_serve (continuous-batching request loop).

run(requests, n_streams, arena) hands an open-loop schedule to the native
loop and returns per-request results.  Each request is a dict with keys
op ('quantize' / 'dequantize'), x (CUDA tensor: values, or a uint8 stream),
n, dtype (torch dtype), q, eb, in_bytes (dequantize), expect (CUDA uint8 /
value tensor or None), expect_bytes, arrival_ns.
"""
import ctypes

import numpy as np

import paper_2407_15037_amd as lcq

_L = lcq.lib()


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("q", ctypes.c_int), ("t", ctypes.c_int),
                ("eb", ctypes.c_double), ("d_in", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("in_bytes", ctypes.c_uint64), ("d_expect", ctypes.c_void_p),
                ("expect_bytes", ctypes.c_uint64), ("arrival_ns", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("admit_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64),
                ("mismatched", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("stream", ctypes.c_int32)]


class Config(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_uint32), ("d_arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_uint64), ("d_scratch", ctypes.c_void_p),
                ("scratch_bytes", ctypes.c_uint64)]


_L.lcq_serve.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(Request), ctypes.c_uint32,
                         ctypes.POINTER(Result)]
_L.lcq_serve.restype = ctypes.c_int

OPS = {"quantize": 0, "dequantize": 1}


def run(requests, n_streams=8, arena=None, arena_bytes=None):
    """Run the schedule (sorted by arrival_ns); returns a dict of numpy arrays
    admit_ns, done_ns, mismatched, status, stream, arrival_ns."""
    import torch
    nreq = len(requests)
    if arena is None:
        arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
    scratch = torch.empty(max(8 * nreq, 8), dtype=torch.uint8, device="cuda")
    reqs = (Request * max(nreq, 1))()
    for i, r in enumerate(requests):
        exp = r.get("expect")
        reqs[i] = Request(OPS[r["op"]], lcq._q(r.get("q", "abs")), lcq._dtype_code(r["dtype"]),
                          float(r.get("eb", 1.0)), r["x"].data_ptr() if r["x"].numel() else None,
                          int(r["n"]), int(r.get("in_bytes", 0)),
                          exp.data_ptr() if exp is not None and exp.numel() else None,
                          int(r.get("expect_bytes", 0)), int(r["arrival_ns"]))
    res = (Result * max(nreq, 1))()
    cfg = Config(int(n_streams), arena.data_ptr(), arena.numel(), scratch.data_ptr(), scratch.numel())
    lcq._check(_L.lcq_serve(ctypes.byref(cfg), reqs, nreq, res), "lcq_serve")
    out = {k: np.array([getattr(res[i], k) for i in range(nreq)])
           for k in ("admit_ns", "done_ns", "mismatched", "status", "stream")}
    out["arrival_ns"] = np.array([r["arrival_ns"] for r in requests], dtype=np.int64)
    return out
