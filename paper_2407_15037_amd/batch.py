"""ctypes binding of the batched entry points (lcq_batch_* in include/lcq.h).

A BatchPlan quantizes / dequantizes many fields (CUDA tensors of uneven size,
float32 or float64, each with its own quantizer and bound) with one graph
launch.  Argument marshalling only; the work runs in the library's kernels.
"""
import ctypes

import paper_2407_15037_amd as lcq

_L = lcq.lib()


class Field(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("t", ctypes.c_int), ("eb", ctypes.c_double),
                ("d_in", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("d_stream", ctypes.c_void_p), ("stream_cap", ctypes.c_uint64),
                ("d_stream_bytes", ctypes.c_void_p), ("d_out", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_L.lcq_batch_variants.argtypes = []
_L.lcq_batch_variants.restype = ctypes.c_int32
_L.lcq_batch_workspace_bytes.argtypes = [ctypes.POINTER(Field), ctypes.c_uint32, ctypes.c_char_p]
_L.lcq_batch_workspace_bytes.restype = ctypes.c_uint64
_L.lcq_batch_plan_create.argtypes = [ctypes.POINTER(Field), ctypes.c_uint32, ctypes.c_char_p, _vp,
                                     ctypes.c_uint64, _vp, ctypes.POINTER(_vp)]
_L.lcq_batch_plan_create.restype = ctypes.c_int
_L.lcq_batch_quantize.argtypes = [_vp, _vp]
_L.lcq_batch_quantize.restype = ctypes.c_int
_L.lcq_batch_dequantize.argtypes = [_vp, _vp]
_L.lcq_batch_dequantize.restype = ctypes.c_int
_L.lcq_batch_status.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_int64)]
_L.lcq_batch_status.restype = ctypes.c_int
_L.lcq_batch_plan_destroy.argtypes = [_vp]
_L.lcq_batch_plan_destroy.restype = None


def variants():
    return int(_L.lcq_batch_variants())


class BatchPlan:
    """fields: list of dicts with keys x (CUDA tensor), q, eb, and optionally
    out (decode tensor), stream (uint8 tensor), nbytes (int64 tensor).
    tune: the plan's tuning string (lcq_batch_plan_create), e.g. the one
    autotune.tune_batch returns; default "batch=<variant>"."""

    def __init__(self, fields, variant=0, stream=None, tune=None):
        import torch
        self.fields = []
        arr = (Field * max(len(fields), 1))()
        for i, f in enumerate(fields):
            x = f["x"]
            if not x.is_cuda or not x.is_contiguous():
                raise ValueError("field tensors must be contiguous CUDA tensors")
            n = x.numel()
            cap = lcq.max_stream_bytes(x.dtype, n)
            st = f.get("stream")
            if st is None:
                st = torch.empty(cap, dtype=torch.uint8, device=x.device)
            nb = f.get("nbytes")
            if nb is None:
                nb = torch.zeros(1, dtype=torch.int64, device=x.device)
            out = f.get("out")
            if out is None:
                out = torch.empty(n, dtype=x.dtype, device=x.device)
            q = lcq._q(f["q"])
            arr[i] = Field(q, lcq._dtype_code(x.dtype), float(f["eb"]),
                           x.data_ptr() if n else None, n, st.data_ptr(), st.numel(),
                           nb.data_ptr(), out.data_ptr() if n else None)
            self.fields.append(dict(x=x, q=f["q"], eb=f["eb"], stream=st, nbytes=nb, out=out))
        tune = (tune if tune is not None else f"batch={int(variant)}").encode()
        self._arr = arr
        need = int(_L.lcq_batch_workspace_bytes(arr, len(fields), tune))
        if need == 0:
            raise lcq.LCQError(lcq.ERR_ARG, "lcq_batch_workspace_bytes")
        dev = fields[0]["x"].device if fields else torch.device("cuda")
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        plan = _vp()
        st = _L.lcq_batch_plan_create(arr, len(fields), tune, self.ws.data_ptr(), need,
                                      lcq._stream_handle(stream), ctypes.byref(plan))
        lcq._check(st, "lcq_batch_plan_create")
        self._plan = plan

    def quantize(self, stream=None):
        lcq._check(_L.lcq_batch_quantize(self._plan, lcq._stream_handle(stream)),
                   "lcq_batch_quantize")

    def dequantize(self, stream=None):
        lcq._check(_L.lcq_batch_dequantize(self._plan, lcq._stream_handle(stream)),
                   "lcq_batch_dequantize")

    def first_bad_field(self, stream=None):
        v = ctypes.c_int64(0)
        lcq._check(_L.lcq_batch_status(self._plan, lcq._stream_handle(stream), ctypes.byref(v)),
                   "lcq_batch_status")
        return int(v.value)

    def close(self):
        if getattr(self, "_plan", None):
            _L.lcq_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
