"""Guaranteed-error-bound ABS / REL / NOA quantizers for MI355X (gfx950).

A thin ctypes binding of liblcq.so (C ABI in include/lcq.h): it only checks
and marshals arguments.  Every step of quantize / dequantize runs in the
library's HIP kernels; PyTorch provides device memory and streams.  There is
no CPU fallback: if the library is missing, importing this package fails.
"""
import ctypes
import os

__all__ = ["ABS", "REL", "NOA", "F32", "F64", "LCQError", "lib", "max_stream_bytes",
           "workspace_bytes", "quantize", "quantize_noalloc", "NOALLOC_SCRATCH_BYTES", "dequantize", "stream_status", "profile_events",
           "set_lookback_spin", "tune_variants", "tune_set", "tune_get",
           "inline_stream_bytes", "inline_workspace_bytes", "quantize_inline",
           "quantize_ablation", "dequantize_ablation", "ABL_ABS_UNCHECKED", "ABL_REL_LIBM",
           "pack_max_bytes", "pack_workspace_bytes", "pack", "unpack", "compress", "decompress",
           "compress_workspace_bytes", "dequantize_inline", "SO_PATH",
           "profile_mid_event"]

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "liblcq.so")

F32, F64 = 0, 1
ABS, REL, NOA = 0, 1, 2
OK, ERR_ARG, ERR_CAPACITY, ERR_STREAM, ERR_HIP = 0, 1, 2, 3, 4
_QNAMES = {"abs": ABS, "rel": REL, "noa": NOA}
ABL_ABS_UNCHECKED, ABL_REL_LIBM = 3, 4  # section 6 ablations (no guarantee by design)
_ABLATIONS = {"abs_unchecked": ABL_ABS_UNCHECKED, "rel_libm": ABL_REL_LIBM}
_OPS = {"quantize": 0, "dequantize": 1}

if not os.path.exists(SO_PATH):
    raise ImportError(f"{SO_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'` "
                      "(or python paper_2407_15037_amd/build.py)")

_lib = ctypes.CDLL(SO_PATH)
_u64, _vp, _i32, _dbl = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_lib.lcq_max_stream_bytes.argtypes = [_i32, _u64]
_lib.lcq_max_stream_bytes.restype = _u64
_lib.lcq_workspace_bytes.argtypes = [_i32, _i32, _u64]
_lib.lcq_workspace_bytes.restype = _u64
_lib.lcq_quantize.argtypes = [_i32, _i32, _dbl, _vp, _u64, _vp, _u64, _vp, _vp, _u64, _vp]
_lib.lcq_quantize.restype = _i32
_lib.lcq_quantize_noalloc.argtypes = [_i32, _i32, _dbl, _vp, _u64, _vp, _u64, _vp, _vp]
_lib.lcq_quantize_noalloc.restype = _i32
NOALLOC_SCRATCH_BYTES = 128 << 20  # LCQ_NOALLOC_SCRATCH_BYTES of include/lcq.h
_lib.lcq_dequantize.argtypes = [_i32, _vp, _u64, _vp, _u64, _vp, _u64, _vp]
_lib.lcq_dequantize.restype = _i32
_lib.lcq_inline_stream_bytes.argtypes = [_i32, _u64]
_lib.lcq_inline_stream_bytes.restype = _u64
_lib.lcq_inline_workspace_bytes.argtypes = [_i32]
_lib.lcq_inline_workspace_bytes.restype = _u64
_lib.lcq_quantize_inline.argtypes = [_i32, _i32, _dbl, _vp, _u64, _vp, _u64, _vp, _u64, _vp]
_lib.lcq_quantize_inline.restype = _i32
_lib.lcq_dequantize_inline.argtypes = [_i32, _vp, _u64, _vp, _u64, _vp, _u64, _vp]
_lib.lcq_dequantize_inline.restype = _i32
_lib.lcq_quantize_ablation.argtypes = [_i32, _i32, _dbl, _vp, _u64, _vp, _u64, _vp, _vp, _u64, _vp]
_lib.lcq_quantize_ablation.restype = _i32
_lib.lcq_dequantize_ablation.argtypes = [_i32, _i32, _vp, _u64, _vp, _u64, _vp, _u64, _vp]
_lib.lcq_dequantize_ablation.restype = _i32
_lib.lcq_pack_max_bytes.argtypes = [_i32, _u64]
_lib.lcq_pack_max_bytes.restype = _u64
_lib.lcq_pack_workspace_bytes.argtypes = [_i32, _u64]
_lib.lcq_pack_workspace_bytes.restype = _u64
for _name in ("lcq_pack", "lcq_unpack"):
    getattr(_lib, _name).argtypes = [_i32, _vp, _u64, _u64, _vp, _u64, _vp, _vp, _u64, _vp]
    getattr(_lib, _name).restype = _i32
_lib.lcq_compress_workspace_bytes.argtypes = [_i32, _i32, _u64]
_lib.lcq_compress_workspace_bytes.restype = _u64
_lib.lcq_compress.argtypes = [_i32, _i32, _dbl, _vp, _u64, _vp, _u64, _vp, _vp, _u64, _vp]
_lib.lcq_compress.restype = _i32
_lib.lcq_decompress.argtypes = [_i32, _vp, _u64, _vp, _u64, _vp, _u64, _vp]
_lib.lcq_decompress.restype = _i32
_lib.lcq_stream_status.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_int32)]
_lib.lcq_stream_status.restype = _i32
_lib.lcq_status_string.argtypes = [_i32]
_lib.lcq_status_string.restype = ctypes.c_char_p
_lib.lcq_profile_events.argtypes = [_vp, _vp]
_lib.lcq_profile_events.restype = None
_lib.lcq_profile_mid_event.argtypes = [_vp]
_lib.lcq_profile_mid_event.restype = None
_lib.lcq_debug_set_lookback_spin.argtypes = [ctypes.c_uint32]
_lib.lcq_debug_set_lookback_spin.restype = None
_lib.lcq_tune_variants.argtypes = []
_lib.lcq_tune_variants.restype = ctypes.c_int32
_lib.lcq_tune_set.argtypes = [ctypes.c_int32, _i32, ctypes.c_int32]
_lib.lcq_tune_set.restype = _i32
_lib.lcq_tune_get.argtypes = [ctypes.c_int32, _i32]
_lib.lcq_tune_get.restype = ctypes.c_int32


def lib():
    return _lib


class LCQError(RuntimeError):
    def __init__(self, status, what):
        msg = _lib.lcq_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})")
        self.status = status


def _check(st, what):
    if st != OK:
        raise LCQError(st, what)


def _q(q):
    return _QNAMES[q] if isinstance(q, str) else int(q)


def _dtype_code(dtype):
    import torch
    if dtype == torch.float32:
        return F32
    if dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {dtype}")


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _empty(numel, dtype, device, stream, zero=False):
    """A buffer a call on `stream` uses.  It is allocated on that stream, so
    torch's caching allocator cannot hand its memory to work on another
    stream while the call's kernels may still run (a temporary dropped when
    the wrapper returns is only reused by later work on the same stream)."""
    import torch
    make = torch.zeros if zero else torch.empty
    if stream is None:
        return make(numel, dtype=dtype, device=device)
    with torch.cuda.stream(stream):
        return make(numel, dtype=dtype, device=device)


def max_stream_bytes(dtype, n):
    return int(_lib.lcq_max_stream_bytes(_dtype_code(dtype), n))


def workspace_bytes(q, dtype, n):
    return int(_lib.lcq_workspace_bytes(_q(q), _dtype_code(dtype), n))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def quantize(x, q, eb, *, out=None, nbytes=None, ws=None, stream=None):
    """Quantize the contiguous CUDA tensor x (float32 / float64).

    Returns (stream, nbytes): `stream` is a uint8 device tensor of capacity
    max_stream_bytes, `nbytes` a one-element int64 device tensor receiving the
    stream's size.  Buffers may be passed in to avoid allocation."""
    import torch
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA tensor")
    dt = _dtype_code(x.dtype)
    n = x.numel()
    cap = int(_lib.lcq_max_stream_bytes(dt, n))
    if out is None:
        out = _empty(cap, torch.uint8, x.device, stream)
    if nbytes is None:
        nbytes = _empty(1, torch.int64, x.device, stream)
    if ws is None:
        ws = _empty(int(_lib.lcq_workspace_bytes(_q(q), dt, n)), torch.uint8, x.device, stream)
    st = _lib.lcq_quantize(_q(q), dt, float(eb), _ptr(x) if n else None, n, _ptr(out),
                           out.numel(), _ptr(nbytes), _ptr(ws), ws.numel(),
                           _stream_handle(stream))
    _check(st, "lcq_quantize")
    return out, nbytes


def quantize_noalloc(x, q, eb, *, out, nbytes, stream=None):
    """quantize() with the library's fixed per-GPU workspace
    (lcq_quantize_noalloc): the caller passes the stream buffer `out` (uint8,
    at least max_stream_bytes) and the size word `nbytes` (int64, one
    element); nothing is allocated.  Calls that overlap on one GPU race."""
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA tensor")
    dt = _dtype_code(x.dtype)
    n = x.numel()
    st = _lib.lcq_quantize_noalloc(_q(q), dt, float(eb), _ptr(x) if n else None, n, _ptr(out),
                                   out.numel(), _ptr(nbytes), _stream_handle(stream))
    _check(st, "lcq_quantize_noalloc")
    return out, nbytes


def dequantize(stream_buf, dtype, n, *, stream_bytes=None, out=None, ws=None, stream=None):
    """Decode a stream (uint8 CUDA tensor) into a new (or given) tensor of n
    values.  stream_bytes defaults to the tensor's size."""
    import torch
    dt = _dtype_code(dtype)
    if out is None:
        out = _empty(n, dtype, stream_buf.device, stream)
    if ws is None:
        ws = _empty(64, torch.uint8, stream_buf.device, stream)
    sb = stream_buf.numel() if stream_bytes is None else int(stream_bytes)
    st = _lib.lcq_dequantize(dt, _ptr(stream_buf), sb, _ptr(out) if n else None, n, _ptr(ws),
                             ws.numel(), _stream_handle(stream))
    _check(st, "lcq_dequantize")
    return out


def _abl(kind):
    return _ABLATIONS[kind] if isinstance(kind, str) else int(kind)


def quantize_ablation(x, kind, eb, *, out=None, nbytes=None, ws=None, stream=None):
    """One of the section 6 ablations ('abs_unchecked' or 'rel_libm'); same
    buffers and return value as quantize().  Not error-bounded by design."""
    import torch
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA tensor")
    dt = _dtype_code(x.dtype)
    n = x.numel()
    k = _abl(kind)
    if out is None:
        out = _empty(int(_lib.lcq_max_stream_bytes(dt, n)), torch.uint8, x.device, stream)
    if nbytes is None:
        nbytes = _empty(1, torch.int64, x.device, stream)
    if ws is None:
        base = ABS if k == ABL_ABS_UNCHECKED else REL
        ws = _empty(int(_lib.lcq_workspace_bytes(base, dt, n)), torch.uint8, x.device, stream)
    st = _lib.lcq_quantize_ablation(k, dt, float(eb), _ptr(x) if n else None, n, _ptr(out),
                                    out.numel(), _ptr(nbytes), _ptr(ws), ws.numel(),
                                    _stream_handle(stream))
    _check(st, "lcq_quantize_ablation")
    return out, nbytes


def dequantize_ablation(stream_buf, kind, dtype, n, *, stream_bytes=None, out=None, ws=None,
                        stream=None):
    """Decode a stream of the given ablation kind (header status in ws)."""
    import torch
    dt = _dtype_code(dtype)
    if out is None:
        out = _empty(n, dtype, stream_buf.device, stream)
    if ws is None:
        ws = _empty(64, torch.uint8, stream_buf.device, stream)
    sb = stream_buf.numel() if stream_bytes is None else int(stream_bytes)
    st = _lib.lcq_dequantize_ablation(_abl(kind), dt, _ptr(stream_buf), sb, _ptr(out) if n else None,
                                      n, _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(st, "lcq_dequantize_ablation")
    return out


def pack_max_bytes(dtype, n):
    return int(_lib.lcq_pack_max_bytes(_dtype_code(dtype), n))


def pack_workspace_bytes(dtype, n):
    return int(_lib.lcq_pack_workspace_bytes(_dtype_code(dtype), n))


def pack(stream_buf, dtype, n, *, stream_bytes=None, out=None, nbytes=None, ws=None, stream=None):
    """Lossless packing stage: LCQ1 stream (uint8 CUDA tensor) -> packed
    stream.  Returns (packed buffer, one-element int64 tensor with its size);
    the input check's status lands in ws (read with stream_status)."""
    import torch
    dt = _dtype_code(dtype)
    if out is None:
        out = _empty(pack_max_bytes(dtype, n), torch.uint8, stream_buf.device, stream)
    if nbytes is None:
        nbytes = _empty(1, torch.int64, stream_buf.device, stream)
    if ws is None:
        ws = _empty(pack_workspace_bytes(dtype, n), torch.uint8, stream_buf.device, stream)
    sb = stream_buf.numel() if stream_bytes is None else int(stream_bytes)
    st = _lib.lcq_pack(dt, _ptr(stream_buf), sb, n, _ptr(out), out.numel(), _ptr(nbytes),
                       _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(st, "lcq_pack")
    return out, nbytes


def unpack(packed_buf, dtype, n, *, packed_bytes=None, out=None, nbytes=None, ws=None, stream=None):
    """Inverse of pack(): (LCQ1 stream buffer, size tensor)."""
    import torch
    dt = _dtype_code(dtype)
    if out is None:
        out = _empty(max_stream_bytes(dtype, n), torch.uint8, packed_buf.device, stream)
    if nbytes is None:
        nbytes = _empty(1, torch.int64, packed_buf.device, stream)
    if ws is None:
        ws = _empty(64, torch.uint8, packed_buf.device, stream)
    pb = packed_buf.numel() if packed_bytes is None else int(packed_bytes)
    st = _lib.lcq_unpack(dt, _ptr(packed_buf), pb, n, _ptr(out), out.numel(), _ptr(nbytes),
                         _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(st, "lcq_unpack")
    return out, nbytes


def compress_workspace_bytes(q, dtype, n):
    return int(_lib.lcq_compress_workspace_bytes(_q(q), _dtype_code(dtype), n))


def compress(x, q, eb, *, out=None, nbytes=None, ws=None, stream=None):
    """Quantize x and pack the codes in one call (lcq_compress): the bytes of
    pack(quantize(x)), the codes never written to memory.  Returns (packed,
    nbytes): a uint8 device tensor of capacity pack_max_bytes and a
    one-element int64 device tensor receiving the packed size."""
    import torch
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA tensor")
    dt = _dtype_code(x.dtype)
    n = x.numel()
    if out is None:
        out = _empty(int(_lib.lcq_pack_max_bytes(dt, n)), torch.uint8, x.device, stream)
    if nbytes is None:
        nbytes = _empty(1, torch.int64, x.device, stream)
    if ws is None:
        ws = _empty(compress_workspace_bytes(q, x.dtype, n), torch.uint8, x.device, stream)
    st = _lib.lcq_compress(_q(q), dt, float(eb), _ptr(x) if n else None, n, _ptr(out),
                           out.numel(), _ptr(nbytes), _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(st, "lcq_compress")
    return out, nbytes


def decompress(packed, dtype, n, *, packed_bytes=None, out=None, ws=None, stream=None):
    """Decode a packed stream straight to n values (lcq_decompress): the
    values of dequantize(unpack(packed)).  The device checks land in ws (read
    them with stream_status); packed_bytes defaults to the tensor's size."""
    import torch
    dt = _dtype_code(dtype)
    if out is None:
        out = _empty(n, dtype, packed.device, stream)
    if ws is None:
        ws = _empty(64, torch.uint8, packed.device, stream)
    pb = packed.numel() if packed_bytes is None else int(packed_bytes)
    st = _lib.lcq_decompress(dt, _ptr(packed), pb, _ptr(out) if n else None, n, _ptr(ws),
                             ws.numel(), _stream_handle(stream))
    _check(st, "lcq_decompress")
    return out


def inline_stream_bytes(dtype, n):
    return int(_lib.lcq_inline_stream_bytes(_dtype_code(dtype), n))


def inline_workspace_bytes(q):
    return int(_lib.lcq_inline_workspace_bytes(_q(q)))


def quantize_inline(x, q, eb, *, out=None, ws=None, stream=None):
    """Quantize x into the in-line layout (one word per value plus a bitmap
    of values stored raw).  Returns the stream, a uint8 device tensor of
    exactly inline_stream_bytes(x.dtype, x.numel()) bytes."""
    import torch
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA tensor")
    dt = _dtype_code(x.dtype)
    n = x.numel()
    if out is None:
        out = _empty(int(_lib.lcq_inline_stream_bytes(dt, n)), torch.uint8, x.device, stream)
    if ws is None:
        ws = _empty(int(_lib.lcq_inline_workspace_bytes(_q(q))), torch.uint8, x.device, stream)
    st = _lib.lcq_quantize_inline(_q(q), dt, float(eb), _ptr(x) if n else None, n, _ptr(out),
                                  out.numel(), _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(st, "lcq_quantize_inline")
    return out


def dequantize_inline(stream_buf, dtype, n, *, out=None, ws=None, stream=None):
    """Decode an in-line layout stream into n values; the header check's
    result lands in ws (read with stream_status)."""
    import torch
    dt = _dtype_code(dtype)
    if out is None:
        out = _empty(n, dtype, stream_buf.device, stream)
    if ws is None:
        ws = _empty(64, torch.uint8, stream_buf.device, stream)
    st = _lib.lcq_dequantize_inline(dt, _ptr(stream_buf), stream_buf.numel(),
                                    _ptr(out) if n else None, n, _ptr(ws), ws.numel(),
                                    _stream_handle(stream))
    _check(st, "lcq_dequantize_inline")
    return out


def stream_status(ws, stream=None):
    """Status (OK / ERR_STREAM) of the last dequantize that used ws; syncs."""
    err = ctypes.c_int32(0)
    _check(_lib.lcq_stream_status(_ptr(ws), _stream_handle(stream), ctypes.byref(err)),
           "lcq_stream_status")
    return int(err.value)


def tune_variants():
    """Number of launch-shape variants of each per-value kernel."""
    return int(_lib.lcq_tune_variants())


def tune_set(op, dtype, variant):
    """Select launch-shape `variant` for op 'quantize' / 'dequantize' and a
    torch dtype (process-wide; every variant gives the same bytes)."""
    _check(_lib.lcq_tune_set(_OPS[op], _dtype_code(dtype), int(variant)), "lcq_tune_set")


def tune_get(op, dtype):
    return int(_lib.lcq_tune_get(_OPS[op], _dtype_code(dtype)))


def set_lookback_spin(polls):
    """Testing hook: polls before the quantize look-back counts a missing
    predecessor tile from its input (default 4096; 0 = always)."""
    _lib.lcq_debug_set_lookback_spin(int(polls))


def profile_mid_event(mid=None):
    """Record a torch.cuda.Event between the two kernels of every following
    two-pass quantize call from this thread (None clears)."""
    _lib.lcq_profile_mid_event(ctypes.c_void_p(mid.cuda_event) if mid is not None else None)


def profile_events(before=None, after=None):
    """Record torch.cuda.Event pairs around the main kernel of every following
    quantize / dequantize call from this thread (None clears)."""
    b = ctypes.c_void_p(before.cuda_event) if before is not None else None
    a = ctypes.c_void_p(after.cuda_event) if after is not None else None
    _lib.lcq_profile_events(b, a)
