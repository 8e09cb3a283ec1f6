"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It loads oracle/liblcq_oracle.so (built by oracle/build.py), works
on numpy arrays in host memory and shares nothing with the HIP library.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblcq_oracle.so")

F32, F64 = 0, 1
ABS, REL, NOA = 0, 1, 2
OK, ERR_ARG, ERR_CAPACITY, ERR_STREAM, ERR_FPENV = 0, 1, 2, 3, 5
ABS_UNCHECKED, REL_LIBM = 3, 4  # the two ablations of section 6
QNAMES = {"abs": ABS, "rel": REL, "noa": NOA, "abs_unchecked": ABS_UNCHECKED,
          "rel_libm": REL_LIBM}


class Params(ctypes.Structure):
    _fields_ = [("step", ctypes.c_uint64), ("inv", ctypes.c_uint64),
                ("bound", ctypes.c_uint64), ("aux0", ctypes.c_uint64),
                ("aux1", ctypes.c_uint64), ("lambda_", ctypes.c_uint64),
                ("degenerate", ctypes.c_int32), ("pad", ctypes.c_int32)]


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


_lib = None


def lib(path=None):
    """Load (once) and return the oracle shared library."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(SO):
            from . import build
            build.build()
        _lib = _bind(ctypes.CDLL(SO))
    return _lib


def _bind(L):
    u64, vp, i32 = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
    L.orc_max_stream_bytes.argtypes = [i32, u64]
    L.orc_max_stream_bytes.restype = u64
    L.orc_params_derive.argtypes = [i32, i32, ctypes.c_double, vp, u64, ctypes.POINTER(Params)]
    L.orc_params_derive.restype = i32
    L.orc_quantize.argtypes = [i32, i32, ctypes.c_double, vp, u64, vp, u64, ctypes.POINTER(u64)]
    L.orc_quantize.restype = i32
    L.orc_dequantize.argtypes = [i32, vp, u64, vp, u64]
    L.orc_dequantize.restype = i32
    L.orc_quantize_mt.argtypes = [i32, i32, ctypes.c_double, vp, u64, vp, u64,
                                  ctypes.POINTER(u64), i32]
    L.orc_quantize_mt.restype = i32
    L.orc_dequantize_mt.argtypes = [i32, vp, u64, vp, u64, i32]
    L.orc_dequantize_mt.restype = i32
    L.orc_threads_used.argtypes = [i32]
    L.orc_threads_used.restype = i32
    L.orc_inline_stream_bytes.argtypes = [i32, u64]
    L.orc_inline_stream_bytes.restype = u64
    L.orc_quantize_inline.argtypes = [i32, i32, ctypes.c_double, vp, u64, vp, u64, ctypes.POINTER(u64)]
    L.orc_quantize_inline.restype = i32
    L.orc_dequantize_inline.argtypes = [i32, vp, u64, vp, u64]
    L.orc_dequantize_inline.restype = i32
    L.orc_pack_max_bytes.argtypes = [i32, u64]
    L.orc_pack_max_bytes.restype = u64
    for name in ("orc_pack", "orc_unpack"):
        getattr(L, name).argtypes = [i32, vp, u64, u64, vp, u64, ctypes.POINTER(u64)]
        getattr(L, name).restype = i32
    for name in ("orc_log2approx_f32", "orc_pow2approx_f32",
                 "orc_log2approx_f64", "orc_pow2approx_f64"):
        getattr(L, name).argtypes = [vp, vp, u64]
        getattr(L, name).restype = None
    return L


def _dt(x):
    if x.dtype == np.float32:
        return F32
    if x.dtype == np.float64:
        return F64
    raise TypeError(f"unsupported dtype {x.dtype}")


def _q(q):
    return QNAMES[q] if isinstance(q, str) else int(q)


def max_stream_bytes(dtype, n, L=None):
    L = L or lib()
    return int(L.orc_max_stream_bytes(F64 if np.dtype(dtype) == np.float64 else F32, n))


def quantize(q, x, eb, L=None):
    """Quantize a contiguous float32/float64 numpy array; returns the stream
    as a uint8 numpy array of exactly the stream's size."""
    L = L or lib()
    x = np.ascontiguousarray(x)
    dt = _dt(x)
    cap = int(L.orc_max_stream_bytes(dt, x.size))
    buf = np.zeros(cap, dtype=np.uint8)
    nbytes = ctypes.c_uint64(0)
    st = L.orc_quantize(_q(q), dt, float(eb), x.ctypes.data, x.size,
                        buf.ctypes.data, cap, ctypes.byref(nbytes))
    if st != OK:
        raise OracleError(st, "orc_quantize")
    return buf[: nbytes.value].copy()


def quantize_mt(q, x, eb, threads=0, L=None):
    """quantize() split over `threads` threads at chunk boundaries (0: one
    per online CPU); the same bytes."""
    L = L or lib()
    x = np.ascontiguousarray(x)
    dt = _dt(x)
    cap = int(L.orc_max_stream_bytes(dt, x.size))
    buf = np.empty(cap, dtype=np.uint8)
    nbytes = ctypes.c_uint64(0)
    st = L.orc_quantize_mt(_q(q), dt, float(eb), x.ctypes.data, x.size,
                           buf.ctypes.data, cap, ctypes.byref(nbytes), int(threads))
    if st != OK:
        raise OracleError(st, "orc_quantize_mt")
    return buf[: nbytes.value]


def dequantize_mt(stream, dtype, n, threads=0, L=None):
    """dequantize() split over `threads` threads (0: one per online CPU)."""
    L = L or lib()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    out = np.empty(n, dtype=dtype)
    st = L.orc_dequantize_mt(_dt(out), stream.ctypes.data, stream.size, out.ctypes.data, n,
                             int(threads))
    if st != OK:
        raise OracleError(st, "orc_dequantize_mt")
    return out


def threads_used(threads=0, L=None):
    """Thread count a `threads` argument of the *_mt calls resolves to."""
    L = L or lib()
    return int(L.orc_threads_used(int(threads)))


def dequantize(stream, dtype, n, L=None):
    L = L or lib()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    out = np.empty(n, dtype=dtype)
    dt = _dt(out)
    st = L.orc_dequantize(dt, stream.ctypes.data, stream.size, out.ctypes.data, n)
    if st != OK:
        raise OracleError(st, "orc_dequantize")
    return out


def quantize_inline(q, x, eb, L=None):
    """In-line layout (one word per value + raw-value bitmap)."""
    L = L or lib()
    x = np.ascontiguousarray(x)
    dt = _dt(x)
    cap = int(L.orc_inline_stream_bytes(dt, x.size))
    buf = np.zeros(cap, dtype=np.uint8)
    nbytes = ctypes.c_uint64(0)
    st = L.orc_quantize_inline(_q(q), dt, float(eb), x.ctypes.data, x.size, buf.ctypes.data, cap,
                               ctypes.byref(nbytes))
    if st != OK:
        raise OracleError(st, "orc_quantize_inline")
    return buf[: nbytes.value].copy()


def dequantize_inline(stream, dtype, n, L=None):
    L = L or lib()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    out = np.empty(n, dtype=dtype)
    st = L.orc_dequantize_inline(_dt(out), stream.ctypes.data, stream.size, out.ctypes.data, n)
    if st != OK:
        raise OracleError(st, "orc_dequantize_inline")
    return out


def pack(stream, dtype, n, L=None):
    """Lossless packing stage: an LCQ1 stream (uint8 array) -> packed stream."""
    L = L or lib()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    dt = F64 if np.dtype(dtype) == np.float64 else F32
    cap = int(L.orc_pack_max_bytes(dt, n))
    buf = np.zeros(cap, dtype=np.uint8)
    nbytes = ctypes.c_uint64(0)
    st = L.orc_pack(dt, stream.ctypes.data, stream.size, n, buf.ctypes.data, cap, ctypes.byref(nbytes))
    if st != OK:
        raise OracleError(st, "orc_pack")
    return buf[: nbytes.value].copy()


def unpack(packed, dtype, n, L=None):
    """Inverse of pack(): the LCQ1 stream, byte for byte."""
    L = L or lib()
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    dt = F64 if np.dtype(dtype) == np.float64 else F32
    cap = int(L.orc_max_stream_bytes(dt, n))
    buf = np.zeros(cap, dtype=np.uint8)
    nbytes = ctypes.c_uint64(0)
    st = L.orc_unpack(dt, packed.ctypes.data, packed.size, n, buf.ctypes.data, cap, ctypes.byref(nbytes))
    if st != OK:
        raise OracleError(st, "orc_unpack")
    return buf[: nbytes.value].copy()


def params(q, dtype, eb, x=None, L=None):
    """Derived per-field parameters, as a dict of numpy scalars of dtype."""
    L = L or lib()
    dtype = np.dtype(dtype)
    dt = F64 if dtype == np.float64 else F32
    p = Params()
    if x is not None:
        x = np.ascontiguousarray(x, dtype=dtype)
        ptr, n = x.ctypes.data, x.size
    else:
        ptr, n = None, 0
    st = L.orc_params_derive(_q(q), dt, float(eb), ptr, n, ctypes.byref(p))
    if st != OK:
        raise OracleError(st, "orc_params_derive")
    ut = np.uint64 if dt == F64 else np.uint32

    def val(bits):
        return np.array([bits], dtype=ut).view(dtype)[0]
    return {"step": val(p.step), "inv": val(p.inv), "bound": val(p.bound),
            "aux0": val(p.aux0), "aux1": val(p.aux1), "lambda": val(p.lambda_),
            "degenerate": bool(p.degenerate)}


def _elementwise(name, x, dtype, L):
    L = L or lib()
    x = np.ascontiguousarray(x, dtype=dtype)
    out = np.empty_like(x)
    getattr(L, name)(x.ctypes.data, out.ctypes.data, x.size)
    return out


def log2approx(x, L=None):
    x = np.asarray(x)
    if x.dtype == np.float64:
        return _elementwise("orc_log2approx_f64", x, np.float64, L)
    return _elementwise("orc_log2approx_f32", x, np.float32, L)


def pow2approx(x, L=None):
    x = np.asarray(x)
    if x.dtype == np.float64:
        return _elementwise("orc_pow2approx_f64", x, np.float64, L)
    return _elementwise("orc_pow2approx_f32", x, np.float32, L)
