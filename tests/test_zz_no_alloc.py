"""lcq_quantize_noalloc: the allocation-free quantize (fixed per-GPU
workspace inside the library) gives the same stream, byte for byte, as
lcq_quantize with a caller workspace, call after call on the shared array,
including a second, smaller input after a larger one."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce, first_diff

pytestmark = pytest.mark.gpu


def _plain(xt, q, eb):
    import torch
    import paper_2407_15037_amd as lcq
    st, nb = lcq.quantize(xt, q, eb)
    torch.cuda.synchronize()
    return st[: int(nb.item())].cpu().numpy()


def _noalloc(xt, q, eb, fill):
    """Through the C ABI with caller buffers; the stream buffer is filled
    with junk first so stale bytes would show."""
    import torch
    import paper_2407_15037_amd as lcq
    cap = lcq.max_stream_bytes(xt.dtype, xt.numel())
    out = torch.full((cap,), fill, dtype=torch.uint8, device="cuda")
    nb = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    lcq.quantize_noalloc(xt, q, eb, out=out, nbytes=nb)
    torch.cuda.synchronize()
    return out[: int(nb.item())].cpu().numpy()


CASES = [
    # (quantizer, dtype, n, eb): each row runs after the one above it on the
    # same array; sizes fall and rise so leftovers of a larger call are seen
    ("noa", np.float32, 5 * (1 << 20) + 4099, 1e-3),
    ("abs", np.float32, 3 * (1 << 20) + 17, 1e-3),
    ("rel", np.float32, (1 << 21) + 1023, 1e-2),
    ("abs", np.float64, (1 << 20) + 77, 1e-6),
    ("noa", np.float64, 70_001, 1e-4),
    ("rel", np.float64, 4_097, 1e-3),
    ("abs", np.float32, 0, 1e-3),
]


def _input(q, dt, n, seed):
    x = synth.sines_1d(n, seed, dtype=dt)
    if q == "rel":
        x = synth.rel_variant(x.astype(np.float64), seed + 1, dtype=dt)
    if n:
        x = synth.with_specials(x, q, max(1, n // 1000), seed + 2, 1e-3)
    return np.ascontiguousarray(x)


def test_noalloc_equals_quantize_call_after_call():
    import torch
    for i, (q, dt, n, eb) in enumerate(CASES):
        x = _input(q, dt, n, 900 + 5 * i)
        xt = torch.from_numpy(x).cuda()
        announce("noalloc", i, q, np.dtype(dt).name, n, eb)
        want = _plain(xt, q, eb)
        got = _noalloc(xt, q, eb, 0x5A if i % 2 else 0xC3)
        assert first_diff(got, want) is None, (i, q, n, first_diff(got, want))
        if n <= (1 << 21):
            assert first_diff(got, O.quantize(q, x, eb)) is None, (i, q, n)


def test_noalloc_twice_second_smaller():
    """The required pair: a call, then a smaller one, both equal to
    lcq_quantize's streams."""
    import torch
    big = _input("abs", np.float32, 6 * (1 << 20) + 333, 950)
    small = _input("abs", np.float32, 100_003, 951)
    for tag, x in (("first", big), ("second", small)):
        xt = torch.from_numpy(x).cuda()
        announce("noalloc pair", tag, x.size)
        want = _plain(xt, "abs", 1e-3)
        got = _noalloc(xt, "abs", 1e-3, 0xEE)
        assert first_diff(got, want) is None, (tag, first_diff(got, want))


def test_noalloc_rejects_sizes_beyond_the_array():
    import ctypes
    import paper_2407_15037_amd as lcq
    L = lcq.lib()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: refused on the host
    big = 1 << 30
    assert L.lcq_workspace_bytes(lcq.ABS, lcq.F32, big) > lcq.NOALLOC_SCRATCH_BYTES
    st = L.lcq_quantize_noalloc(lcq.ABS, lcq.F32, 1e-3, fake, big, fake, 1 << 62, fake, None)
    assert st == lcq.ERR_CAPACITY
