"""CPU checks of the C ABI library: it loads, exports every function that
include/lcq.h declares, rejects bad arguments on the host without touching a
GPU, and its gfx950 code keeps the parity rules of section 3.2 (no fused
multiply-add and no packed-FP32 arithmetic in the per-value kernels,
float32 subnormals kept)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcq.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lcq_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("lcq_quantize", "lcq_dequantize", "lcq_max_stream_bytes",
                 "lcq_workspace_bytes", "lcq_stream_status"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_2407_15037_amd as lcq
    out = subprocess.run(["nm", "-D", "--defined-only", lcq.SO_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        assert hasattr(lcq.lib(), f)


def test_sizes_and_host_argument_errors():
    import paper_2407_15037_amd as lcq
    L = lcq.lib()
    # layout arithmetic (no GPU involved)
    assert L.lcq_max_stream_bytes(0, 0) == 64
    assert L.lcq_max_stream_bytes(0, 1) == 64 + 16 + 16 + 4
    n = 1 << 20
    ct = (64 + 4 * n + 15) // 16 * 16
    out = (ct + 8 * (n // 1024) + 15) // 16 * 16
    assert L.lcq_max_stream_bytes(0, n) == out + 4 * n
    assert L.lcq_max_stream_bytes(1, n) == out + 8 * n
    assert L.lcq_max_stream_bytes(2, n) == 0
    assert L.lcq_workspace_bytes(0, 0, n) > 0 and L.lcq_workspace_bytes(3, 0, n) == 0
    vp = ctypes.c_void_p
    fake = vp(1 << 20)  # never dereferenced: every call below fails on the host
    cases = [
        (7, 0, 1e-3), (0, 9, 1e-3), (0, 0, 0.0), (0, 0, -1.0), (0, 0, float("nan")),
        (0, 0, float("inf")), (1, 0, 1.0), (1, 0, 1.5),
    ]
    for q, t, eb in cases:
        st = L.lcq_quantize(q, t, eb, fake, 16, fake, 1 << 30, fake, fake, 1 << 30, None)
        assert st == lcq.ERR_ARG, (q, t, eb, st)
    # misaligned pointer
    st = L.lcq_quantize(0, 0, 1e-3, vp((1 << 20) + 4), 16, fake, 1 << 30, fake, fake, 1 << 30, None)
    assert st == lcq.ERR_ARG
    # capacity
    st = L.lcq_quantize(0, 0, 1e-3, fake, 1000, fake, 100, fake, fake, 1 << 30, None)
    assert st == lcq.ERR_CAPACITY
    st = L.lcq_quantize(0, 0, 1e-3, fake, 1000, fake, 1 << 30, fake, fake, 8, None)
    assert st == lcq.ERR_CAPACITY
    # dequantize: stream too short for the codes of n values
    st = L.lcq_dequantize(0, fake, 100, fake, 1000, fake, 64, None)
    assert st == lcq.ERR_STREAM
    assert L.lcq_dequantize(5, fake, 1 << 20, fake, 10, fake, 64, None) == lcq.ERR_ARG
    assert L.lcq_status_string(3).decode().startswith("stream")


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    from paper_2407_15037_amd import build
    path = str(tmp_path_factory.mktemp("asm") / "lcq.s")
    build.asm(path)
    return open(path).read()


def kernel_bodies(asm):
    bodies = {}
    for m in re.finditer(r"^(_Z\w+):[^\n]*$(.*?)^\.Lfunc_end", asm, flags=re.M | re.S):
        bodies[m.group(1)] = m.group(2)
    return bodies


PER_VALUE = ("k_quantize", "k_dequantize", "k_quant_stage", "k_quant_finish")
# the library-log2/exp2 ablation (quantizer code 4) runs the device math
# library's own code, which may fuse; it is outside the parity rule by design
LIBM_ABLATION = re.compile(r"k_quant_stageI[fd]Li4E|k_dequantize_ablationI[fd]Li4E")


def test_per_value_kernels_have_no_fused_or_packed_fp(device_asm):
    bodies = kernel_bodies(device_asm)
    per_value = {k: v for k, v in bodies.items() if any(p in k for p in PER_VALUE)}
    assert len(per_value) >= 8, sorted(bodies)
    assert any("k_quant_stage" in k for k in per_value) and any("k_quant_finish" in k for k in per_value)
    # floating-point multiply-adds of any form (integer address mads are fine)
    fused = re.compile(r"^\s*(v_(?:fma|fmac|mad|mac)\w*_f(?:16|32|64)\w*|v_mad_legacy\w*|"
                       r"v_fma_legacy\w*)\b", flags=re.M)
    packed = re.compile(r"^\s*(v_pk_fma_f32|v_pk_mul_f32|v_pk_add_f32)\b", flags=re.M)
    libm = 0
    for name, body in per_value.items():
        hits = packed.findall(body)
        assert not hits, (name, hits[:5])
        if LIBM_ABLATION.search(name):
            libm += 1
            continue
        hits = fused.findall(body)
        assert not hits, (name, hits[:5])
    assert libm == 4, libm


@pytest.fixture(scope="module")
def compress_asm(tmp_path_factory):
    from paper_2407_15037_amd import build
    path = str(tmp_path_factory.mktemp("asm") / "lcq_compress.s")
    build.asm(path, src=os.path.join(ROOT, "paper_2407_15037_amd", "csrc", "lcq_compress.hip"))
    return open(path).read()


def test_fused_kernels_have_no_fused_or_packed_fp(compress_asm):
    """The fused compress / decompress encode and decode every value too:
    the same rule holds for their kernels."""
    bodies = kernel_bodies(compress_asm)
    fused_path = {k: v for k, v in bodies.items()
                  if any(p in k for p in ("k_cmp_stage", "k_cmp_write", "k_cmp_finish",
                                          "k_decompress"))}
    assert len(fused_path) == 3 * 2 * 3 + 2, sorted(bodies)
    fused = re.compile(r"^\s*(v_(?:fma|fmac|mad|mac)\w*_f(?:16|32|64)\w*|v_mad_legacy\w*|"
                       r"v_fma_legacy\w*|v_pk_fma_f32|v_pk_mul_f32|v_pk_add_f32)\b", flags=re.M)
    for name, body in fused_path.items():
        hits = fused.findall(body)
        assert not hits, (name, hits[:5])
    modes = re.findall(r"\.amdhsa_float_denorm_mode_32\s+(\d+)", compress_asm)
    assert modes and all(m == "3" for m in modes), modes


@pytest.fixture(scope="module")
def pack_asm(tmp_path_factory):
    from paper_2407_15037_amd import build
    path = str(tmp_path_factory.mktemp("asm") / "lcq_pack.s")
    build.asm(path, src=os.path.join(ROOT, "paper_2407_15037_amd", "csrc", "lcq_pack.hip"))
    return open(path).read()


# cross-lane (DPP) instruction forms measured right on gfx950 by a lane-layout
# check; a subtraction with a DPP operand measured wrong there
DPP_FORMS = {"v_mov_b32_dpp", "v_add_u32_dpp", "v_or_b32_dpp"}


def test_only_checked_dpp_forms(device_asm, compress_asm, pack_asm, tmp_path):
    from paper_2407_15037_amd import build
    others = []
    for name in ("lcq_batch.hip", "lcq_serve.hip"):
        path = str(tmp_path / (name + ".s"))
        build.asm(path, src=os.path.join(ROOT, "paper_2407_15037_amd", "csrc", name))
        others.append(open(path).read())
    for asm in [device_asm, compress_asm, pack_asm] + others:
        used = set(re.findall(r"^\s*(v_\w+_dpp)\b", asm, flags=re.M))
        assert used <= DPP_FORMS, sorted(used - DPP_FORMS)
    assert re.search(r"^\s*v_mov_b32_dpp\b.*wave_shr:1", compress_asm, flags=re.M)


def test_fused_entry_points_refuse_bad_arguments():
    import paper_2407_15037_amd as lcq
    L = lcq.lib()
    vp = ctypes.c_void_p
    fake = vp(1 << 20)  # never dereferenced: every call below fails on the host
    n = 1 << 20
    assert L.lcq_compress_workspace_bytes(0, 0, n) > L.lcq_compress_workspace_bytes(0, 0, 1000) > 0
    assert L.lcq_compress_workspace_bytes(2, 1, n) > L.lcq_compress_workspace_bytes(0, 1, n)
    assert L.lcq_compress_workspace_bytes(3, 0, n) == 0
    assert L.lcq_compress_workspace_bytes(0, 2, n) == 0
    big = 1 << 40
    for q, t, eb in [(7, 0, 1e-3), (0, 9, 1e-3), (0, 0, 0.0), (0, 0, float("nan")), (1, 0, 1.0)]:
        st = L.lcq_compress(q, t, eb, fake, 16, fake, big, fake, fake, big, None)
        assert st == lcq.ERR_ARG, (q, t, eb, st)
    st = L.lcq_compress(0, 0, 1e-3, vp((1 << 20) + 4), 16, fake, big, fake, fake, big, None)
    assert st == lcq.ERR_ARG
    # packed capacity below pack_max_bytes, workspace below its size
    cap = L.lcq_pack_max_bytes(0, 1000)
    st = L.lcq_compress(0, 0, 1e-3, fake, 1000, fake, cap - 1, fake, fake, big, None)
    assert st == lcq.ERR_CAPACITY
    wsb = L.lcq_compress_workspace_bytes(0, 0, 1000)
    st = L.lcq_compress(0, 0, 1e-3, fake, 1000, fake, cap, fake, fake, wsb - 1, None)
    assert st == lcq.ERR_CAPACITY
    # decompress: too short for the offset table, bad dtype, small workspace
    assert L.lcq_decompress(0, fake, 64, fake, 1000, fake, 64, None) == lcq.ERR_STREAM
    assert L.lcq_decompress(5, fake, 1 << 20, fake, 10, fake, 64, None) == lcq.ERR_ARG
    assert L.lcq_decompress(0, fake, 1 << 20, fake, 10, fake, 4, None) == lcq.ERR_CAPACITY


def test_float32_subnormals_kept(device_asm):
    modes = re.findall(r"\.amdhsa_float_denorm_mode_32\s+(\d+)", device_asm)
    assert modes and all(m == "3" for m in modes), modes


def test_batch_tuning_strings():
    """The batch plan's tuning string is read on the host: both spellings of
    the same tuning give the same workspace, chunks per wavefront change the
    plan's layout, and a malformed value is refused (workspace 0)."""
    import paper_2407_15037_amd as lcq
    from paper_2407_15037_amd.batch import Field
    L = lcq.lib()
    arr = (Field * 3)()
    fake = 1 << 20  # never dereferenced by the size query
    for i, (q, t, n) in enumerate([(0, 0, 100000), (1, 1, 5000), (2, 0, 3 << 20)]):
        arr[i] = Field(q, t, 1e-3, fake, n, fake, 1 << 40, fake, fake)

    def ws(tune):
        return int(L.lcq_batch_workspace_bytes(arr, 3, None if tune is None else tune.encode()))

    base = ws(None)
    assert base > 0 and ws("batch=0") == base and ws("batch=0 f32=1 f64=1") == base
    assert ws("batch=0 f32=4 f64=2") == ws('{"batch": 0, "f32": 4, "f64": 2}') > 0
    assert ws("batch=0 f32=4 f64=2") != base  # fewer quantize items, fewer group sums
    for bad in ("batch=99", "batch=0 f32=3", "f64=0", "f32=32", "batch=x"):
        assert ws(bad) == 0, bad
