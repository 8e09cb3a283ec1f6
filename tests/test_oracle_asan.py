"""The oracle has no out-of-bounds or use-after-free access: a build with
AddressSanitizer runs every pin (quantize / dequantize of both layouts,
corrupted-stream rejection, the packing stage, the section 6 ablations) and
the chunk-parallel wrapper on ragged sizes in a child process; a control
shows the same build stops a planted one-past-the-end write.  CPU only."""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import numpy as np
import oracle as O
import pins
import synth
L = O.lib({so!r})
for p in pins.PINS:
    p(L)
# the chunk-parallel wrapper: thread counts below and above the chunk count
for n in (0, 1, 1023, 1025, 5 * 1024 + 77):
    x = synth.sines_1d(max(n, 1), 7, dtype=np.float32)[:n]
    for q in ("abs", "rel", "noa"):
        for th in (1, 3, 64):
            a = O.quantize(q, x, 1e-3, L=L)
            b = O.quantize_mt(q, x, 1e-3, th, L=L)
            assert np.array_equal(a, b)
            d = O.dequantize_mt(b, np.float32, n, th, L=L)
            assert np.array_equal(d.view(np.uint32), O.dequantize(a, np.float32, n, L=L).view(np.uint32))
print("ASAN-CLEAN")
"""


def _asan_env():
    lib = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                         text=True).stdout.strip()
    if not (os.path.isabs(lib) and os.path.exists(lib)):
        return None
    env = dict(os.environ)
    # the interpreter itself is not instrumented: its own allocations are
    # not leak-checked, and the runtime must be loaded first
    env["LD_PRELOAD"] = (lib + " " + env.get("LD_PRELOAD", "")).strip()
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    return env


FLAGS = ["-fsanitize=address", "-fno-omit-frame-pointer", "-g"]


def test_oracle_under_asan(tmp_path):
    env = _asan_env()
    if env is None:
        pytest.skip("libasan not available")
    so = str(tmp_path / "liblcq_oracle_asan.so")
    try:
        obuild.build(extra_flags=FLAGS, out=so, quiet=True)
    except RuntimeError as e:
        pytest.skip(f"ASan build unavailable: {e}")
    code = CHILD.format(root=ROOT, tests=HERE, so=so)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=900)
    assert res.returncode == 0 and "ASAN-CLEAN" in res.stdout, res.stdout[-2000:] + res.stderr[-4000:]
    assert "AddressSanitizer" not in res.stderr, res.stderr[-4000:]


def test_asan_catches_planted_overflow(tmp_path):
    """Control: a copy of the oracle whose dequantize writes one value past
    the end of its output is stopped by the same build."""
    env = _asan_env()
    if env is None:
        pytest.skip("libasan not available")
    src = open(os.path.join(ROOT, "oracle", "lcq_oracle.c")).read()
    marker = "/* ASAN-CONTROL: dequantize output end */"
    assert src.count(marker) == 1
    planted = src.replace(marker, "((unsigned char *)out_v)[n * s] = 0;")
    (tmp_path / "lcq_oracle.c").write_text(planted)
    (tmp_path / "lcq_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "lcq_oracle.h")).read())
    so = str(tmp_path / "planted.so")
    cmd = ["gcc", *obuild.CFLAGS, "-w", *FLAGS, str(tmp_path / "lcq_oracle.c"), "-o", so,
           "-lm", "-lpthread"]
    if subprocess.run(cmd, capture_output=True).returncode != 0:
        pytest.skip("ASan build unavailable")
    code = (f"import sys; sys.path[:0] = [{ROOT!r}, {HERE!r}]\n"
            "import numpy as np, oracle as O, synth\n"
            f"L = O.lib({so!r})\n"
            "x = synth.sines_1d(5000, 3, dtype=np.float32)\n"
            "st = O.quantize('abs', x, 1e-3, L=L)\n"
            "O.dequantize(st, np.float32, x.size, L=L)\n"
            "print('SURVIVED')")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=300)
    assert res.returncode != 0 and "heap-buffer-overflow" in res.stderr, res.stderr[-3000:]
