"""The oracle is free of undefined behaviour on the inputs that trip the
paper's printed routines (section 3.2 type punning and shifts, section 3.3
INT_MIN bins): a build with UBSan (float-cast-overflow included, no recovery)
runs the special-value, bin-range and bound pins in a child process.  CPU
only."""
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
import oracle as O
import pins
L = O.lib({so!r})
for p in (pins.pin_specials, pins.pin_bin_range, pins.pin_bounds, pins.pin_roundtrip_sizes,
          pins.pin_noa_degenerate, pins.pin_mitchell_golden, pins.pin_mitchell_powers_of_two):
    p(L)
print("UBSAN-CLEAN")
"""


def test_oracle_under_ubsan(tmp_path):
    so = str(tmp_path / "liblcq_oracle_ubsan.so")
    try:
        obuild.build(extra_flags=["-fsanitize=undefined,float-cast-overflow",
                                  "-fno-sanitize-recover=all", "-g"], out=so, quiet=True)
    except RuntimeError as e:
        pytest.skip(f"UBSan build unavailable: {e}")
    env = dict(os.environ)
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    # the sanitizer runtime must be loaded before the instrumented library
    libubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True,
                              text=True).stdout.strip()
    if os.path.isabs(libubsan) and os.path.exists(libubsan):
        env["LD_PRELOAD"] = (libubsan + " " + env.get("LD_PRELOAD", "")).strip()
    code = CHILD.format(root=ROOT, tests=HERE, so=so)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=600)
    assert res.returncode == 0 and "UBSAN-CLEAN" in res.stdout, res.stdout[-2000:] + res.stderr[-4000:]
    assert "runtime error" not in res.stderr, res.stderr[-4000:]


def test_ubsan_catches_conversion_before_range_test(tmp_path):
    """Control: the same sanitizer build does flag the section 3.3 hazard when
    the float bin is converted to int before the range test (planted in a
    copy of the oracle source, CPU only)."""
    src = open(os.path.join(ROOT, "oracle", "lcq_oracle.c")).read()
    old = ("if (!(qf > -(float)MAXBIN && qf < (float)MAXBIN)) return 1;\n  int32_t b = (int32_t)qf;\n"
           "  float rec = (float)b * p->stepf;")
    new = ("int32_t b = (int32_t)qf;\n  if (!(qf > -(float)MAXBIN && qf < (float)MAXBIN)) return 1;\n"
           "  float rec = (float)b * p->stepf;")
    assert src.count(old) == 1
    (tmp_path / "lcq_oracle.c").write_text(src.replace(old, new))
    (tmp_path / "lcq_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "lcq_oracle.h")).read())
    so = str(tmp_path / "planted.so")
    cmd = ["gcc", *obuild.CFLAGS, "-w", "-fsanitize=undefined,float-cast-overflow",
           "-fno-sanitize-recover=all", str(tmp_path / "lcq_oracle.c"), "-o", so, "-lm"]
    if subprocess.run(cmd, capture_output=True).returncode != 0:
        pytest.skip("UBSan build unavailable")
    env = dict(os.environ)
    libubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True,
                              text=True).stdout.strip()
    if os.path.isabs(libubsan) and os.path.exists(libubsan):
        env["LD_PRELOAD"] = (libubsan + " " + env.get("LD_PRELOAD", "")).strip()
    code = (f"import sys; sys.path[:0] = [{ROOT!r}, {HERE!r}]\n"
            f"import oracle as O, pins\npins.pin_bin_range(O.lib({so!r}))\nprint('SURVIVED')")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=300)
    assert res.returncode != 0 and "outside the range of representable values" in res.stderr
