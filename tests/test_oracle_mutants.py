"""The pins are strong enough: each plausible mistake, planted in a copy of the
oracle's source and built on the CPU, makes at least one pin fail.  CPU only.

Every mutant names an exact snippet of oracle/lcq_oracle.c; if the snippet
is no longer there the test fails loudly instead of silently passing.
"""
import os
import tempfile

import pytest

import oracle as O
from oracle import build as obuild
from pins import PINS

SRC = os.path.join(os.path.dirname(O.__file__), "lcq_oracle.c")

MUTANTS = {
    # section 3.2 log2: de-biasing off by one
    "log2_bias": ("float e_minus = (float)((int32_t)E - 128);",
                  "float e_minus = (float)((int32_t)E - 127);"),
    # section 3.2 pow2: fraction rebuilt from the wrong integer
    "pow2_frac": ("float g = t - (float)(k - 1);", "float g = t - (float)k;"),
    # double-check against the bin width instead of the bound (sec. 3.1)
    "abs_verify_loose": ("if (p->q != ORC_ABS_UNCHECKED && !(fabsf(x - rec) <= p->boundf)) return 1;",
                         "if (p->q != ORC_ABS_UNCHECKED && !(fabsf(x - rec) <= p->stepf)) return 1;"),
    # double-check dropped entirely for float64
    "abs_verify_dropped_f64": ("if (p->q != ORC_ABS_UNCHECKED && !(fabs(x - rec) <= p->bound)) return 1;", ""),
    # nearest bin replaced by truncation
    "bin_trunc": ("float qf = rintf(x * p->invf);", "float qf = truncf(x * p->invf);"),
    # bin range test admits +2^30 (sec. 3.3)
    "range_inclusive": ("if (!(qf > -(float)MAXBIN && qf < (float)MAXBIN)) return 1;\n  int32_t b = (int32_t)qf;\n  float rec = (float)b * p->stepf;",
                        "if (!(qf > -(float)MAXBIN && qf <= (float)MAXBIN)) return 1;\n  int32_t b = (int32_t)qf;\n  float rec = (float)b * p->stepf;"),
    # denormals quantized instead of stored losslessly
    "denormal_binned": ("  if (E == 0 && F != 0) return 1;\n  if (is_rel(p->q) && E == 0) return 1;\n  if (p->q == ORC_NOA && p->degenerate) return 1;\n\n  if (is_rel(p->q)) {\n    const int libm = p->q == ORC_REL_LIBM;\n    float a",
                        "  if (is_rel(p->q) && E == 0) return 1;\n  if (p->q == ORC_NOA && p->degenerate) return 1;\n\n  if (is_rel(p->q)) {\n    const int libm = p->q == ORC_REL_LIBM;\n    float a"),
    # REL lower side checked against eh instead of eb/(1+eb)
    "rel_low_side": ("else ok = (a - rec) < (p->aux0f * a);", "else ok = (a - rec) < (p->boundf * a);"),
    # REL sign bit lost
    "rel_sign": ("*code = (int32_t)(((uint32_t)b << 1) | (u >> 31));",
                 "*code = (int32_t)((uint32_t)b << 1);"),
    # NOA range over all values, infinities included
    "noa_nonfinite": ("    if (!isfinite(v)) continue;\n    if (v == 0.0f) v = 0.0f;",
                      "    if (isnan(v)) continue;\n    if (v == 0.0f) v = 0.0f;"),
    # NOA: ebR rounded to nearest, not stepped down
    "noa_no_stepdown": ("    if (b > 0.0) ebr = nextafter(b, 0.0);", ""),
    # chunk table written after the value is counted
    "chunk_off_by_one": ("    if (i % CHUNK == 0) put_u64(S + ct + 8 * (i / CHUNK), k);\n",
                         "    if (i % CHUNK == 1) put_u64(S + ct + 8 * (i / CHUNK), k);\n"),
    # outliers stored as floats through a conversion (NaN payload / sNaN lost)
    "outlier_via_float": ("      memcpy(S + out + s * k, (const uint8_t *)in + s * i, s);",
                          "      if (s == 4) { float v; memcpy(&v, (const uint8_t *)in + s * i, 4); volatile double w = v; v = (float)w; memcpy(S + out + s * k, &v, 4); } else memcpy(S + out + s * k, (const uint8_t *)in + s * i, s);"),
    # REL el derived as round-down of eb instead of eb/(1+eb)
    "rel_el": ("float el = round_down_f32(rel_low_double(eb));", "float el = round_down_f32(eb);"),
    # ABS step taken as e instead of 2e
    "abs_step": ("    p->stepf = e + e;", "    p->stepf = e;"),
    # packing: zigzag with a logical shift (negative values mapped wrongly)
    "pack_zigzag": ("static uint32_t zigzag32(uint32_t v) { return (v << 1) ^ (uint32_t)((int32_t)v >> 31); }",
                    "static uint32_t zigzag32(uint32_t v) { return (v << 1) ^ (v >> 31); }"),
    # packing: delta mode taken on a tie
    "pack_tie": ("  *mode = wd < wp;", "  *mode = wd <= wp;"),
    # packing: most significant bit of each byte first
    "pack_bit_order": ("if ((z >> t) & 1u) bits[(j * w + t) / 8] |= (uint8_t)(1u << ((j * w + t) % 8));",
                       "if ((z >> t) & 1u) bits[(j * w + t) / 8] |= (uint8_t)(0x80u >> ((j * w + t) % 8));"),
    # ablation: the unchecked ABS still runs the double-check
    "unchecked_checks": ("if (p->q != ORC_ABS_UNCHECKED && !(fabsf(x - rec) <= p->boundf)) return 1;",
                         "if (!(fabsf(x - rec) <= p->boundf)) return 1;"),
    # ablation: library-log2 REL keeps the approximation's bin width
    "libm_lambda": ("float lam = q == ORC_REL_LIBM ? log2f(1.0f + eh) : log2approx_f32(1.0f + eh);",
                    "float lam = log2approx_f32(1.0f + eh);"),
    # ablation: library-log2 REL decoded with the approximate 2^y
    "libm_decode": ("float a = q == ORC_REL_LIBM ? exp2f((float)b * step) : pow2approx_f32((float)b * step);",
                    "float a = pow2approx_f32((float)b * step);"),
}


@pytest.fixture(scope="module")
def source():
    return open(SRC).read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutant {name}: snippet not found exactly once"
    msrc = tmp_path / "lcq_oracle.c"
    msrc.write_text(source.replace(old, new))
    (tmp_path / "lcq_oracle.h").write_text(open(os.path.join(os.path.dirname(SRC), "lcq_oracle.h")).read())
    so = str(tmp_path / f"mut_{name}.so")
    import subprocess
    cmd = ["gcc", *obuild.CFLAGS, "-w", str(msrc), "-o", so, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    L = O.lib(so)
    caught = []
    for pin in PINS:
        try:
            pin(L)
        except AssertionError:
            caught.append(pin.__name__)
            break
        except O.OracleError:
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} survived every pin"
