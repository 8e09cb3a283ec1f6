"""Build the gfx950 HIP library paper_2407_15037_amd/liblcq.so with hipcc.

Flags: no floating-point contraction and no fast-math on host and device
(the parity rule of section 3.2 of the paper), packed-FP32 instructions
disabled, subnormals kept (the HIP default for gfx950).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "liblcq.so")
SRCS = [os.path.join(HERE, "csrc", f) for f in ("lcq.hip", "lcq_batch.hip", "lcq_serve.hip",
                                                       "lcq_pack.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(out=SO, extra=(), quiet=True):
    cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), *SRCS, "-o", out + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    os.replace(out + ".tmp", out)
    if res.stderr and not quiet:
        print(res.stderr)
    return out


def asm(out_path, extra=(), src=None):
    """Device assembly of one source of the library (for instruction checks)."""
    cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC")], *extra,
           "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), src or SRCS[0], "-o", out_path]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out_path


if __name__ == "__main__":
    print(build(quiet=False))
