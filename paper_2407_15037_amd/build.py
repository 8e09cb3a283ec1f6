"""Build the gfx950 HIP library paper_2407_15037_amd/liblcq.so with hipcc.

Flags: no floating-point contraction and no fast-math on host and device
(the parity rule of section 3.2 of the paper), packed-FP32 instructions
disabled, subnormals kept (the HIP default for gfx950).  Each source is
compiled to an object in its own hipcc process (in parallel), then linked.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "liblcq.so")
OBJDIR = os.path.join(HERE, "_build")
SRCS = [os.path.join(HERE, "csrc", f) for f in ("lcq.hip", "lcq_batch.hip", "lcq_serve.hip",
                                                       "lcq_pack.hip", "lcq_compress.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _incs():
    return ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def _compile(src, extra):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, *_incs(), "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    return obj, res.stderr


def build(out=SO, extra=(), quiet=True):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SRCS), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, extra), SRCS))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *extra,
           *[o for o, _ in results], "-o", out + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    os.replace(out + ".tmp", out)
    if not quiet:
        for _, err in results:
            if err:
                print(err)
    return out


def asm(out_path, extra=(), src=None):
    """Device assembly of one source of the library (for instruction checks)."""
    cmd = [HIPCC, *[f for f in FLAGS if f != "-fPIC"], *extra,
           "--cuda-device-only", "-S", *_incs(), src or SRCS[0], "-o", out_path]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out_path


if __name__ == "__main__":
    print(build(quiet=False))
