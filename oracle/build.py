"""Build the CPU oracle (test infrastructure) into oracle/liblcq_oracle.so.

Flags follow the paper's parity rule (section 3.2): no floating-point
contraction, no fast-math, SSE arithmetic (x86-64 default) in round-to-nearest.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblcq_oracle.so")

CFLAGS = [
    "-std=gnu11", "-O2", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
    "-mfpmath=sse", "-msse2", "-Wall", "-Wextra",
]


def build(extra_flags=(), out=SO, quiet=False):
    """Compile lcq_oracle.c with gcc; returns the path of the shared object."""
    cmd = ["gcc", *CFLAGS, *extra_flags, os.path.join(HERE, "lcq_oracle.c"),
           "-o", out, "-lm", "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    if res.stderr and not quiet:
        print(res.stderr)
    return out


if __name__ == "__main__":
    print(build())
