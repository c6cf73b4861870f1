"""Build the C-ABI library ``libsph.so`` for gfx950 with hipcc (in-tree).

Flags: -O3, gfx950 only, packed FP32 instructions disabled
(``-target-feature -packed-fp32-ops``); the float arithmetic is plain
per-lane FP32.  ``-ffp-contract=on`` fuses a multiply and an add only
within one source expression, so a formula rounds the same way in every
kernel and code path that inlines it (the cell walk, the masked sweeps and
their staged forms give bit-identical sums).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", "sph_kernels.hip"), os.path.join(HERE, "csrc", "sph_adjoint.hip")]
DEPS = SRC + [os.path.join(HERE, "csrc", n) for n in ("sph_device.h", "sph_host.h")] + \
    [os.path.join(ROOT, "include", "sph.h")]
LIB = os.path.join(HERE, "libsph.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def command(out=LIB):
    return [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
            "-Wall", "-Wno-unused-function", "-Wno-unused-lambda-capture",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-o", out] + SRC


def build(verbose=False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
