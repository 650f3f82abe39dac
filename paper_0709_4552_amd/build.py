"""Build libnbody.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libnbody.so")

HIPFLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-variable",
    "-Wno-unused-but-set-variable",
    "-munsafe-fp-atomics",
    # loop heads on 64-byte boundaries: the force kernel's j loop otherwise
    # runs up to 10% slower or faster depending on where unrelated code
    # changes happen to put it
    "-falign-loops=64",
    # no packed FP32 (v_pk_*) instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def device_asm(src: str, out: str | None = None) -> str:
    """gfx950 assembly of one source file (device code only)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = out or os.path.join(HERE, "_build", os.path.basename(src) + ".s")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    flags = [f for f in HIPFLAGS if f not in ("-shared", "-fPIC")]
    cmd = [hipcc, *flags, "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), "-o", out, src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc -S failed for {src}")
    with open(out) as f:
        return f.read()


def check_barriers(srcs) -> None:
    """Refuse a build whose kernels hold a barrier inside a divergent loop."""
    from . import isa_check
    problems = []
    for src in srcs:
        problems += isa_check.check_asm(device_asm(src))
    if problems:
        raise RuntimeError("barrier inside a divergent loop (would risk a workgroup "
                           f"deadlock): {problems}")


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    check_barriers([x for x in srcs if os.path.basename(x).startswith("kernels_")])
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPFLAGS, "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(HERE, "csrc"), "-o", tmp, *srcs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libnbody.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_0709_4552_amd import build as _b
    print(_b.build(verbose=True))
