"""Builds the HIP library libvls.so in-tree for gfx950.

    python paper_2105_13168_amd/build.py

(run it as a script: importing the package loads the library it builds)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvls.so")
SOURCES = [os.path.join(CSRC, "vls_api.cpp"), os.path.join(CSRC, "vls_kernels.hip"),
           os.path.join(CSRC, "vls_passes.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the field must be evaluated exactly as written: no FMA contraction
    "-ffp-contract=off", "-fno-fast-math",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in device code: the
    # feature is known to the gfx950 device pass, which then emits none (a
    # float2 multiply-add that compiles to v_pk_fma_f32 without the flag
    # compiles to scalar v_fma_f32 with it; tests/test_build_flags.py checks
    # this); the host pass, which has no such feature, warns and ignores it
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libvls.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
