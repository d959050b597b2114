"""The library's device code is built without packed FP32 instructions: the
build flag that disables them is honoured by the gfx950 device pass.  A
float2 multiply-add that the compiler turns into v_pk_fma_f32 by default
must come out as scalar FP32 instructions under the library's flags."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void k(float2 *a, const float2 *b, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { float2 x = a[i], y = b[i]; x.x = x.x * y.x + y.y; x.y = x.y * y.y + y.x; a[i] = x; }
}
"""


def _device_asm(extra):
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.hip")
        out = os.path.join(d, "probe.s")
        with open(src, "w") as f:
            f.write(PROBE)
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-S", "--cuda-device-only", src, "-o", out] + extra,
                       check=True, capture_output=True)
        return open(out).read()


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_packed_fp32_disabled_by_the_library_flags():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_b", os.path.join(ROOT, "paper_2105_13168_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    i = b.FLAGS.index("-packed-fp32-ops")
    flag = b.FLAGS[i - 3:i + 1]
    assert flag == ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    assert "v_pk_fma_f32" in _device_asm([])          # the probe does produce them by default
    asm = _device_asm(flag)
    for op in ("v_pk_fma_f32", "v_pk_mul_f32", "v_pk_add_f32"):
        assert op not in asm
