"""The build's no-packed-FP32 flag takes effect in the gfx950 device code.

The library is compiled with ``-Xclang -target-feature -Xclang
-packed-fp32-ops``.  The host pass warns that x86 does not know the feature;
this test shows that the device pass honours it: a float2 multiply-add probe
compiled for gfx950 contains packed f32 instructions without the flag and
none with it.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1411_4942_amd import build as libbuild

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(float2 *a, float2 b, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        float2 x = a[i];
        x.x = x.x * b.x + b.y;
        x.y = x.y * b.x + b.y;
        a[i] = x;
    }
}
"""

PACKED_F32 = re.compile(r"\bv_pk_(add|mul|fma|mov)_f32\b")


def _device_asm(tmp_path, flags):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    out = tmp_path / ("probe%d.s" % len(flags))
    subprocess.run([libbuild.hipcc(), f"--offload-arch={libbuild.ARCH}", "-O3", "--cuda-device-only", "-S",
                    "-o", str(out), str(src), *flags], check=True, capture_output=True)
    return out.read_text()


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not installed")
def test_device_pass_honours_no_packed_fp32(tmp_path):
    plain = _device_asm(tmp_path, [])
    flagged = _device_asm(tmp_path, libbuild.FLAGS_NO_PACKED_F32)
    assert PACKED_F32.search(plain), "probe should use packed f32 without the flag (else the test shows nothing)"
    assert not PACKED_F32.search(flagged)
    assert "v_fma_f32" in flagged or "v_fmac_f32" in flagged
