"""The HIP build keeps packed FP32 instructions out of device code.

The library's hipcc flags include -target-feature -packed-fp32-ops; hipcc
warns that its host pass does not know the feature, so this checks on the
CPU that the device pass honours it: a kernel of float2 multiply-adds
compiles to v_pk_fma_f32 without the flag and to no packed FP32
instruction with the library's flags.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1504_04804_amd import build

KERNEL = r"""
#include <hip/hip_runtime.h>
__global__ void k(float2* a, const float2* b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float2 x = a[i], y = b[i];
    x.x = x.x * y.x + 1.0f;
    x.y = x.y * y.y + 1.0f;
    a[i] = x;
  }
}
"""

PACKED = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")


def device_asm(tmp_path, flags):
    src = tmp_path / "k.hip"
    src.write_text(KERNEL)
    out = tmp_path / "k.s"
    cmd = [build.hipcc(), "--cuda-device-only", "-S", "-o", str(out), str(src)] + flags
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not installed")
def test_packed_fp32_kept_out_of_device_code(tmp_path):
    lib_flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    assert "-packed-fp32-ops" in lib_flags
    plain = [f for f in lib_flags if f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    assert PACKED.search(device_asm(tmp_path, plain)), "the probe no longer produces packed FP32"
    assert not PACKED.search(device_asm(tmp_path, lib_flags))
