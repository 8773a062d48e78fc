"""The device code is built without packed FP32 arithmetic.

The library's flags switch the gfx950 target feature `packed-fp32-ops` off
(`-Xclang -target-feature -Xclang -packed-fp32-ops`).  hipcc's host pass does
not know the feature and says so ("not a recognized feature ... ignoring"); the
device pass honours it.  These tests show both halves: a float2 probe compiles
to a packed FMA without the switch and to none with it, and the device assembly
of every HIP source of the library, built with the library's own flags,
contains no packed FP32 add, multiply or FMA.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1908_08292_amd import build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")
PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(const float2* a, const float2* b, float2* c, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        float2 x = a[i], y = b[i];
        c[i] = make_float2(x.x * y.x + x.x, x.y * y.y + x.y);
    }
}
"""

pytestmark = pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc missing")


def device_flags():
    return [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]


def device_asm(src, out, flags):
    subprocess.check_call([HIPCC] + flags + ["--cuda-device-only", "-S", src, "-o", out],
                          stderr=subprocess.DEVNULL)
    return open(out).read()


def test_switch_removes_packed_fp32_from_a_probe(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    base = ["--offload-arch=gfx950", "-O3", "-std=c++17"]
    with_pk = device_asm(str(src), str(tmp_path / "a.s"), base)
    without = device_asm(str(src), str(tmp_path / "b.s"), device_flags())
    assert PACKED.search(with_pk), "probe no longer exercises packed FP32; pick another"
    assert not PACKED.search(without)


def test_library_device_code_has_no_packed_fp32(tmp_path):
    flags = device_flags()
    procs = []
    for s in build.SOURCES:
        if s.endswith(".hip"):
            out = str(tmp_path / (s + ".s"))
            cmd = [HIPCC] + flags + ["--cuda-device-only", "-S", os.path.join(build.CSRC, s), "-o", out]
            procs.append((s, out, subprocess.Popen(cmd, stderr=subprocess.DEVNULL)))
    assert procs
    for s, out, p in procs:
        assert p.wait() == 0, s
        hits = PACKED.findall(open(out).read())
        assert not hits, f"{s}: {len(hits)} packed FP32 instructions"
