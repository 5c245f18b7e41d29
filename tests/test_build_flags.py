"""Build checks of the library's device code as build.py compiles it: no
packed FP32 VALU instructions (the build turns that target feature off, and
the flag does what it says: the same probe kernel compiled without it does
get them), and no kernel spills vector registers to scratch memory."""
import os
import re
import subprocess

import pytest

from paper_1803_08833_amd import build as B

PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(float2* a, const float2* b) {
    int i = threadIdx.x;
    float2 x = a[i], y = b[i];
    x.x = x.x * y.x + 1.0f;
    x.y = x.y * y.y + 1.0f;
    a[i] = x;
}
"""


def _device_asm(src, out, flags):
    cmd = [B.HIPCC, "--cuda-device-only", "-S", *flags, "-o", out, src]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


@pytest.fixture(scope="module")
def hipcc():
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not installed")
    return B.HIPCC


def test_flag_removes_packed_fp32(hipcc, tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    base = [f"--offload-arch={B.ARCH}", "-O3"]
    with_flag = _device_asm(str(src), str(tmp_path / "a.s"), B.DEVICE + ["-O3"])
    without = _device_asm(str(src), str(tmp_path / "b.s"), base)
    assert PACKED.search(without), "probe no longer exercises packed FP32; pick another probe"
    assert not PACKED.search(with_flag)


@pytest.mark.parametrize("src", [s for s in B.SOURCES if s.endswith(".hip")])
def test_library_device_code_has_no_packed_fp32(hipcc, tmp_path, src):
    asm = _device_asm(os.path.join(B.CSRC, src), str(tmp_path / (src + ".s")), B.DEVICE + B.COMMON)
    found = sorted(set(m.group(0) for m in PACKED.finditer(asm)))
    assert not found, f"{src}: {found}"


@pytest.mark.parametrize("src", [s for s in B.SOURCES if s.endswith(".hip")])
def test_no_vgpr_spills(hipcc, tmp_path, src):
    """Every kernel keeps its vector registers within the hardware budget of
    its launch shape: no VGPR spills to scratch memory (as build.py compiles)."""
    cmd = [B.HIPCC, "--cuda-device-only", "-c", *B.DEVICE, *B.COMMON, "-Rpass-analysis=kernel-resource-usage",
           os.path.join(B.CSRC, src), "-o", str(tmp_path / "k.o")]
    out = subprocess.run(cmd, check=True, capture_output=True, text=True).stderr
    found = {}
    for block in out.split("Function Name: ")[1:]:
        name = block.split()[0]
        m = re.search(r"VGPRs Spill: (\d+)", block)
        assert m, f"{src}: no spill figure for {name}"
        found[name] = int(m.group(1))
    assert found, f"{src}: no kernel resource report"
    spilled = {k: v for k, v in found.items() if v}
    assert not spilled, f"{src}: VGPR spills {spilled}"
