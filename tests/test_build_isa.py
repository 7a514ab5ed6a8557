"""The built library's gfx950 code holds no packed FP32 instruction.

The library is compiled with the packed-FP32 target feature switched off
(some forms of those instructions have produced wrong results on the target
machines without any error); the host pass of hipcc warns that it does not
know the feature, so this test checks the device code itself: it unbundles
the gfx950 code object from libpimc.so, disassembles it with the ROCm LLVM
tools and looks for any v_pk_*_f32 instruction.  It also confirms that the
check can see such instructions at all, on a small kernel compiled here with
the feature left on.
"""

import os
import re
import shutil
import subprocess

import pytest

from paper_1103_4887_amd import _lib as L
from paper_1103_4887_amd import build as B

LLVM = "/opt/rocm/llvm/bin"
PK32 = re.compile(r"\bv_pk_(?:fma|mul|add|mov)_f32\b")


def _tools():
    need = [os.path.join(LLVM, t) for t in ("clang-offload-bundler", "llvm-objdump")]
    if not all(os.path.exists(t) for t in need) or shutil.which("objcopy") is None:
        pytest.skip("ROCm LLVM tools or objcopy not available")


def _device_asm(so_path, tmp_path):
    fat = tmp_path / "fatbin.bin"
    co = tmp_path / "dev.co"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", so_path, str(fat)], check=True)
    subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fat}", f"--output={co}"], check=True)
    r = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", str(co)], check=True, capture_output=True,
                       text=True)
    return r.stdout


def test_library_has_no_packed_fp32(tmp_path):
    _tools()
    assert os.path.exists(L.LIB_PATH), "run __graft_entry__.build() first"
    asm = _device_asm(L.LIB_PATH, tmp_path)
    assert "v_add_f32" in asm or "v_fma_f32" in asm   # the disassembly is the library's code
    hits = sorted(set(PK32.findall(asm)))
    assert not hits, f"packed FP32 instructions in libpimc.so: {hits}"


def test_check_sees_packed_fp32_when_allowed(tmp_path):
    """Without the switch, hipcc -O3 packs this loop; the same check finds it."""
    _tools()
    src = tmp_path / "pk.hip"
    src.write_text(
        "#include <hip/hip_runtime.h>\n"
        "extern \"C\" __global__ void k(float2* a, const float2* b, float s) {\n"
        "  const int i = blockIdx.x * blockDim.x + threadIdx.x;\n"
        "  float2 x = a[i], y = b[i];\n"
        "  x.x = x.x * s + y.x; x.y = x.y * s + y.y;\n"
        "  a[i] = x;\n"
        "}\n")
    so = tmp_path / "pk.so"
    flags = [f for f in B.FLAGS if f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    subprocess.run([B.hipcc(), *flags, str(src), "-o", str(so)], check=True, capture_output=True)
    assert PK32.search(_device_asm(str(so), tmp_path))
