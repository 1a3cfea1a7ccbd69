"""Compile-time properties the HIP path relies on (hipcc cross-compiles for gfx950 without a GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_10128_amd", "csrc")

KERNEL = r'''
#include "ges_internal.h"
__global__ void k(float* p, const float* g, float* m, float* v, float b1, float b2, float eps, float ss, float ib) {
  const int i = threadIdx.x;
  float pp = p[i], mm = m[i], vv = v[i];
  ges::adam_update(pp, g[i], mm, vv, b1, b2, eps, ss, ib);
  p[i] = pp; m[i] = mm; v[i] = vv;
}
'''


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_adam_update_code_does_not_depend_on_contraction(tmp_path):
    """The Adam update is compiled into a file built without contraction (the stand-alone step) and into one
    built with it (the preprocess backward, where it is fused).  Both must emit the same instructions, or the
    fused and stand-alone steps would round differently."""
    src = tmp_path / "t.hip"
    src.write_text(KERNEL)
    asm = {}
    for mode in ("off", "fast"):
        out = tmp_path / f"t_{mode}.s"
        cmd = ["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", f"-I{CSRC}", "--cuda-device-only", "-S",
               "-fno-gpu-flush-denormals-to-zero", "-fhip-fp32-correctly-rounded-divide-sqrt",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-ffp-contract={mode}",
               str(src), "-o", str(out)]
        subprocess.run(cmd, check=True, capture_output=True, cwd=tmp_path)
        asm[mode] = [l.strip() for l in out.read_text().splitlines() if l.strip().startswith("v_")]
    assert asm["off"] and asm["off"] == asm["fast"]
