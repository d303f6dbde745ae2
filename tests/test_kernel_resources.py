"""Register budget of the operator-apply kernels on the headline discretisation (3D Q2, dG(1), the
M = 4, p_xi = 3 index set), checked at compile time with hipcc for gfx950 (no GPU needed).

The coupled apply and the mean-block apply hold the (k+1)^d point values and integrand of a
(cell, component) pair in registers; scratch spills there cost HBM traffic (they were a third of the
apply's traffic once) and occupancy decides how well the exchange barriers are hidden.  This pins
what the kernels are built for: no spills, 2 waves per SIMD for the coupled FP64 kernel, 3 for the
FP64 mean block.
"""
import os
import re
import shutil
import subprocess

import pytest

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_21046_amd", "csrc")

TU = r"""
#include "apply_impl.hpp"
namespace sg {
void instantiate(ApplyArgs<double> a, Tables<double> tb, hipStream_t s) {
    hipLaunchKernelGGL((k_apply<3, 2, 2, double, false, 4, 3, false>), dim3(1), dim3(210), 0, s, a, tb);
    hipLaunchKernelGGL((k_apply<3, 2, 2, double, true, 0, 0, false>), dim3(1), dim3(210), 0, s, a, tb);
}
}
"""


def _usage(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    src = tmp_path / "apply_resources.hip"
    src.write_text(TU)
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-I", CSRC, "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "--cuda-device-only", "-c", str(src), "-o", str(tmp_path / "apply_resources.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    out = {}
    for block in r.stderr.split("Function Name: ")[1:]:
        name = block.split()[0]
        m = re.search(r"k_applyILi3ELi2ELi2EdLb([01])ELi(\d)ELi(\d)E", name)
        if not m:
            continue

        def field(key):
            return int(re.search(re.escape(key) + r": (\d+)", block).group(1))

        kind = "mean" if m.group(1) == "1" else "coupled"
        out[kind] = {"vgpr": field("VGPRs"), "spill": field("VGPRs Spill"), "scratch": field("ScratchSize [bytes/lane]"),
                     "occupancy": field("Occupancy [waves/SIMD]")}
    assert set(out) == {"mean", "coupled"}, out
    return out


def test_apply_kernels_do_not_spill(tmp_path):
    u = _usage(tmp_path)
    for kind, v in u.items():
        assert v["spill"] == 0 and v["scratch"] == 0, (kind, v)
    assert u["coupled"]["occupancy"] >= 2, u
    assert u["mean"]["occupancy"] >= 3, u
