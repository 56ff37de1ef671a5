"""Resource use of the hot kernels as the HIP compiler reports it for gfx950
(CPU only: the compiler's kernel-resource-usage remarks).

The fused re-walk keeps its per-pixel state (the moment bound, its zeros, the
continuation state, the walk position) in registers: an array read with a
run-time index, or a structure whose address is taken, would put that state
in scratch memory, which every evaluated piece would then read and write
through the vector memory path."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2501_12581_amd", "csrc", "apc_kernels.hip")


@pytest.fixture(scope="module")
def usage(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("res") / "k.o")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c", SRC, "-o", out,
           "-Rpass-analysis=kernel-resource-usage"]
    text = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    kernels, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1).strip()] = int(m.group(2))
    return kernels


def _find(usage, pattern):
    hits = [v for k, v in usage.items() if re.search(pattern, k)]
    assert len(hits) == 1, (pattern, [k for k in usage if "k_" in k])
    return hits[0]


@pytest.mark.parametrize("pattern", [r"k_momentsILi9ELb0ELb0E", r"k_momentsILi7ELb0ELb0E", r"k_momentsILi5ELb0ELb0E"])
def test_stage_one_uses_no_scratch(usage, pattern):
    u = _find(usage, pattern)
    assert u["ScratchSize"] == 0 and u["VGPRs Spill"] == 0, u


@pytest.mark.parametrize("pattern", [r"k_resolveILi4EdLb0ELb0E", r"k_resolveILi3EdLb0ELb0E", r"k_resolveILi2EfLb0ELb0E",
                                     r"k_resolveILi4EdLb0ELb1E", r"k_resolveILi3EdLb0ELb1E", r"k_resolveILi2EfLb0ELb1E"])
def test_fused_rewalk_fits_three_workgroups_per_simd(usage, pattern):
    """The walker/evaluator pair (one workgroup per tile, or per (tile, subdomain) pair) is compiled for three
    workgroups of two wavefronts per SIMD (168 VGPRs): a few registers of the walk may spill there, not the
    per-lane state (which took 848 bytes per lane)."""
    u = _find(usage, pattern)
    assert u["Occupancy"] >= 3 and u["ScratchSize"] <= 64 and u["VGPRs Spill"] <= 16, u
    assert u["LDS Size"] * 6 <= 160 * 1024 - 6 * 256 * 16, u  # six workgroups per CU with a 256-entry table
