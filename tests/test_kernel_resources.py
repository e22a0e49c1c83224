"""Register and scratch budget of the GEMM kernels, read from the gfx950
assembly of this repository's own kernel source (CPU: hipcc cross-compiles).

The three-product GEMM relies on three waves per SIMD (at most 168 VGPRs a
wave) to hide its barrier and LDS waits, and no GEMM may spill to scratch;
a compiler or source change that breaks either fails here before it costs
time on the device."""

import os
import re
import subprocess

import pytest

from paper_2011_02621_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2011_02621_amd", "csrc", "kernels_contract.hip")


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("asm") / "kernels_contract.s")
    subprocess.run([B.HIPCC] + B.HIP_FLAGS + ["--cuda-device-only", "-S", "-o", out, SRC],
                   check=True, capture_output=True, timeout=900)
    res, name = {}, None
    for ln in open(out):
        m = re.match(r"^(_Z\S+):\s*; @", ln)
        if m:
            name = m.group(1)
            res[name] = {}
            continue
        m = re.match(r"^; (NumVgprs|ScratchSize|Occupancy): (\d+)", ln)
        if m and name:
            res[name][m.group(1)] = int(m.group(2))
    return res


def _select(kernels, pattern):
    sel = {k: v for k, v in kernels.items() if re.search(pattern, k)}
    assert sel, pattern
    return sel


def test_three_product_gemm_runs_three_waves_per_simd(kernels):
    for name, r in _select(kernels, r"k_gemm_3mIL").items():
        assert r["ScratchSize"] == 0, name
        assert r["NumVgprs"] <= 168, name
        assert r["Occupancy"] >= 3, name


def test_no_gemm_spills(kernels):
    for name, r in _select(kernels, r"k_gemm_|k_splitk_|k_small").items():
        assert r["ScratchSize"] == 0, name
