"""Consistency of the committed measurement records with the sources (CPU).

The bench reads the HBM traffic of its dominant kernel from a profile entry
keyed by the kernel source's hash; these tests fail when the kernels change
without the counters being taken again, and check that every profile names
the command that produced it."""

import glob
import hashlib
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNELS = os.path.join(ROOT, "paper_2011_02621_amd", "csrc", "kernels_contract.hip")


def _kernel_sha():
    return hashlib.sha256(open(KERNELS, "rb").read()).hexdigest()[:16]


def _entries():
    text = open(os.path.join(ROOT, "profiles", "gemm3m_diag53_d12_traffic.md")).read()
    out = []
    for ln in text.splitlines():
        if ln.startswith("traffic_entry:"):
            out.append(dict(kv.split("=", 1) for kv in ln.split(":", 1)[1].split()))
    return out


def test_traffic_entries_match_the_kernel_source():
    sha = _kernel_sha()
    have = {(e["kernel_sha"], e["workload"]) for e in _entries()}
    assert (sha, "diag53_d12") in have, "counters not retaken for kernel source %s" % sha
    assert (sha, "grid5x5_d10") in have, "counters not retaken for kernel source %s" % sha
    for e in _entries():
        # counted bytes at or above the algorithmic bytes (nothing is read less than once)
        assert float(e["bytes_per_launch"]) >= float(e["alg_mib_per_launch"]) * 2 ** 20


def test_headline_profiles_name_the_current_kernel_source():
    sha = _kernel_sha()
    for name in ("gemm3m_diag53_d12.md", "gemm3m_diag53_d12_traffic.md", "gemm3m_diag53_d12_mfma.md",
                 "gemm_f32_grid5x5_d10.md", "gemm_f32_grid5x5_d10_traffic.md"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "sha256 prefix %s" % sha in text, name


def test_every_profile_gives_its_command():
    files = glob.glob(os.path.join(ROOT, "profiles", "*"))
    assert files
    for f in files:
        assert f.endswith((".md", ".txt")), f
        text = open(f).read()
        assert re.search(r"^\s+rocprofv3 .* -- python3 ", text, re.M), f
        assert len(text) < 16384, f


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
