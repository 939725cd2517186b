"""Every HIP kernel of the library compiles for gfx950 without scratch
memory: no register spills and no private arrays (a spill in a filter GEMM
costs it 40-70% of its speed), and the GEMM kernels keep the occupancy
their tiles are designed for (two waves per SIMD for the 512-thread
workgroups with 64 x 64 or 32 x 32 wave tiles)."""
import concurrent.futures
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_02491_amd", "csrc")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
SOURCES = ["gemm.hip", "gemm_bf16.hip", "kernels.hip", "eigh.hip", "crt.hip", "chol.hip",
           "solver.hip"]


def _resources(src):
    """{kernel: {field: value}} from the compiler's resource-usage remarks."""
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
                        "-c", os.path.join(CSRC, src), "-o", os.devnull,
                        "-Rpass-analysis=kernel-resource-usage"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([^:]+): (\d+)\s", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = int(m.group(2))
    return out


@pytest.fixture(scope="module")
def resources():
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        return dict(zip(SOURCES, ex.map(_resources, SOURCES)))


def test_no_kernel_uses_scratch(resources):
    kernels = {k: v for per in resources.values() for k, v in per.items()}
    assert len(kernels) > 40
    bad = {k: v for k, v in kernels.items()
           if v.get("ScratchSize [bytes/lane]", 1) or v.get("VGPRs Spill", 1)
           or v.get("SGPRs Spill", 1)}
    assert not bad, bad


def test_filter_gemms_run_two_waves_per_simd(resources):
    per = resources["gemm_bf16.hip"]
    per.update(resources["gemm.hip"])
    filt = {k: v for k, v in per.items()
            if "gemm_bf16x2_k32_kernel" in k or "gemm_bf16x3_kernel" in k
            or re.search(r"gemm_kernelI[df][df]Lb1ELi0ELi0ELi1E", k)}
    assert len(filt) >= 12
    for k, v in filt.items():
        assert v["Occupancy [waves/SIMD]"] >= 2, (k, v)
