"""Resources of the stage kernels as the compiler reports them (CPU only: hipcc
cross-compiles for gfx950). A persistent worker grid needs every workgroup resident
at once: each stage kernel must fit twice per CU (at most 256 registers per lane,
at most 80 KB of LDS per workgroup) and must need no scratch, since the runtime may
start fewer waves than the grid when it cannot back all of their scratch. The
library refuses such a kernel at launch; this test catches it at build time."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def usage(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("ru") / "stages.o"
    cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-x", "hip", "-c", os.path.join(ROOT, "paper_2005_02088_amd", "csrc", "stages.hip"),
           "-o", str(out), "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+) \[-Rpass", line)
        if m and cur:
            kernels[cur][m.group(1).strip()] = int(m.group(2))
    return {k: v for k, v in kernels.items() if "stage_worker" in k or "stage_bench" in k}


def test_every_stage_kernel_fits_twice_per_cu_without_scratch(usage):
    # 11 stage kinds, a worker and a one-shot kernel each (the compiler may merge
    # identical instantiations, so at least one per kind)
    assert len(usage) >= 11
    for name, u in usage.items():
        assert u["VGPRs"] + u.get("AGPRs", 0) <= 256, (name, u)
        assert u["LDS Size"] <= 80 * 1024, (name, u)
        assert u["ScratchSize"] == 0, (name, u)
        assert u.get("VGPRs Spill", 0) == 0, (name, u)
