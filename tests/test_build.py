"""Compile-time properties of the relaxation and boundary-scan kernels (no
GPU needed): the relaxation's in-flight loads and atomics must stay in
registers (no scratch spills) at four or more waves per SIMD, and the scan
(bound by the latency of its dependent loads) keeps seven waves per SIMD
with four independent steps in flight."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_14503_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_round_kernel_occupancy(tmp_path):
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, "kernels.hip"),
           "-o", str(tmp_path / "k.o"), "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    blocks = re.split(r"remark: Function Name: ", out)
    info = {}
    for b in blocks[1:]:
        name = b.split()[0]
        fields = dict(re.findall(r"remark:\s+([A-Za-z \[\]/]+?):\s+(\d+)", b))
        info[name] = fields
    rounds = [v for k, v in info.items() if "k_round" in k]
    assert len(rounds) == 2, list(info)  # the general instance and the one for rows of at most 4 entries
    for rnd in rounds:
        assert int(rnd["Occupancy [waves/SIMD]"]) >= 4, rnd
        assert int(rnd["ScratchSize [bytes/lane]"]) == 0, rnd
    # the boundary scan's instances without event counters (forward and reversed edge direction)
    scans = [v for k, v in info.items() if k.startswith("_ZN3stn6k_scan") and k.endswith("ELb0EEEvNS_10ScanParamsE")]
    assert len(scans) == 2, list(info)
    for scan in scans:
        assert int(scan["Occupancy [waves/SIMD]"]) >= 7, scan
        assert int(scan["ScratchSize [bytes/lane]"]) == 0, scan
