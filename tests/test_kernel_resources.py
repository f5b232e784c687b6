"""Resource use of the HIP kernels, from the compiler's own report (hipcc
cross-compiles for gfx950 without a GPU): no kernel may spill to scratch,
which would cost every launch its scratch set-up."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1202_2355_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
UNITS = ("m2m_kernels.hip", "m2m_step_f32d.hip", "m2m_step_f32f.hip", "m2m_step_f64.hip")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_no_kernel_uses_scratch(tmp_path):
    from paper_1202_2355_amd.build import HIPCC_FLAGS
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC", "-Wall")]
    procs = []
    for u in UNITS:
        cmd = [HIPCC, *flags, "--offload-device-only", "-Rpass-analysis=kernel-resource-usage",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", "-o",
               str(tmp_path / (u + ".o")), os.path.join(CSRC, u)]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                      text=True))
    spills = []
    n = 0
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err[-2000:]
        name = None
        for line in err.splitlines():
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
                n += 1
                continue
            m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
            if m and int(m.group(1)) > 0:
                spills.append((name, int(m.group(1))))
    assert n > 100, "no resource report parsed"
    assert not spills, spills[:10]
