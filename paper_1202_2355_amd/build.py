"""Build the gfx950 HIP library ``libm2m.so`` in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libm2m.so")
SOURCES = [os.path.join(CSRC, f) for f in ("m2m_kernels.hip", "m2m_step_f32d.hip", "m2m_step_f32f.hip",
                                            "m2m_step_f64.hip", "m2m_api.cpp", "m2m_smooth.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # single-precision division and sqrt at hardware accuracy (about 1 ulp)
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-Wall",
]


def build(verbose: bool = False) -> str:
    """Compile the library (always; a previous build is replaced). The units
    compile in parallel, then link into one shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory() as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            cmd = [hipcc, *compile_flags, "-I", INCLUDE, "-I", CSRC, "-c", "-o", obj, src]
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.PIPE, text=True)))
            objs.append(obj)
        logs = []
        for src, p in procs:
            out, err = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + out + err)
            logs.append(err)
        tmp = LIB + ".tmp"
        res = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                             capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    if verbose:
        print("".join(logs) + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
