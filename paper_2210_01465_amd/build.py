"""Compile the HIP engine into ``libfl.so`` for gfx950 (MI355X).

Run ``python -m paper_2210_01465_amd.build``.  hipcc cross-compiles, so no GPU
is needed to build.  Packed-FP32 instructions are disabled for every device
pass (``-packed-fp32-ops``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfl.so")
SOURCES = ["fl_kernels.hip", "fl_engine.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(out: str = LIB, extra: tuple = (), verbose: bool = False) -> str:
    """Always recompiles; writes the library atomically."""
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", INCLUDE, "-I", CSRC, *extra, "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def kernel_resources(source: str = "fl_kernels.hip") -> dict:
    """Per-kernel register and scratch use of one source, from the compiler's
    resource report (device pass only; nothing is linked).
    Returns {mangled name: {"vgprs": int, "sgprs": int, "scratch": int, "occupancy": int}}."""
    import re
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "--cuda-device-only", "-c",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Rpass-analysis=kernel-resource-usage", "-I", INCLUDE, "-I", CSRC,
               "-o", os.path.join(tmp, "k.o"), os.path.join(CSRC, source)]
        text = subprocess.run(cmd, check=True, capture_output=True, text=True).stderr
    out, cur = {}, None
    keys = {"VGPRs": "vgprs", "TotalSGPRs": "sgprs", "ScratchSize [bytes/lane]": "scratch",
            "Occupancy [waves/SIMD]": "occupancy"}
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z \[\]/]+): (\d+)", line)
        if m and cur is not None and m.group(1).strip() in keys:
            cur[keys[m.group(1).strip()]] = int(m.group(2))
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
