"""Build the native library librsl.so (HIP kernels for gfx950 + C-ABI host code).

Usage: python paper_1010_1386_amd/build.py   (or build() from __graft_entry__)

Every source is compiled with hipcc for --offload-arch=gfx950 into _build/
and linked into paper_1010_1386_amd/librsl.so (in-tree, so that a snapshot of
the repository carries it to the GPU machine).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librsl.so")
PEAK_LIB = os.path.join(PKG, "libpeak.so")

SOURCES = ["kernels.hip", "api.cpp", "plan.cpp", "job.cpp", "tune.cpp", "server.cpp", "persistent.hip", "gcd.cpp",
           "noalloc.cpp"]
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed fp32 forms are never wanted in this integer code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core accumulators in ordinary VGPRs: no AGPR copies before the
         # VALU reads them, and a smaller register footprint per wave
         "-mllvm", "-amdgpu-mfma-vgpr-form=1",
         "-fno-strict-aliasing", "-Wall", "-Wno-unused-result"]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return exe


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc()] + FLAGS + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
    return obj, msg


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    for obj, msg in results:
        if verbose and msg.strip():
            print(msg, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    # issue-rate microbenchmarks of the units the kernels use (measurement only)
    pk_obj, _ = _compile("peak.hip")
    r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", PEAK_LIB + ".tmp", pk_obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("peak library link failed:\n" + r.stdout + r.stderr)
    os.replace(PEAK_LIB + ".tmp", PEAK_LIB)
    # host build of the per-lane arithmetic, used only by CPU tests
    hs_src = os.path.join(ROOT, "tests", "hostsim", "hostsim.cpp")
    if os.path.exists(hs_src):
        hs_lib = os.path.join(ROOT, "tests", "hostsim", "libhostsim.so")
        r = subprocess.run([hipcc(), "-O2", "-fPIC", "-shared", "-o", hs_lib, hs_src],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hostsim build failed:\n" + r.stdout + r.stderr)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
