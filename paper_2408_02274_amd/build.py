"""Build libifgf.so in-tree for gfx950 (host C++ with g++, kernels with hipcc)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libifgf.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = os.environ.get("IFGF_OFFLOAD_ARCH", "gfx950")

CXXFLAGS = ["-O2", "-fPIC", "-std=c++17", "-fopenmp", "-ffp-contract=off",
            f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__", "-Wall", "-Wno-unused-function"]
HIPFLAGS = ["-O3", "-fPIC", "-std=c++20", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result", "-munsafe-fp-atomics"]


def _sources():
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    return cpp, hip


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objdir = os.path.join(OUT_DIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    cpp, hip = _sources()
    jobs = []
    for f in cpp:
        jobs.append(["g++", *CXXFLAGS, "-c", os.path.join(CSRC, f), "-o",
                     os.path.join(objdir, f + ".o")])
    for f in hip:
        jobs.append([HIPCC, *HIPFLAGS, "-c", os.path.join(CSRC, f), "-o",
                     os.path.join(objdir, f + ".o")])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    objs = [os.path.join(objdir, f + ".o") for f in cpp + hip]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-lgomp", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
