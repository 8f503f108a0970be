"""Build librq.so (HIP for gfx950) in-tree.

Every HIP source is compiled with hipcc for gfx950 with packed-FP32
instructions disabled; plain C++ sources with the host compiler.  Objects go
to ``paper_2506_23775_amd/_build/``; the shared library to
``paper_2506_23775_amd/librq.so``.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librq.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp_hip = ["rq_api.cpp"]           # host code calling the HIP runtime
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp") and f not in cpp_hip)
    return hip, cpp_hip, cpp


def _compile(src: str, kind: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if kind == "hip":
        cmd = [HIPCC] + HIP_FLAGS + ["-c", path, "-o", obj]
    elif kind == "hiphost":
        cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__",
               "-c", path, "-o", obj]
    else:
        cmd = ["g++"] + CXX_FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp_hip, cpp = _sources()
    work = [(s, "hip") for s in hip] + [(s, "hiphost") for s in cpp_hip] + [(s, "cxx") for s in cpp]
    # heaviest first
    work.sort(key=lambda w: -os.path.getsize(os.path.join(CSRC, w[0])) if w[1] != "hip" else -10**9)
    jobs = jobs or min(len(work), max(1, min(16, os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda w: _compile(*w), work))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
