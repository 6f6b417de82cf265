"""Build libbdeg.so (the C-ABI library) in-tree with hipcc for gfx950.

    python -m paper_1501_02237_amd.build

Every source is compiled by hipcc; kernels are compiled for gfx950 only with
packed-FP32 instruction selection disabled."""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbdeg.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["algebra.cpp", "tiles.cpp", "runtime.cpp", "tune.cpp", "api.cpp", "serve.cpp", "kernels.hip",
           "kernels_mixed12.hip", "kernels_mixed7.hip", "kernels_cells.hip", "kernels_extend.hip", "pivot.cpp",
           "kernels_prune.hip", "noalloc.hip", "kernels_pivot_a.hip", "kernels_pivot_b.hip", "kernels_pivot_c.hip", "kernels_pivot_d.hip"] + [f"kernels_k{k}.hip" for k in range(18, 0, -1)]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _flags(src: str) -> list[str]:
    f = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]
    f += [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    if src.startswith(("kernels_pivot", "kernels_prune", "kernels_k", "kernels_mixed")):
        # the work-item claims of the enumeration, the walk and the prefix filter are atomic adds with a
        # per-lane value (one lane adds 1): a DPP scan instead of a 64-step scalar loop
        f += ["-mllvm", "-amdgpu-atomic-optimizer-strategy=DPP"]
    return f


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    t0 = time.time()
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    for s in SOURCES:
        while sum(p.poll() is None for _, p in procs) >= jobs:
            time.sleep(0.05)
        src = os.path.join(CSRC, s)
        obj = os.path.join(BUILD, s + ".o")
        cmd = [HIPCC, *_flags(s), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        objs.append(obj)
    bad = [s for s, p in procs if p.wait() != 0]
    if bad:
        raise RuntimeError(f"hipcc failed on {bad}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
