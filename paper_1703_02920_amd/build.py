"""Build the uvmem HIP library (libuvmem.so) for gfx950 with hipcc.

Every HIP source under csrc/ is compiled to an object and linked into one
shared library next to this file.  Packed FP32 instructions are disabled
(-packed-fp32-ops).  Run as `python -m paper_1703_02920_amd.build`.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libuvmem.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "k_dft.hip", "k_aux.hip", "k_grid.hip", "noalloc.hip"]
ARCH = os.environ.get("UVMEM_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if out:
        sys.stderr.write(out + "\n")
    return obj


# matrix-core peak microbenchmark used by bench.py (measurement only; not
# part of the library)
PEAK_SRC = os.path.join(os.path.dirname(HERE), "mfma_peak.hip")
PEAK_OUT = os.path.join(os.path.dirname(HERE), "libmfma_peak.so")


def build_peak() -> str:
    tmp = PEAK_OUT + ".tmp%d" % os.getpid()
    # matrix instructions in the VGPR form: with accumulators in AGPRs the
    # compiler copies them between registers inside the loop, and the copies
    # (not the matrix cores) set the rate of the 16-wide forms
    cmd = ["hipcc", *FLAGS, "-mllvm", "--amdgpu-mfma-vgpr-form=1", "-shared", "-o", tmp, PEAK_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for mfma_peak.hip:\n" + r.stdout + r.stderr)
    os.replace(tmp, PEAK_OUT)
    return PEAK_OUT


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    build_peak()
    if verbose:
        print("built", OUT, "and", PEAK_OUT)
    return OUT


if __name__ == "__main__":
    build()
