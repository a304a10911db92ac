"""Build liblbe.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1109_3277_amd.build

Every source under csrc/ is compiled for gfx950 only; the shared library is
written next to this file so that it travels with the source tree. The
counter-calibration copy (csrc/probe/) becomes a separate liblbe_probe.so,
loaded only by the profiling driver.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbe.so")
PROBE_LIB = os.path.join(HERE, "liblbe_probe.so")
PROBE_SRC = os.path.join(CSRC, "probe", "lbe_probe.hip")
SOURCES = ["lbe_fluid.hip", "lbe_particles.hip", "lbe_pairs.hip", "lbe_runtime.hip", "lbe_batch.hip",
           "lbe_noalloc.hip", "lbe_analysis.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of generated code on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(HERE, "..", "include"),
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, out: str):
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(5, len(SOURCES) + 1)) as ex:
        objs = list(ex.map(_compile, SOURCES + [os.path.join("probe", "lbe_probe.hip")]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], PROBE_LIB)
    if verbose:
        print("built", LIB, "and", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
