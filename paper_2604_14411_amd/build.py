"""Build libhgp.so (hipcc, gfx950), the LDS-atomic micro-benchmark
libhgp_probe.so and the synthetic-input generator in-tree."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhgp.so")
PROBE_LIB = os.path.join(HERE, "libhgp_probe.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["prims.hip", "coarsen.hip", "refine.hip", "seg.hip", "tail.hip", "events.hip", "learned.hip", "training.hip", "checkpoint.hip", "driver.hip"]

HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions stay disabled in every device code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build_lib() -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def build_probe() -> str:
    """The micro-benchmark of LDS atomic adds (bench.py --lds-probe)."""
    os.makedirs(OBJDIR, exist_ok=True)
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, "-shared", os.path.join(CSRC, "probe.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on probe.hip:\n{r.stderr}")
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def build_all() -> None:
    from paper_2604_14411_amd import synth

    synth.build(force=True)
    build_lib()
    build_probe()


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    build_all()
    print(LIB)
