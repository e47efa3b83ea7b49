"""Build libosbli.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2007_14933_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libosbli.so")
SOURCES = ["abi.hip", "convective.hip", "convective_teno6.hip", "convective_wenojs5.hip", "convective_wenoz3.hip", "convective_wenoz7.hip",
           "viscous.hip", "central.hip", "bc.hip", "metrics.hip", "sensor.hip", "batch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no packed-FP32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-Wall", "-Wno-unused-function",
]


# translation units compiled without FMA contraction: the sensor's features
# and training arithmetic follow their FP64 definitions operation by operation
NO_CONTRACT = {"sensor.hip"}

# translation units built without loop strength reduction: in the z-marching
# viscous kernel it turns every address stream of the march into a 64-bit
# induction variable of its own, which spills the registers the loads issued
# ahead need
NO_LSR = {"viscous.hip"}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    extra = ["-ffp-contract=off"] if src in NO_CONTRACT else []
    if src in NO_LSR:
        extra += ["-mllvm", "-disable-lsr"]
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libosbli.so (always recompiles)."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
