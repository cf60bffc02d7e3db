"""Build librbstep.so (the HIP kernels and the C ABI) for gfx950 with hipcc, in-tree.

The step kernel's source is compiled as several translation units in parallel (RB_PART = 0 ..
RB_NPARTS - 1, each defining a share of the kernel instantiations), beside the other sources;
the objects go to csrc/_build/ and are linked into one shared library."""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ_DIR = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "librbstep.so")
SOURCES = ["runtime.hip", "step_kernel.hip", "aux_kernels.hip", "model_json.cpp"]
PARTED = "step_kernel.hip"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: multiply-adds are fused only inside one source expression, so every kernel
# instantiation (plain or fused launch, any chain bound) rounds a world's arithmetic the same way
# and the batched forms reproduce the plain launch bit for bit.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
         "-Wall", "-Wno-unused-result", "-Wno-unused-variable"]
LINK_FLAGS = ["-shared", "-fPIC", "--offload-arch=gfx950"]


def nparts() -> int:
    """The number of parts the step kernel's source declares (its RB_NPARTS)."""
    with open(os.path.join(CSRC, PARTED)) as f:
        m = re.search(r"^#define RB_NPARTS (\d+)", f.read(), flags=re.M)
    if not m:
        raise RuntimeError(f"{PARTED}: no RB_NPARTS")
    return int(m.group(1))


def _jobs() -> int:
    n = os.cpu_count() or 1
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(var, "")
        if v.isdigit() and int(v) > 0:
            n = min(n, int(v))
    return max(1, min(n, 16))


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    # the last parts hold the fused launchers, which inline the most steps: started first
    units = [(PARTED, [f"-DRB_PART={k}"], f"step_kernel.part{k}.o") for k in reversed(range(nparts()))]
    units += [(s, [], os.path.splitext(s)[0] + ".o") for s in SOURCES if s != PARTED]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cmds = []
    for src, defs, obj in units:
        cmds.append([HIPCC] + FLAGS + (extra or []) + defs + inc
                    + ["-c", os.path.join(CSRC, src), "-o", os.path.join(OBJ_DIR, obj)])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return cmd, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(run, cmds))
    failed = None
    for cmd, r in results:
        out = (r.stdout + r.stderr).strip()
        if out and (verbose or r.returncode != 0):
            print(out, flush=True)
        if r.returncode != 0 and failed is None:
            failed = (cmd, r.returncode)
    if failed:
        raise subprocess.CalledProcessError(failed[1], failed[0])
    link = [HIPCC] + LINK_FLAGS + [os.path.join(OBJ_DIR, obj) for _, _, obj in units] + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
