"""Build libbsh.so (the HIP library behind include/bsh.h) in-tree for gfx950.

Each source is compiled to its own object (in parallel), then the objects are linked into
the shared library; no device code calls across sources, so no relocatable device code is
needed."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbsh.so")
SOURCES = ["bsh_api.hip", "bsh_count.hip", "bsh_count_batch.hip", "bsh_count_table.hip", "bsh_batch.hip",
           "bsh_power.hip", "bsh_topk.hip", "bsh_post.hip"]
ARCH = os.environ.get("BSH_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # the frequency track is evaluated in one fixed FP64 operation order
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]

# Per-source additions.  The table variant of the count is scheduled for instruction-level
# parallelism (its table reads issue in longer runs ahead of their adds at the same occupancy);
# the select variants, in other sources, would spill under that scheduler.
SOURCE_FLAGS: dict[str, list[str]] = {
    "bsh_count_table.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed: {' '.join(cmd[-3:])}")


def build(verbose: bool = False, extra: list | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    jobs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(OBJ, src.replace(".hip", ".o"))
        objs.append(obj)
        jobs.append([cc] + FLAGS + SOURCE_FLAGS.get(src, []) + (extra or []) +
                    ["-c", "-o", obj, os.path.join(CSRC, src)])
    with ThreadPoolExecutor(max_workers=min(len(jobs), 8)) as pool:
        list(pool.map(lambda c: _run(c, verbose), jobs))
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
