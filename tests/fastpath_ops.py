"""VALU instructions per template x segment on the fast path of the stage-1 table count, counted
in its gfx950 assembly.

The count kernel is compiled to assembly with the library's own flags; in the kernel of the
given mode and chunk size (by default mode 10, the table variant for a launch whose tracks the
host has proven to stay inside the staged rows, which the benchmark's launches are; mode 2 is
the same kernel with the per-track range checks) the loop over segment groups is walked along
the path that every group takes
when no lane of the wave meets an f0-shift step and no partial-sum flush is due.  Exec-mask
regions (s_cbranch_execz) are entered, except the innermost ones that hold the step's position
guess (v_rcp_f32) and the ones that store to global memory (the flush).  Each VALU instruction
on that path is one 64-lane wave instruction; a pair of lanes shares one binary template, so a
lane covers a group's 8 segments x 45 f0 bins (the pair, 90), and the count divided by 8 x 45
is the lane-operation cost of one template x segment that bench.py reports as the issued work.

    python tests/fastpath_ops.py [chunk ...]      (BSH_FASTPATH_MODE=2 for the checked kernel)
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(os.path.dirname(HERE), "paper_1904_04873_amd"))
import build  # noqa: E402

N_F0 = 90
BINS_PER_LANE = N_F0 // 2      # two lanes share a binary template's 90 f0 bins
SEGMENTS_PER_GROUP = 8


def assembly() -> str:
    src = "bsh_count_table.hip"
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "count.s")
        cmd = ([build.hipcc()] + build.FLAGS + build.SOURCE_FLAGS.get(src, []) +
               ["--cuda-device-only", "-S", "-o", out, os.path.join(build.CSRC, src)])
        subprocess.run(cmd, check=True, capture_output=True)
        with open(out) as f:
            return f.read()


PROVEN_MODE = 10


def kernel_lines(asm: str, chunk: int, mode: int = PROVEN_MODE) -> list[str]:
    sym = f"_ZN3bsh18hough_count_kernelILi{mode}ELi{chunk}EEEvNS_11PlainLaunchE:"
    lines = asm.splitlines()
    start = next(i for i, l in enumerate(lines) if l.startswith(sym))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    return lines[start:end]


def _labels(lines: list[str]) -> dict[str, int]:
    out = {}
    for i, l in enumerate(lines):
        m = re.match(r"^(\.LBB\d+_\d+):", l)
        if m:
            out[m.group(1)] = i
    return out


def _region(lines: list[str], labels: dict[str, int], a: int, b: int) -> set[int]:
    """Lines executed from the fall-through of the exec-mask branch at line a until control
    reaches its target (line b): fall-through and unconditional jumps are followed (the compiler
    may place a region's tail, and its target, before the branch)."""
    seen: set[int] = set()
    i = a + 1
    for _ in range(20000):
        if i >= len(lines) or i == b or i in seen:
            break
        seen.add(i)
        t = lines[i].split()
        if t and t[0] == "s_branch":
            i = labels[t[1]]
            continue
        i += 1
    return seen


def _rare_regions(lines: list[str], labels: dict[str, int]) -> set[int]:
    """Lines of the exec-mask branches whose regions the fast path skips."""
    regions = {}
    for i, l in enumerate(lines):
        t = l.split()
        if t and t[0] == "s_cbranch_execz":
            regions[i] = _region(lines, labels, i, labels[t[1]])
    has = lambda r, what: any(what in lines[k] for k in r)
    with_rcp = {a: r for a, r in regions.items() if has(r, "v_rcp_f32")}
    rare = set()
    for a, r in with_rcp.items():
        if not any(a2 != a and a2 in r for a2 in with_rcp):
            rare.add(a)                       # innermost region holding the step's guess
    for a, r in regions.items():
        if has(r, "global_store"):
            rare.add(a)                       # the flush of the partial sums
    return rare


def walk(lines: list[str], head: int) -> dict[str, int]:
    labels = _labels(lines)
    rare = _rare_regions(lines, labels)
    counts: dict[str, int] = {}
    i = head + 1
    for _ in range(100000):
        # back at the header: by a branch (below) or, when the loop's latch is placed before its
        # header, by falling through into it
        if i >= len(lines) or i == head:
            break
        l = lines[i].strip()
        if not l or l.startswith(";") or l.startswith("."):
            i += 1
            continue
        ins = l.split()[0]
        counts[ins] = counts.get(ins, 0) + 1
        if ins == "s_cbranch_execz":
            i = labels[l.split()[1]] if i in rare else i + 1
            continue
        if ins == "s_branch" or (ins.startswith("s_cbranch") and ins != "s_cbranch_execnz"):
            tgt = labels[l.split()[1]]
            if tgt == head:
                break
            if ins == "s_branch":
                i = tgt
                continue
        i += 1
    return counts


def fast_path(chunk: int, asm: str | None = None, mode: int = PROVEN_MODE) -> tuple[int, int]:
    """(VALU instructions per group on the fast path, segments per group)."""
    lines = kernel_lines(asm or assembly(), chunk, mode)
    best = None
    for i, l in enumerate(lines):
        if re.match(r"^\.LBB\d+_\d+:", l) and i + 1 < len(lines) and "This Loop Header: Depth=2" in lines[i + 1]:
            c = walk(lines, i)
            adds = c.get("v_add_f32_e32", 0) + c.get("v_add_f32_e64", 0)
            valu = sum(n for k, n in c.items() if k.startswith("v_"))
            if best is None or adds > best[0]:
                best = (adds, valu)
    if best is None:
        raise RuntimeError("segment-group loop not found")
    return best[1], SEGMENTS_PER_GROUP


if __name__ == "__main__":
    chunks = [int(c) for c in sys.argv[1:]] or [128, 256, 512]
    mode = int(os.environ.get("BSH_FASTPATH_MODE", PROVEN_MODE))
    asm = assembly()
    for c in chunks:
        valu, seg = fast_path(c, asm, mode)
        print(f"chunk {c}: {valu} VALU per group of {seg} segments x {BINS_PER_LANE} bins = "
              f"{valu / (seg * BINS_PER_LANE):.3f} per template x segment")
