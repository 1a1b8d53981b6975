"""Tile-shape autotuner for the stage-1 count (binary templates per block x segments per LDS
stage).

Every shape gives bit-identical results (the per-lane summation order does not depend on it),
so the choice is purely a matter of speed.  Candidates are timed with HIP events on a sample of
the real work items through the batched plan; the winner is cached on disk keyed by the device
name and a signature of the workload (f0 bins, row words, segment-count bucket, items).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Sequence, Tuple

import torch

from . import bsh

SHAPES: Tuple[Tuple[int, int], ...] = tuple((l, c) for l in (64, 128, 256, 512) for c in (128, 256, 512))
CACHE = os.environ.get("BSH_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "bsh", "tune.json"))


def _signature(items, grids) -> str:
    ds = [it[0] for it in items]
    nseg = sorted(d.n_seg for d in ds)
    words = sorted({(d.n_bins + 31) // 32 for d in ds})
    nf0 = sorted({grids[it[1]].n_f0 for it in items})
    med = nseg[len(nseg) // 2] if nseg else 0
    return f"nf0={nf0}|words={words}|seg~{1 << max(0, med.bit_length() - 1)}|items={len(items)}"


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: Dict[str, dict]) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def time_plan(plan: "bsh.Plan", reps: int = 2, plain: bool = False) -> float:
    """Median milliseconds of plan.run() (or plan.run_plain()) over reps runs after one warmup."""
    run = plan.run_plain if plain else plan.run
    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune_plain(seg: "bsh.DeviceSegments", grid: "bsh.DeviceGrid", shapes=SHAPES, reps: int = 3,
               use_cache: bool = True, verbose: bool = False):
    """Best (lanes, chunk) for one item's plain launch (bsh_hough_count_ex); ({shape: ms})."""
    dev = torch.cuda.get_device_name(0)
    key = (dev + f"|plain|nf0={grid.n_f0}|words={(seg.n_bins + 31) // 32}|seg={seg.n_seg}"
           f"|sky={grid.n_sky}|bin={grid.n_bin}")
    db = _load() if use_cache else {}
    if use_cache and key in db:
        e = db[key]
        return (int(e["lanes"]), int(e["chunk"])), {tuple(map(int, k.split("x"))): v
                                                     for k, v in e.get("times", {}).items()}
    out = torch.empty(grid.n_templates, dtype=torch.float32, device=seg.t_mid.device)
    times = {}
    for shape in shapes:
        run = lambda: bsh.bsh_hough_count(seg, grid, wsum_out=out, lanes=shape[0], chunk=shape[1])
        run()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            run()
        b.record()
        torch.cuda.synchronize()
        times[shape] = a.elapsed_time(b) / reps
        if verbose:
            print(f"[autotune] plain lanes={shape[0]} chunk={shape[1]}: {times[shape]:.3f} ms", flush=True)
    best = min(times, key=times.get)
    if use_cache:
        db[key] = {"lanes": best[0], "chunk": best[1],
                   "times": {f"{l}x{c}": t for (l, c), t in times.items()}}
        _store(db)
    return best, times


def tune(items: Sequence, grids: Sequence["bsh.DeviceGrid"], n_bands: int, sample: int = 16,
         shapes: Sequence[Tuple[int, int]] = SHAPES, use_cache: bool = True, verbose: bool = False,
         plain: bool = False):
    """Best (lanes, chunk) for these items; returns (shape, {shape: ms}).

    Times the batched count (no top-lists) over an evenly spaced sample of the items, or with
    ``plain`` the same items as one launch each (the tile that form runs fastest with)."""
    dev = torch.cuda.get_device_name(0)
    key = dev + ("|plain-items|" if plain else "|") + _signature(items, grids)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        e = db[key]
        return (int(e["lanes"]), int(e["chunk"])), {tuple(map(int, k.split("x"))): v
                                                     for k, v in e.get("times", {}).items()}
    step = max(1, len(items) // max(1, sample))
    sub = list(items[::step])[:sample]
    # renumber bands so that the sample is still ordered and contiguous
    bands = sorted({it[4] for it in sub})
    sub = [(it[0], it[1], it[2], it[3], bands.index(it[4])) for it in sub]
    times = {}
    for shape in shapes:
        plan = bsh.Plan(sub, grids, len(bands), lanes=shape[0], chunk=shape[1], use_graph=False)
        times[shape] = time_plan(plan, plain=plain)
        plan.close()
        if verbose:
            print(f"[autotune] {'plain ' if plain else ''}lanes={shape[0]} chunk={shape[1]}: "
                  f"{times[shape]:.3f} ms", flush=True)
    best = min(times, key=times.get)
    if use_cache:
        db[key] = {"lanes": best[0], "chunk": best[1],
                   "times": {f"{l}x{c}": t for (l, c), t in times.items()}}
        _store(db)
    return best, times
