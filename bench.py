#!/usr/bin/env python3
"""Throughput of the binary Hough hot path on one MI355X.

One step = one pass of the whole hot path over one band of synthetic data already resident
in HBM: peakgram, stage-1 weighted count over every template, stage-1 top-k, decoding of the
winners, stage-2 power (and the winners' counts) on the exact track, stage-2 top-k.

Default workload: 4000 segments (2 detectors x 2000, gapped), one sky pixel, band
200.0-200.1 Hz (90 f0 bins), a_p 64 x P 32 x t_asc 64 -> 11 796 480 templates; stage-1
top-10^4 then stage-2 top-100.  Work unit: template x segment of stage 1.

The same line carries the batched-versus-plain comparison on the full batching workload: 256 sky
patches x 4 bands of 0.1 Hz in 100-300 Hz (1024 items, 3000-6000 gapped segments each, uneven
t_asc counts per cell; 9.01e9 templates, ~4e13 template x segments), stage 1 plus per-item top-1000
and per-band top-1000 lists, once as one graph-captured persistent launch and once as one plain
launch (and top-k) per item.

Prints one JSON line.  The CPU oracle is timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hough templates·segments/s on 1 GPU, batched vs plain, at oracle-exact top-k"
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: 32-bit VALU lane-operations per second
VALU_PEAK_OPS = 256 * 64 * 2.4e9
# VALU lane-operations per template x segment on the fast path of the subset-sum table count:
# the VALU instructions of the segment-group loop in its gfx950 assembly along the path with no
# f0-shift step and no flush (paper_1904_04873_amd/fastpath_ops.py counts them: 664 per group
# of 8 segments at the 128- and 256-segment chunks), divided by the group's 8 x 90 template x
# segments.
TABLE_OPS_PER_TS = 664 / 720
# the same figure for plain select-and-add: extract the peak bit, select the weight, add
SELECT_OPS_PER_TS = 3
# HBM bytes per count launch, measured with rocprofv3 counters for one kernel source and tile
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hough_count_table_band200Hz_traffic.txt")
# the plain count kernel's sources and the build script (which holds its compiler flags)
COUNT_SOURCES = ("paper_1904_04873_amd/csrc/bsh_count.hip", "paper_1904_04873_amd/csrc/bsh_count_tile.h",
                 "paper_1904_04873_amd/csrc/bsh_count.h", "paper_1904_04873_amd/csrc/bsh_internal.h",
                 "paper_1904_04873_amd/build.py")


def count_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in COUNT_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(lanes: int, chunk: int):
    """HBM bytes per launch from the committed counter summary, or None when the count kernel's
    sources or the tile differ from those the counters were taken on."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                parts = line.split()
                if len(parts) == 2 and not line.startswith("#"):
                    kv[parts[0]] = parts[1]
        if kv.get("sources_sha256") != count_sources_digest():
            return None
        if (int(kv["lanes"]), int(kv["chunk"])) != (lanes, chunk):
            return None
        return float(kv["traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def oracle_one_thread(n_ap: int) -> dict:
    """The same oracle count on one host thread (OMP_NUM_THREADS=1 in a child process), over the
    first n_ap a_p values of the 200 Hz band grid."""
    import subprocess
    code = (
        "import json, sys, time\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import bsh_synth as S\n"
        "import oracle as O\n"
        "w = S.config2(); seg, spec = w.segments[0], w.grids[0]\n"
        "a_p, per, off, t_asc = O.grid_tables(spec, seg.t_span_mid())\n"
        f"n_ap = max(1, min({n_ap}, spec.n_ap)); sub = off[:n_ap * spec.n_per + 1]\n"
        "t0 = time.perf_counter()\n"
        "O.hough_count(seg, w.sky, spec.k0, spec.n_f0, a_p[:n_ap], per, sub, t_asc[:sub[-1]])\n"
        "dt = time.perf_counter() - t0\n"
        "ts = int(sub[-1]) * spec.n_f0 * seg.n_seg\n"
        "print(json.dumps({'value': ts / dt, 'threads': O.num_threads(), 'sample': "
        "f'first {n_ap} a_p values: {ts:.3e} template*segments in {dt:.1f} s'}))\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if res.returncode != 0:
        raise RuntimeError(f"one-thread oracle run failed: {res.stderr[-2000:]}")
    return json.loads(res.stdout.strip().splitlines()[-1])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="enqueue every step eagerly")
    ap.add_argument("--cpu-one-thread-ap", type=int, default=1,
                    help="a_p values of the one-thread oracle sample (0: skip it)")
    ap.add_argument("--cpu-sample-ap", type=int, default=32,
                    help="a_p values (of 64) in the oracle's timed sample")
    ap.add_argument("--skip-batched", action="store_true",
                    help="omit the batched-versus-plain comparison")
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--allsky-pixels", type=int, default=16,
                    help="pixels of the all-sky slice to time (0: skip it)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB (a known-size "
                         "kernel for scaling HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; sharding the "
                                   "items over several GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import bsh_synth as S
    from paper_1904_04873_amd import bsh

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    w = S.config2()
    seg, spec = w.segments[0], w.grids[0]
    k1, k2 = w.topk_stage1, w.topk_stage2
    print(f"[bench] workload cfg2: {seg.n_seg} segments, building device tables", file=sys.stderr, flush=True)
    ds = bsh.DeviceSegments.from_host(seg)
    g = bsh.DeviceGrid.build(spec, seg.t_span_mid(), w.sky)
    n_t = g.n_templates
    ts_per_step = n_t * seg.n_seg
    st = bsh.Status(dev)
    ws_map = torch.empty(n_t, dtype=torch.float32, device=dev)
    top1 = bsh.TopK(n_t, k1, dev)
    top2 = bsh.TopK(k1, k2, dev)
    s1_score = torch.empty(k1, dtype=torch.float32, device=dev)
    s1_index = torch.empty(k1, dtype=torch.int64, device=dev)
    s2_score = torch.empty(k2, dtype=torch.float32, device=dev)
    s2_pos = torch.empty(k2, dtype=torch.int64, device=dev)
    P = torch.empty(k1, dtype=torch.float32, device=dev)
    from paper_1904_04873_amd import autotune
    (lanes, chunk), tune_ms = autotune.tune_plain(ds, g, use_cache=False)
    print(f"[bench] tile {lanes} x {chunk}", file=sys.stderr, flush=True)

    def step():
        bsh.bsh_peakgram(ds.power, 1.6, out=ds.peak_bits)
        bsh.bsh_hough_count(ds, g, status=st, wsum_out=ws_map, lanes=lanes, chunk=chunk)
        top1(ws_map, out_score=s1_score, out_index=s1_index)
        cs, cp = bsh.bsh_decode_templates(g, s1_index)
        bsh.bsh_power_stat(ds, g.sky, cs, cp, mode=0, with_counts=True, status=st, out=P)
        top2(P, out_score=s2_score, out_index=s2_pos)

    if args.calibrate_copy_mb > 0:
        n_f = args.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n_f, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st.raise_if_set("warmup")

    # One step is one HIP graph replay: the ~50 launches of a step are enqueued once at capture
    # time, so host launch latency does not stretch the step.
    run_step = step
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
        run_step = graph.replay
        for _ in range(args.warmup):
            run_step()
        torch.cuda.synchronize()
        st.raise_if_set("graph warmup")
    print(f"[bench] warmup done, timing {args.steps} steps", file=sys.stderr, flush=True)

    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for _ in range(args.steps):
        run_step()
    t_end.record()
    torch.cuda.synchronize()
    st.raise_if_set("timed steps")
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / max(args.steps, 1)

    # The dominant kernel alone: the same stage-1 launch, back to back on the stream it runs on,
    # bracketed by HIP events.
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    n_count = max(args.steps, 3)
    c0.record()
    for _ in range(n_count):
        bsh.bsh_hough_count(ds, g, status=st, wsum_out=ws_map, lanes=lanes, chunk=chunk)
    c1.record()
    torch.cuda.synchronize()
    st.raise_if_set("count kernel")
    count_ms = c0.elapsed_time(c1) / n_count
    value = ts_per_step / (ms_step / 1e3)
    ops_per_ts = TABLE_OPS_PER_TS
    achieved = ops_per_ts * ts_per_step / (count_ms / 1e3)
    achieved_select = SELECT_OPS_PER_TS * ts_per_step / (count_ms / 1e3)
    print(f"[bench] {ms_step:.3f} ms/step, count kernel {count_ms:.3f} ms", file=sys.stderr, flush=True)

    post = run_post(bsh, ds, g, s1_score, s1_index, seg.t_coh, seg.t_span_mid(), st)
    refine = run_refine(bsh, spec, st)
    beside = run_beside(bsh, w, st, *bsh.bsh_decode_templates(g, s1_index))

    batched = None if args.skip_batched else run_batched(args)
    allsky = run_allsky(args) if (args.allsky_pixels > 0 and not args.skip_batched) else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        a_p, per, off, t_asc = O.grid_tables(spec, seg.t_span_mid())
        n_ap = max(1, min(args.cpu_sample_ap, spec.n_ap))
        cells = n_ap * spec.n_per
        sub_off = off[:cells + 1]
        t0 = time.perf_counter()
        O.hough_count(seg, w.sky, spec.k0, spec.n_f0, a_p[:n_ap], per, sub_off, t_asc[:sub_off[-1]])
        dt = time.perf_counter() - t0
        ts_cpu = int(sub_off[-1]) * spec.n_f0 * seg.n_seg
        cpu = {"value": ts_cpu / dt, "unit": "template*segments/s", "cores": O.num_threads(),
               "kind": "oracle",
               "sample": f"stage-1 count of the first {n_ap} of {spec.n_ap} a_p values (all P, t_asc, f0 "
                         f"and {seg.n_seg} segments): {ts_cpu:.3e} template*segments in {dt:.1f} s",
               "affinity": sorted(os.sched_getaffinity(0))}
        if args.cpu_one_thread_ap > 0:
            cpu["one_thread"] = oracle_one_thread(args.cpu_one_thread_ap)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "template*segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32",
        "data": "synthetic",
        "config": {
            "workload": "band 200.0-200.1 Hz: 4000 segments (2 detectors x 2000, gapped), 1 sky "
                        "pixel, 90 f0 x 64 a_p x 32 P x 64 t_asc = 11796480 templates; stage-1 "
                        "weighted count -> top-10^4 -> stage-2 power -> top-100",
            "templates": n_t,
            "segments": seg.n_seg,
            "template_segments_per_step": ts_per_step,
            "topk_stage1": k1,
            "topk_stage2": k2,
            "parallelism": "single GPU",
            "step_launch": "eager" if args.no_graph else "hip graph replay",
        },
        "roofline": {
            "bound": "alu",
            "kernel": f"hough_count_kernel<2, {chunk}> (subset-sum tables of 8 segments)",
            "achieved": achieved / 1e12,
            "peak": VALU_PEAK_OPS / 1e12,
            "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_OPS,
            "traffic": measured_traffic(lanes, chunk),
            "count_kernel_ms": count_ms,
            "ops_per_template_segment": ops_per_ts,
            "select_add_equivalent": {"ops_per_template_segment": SELECT_OPS_PER_TS,
                                      "achieved": achieved_select / 1e12,
                                      "frac": achieved_select / VALU_PEAK_OPS},
            "tile": {"lanes": lanes, "chunk": chunk},
            "autotune_ms": {f"{l}x{c}": t for (l, c), t in tune_ms.items()},
        },
        "cpu_baseline": cpu,
        "post": post,
        "refine": refine,
        "beside_path": beside,
        "batched": batched,
        "allsky": allsky,
    }
    print(json.dumps(out), flush=True)


def run_post(bsh, ds, g, s1_score, s1_index, t_coh, t_mid, st):
    """Post-processing of the stage-1 top-10^4 (not part of the step): rows, s_H significances,
    clusters in a sqrt(14) window and their centroids, timed with HIP events."""
    import torch
    seg_w = ds.weight
    pp = bsh.post_params(t_coh=t_coh, t_obs=2.0 * (t_mid - float(ds.t_mid.min().item())) + t_coh)

    def run():
        cs, cp = bsh.bsh_decode_templates(g, s1_index)
        rows = bsh.bsh_post_rows(g.sky, cs, cp, t_coh)
        sig = bsh.bsh_significance(s1_score, seg_w, 0, 1.6)
        lab = bsh.bsh_cluster(pp, rows, 14.0 ** 0.5)
        return lab, bsh.bsh_cluster_centroids(pp, rows, sig, lab, status=st)

    run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    reps = 5
    a.record()
    for _ in range(reps):
        lab, (cen, weight, top, best) = run()
    b.record()
    torch.cuda.synchronize()
    st.raise_if_set("post-processing")
    n_clusters = int((lab == torch.arange(lab.numel(), device=lab.device, dtype=lab.dtype)).sum().item())
    return {"candidates": int(s1_index.numel()), "clusters": n_clusters, "ms": a.elapsed_time(b) / reps,
            "window": "sqrt(14)", "best_cluster_weight": float(weight[int(best.item())].item())}


def run_refine(bsh, spec, st):
    """The differentiable stage 2 at its real size (not part of the step): 10^5 off-grid
    candidates over 4000 segments (the 200 Hz band layout, noise only), one forward
    (interpolated power), one backward (adjoint kernel), both from one pass, and 20 Adam steps
    with the one-pass kernel and through autograd (forward and backward kernels)."""
    import numpy as np
    import torch
    import bsh_synth as S
    from paper_1904_04873_amd.refine import refine

    w = S.config4()
    seg = w.segments[0]
    ds = bsh.DeviceSegments.from_host(seg)
    sky = torch.from_numpy(w.sky).cuda()
    rng = w.rng["candidates"]
    n = 100_000
    centre = np.stack([spec.k0 + rng.uniform(5, 85, 10), rng.uniform(0.5, 2.8, 10),
                       rng.uniform(spec.per_lo * 1.1, spec.per_hi * 0.9, 10), np.zeros(10)], axis=1)
    centre[:, 3] = seg.t_span_mid() + rng.uniform(-0.5, 0.5, 10) * centre[:, 2]
    steps = np.array([1.0, (spec.ap_hi - spec.ap_lo) / (spec.n_ap - 1),
                      (spec.per_hi - spec.per_lo) / (spec.n_per - 1), 0.0])
    cand = np.repeat(centre, n // 10, axis=0)
    st_steps = np.repeat(steps[None, :], n, axis=0)
    st_steps[:, 3] = cand[:, 2] / 64.0
    cand = cand + rng.uniform(0, 2, cand.shape) * rng.choice([-1.0, 1.0], cand.shape) * st_steps
    th = torch.from_numpy(cand).cuda()
    cs = torch.zeros(n, dtype=torch.int32, device="cuda")
    stp = torch.from_numpy(st_steps).cuda()

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    fwd = timed(lambda: bsh.bsh_power_stat(ds, sky, cs, th, mode=1, status=st))
    bwd = timed(lambda: bsh.bsh_power_stat_grad(ds, sky, cs, th, status=st))
    both = timed(lambda: bsh.bsh_power_stat_value_and_grad(ds, sky, cs, th, status=st))
    adam = timed(lambda: refine(th, stp, ds, sky, cs, n_iter=20, lr=0.05, status=st), reps=1)
    adam_ag = timed(lambda: refine(th, stp, ds, sky, cs, n_iter=20, lr=0.05, status=st, fused=False), reps=1)
    st.raise_if_set("refinement")
    cs_n = n * seg.n_seg
    return {"candidates": n, "segments": seg.n_seg, "forward_ms": fwd, "backward_ms": bwd,
            "value_and_grad_ms": both, "adam_20_steps_ms": adam, "adam_20_steps_autograd_ms": adam_ag,
            "forward_cand_seg_per_s": cs_n / (fwd / 1e3), "backward_cand_seg_per_s": cs_n / (bwd / 1e3)}


def run_beside(bsh, w, st, cs, cp):
    """The steps beside the path, timed on the 200 Hz band layout (not part of the step): the
    running-median normalization of the raw spectra, stage 2 on the Tc/2-shifted doubled segment
    set, and stage 2 on the low-eccentricity track, each for the step's 10^4 stage-1 winners."""
    import numpy as np
    import torch
    import bsh_synth as S

    seg = w.segments[0]
    sky = torch.from_numpy(w.sky).cuda()

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # normalization: raw rows 100 bins wider than the band's row, window 101
    raw = torch.from_numpy(S.raw_sft_powers(np.random.default_rng(5), seg.n_seg, seg.n_bins + 100,
                                            seg.k_lo - 50)).cuda()
    rho = torch.empty((seg.n_seg, seg.n_bins), dtype=torch.float32, device="cuda")
    ms_norm = timed(lambda: bsh.bsh_normalize(raw, 101, out=rho))
    # the doubled set: the band's segments and their Tc/2-shifted companions in one table
    comp = S.half_shifted(seg, np.random.default_rng(21))
    du = bsh.DeviceSegments.from_host(S.concat_segments(seg, comp))
    ms_dbl = timed(lambda: bsh.bsh_power_stat(du, sky, cs, cp, mode=0, status=st))
    # the ELL1 track: the winners with e cos w = 0.01, e sin w = -0.005
    n = int(cs.numel())
    cpe = torch.cat([cp, torch.tensor([[0.01, -0.005]], dtype=torch.float64, device="cuda").expand(n, 2)],
                    dim=1).contiguous()
    ds = bsh.DeviceSegments.from_host(seg)
    ms_ecc = timed(lambda: bsh.bsh_power_stat_ecc(ds, sky, cs, cpe, mode=0, status=st))
    st.raise_if_set("steps beside the path")
    return {
        "normalize": {"segments": seg.n_seg, "raw_bins": seg.n_bins + 100, "window": 101, "ms": ms_norm,
                      "output_bins_per_s": seg.n_seg * seg.n_bins / (ms_norm / 1e3)},
        "stage2_doubled_set": {"candidates": n, "segments": du.n_seg, "ms": ms_dbl,
                               "cand_seg_per_s": n * du.n_seg / (ms_dbl / 1e3)},
        "stage2_ell1": {"candidates": n, "segments": seg.n_seg, "ms": ms_ecc,
                        "cand_seg_per_s": n * seg.n_seg / (ms_ecc / 1e3)},
    }


def run_allsky(args):
    """The all-sky slice's shape (2 x 4000 segments over 240 d, band 300.0-300.1 Hz, 128 a_p x 64 P
    x rule t_asc = 581 531 binary templates per pixel) on `allsky_pixels` of its 2000 pixels, one
    batched plan with per-pixel and per-band top-10^5."""
    import numpy as np
    import torch

    import bsh_synth as S
    from paper_1904_04873_amd import bsh

    dev = torch.device("cuda:0")
    n_pix = args.allsky_pixels
    print(f"[bench] all-sky slice: {n_pix} pixels", file=sys.stderr, flush=True)
    w = S.config5()
    seg, spec = w.segments[0], w.grids[0]
    ds = bsh.DeviceSegments.from_host(seg, device=dev)
    g = bsh.DeviceGrid.build(spec, seg.t_span_mid(), w.sky, device=dev)
    pixels = [int(p) for p in np.linspace(0, len(w.sky) - 1, n_pix).round()]
    items = [(ds, 0, p, 1, 0) for p in pixels]
    k = 100000
    st = bsh.Status(dev)
    plan = bsh.Plan(items, [g], 1, k_item=k, k_band=k, use_graph=True, lpt=True, status=st)
    plan.run()
    torch.cuda.synchronize()
    out = []
    for _ in range(max(1, args.batched_steps)):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.run()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    st.raise_if_set("all-sky plan")
    plan.close()
    ms = float(np.median(out))
    ts = n_pix * g.n_bin * g.n_f0 * seg.n_seg
    return {"workload": f"band 300.0-300.1 Hz, 2 x 4000 segments over 240 d, {n_pix} of 2000 pixels, "
                        f"90 f0 x 128 a_p x 64 P x rule t_asc = {g.n_bin} binary templates per pixel; "
                        "per-pixel and per-band top-10^5",
            "pixels": n_pix, "template_segments": ts, "ms": ms, "value": ts / (ms / 1e3),
            "unit": "template*segments/s", "k": k}


def run_batched(args):
    """Full batching workload: one graph-captured persistent launch vs one plain launch per item,
    each form with the tile the autotuner finds fastest for it."""
    import numpy as np
    import torch

    import bsh_synth as S
    from paper_1904_04873_amd import autotune, bsh

    dev = torch.device("cuda:0")
    print("[bench] batching workload: generating 1024 items", file=sys.stderr, flush=True)
    w = S.config3()
    items, grids = [], []
    ts_total = 0
    for it in range(len(w.segments)):
        seg = w.segments[it]
        band = w.item_grid[it]
        g = bsh.DeviceGrid.build(w.grids[band], seg.t_span_mid(), w.sky, device=dev)
        ds = bsh.DeviceSegments.from_host(seg, device=dev)
        lo, hi = w.item_sky[it]
        items.append((ds, it, lo, hi - lo, band))
        grids.append(g)
        ts_total += (hi - lo) * g.n_bin * g.n_f0 * seg.n_seg
        w.segments[it] = None        # drop the host copy
    torch.cuda.synchronize()
    print(f"[bench] batching workload resident: {ts_total:.3e} template*segments; autotuning",
          file=sys.stderr, flush=True)
    (lanes, chunk), tune_ms = autotune.tune(items, grids, 4, sample=16, use_cache=False)
    # the plain baseline runs with the tile that suits one launch per item best
    (lanes_p, chunk_p), tune_p_ms = autotune.tune(items, grids, 4, sample=16, use_cache=False, plain=True)
    k_item, k_band = 1000, 1000
    st = bsh.Status(dev)
    plan = bsh.Plan(items, grids, 4, k_item=k_item, k_band=k_band, lanes=lanes, chunk=chunk,
                    use_graph=True, lpt=True, status=st)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.median(out))

    print("[bench] batched runs", file=sys.stderr, flush=True)
    ms_b = timed(plan.run, args.batched_steps)
    st.raise_if_set("batched")
    ref = plan.band_index.clone()
    units, blocks = plan.units, plan.blocks
    if (lanes_p, chunk_p) != (lanes, chunk):
        plan.close()
        plan = bsh.Plan(items, grids, 4, k_item=k_item, k_band=k_band, lanes=lanes_p, chunk=chunk_p,
                        use_graph=True, lpt=True, status=st)
    print("[bench] plain runs", file=sys.stderr, flush=True)
    ms_p = timed(plan.run_plain, args.batched_steps)
    st.raise_if_set("plain")
    same = bool(torch.equal(ref, plan.band_index))
    plan.close()
    return {
        "workload": "256 sky patches x 4 bands of 0.1 Hz (f_lo 100.0/166.6/233.2/299.8 Hz): 1024 items "
                    "of 3000-6000 gapped segments, a_p 64 x P 32 x t_asc 4-256 per cell, 90 f0; "
                    "per-item top-1000 and per-band top-1000",
        "items": len(items),
        "template_segments": ts_total,
        "batched_ms": ms_b,
        "plain_ms": ms_p,
        "batched_value": ts_total / (ms_b / 1e3),
        "plain_value": ts_total / (ms_p / 1e3),
        "speedup": ms_p / ms_b,
        "lists_identical": same,
        "tile": {"lanes": lanes, "chunk": chunk},
        "plain_tile": {"lanes": lanes_p, "chunk": chunk_p},
        "autotune_ms": {f"{l}x{c}": t for (l, c), t in tune_ms.items()},
        "autotune_plain_ms": {f"{l}x{c}": t for (l, c), t in tune_p_ms.items()},
        "units": units,
        "persistent_blocks": blocks,
    }


if __name__ == "__main__":
    main()
