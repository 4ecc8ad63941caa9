#!/usr/bin/env python3
"""Benchmark of the gaze-line stereo graph-cut hot path on one MI355X.

One step = the whole path on one synthetic stereo pair already resident in
HBM: stereo_cost_volume -> graph_build -> maxflow_solve -> extract_labels
(exact minimum cut, canonical labels, energy and flow).  The workload is the
384x288 pair with 16 depth numbers (slanted-plane scene, truncated AD cap 30,
penalty 1, inhibit 1023).

Prints one JSON line (rank 0) with throughput in pairs/s, per-pair latency,
Medge-pushes/s, a roofline entry for the dominant kernel (device time from
HIP events recorded on the solve stream during the timed steps) and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ms/stereo pair + Medge-pushes/s at 384×288×16; "
          "batched pairs/s at p99 latency")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pairs", type=int, default=8, help="distinct resident pairs cycled")
    ap.add_argument("--lam", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=5, help="pairs the oracle solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--no-approx", action="store_true",
                    help="skip the variant sections (approximate cuts, pairwise and colour "
                         "variants, the larger 450x375x64 pair)")
    ap.add_argument("--batch-pairs", type=int, default=64, help="pairs of the uneven batch (0: skip)")
    ap.add_argument("--batch-runs", type=int, default=3,
                    help="interleaved runs of each batch mode (each reports its median run)")
    ap.add_argument("--serve-requests", type=int, default=60, help="requests of the serving stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-low-rate", type=float, default=8.0,
                    help="second stream below the GPU's capacity (0: skip)")
    ap.add_argument("--serve-low-requests", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 5 plain 256 MiB device copies (reference for HBM counters)")
    ap.add_argument("--sections", default="all",
                    help="comma list of the parts to run besides the timed headline steps: "
                         "variants, rgb, approx, larger, batch, serving, cpu (default all)")
    ap.add_argument("--larger-pairs", type=int, default=3,
                    help="seeded pairs of each larger DRAM-resident configuration")
    ap.add_argument("--larger-shapes", default="450x375x64,640x480x64",
                    help="which larger configurations the 'larger' section runs")
    args = ap.parse_args()
    every = {"variants", "rgb", "approx", "larger", "batch", "serving", "cpu"}
    sec = every if args.sections == "all" else {x for x in args.sections.split(",") if x}
    if not sec <= every:
        ap.error(f"unknown sections {sorted(sec - every)}")
    if args.no_approx:
        sec -= {"variants", "rgb", "approx", "larger"}
    if args.batch_pairs <= 0:
        sec.discard("batch")
    if args.serve_requests <= 0:
        sec.discard("serving")
    if args.no_cpu_baseline:
        sec.discard("cpu")
    args.sec = sec
    return args


BYTES_PER_VISIT = 72.0     # one node's 9-word record read and written per sweep


def algorithmic_bytes(kind: str, nodes: int, visits_per_sweep: float) -> float:
    """Algorithmic bytes of one launch.

    push / relabel / fused sweep: a sweep reads and writes the 9-word record
    (excess, height, 7 stored pair words: 36 B) of every node it finds with
    excess and a finite height, 72 B per such visit.  The visits are counted
    on the device by the push (or fused) sweep; inactive nodes cost nothing
    algorithmically (their 64-node groups are skipped by a flag test).
    relax: one tiled BFS pass reads every node's 16-bit arc mask and 32-bit
    value and writes the value back: 10 B per node (an upper bound: tiles
    whose neighbourhood did not change are skipped).
    """
    if kind == "relax":
        return 10.0 * nodes
    return BYTES_PER_VISIT * visits_per_sweep


PROFILES = os.path.join(ROOT, "profiles")
HIP_SOURCE = os.path.join(ROOT, "paper_1803_01516_amd", "csrc", "gazecut.hip")


def measured_traffic(kernel: str, shape: str):
    """HBM bytes per launch of `kernel` on the workload `shape` (WxHxM) from
    the committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by the ratio the same counter shows on a plain
    device copy of known size), or None when no summary covers the kernel or
    the HIP source has changed since the counters were taken (the summary
    records the source's SHA-1)."""
    import hashlib
    path = os.path.join(PROFILES, f"{kernel}_{shape}_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
    if not rec or rec.get("kernel") != kernel:
        return None
    with open(HIP_SOURCE, "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != rec.get("source_sha1"):
            return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])


KERNEL_NAMES = {"relax": "k_relax", "push": "k_push", "relabel": "k_relabel"}


def roofline_block(stats, nodes, shape, fused, state_bytes, steps):
    """Roofline entry of the dominant kernel class over a list of solve
    statistics (GC_OPT_TIME_KERNELS): algorithmic bytes of its average launch
    over that launch's average device time (sampled HIP events on the solve
    stream), against MI355X's 8 TB/s."""
    tot = {k: sum(s[f"{k}_ms"] for s in stats) for k in ("push", "relabel", "relax")}
    launches = {k: sum(s[f"{k}_launches"] for s in stats) for k in ("push", "relabel", "relax")}
    # the entry is the push-relabel sweep's (push or fused sweep): the class
    # the HBM target is set for, and the largest or nearly so wherever the
    # state leaves the Infinity Cache.  The relaxation's bytes depend on how
    # many tiles a pass processes, which is not counted, so it is reported
    # beside it by time and measured traffic only.
    kind = "push"
    dominant = max(tot, key=tot.get)
    sweeps = max(1, sum(s["sweeps"] for s in stats))
    visits = sum(s["active_visits"] for s in stats)
    per_launch_ms = tot[kind] / max(1, launches[kind])
    bytes_launch = algorithmic_bytes(kind, nodes, visits / sweeps)
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    kname = "k_sweep" if (kind == "push" and fused) else KERNEL_NAMES[kind]
    traffic = measured_traffic(kname, shape)
    resident = state_bytes < 256e6
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else int(traffic),
            "traffic_over_algorithmic": None if traffic is None else round(traffic / bytes_launch, 3),
            "traffic_GBs": None if traffic is None else round(traffic / (per_launch_ms * 1e-3) / 1e9, 1),
            "kernel": kname, "workload": shape,
            "state_mb": round(state_bytes / 1e6, 1),
            "measure": ("effective algorithmic bandwidth: the state fits the 256 MB Infinity "
                        "Cache, so these bytes are not DRAM traffic" if resident else
                        "algorithmic bytes of a DRAM-resident state (larger than the 256 MB "
                        "Infinity Cache)"),
            "avg_launch_us": round(per_launch_ms * 1e3, 2),
            "active_visits_per_sweep": round(visits / sweeps, 1),
            "bytes_per_visit": BYTES_PER_VISIT,
            "launches_per_solve": round(launches[kind] / steps, 1),
            "bytes_per_launch": int(bytes_launch),
            "device_ms_per_solve": {k: round(v / steps, 3) for k, v in tot.items()},
            "largest_class": KERNEL_NAMES[dominant] if dominant != "push" or not fused else "k_sweep",
            "relax": relax_entry(tot, launches, shape)}


def relax_entry(tot, launches, shape):
    """The relaxation pass beside the sweep: average launch time and the HBM
    traffic of the committed counter summary (no algorithmic fraction)."""
    per_launch_ms = tot["relax"] / max(1, launches["relax"])
    traffic = measured_traffic("k_relax", shape)
    return {"kernel": "k_relax", "avg_launch_us": round(per_launch_ms * 1e3, 2),
            "traffic": None if traffic is None else int(traffic),
            "traffic_GBs": None if traffic is None or per_launch_ms <= 0 else
            round(traffic / (per_launch_ms * 1e-3) / 1e9, 1)}


def _log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _pct(xs, q):
    return round(float(np.percentile(np.array(xs) * 1e3, q)), 2)


def bench_batch(args, gc, sg, torch):
    """Uneven batch: pairs drawn uniformly from 320x240x16, 384x288x16,
    450x375x64 and 640x480x64, solved three ways: one pair per launch, by the
    batch engine (every member advancing on the device, each step's launches
    shared by all members, relabel period and tile autotuned), and by four
    concurrent lanes (host threads running single solves, options autotuned).
    Latency of a pair = its completion time from the start of the run."""
    from paper_1803_01516_amd import runtime as rt
    stream = torch.cuda.Stream()
    mix = rt.batch_mix(args.batch_pairs, sg.BATCH_SHAPES, seed=4)
    with torch.cuda.stream(stream):
        # autotune on one pair of every shape class, for each engine
        seen, tune = set(), []
        for i, (spec, pair) in enumerate(mix):
            key = (spec.w, spec.h, spec.m)
            if key not in seen:
                seen.add(key)
                tune.append(rt.make_item(i, spec, pair))
        t = time.perf_counter()
        best_lanes, trials_l = rt.autotune(tune, stream=stream, use_graph=True)
        best_eng, trials_e = rt.autotune(tune, tiles=((8, 8, 16), (16, 16, 8)), periods=(0, 24, 32, 48),
                                         sweeps=(0,), stream=stream, extra_flags=gc.GC_OPT_BATCH_MERGED)
        tune_s = time.perf_counter() - t
        _log(f"batch: autotuned over {len(trials_l) + len(trials_e)} candidates in {tune_s:.1f} s")
        for it in tune:
            rt.release(it)

        def run(fn, opts, name):
            items = [rt.make_item(i, spec, pair) for i, (spec, pair) in enumerate(mix)]
            times, total = fn(items, opts, stream)
            _log(f"batch: {name} {total:.2f} s")
            out = [(it.energy, it.flow, it.labels.cpu()) for it in items]
            for it in items:
                rt.release(it)
            del items
            torch.cuda.empty_cache()
            return times, total, out

        # three interleaved runs of each mode; each reports its run of median total
        runs = {"one": [], "eng": [], "lan": []}
        same = True
        ref = None
        for r in range(args.batch_runs):
            for key, fn, opts, name in (("one", rt.run_one_per_launch, None, "one pair per launch"),
                                        ("eng", rt.run_batched, best_eng, "batch engines"),
                                        ("lan", rt.run_batched, best_lanes, "concurrent lanes")):
                times, total, got = run(fn, opts, name)
                runs[key].append((total, times))
                if ref is None:
                    ref = got
                same = same and all(a[0] == b[0] and a[1] == b[1] and bool((a[2] == b[2]).all())
                                    for a, b in zip(ref, got))

        def median_run(v):
            v = sorted(v, key=lambda x: x[0])
            return v[len(v) // 2]
        tot_one, t_one = median_run(runs["one"])
        tot_eng, t_eng = median_run(runs["eng"])
        tot_lan, t_lan = median_run(runs["lan"])
    n = len(mix)
    nodes = sum(s.w * s.h * (s.m - 1) for s, _ in mix)

    def block(times, total):
        return {"pairs_per_s": round(n / total, 2), "total_s": round(total, 3),
                "p50_ms": _pct(times, 50), "p99_ms": _pct(times, 99)}

    def opts_of(o):
        return {"tile": [o.tile_w, o.tile_h, o.tile_j],
                "relabel_period": o.relabel_period or "by depth (24 below 32 levels, else 32)",
                "sweep": "split" if o.flags & gc.GC_OPT_SPLIT_SWEEP else "fused"}

    return {"workload": f"{n} seeded pairs uniform over 320x240x16, 384x288x16, 450x375x64, "
                        "640x480x64 (6-10 slanted planes, sigma 3, cap 30, penalty 1, inhibit 1023)",
            "nodes_total": nodes,
            "batched": dict(block(t_eng, tot_eng),
                            mode=f"{gc.GC_BATCH_ENGINES} batch engines on their own streams, driven "
                                 "from one host thread: members advance on the device, 32 captured "
                                 "steps per read-back, one work queue per unit kind",
                            options=opts_of(best_eng)),
            "one_per_launch": block(t_one, tot_one),
            "concurrent_lanes": dict(block(t_lan, tot_lan),
                                     mode=f"{gc.GC_BATCH_LANES} host threads each running single solves",
                                     options=opts_of(best_lanes)),
            "runs_total_s": {k: [round(x[0], 3) for x in v] for k, v in
                             (("one_per_launch", runs["one"]), ("batched", runs["eng"]),
                              ("concurrent_lanes", runs["lan"]))},
            "speedup_vs_one_per_launch": round(tot_one / tot_eng, 3),
            "speedup_vs_lanes": round(tot_lan / tot_eng, 3),
            "autotune": {"tuning_s": round(tune_s, 2), "candidates": len(trials_l) + len(trials_e)},
            "identical_results": same}


def bench_approx(gc, sg, torch, spec, pairs, lefts, rights, n_timed, stream, dev, lam):
    """The exact cut, the exact cut warm-started from the level-1 skin
    (b = 3), and the approximate cuts of Sec. 4.5 (level 1 b = 2, 3; level 2
    b = 3 with max(32, labels) wave steps) on the same pairs, each timed from
    the cost volume to the labels (median over n_timed pairs after a warm-up
    pass), with its energy gap to the optimum and eq. (2) error."""
    p = gc.problem(spec.w, spec.h, spec.m, spec.cap, lam, spec.inhibit)
    ws, ws2 = gc.alloc_workspace(p, dev), gc.alloc_workspace(p, dev)
    cost = torch.empty((spec.m, spec.h, spec.w), dtype=torch.int32, device=dev)
    labels = torch.empty((spec.h, spec.w), dtype=torch.int32, device=dev)
    result = torch.zeros(2, dtype=torch.int64, device=dev)

    def exact(k):
        g = gc.graph_build(p, cost, ws, stream)
        gc.maxflow_solve(g, None, stream)
        gc.extract_labels(g, cost, labels, result, stream)
        return labels, int(result.cpu()[0])

    def warm(k):
        lab, e, _, _, _ = gc.solve_warm(p, cost, 3, None, stream, ws=ws, ws_skin=ws2)
        return lab, e

    def approx(level, b):
        def run(k):
            lab, e, _, _, _ = gc.approx_level1(p, cost, b, None, stream, ws=ws, level=level)
            return lab, e
        return run

    out, best = {}, {}
    for name, fn in (("exact", exact), ("warm_start_b3", warm), ("level1_b2", approx(1, 2)),
                     ("level1_b3", approx(1, 3)), ("level2_b3", approx(2, 3))):
        lat, gaps, errs, pcts = [], [], [], []
        for i in range(n_timed + 1):
            k = i % len(pairs)
            torch.cuda.synchronize()
            a = time.perf_counter()
            if lefts[k].dim() == 3:
                gc.stereo_cost_volume_rgb(lefts[k], rights[k], p, cost, stream)
            else:
                gc.stereo_cost_volume(lefts[k], rights[k], p, cost, stream)
            lab, e = fn(k)
            torch.cuda.synchronize()
            if i == 0 and n_timed >= len(pairs):
                continue                                   # warm-up pass
            lat.append(time.perf_counter() - a)
            if name == "exact":
                best[k] = e
            gaps.append(e - best[k])
            er, pc = sg.eq2_error(pairs[k].gt, lab.cpu().numpy())
            errs.append(er)
            pcts.append(pc)
        out[name] = {"ms_per_pair": round(1e3 * float(np.median(lat)), 3),
                     "energy_gap_mean": round(float(np.mean(gaps)), 1),
                     "energy_gap_rel": round(float(np.mean(gaps)) / float(np.mean(list(best.values()))), 6),
                     "eq2_error_mean": round(float(np.mean(errs)), 1),
                     "pct_exact_mean": round(float(np.mean(pcts)), 1)}
        _log(f"approx {spec.w}x{spec.h}x{spec.m} {name}: {out[name]['ms_per_pair']} ms/pair, "
             f"eq2 error {out[name]['eq2_error_mean']}")
    for name in ("warm_start_b3", "level1_b2", "level1_b3", "level2_b3"):
        out[name]["time_over_exact"] = round(out[name]["ms_per_pair"] / out["exact"]["ms_per_pair"], 3)
    # Table 2 of the paper: eq. (2) error 21294 at level 2 b=3 against 20657
    # at level 1 b=3 on its own pair (ratio 1.031)
    out["level2_over_level1_b3_eq2"] = round(out["level2_b3"]["eq2_error_mean"] /
                                             out["level1_b3"]["eq2_error_mean"], 4)
    out["paper_table2_level2_over_level1_b3_eq2"] = round(21294 / 20657, 4)
    out["workload"] = (f"{spec.w}x{spec.h}x{spec.m}, {len(pairs)} seeded "
                       f"{'colour (SAD, untruncated) ' if lefts[0].dim() == 3 else ''}pairs, penalty {lam}, "
                       f"inhibit {spec.inhibit}")
    del ws, ws2
    return out


def bench_larger(args, gc, torch, sg, lspec, seed0, stream, dev):
    """Exact solves of seeded pairs of one larger configuration, with the
    roofline entry of their dominant kernel."""
    lp = gc.problem(lspec.w, lspec.h, lspec.m, lspec.cap, 1, lspec.inhibit)
    lws = gc.alloc_workspace(lp, dev)
    lpairs = [sg.make_pair(lspec, (seed0, i)) for i in range(args.larger_pairs)]
    ll = [torch.from_numpy(q.left).to(dev) for q in lpairs]
    lr = [torch.from_numpy(q.right).to(dev) for q in lpairs]
    opts = gc.GcSolveOpts(flags=0 if args.no_timing else gc.GC_OPT_TIME_KERNELS)
    gc.solve_pair(ll[0], lr[0], lp, None, stream, lws)          # warm-up
    lat, stats, errs, pcts, exact = [], [], [], [], True
    for k in range(len(lpairs)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        lab, _, e, f, st = gc.solve_pair(ll[k], lr[k], lp, opts, stream, lws)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
        exact = exact and e == f                     # min-cut energy = max flow
        stats.append(st.as_dict())
        er, pc = sg.eq2_error(lpairs[k].gt, lab.cpu().numpy())
        errs.append(er)
        pcts.append(pc)
    nodes = lspec.w * lspec.h * (lspec.m - 1)
    out = {"workload": f"{lspec.w}x{lspec.h} grayscale pairs, {lspec.m} depth numbers, "
                       f"{lspec.planes[0]}-{lspec.planes[1]} slanted planes, "
                       f"{int(round(100 * lspec.textureless))} % textureless, sigma {lspec.sigma:g}, "
                       f"cap {lspec.cap}, penalty 1, inhibit {lspec.inhibit}, "
                       f"seeds ({seed0}, 0..{args.larger_pairs - 1})",
           "nodes": nodes,
           "ms_per_pair": round(1e3 * float(np.median(lat)), 3),
           "ms_per_pair_all": [round(1e3 * x, 2) for x in lat],
           "sweeps_per_pair": round(float(np.mean([s["sweeps"] for s in stats])), 1),
           "global_relabels_per_pair": round(float(np.mean([s["global_relabels"] for s in stats])), 2),
           "bfs_passes_per_pair": round(float(np.mean([s["bfs_passes"] for s in stats])), 1),
           "eq2_error_mean": round(float(np.mean(errs)), 1),
           "pct_exact_mean": round(float(np.mean(pcts)), 1),
           "energy_equals_flow": exact}
    if not args.no_timing:
        out["roofline"] = roofline_block(stats, nodes, f"{lspec.w}x{lspec.h}x{lspec.m}",
                                         True, gc.footprint_bytes(lp), len(stats))   # fused sweeps (the default)
    del lws, ll, lr
    return out


def bench_serving(args, gc, sg, torch, rate, n_req):
    """Poisson request stream over 384x288x16, 640x480x64 and 1280x720x128
    pairs, served by continuous batching with admission by workspace
    footprint, one batch engine (lane) per footprint class on its own stream.
    Latency = completion - arrival."""
    from paper_1803_01516_amd import runtime as rt
    pools = {s: [(sg.spec_like(sg.MID, *s), sg.make_pair(sg.spec_like(sg.MID, *s), (5, k, i)))
                 for i in range(2)] for k, s in enumerate(sg.SERVE_SHAPES)}
    reqs = rt.poisson_requests(n_req, rate, sg.SERVE_SHAPES, 2, seed=5)
    opts = gc.GcSolveOpts()                  # relabel period and pass cap by depth
    _log(f"serving: {len(reqs)} requests at {rate:g}/s")
    done, wall, srv = rt.serve(reqs, pools, int(args.serve_budget_gb * 1e9), opts,
                               progress=lambda k, t: _log(f"serving: {k} done at {t:.1f} s"))
    _log(f"serving: done in {wall:.1f} s")
    torch.cuda.empty_cache()
    out = {"workload": f"{len(reqs)} Poisson requests at {rate:g}/s, uniform over "
                       "384x288x16, 640x480x64, 1280x720x128",
           "completed": len(done), "wall_s": round(wall, 3),
           "pairs_per_s": round(len(done) / wall, 2), "rounds": srv.rounds,
           "lanes": [{"max_mb": None if l.limit is None else l.limit >> 20, "max_graphs": l.max_members,
                      "rounds": l.rounds} for l in srv.lanes],
           "peak_members": srv.peak_members, "peak_gb": round(srv.peak_used / 1e9, 2),
           "budget_gb": args.serve_budget_gb}
    out.update(rt.latency_summary(done))
    out["by_shape"] = {"x".join(map(str, s)): rt.latency_summary([r for r in done if r.shape == s])
                       for s in sg.SERVE_SHAPES}
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(independent pairs would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1803_01516_amd import gazecut as gc
    from paper_1803_01516_amd import scenegen as sg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    gc.load()
    spec = sg.MID
    p = gc.problem(spec.w, spec.h, spec.m, spec.cap, args.lam, spec.inhibit)
    nodes = spec.w * spec.h * (spec.m - 1)

    pairs = [sg.make_pair(spec, (2, i)) for i in range(args.pairs)]
    lefts = [torch.from_numpy(q.left).to(dev) for q in pairs]
    rights = [torch.from_numpy(q.right).to(dev) for q in pairs]
    cost = torch.empty((spec.m, spec.h, spec.w), dtype=torch.int32, device=dev)
    labels = torch.empty((spec.h, spec.w), dtype=torch.int32, device=dev)
    result = torch.zeros(2, dtype=torch.int64, device=dev)
    ws = gc.alloc_workspace(p, dev)
    stream = torch.cuda.current_stream()
    opts = gc.GcSolveOpts()
    if not args.no_timing:
        opts.flags = gc.GC_OPT_TIME_KERNELS

    def step(i):
        k = i % len(pairs)
        gc.stereo_cost_volume(lefts[k], rights[k], p, cost, stream)
        g = gc.graph_build(p, cost, ws, stream)
        st = gc.maxflow_solve(g, opts, stream)
        gc.extract_labels(g, cost, labels, result, stream)
        return st

    _log(f"{args.pairs} pairs resident; {args.warmup} warm-up steps")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    lat = []
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        stats.append(step(i).as_dict())
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    elapsed = t1 - t0
    _log(f"{args.steps} timed steps: {1e3 * elapsed / args.steps:.3f} ms/step")
    pushes = sum(s["pushes"] for s in stats)
    ms_per_step = 1e3 * elapsed / args.steps
    lat_ms = np.array(lat) * 1e3

    # energy/flow of the last step and of the first pair, for the record
    r = result.cpu().numpy()
    last_pair = (args.steps - 1) % len(pairs)
    err, pct = sg.eq2_error(pairs[last_pair].gt, labels.cpu().numpy())

    roof = None
    if not args.no_timing:
        roof = roofline_block(stats, nodes, f"{spec.w}x{spec.h}x{spec.m}", True,   # fused sweeps (the default)
                              gc.footprint_bytes(p), args.steps)

    # pairwise-term variants on the same pairs (Fig. 6 compares inhibit 0 and
    # 1023; the vertical pairs' inhibit is a reading of Sec. 3): exact cuts,
    # quality by eq. (2) against the generated truth
    variants = {}
    if "variants" in args.sec:
        for name, (pen, inh_h, inh_v) in (("inhibit_1023", (args.lam, 1023, 1023)),
                                          ("inhibit_0", (args.lam, 0, 0)),
                                          ("inhibit_horizontal_only", (args.lam, 1023, 0))):
            pv = gc.problem(spec.w, spec.h, spec.m, spec.cap, pen, inh_h, pen, inh_v)
            lat_v, errs, pcts = [], [], []
            for i in range(len(pairs) + 1):
                k = i % len(pairs)
                torch.cuda.synchronize()
                a = time.perf_counter()
                gc.stereo_cost_volume(lefts[k], rights[k], pv, cost, stream)
                g = gc.graph_build(pv, cost, ws, stream)
                gc.maxflow_solve(g, None, stream)
                gc.extract_labels(g, cost, labels, result, stream)
                torch.cuda.synchronize()
                if i >= 1:
                    lat_v.append(time.perf_counter() - a)
                    er, pc = sg.eq2_error(pairs[k].gt, labels.cpu().numpy())
                    errs.append(er)
                    pcts.append(pc)
            variants[name] = {"penalty": pen, "inhibit_h": inh_h, "inhibit_v": inh_v,
                              "ms_per_pair": round(1e3 * float(np.median(lat_v)), 3),
                              "eq2_error_mean": round(float(np.mean(errs)), 1),
                              "pct_exact_mean": round(float(np.mean(pcts)), 1)}
            _log(f"variant {name}: {variants[name]['ms_per_pair']} ms/pair, "
                 f"eq2 error {variants[name]['eq2_error_mean']}")

    # the paper's own data term (Sec. 4.3): colour pairs of the same shape,
    # RGB sum of absolute differences, inhibit 1023, a penalty sweep around
    # the paper's 14 and its inhibit-0 comparison (Fig. 6 analogue)
    rgb = {}
    if "rgb" in args.sec:
        rspec = sg.MID_RGB
        rpairs = [sg.make_pair(rspec, (2, i)) for i in range(args.pairs)]
        rl = [torch.from_numpy(q.left).to(dev) for q in rpairs]
        rr = [torch.from_numpy(q.right).to(dev) for q in rpairs]
        for pen, inh in ((4, 1023), (8, 1023), (14, 1023), (20, 1023), (14, 0)):
            pv = gc.problem(rspec.w, rspec.h, rspec.m, rspec.cap, pen, inh)
            lat_v, errs, pcts = [], [], []
            for i in range(len(rpairs) + 1):
                k = i % len(rpairs)
                torch.cuda.synchronize()
                a = time.perf_counter()
                gc.stereo_cost_volume_rgb(rl[k], rr[k], pv, cost, stream)
                g = gc.graph_build(pv, cost, ws, stream)
                gc.maxflow_solve(g, None, stream)
                gc.extract_labels(g, cost, labels, result, stream)
                torch.cuda.synchronize()
                if i >= 1:
                    lat_v.append(time.perf_counter() - a)
                    er, pc = sg.eq2_error(rpairs[k].gt, labels.cpu().numpy())
                    errs.append(er)
                    pcts.append(pc)
            key = f"penalty_{pen}_inhibit_{inh}"
            rgb[key] = {"ms_per_pair": round(1e3 * float(np.median(lat_v)), 3),
                        "eq2_error_mean": round(float(np.mean(errs)), 1),
                        "pct_exact_mean": round(float(np.mean(pcts)), 1)}
            _log(f"rgb {key}: {rgb[key]['ms_per_pair']} ms/pair, eq2 error {rgb[key]['eq2_error_mean']}")

    # the paper's approximate cuts (Sec. 4.5) and the warm-started exact cut,
    # beside the exact cut, on the headline pairs and on 450x375x64 pairs
    approx = approx_large = approx_paper = None
    if "approx" in args.sec:
        approx = bench_approx(gc, sg, torch, spec, pairs, lefts, rights, max(4, args.steps // 4),
                              stream, dev, args.lam)
        lspec = sg.LARGE
        lp = [sg.make_pair(lspec, (3, i)) for i in range(2)]
        approx_large = bench_approx(gc, sg, torch, lspec, lp, [torch.from_numpy(q.left).to(dev) for q in lp],
                                    [torch.from_numpy(q.right).to(dev) for q in lp], 2, stream, dev, 1)
        # the paper's own cuboid (Sec. 4.1, Table 2): 372 gaze lines x 288 rows
        # x 24 depth numbers, colour sum of absolute differences, penalty 14,
        # inhibit 1023, on seeded synthetic colour pairs of that shape
        pspec = sg.spec_like(sg.MID_RGB, 372, 288, 24)
        pp = [sg.make_pair(pspec, (8, i)) for i in range(4)]
        approx_paper = bench_approx(gc, sg, torch, pspec, pp, [torch.from_numpy(q.left).to(dev) for q in pp],
                                    [torch.from_numpy(q.right).to(dev) for q in pp], 4, stream, dev, pspec.lam)
        approx_paper["paper_table2_gtx1080_ms"] = {"exact": 122, "level1_b2": 14, "level1_b3": 14, "level2_b3": 5}
        torch.cuda.empty_cache()

    # the larger configurations, whose state does not fit the Infinity Cache:
    # 450x375 pairs with 64 depth numbers (12 slanted planes, 10 % textureless)
    # and the 640x480x64 class of the batched mix; exact solves, default
    # options, kernel time sampled as in the headline steps
    larger = {}
    if "larger" in args.sec:
        for key, lspec, seed0 in (("450x375x64", sg.LARGE, 3),
                                  ("640x480x64", sg.spec_like(sg.MID, 640, 480, 64), 5)):
            if key not in args.larger_shapes.split(","):
                continue
            larger[key] = bench_larger(args, gc, torch, sg, lspec, seed0, stream, dev)
            _log(f"larger pair {key}: {larger[key]['ms_per_pair']} ms/pair")
        torch.cuda.empty_cache()

    calib = None
    if args.copy_calibration:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # calibrates the counters that give the solve kernels' HBM traffic
        src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        calib = {"copy_bytes": src.numel() * 4, "copies": 5}
        del src, dst

    batch = bench_batch(args, gc, sg, torch) if "batch" in args.sec else None
    serving = serving_low = None
    if "serving" in args.sec:
        serving = bench_serving(args, gc, sg, torch, args.serve_rate, args.serve_requests)
        if args.serve_low_rate > 0:
            serving_low = bench_serving(args, gc, sg, torch, args.serve_low_rate,
                                        args.serve_low_requests)

    cpu = None
    parity = None
    if "cpu" in args.sec:
        import oracle
        n = max(1, args.cpu_sample)
        t = 0.0
        ok = True
        for i in range(n):
            q = pairs[i % len(pairs)]
            a = time.perf_counter()
            c = oracle.cost_volume(q.left, q.right, spec.m, spec.cap)
            lab, flow, energy = oracle.solve(c, args.lam, spec.inhibit)
            t += time.perf_counter() - a
            # the GPU result for the same pair
            gc.stereo_cost_volume(lefts[i % len(pairs)], rights[i % len(pairs)], p, cost, stream)
            g = gc.graph_build(p, cost, ws, stream)
            gc.maxflow_solve(g, None, stream)
            gc.extract_labels(g, cost, labels, result, stream)
            rr = result.cpu().numpy()
            ok = ok and int(rr[0]) == energy and int(rr[1]) == flow and \
                bool((labels.cpu().numpy() == lab).all())
        _log(f"cpu oracle: {n} pairs in {t:.1f} s")
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": round(n / t, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "host": {"cpus_visible": os.cpu_count(), "model": model},
               "sample": f"{n} pairs of the same 384x288x16 workload (seeds (2,0..{n - 1})), "
                         f"cost volume + graph + FIFO push-relabel max-flow + labels, "
                         f"single-threaded C -O2"}
        parity = {"pairs_checked": n, "bit_exact": ok}

    out = {
        "metric": METRIC,
        "value": round(args.steps / elapsed, 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "384x288 grayscale pair, 16 depth numbers, seeded 6-10 slanted "
                               "planes, sigma 3, truncated AD cap 30, penalty "
                               f"{args.lam}, inhibit 1023, exact min cut",
                   "width": spec.w, "height": spec.h, "labels": spec.m, "nodes": nodes,
                   "pairs_cycled": len(pairs)},
        "ms_per_pair_p50": round(float(np.percentile(lat_ms, 50)), 3),
        "ms_per_pair_p99": round(float(np.percentile(lat_ms, 99)), 3),
        "medge_pushes_per_s": round(pushes / elapsed / 1e6, 2),
        "sweeps_per_pair": round(sum(s["sweeps"] for s in stats) / args.steps, 2),
        "global_relabels_per_pair": round(sum(s["global_relabels"] for s in stats) / args.steps, 2),
        "bfs_passes_per_pair": round(sum(s["bfs_passes"] for s in stats) / args.steps, 2),
        "energy_last": int(r[0]), "flow_last": int(r[1]),
        "eq2_error_last": err, "pct_exact_last": pct,
        "approx": approx,
        "approx_450x375x64": approx_large,
        "approx_372x288x24_rgb": approx_paper,
        "pairwise_variants": variants or None,
        "larger_pair": larger.get("450x375x64"),
        "larger_640x480x64": larger.get("640x480x64"),
        "rgb_sad": ({"workload": "384x288 colour pairs, 16 depth numbers, RGB sum of absolute "
                                 "differences (untruncated), seeds (2, 0..7)", **rgb} if rgb else None),
        "copy_calibration": calib,
        "batch": batch,
        "serving": serving,
        "serving_below_capacity": serving_low,
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
