#!/usr/bin/env python3
"""Throughput of the MI355X guided extension aligner.

Default workload (--workload ont): the ONT-like batch -- 100,000 seeded
synthetic pairs, target length clip(round(LogNormal(ln 2000, 0.8)), 1, 20000),
query = target with 10% errors (subst:ins:del 1:1:1), 0.1% N bases scored -1,
scoring a=2 b=4 q=4 e=2 q2=24 e2=1, band w=751, z-drop Z=400. The real
long-read datasets the paper measures on (GIAB reads after Minimap2 seeding)
are not available; these pairs stand in for them. --workload longread (20k
HiFi-like pairs, w=2000) and --workload mixed (1M heavy-tailed pairs) measure
the other two stand-in workloads.

One step = one ga_align_batch call over the whole batch: base unpacking,
pair planning and the anti-diagonal sweep with z-drop for every pair. Inputs
are packed and resident in HBM before the timed region starts.

Prints one JSON line: GCUPS = algorithmic in-band cells up to each pair's
termination anti-diagonal, per second. The line also gives the median device
time of one step and, measured after the timed steps and not part of
`value`, the end-to-end time from host ASCII (upload, packing, alignment,
results back to the host).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (seqgen workload, description)
    "ont": ("ont", "ONT-like batch: 100k pairs, target LogNormal(median 2 kb, sigma 0.8) capped at 20 kb, "
               "10% errors 1:1:1, 0.1% N scored -1, a=2 b=4 q=4 e=2 q2=24 e2=1, w=751, Z=400, seed 0"),
    "longread": ("longread", "HiFi-like long reads: 20k pairs, target U{10000..25000}, 1% errors 1:1:1 plus 1-3 "
                    "indels of U{50..500} bp, a=2 b=4 q=4 e=2 q2=24 e2=1, w=2000, Z=5000, seed 0"),
    "uniform": ("uniform", "uniform: 500 pairs, target U{100..1000}, 5% errors 2:1:1, a=2 b=4 q=4 e=2 q2=24 "
                           "e2=1, w=500, Z=400, seed 0"),
    "mixed": ("mix", "heavy-tailed mix: 1M pairs, target min(50000, 50 U^(-1/1.5)), 8% errors 1:1:1, 20% of "
                 "queries with a U{2000..5000} random insert, a=2 b=4 q=4 e=2 q2=24 e2=1, w=751, Z=400, "
                 "seed 0"),
}

E2E_RUNS = 3                # end-to-end repetitions after the timed steps (median reported)
OPS_PER_CELL = 16           # int32 VALU lane-ops per cell (the roofline convention)
PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # int32 lane-ops/s: CUs x SIMDs x lanes x clock
DOMINANT_KERNEL_SRC = os.path.join(ROOT, "paper_2403_06478_amd", "csrc", "ga_kernels.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "ga_dp_kernel_k24_ont100k_pmc.md")


def log(msg: str):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def kernel_source_hash() -> str:
    with open(DOMINANT_KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from a committed
    rocprofv3 --pmc summary, or None if there is none for them or the kernel
    source changed since it was taken."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m = re.search(r"kernel:\s*(\S+)", text)
    if not m or m.group(1) != kernel:
        return None
    m = re.search(r"workload:\s*(\S+)", text)
    if not m or m.group(1) != workload:
        return None
    m = re.search(r"source_sha256_16:\s*([0-9a-f]{16})", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    return float(m.group(1)) if m else None


def cpu_threads():
    """Host threads for the oracle baseline: every CPU this process may run
    on, capped at the CPU share the job was given (OMP_NUM_THREADS, when
    set). Returns (threads, CPUs the host reports)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS")
    threads = avail
    if share and share.isdigit() and int(share) > 0:
        threads = min(avail, int(share))
    return max(1, threads), os.cpu_count() or avail


def cpu_baseline(batch, n_sample: int):
    import numpy as np

    import oracle
    cores, host_cpus = cpu_threads()
    sub = batch.subset(np.arange(min(n_sample, batch.n_pairs)))
    oracle.build(force=True, native=True)  # -O3 -march=native for this host
    log(f"cpu baseline: oracle (-O3 -march=native) on {sub.n_pairs} pairs, {cores} threads "
        f"({host_cpus} CPUs on the host)")
    t0 = time.perf_counter()
    _, cells = oracle.align_batch(sub, nthreads=cores, native=True)
    dt = time.perf_counter() - t0
    # one thread on a sixteenth of the sample (about as long again)
    one = sub.subset(np.arange(max(1, sub.n_pairs // 16)))
    t0 = time.perf_counter()
    _, cells1 = oracle.align_batch(one, nthreads=1, native=True)
    dt1 = time.perf_counter() - t0
    return {"value": round(float(cells.sum()) / dt / 1e9, 4), "unit": "GCUPS", "cores": cores,
            "host_cpus": host_cpus, "kind": "oracle", "build": "gcc -O3 -march=native",
            "sample": f"first {sub.n_pairs} pairs of the benchmark batch "
                      f"({int(cells.sum())} cells, {dt:.1f} s)",
            "one_core": {"value": round(float(cells1.sum()) / dt1 / 1e9, 4),
                         "sample": f"first {one.n_pairs} pairs ({int(cells1.sum())} cells, {dt1:.1f} s)"}}


def batching_comparison(ctx, steps: int = 3):
    """The heavy-tailed 1M-pair mix under the persistent schedule (this
    context's class order) and the plain per-length-bucket launches: median
    step time of `steps` timed calls each after one warm-up, GCUPS from the
    algorithmic cells, and the two schedules' results compared pair by
    pair."""
    import numpy as np
    import torch

    import paper_2403_06478_amd as ga
    import seqgen

    wid, wdesc = WORKLOADS["mixed"]
    batch = seqgen.make_workload(wid)
    packed = ga.pack_batch(ctx, batch)
    stream = torch.cuda.current_stream()
    res, ms = {}, {}
    for sched in ("persistent", "bucketed"):
        ctx.set_schedule(sched)
        out = torch.empty((batch.n_pairs, 7), dtype=torch.int32, device="cuda")
        ga.ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop, out=out, stream=stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ga.ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop, out=out, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ctx.check()
        res[sched] = out.cpu().numpy()
        ms[sched] = float(np.median(times))
        log(f"batching: {sched} {[round(t, 2) for t in times]} ms")
    ctx.set_schedule("persistent")
    same = bool(np.array_equal(res["persistent"], res["bucketed"]))
    if not same:
        raise RuntimeError("persistent and bucketed schedules gave different results on the mix")
    cells = int(ga.count_cells(batch.t_len, batch.q_len, batch.w, res["persistent"]).sum())
    del packed
    torch.cuda.empty_cache()
    g = {k: cells / (v / 1e3) / 1e9 for k, v in ms.items()}
    return {"workload": wdesc, "pairs": batch.n_pairs, "cells": cells, "steps": steps,
            "persistent_ms": round(ms["persistent"], 3), "bucketed_ms": round(ms["bucketed"], 3),
            "persistent_gcups": round(g["persistent"], 3), "bucketed_gcups": round(g["bucketed"], 3),
            "speedup": round(ms["bucketed"] / ms["persistent"], 3), "same_results": same,
            "statistic": "median device time per call (HIP events)"}


def serving_summary(duration_s: float):
    """Serving at 0.5 and 0.8 of the server's saturated throughput (the
    serving workload, native host loop, captured graphs): p50/p99 per rate
    for short and long requests, every result checked against the offline
    batch. Runs as a child process with a HIP runtime of its own: the
    streams this process already made would share the GPU's few hardware
    queues with the server's slot streams and serialise its batches."""
    import subprocess

    cmd = [sys.executable, "-u", "-m", "paper_2403_06478_amd.serve", "--requests", "20000",
           "--rates", "0.5", "0.8", "--duration", str(duration_s)]
    log(f"serving: {' '.join(cmd[2:])}")
    res = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True)
    for line in res.stderr.splitlines():
        if line.startswith("[serve]"):
            log(line)
    if res.returncode != 0:
        raise RuntimeError(f"serving benchmark failed ({res.returncode}): {res.stderr[-2000:]}")
    lines = [json.loads(l) for l in res.stdout.splitlines() if l.startswith("{")]
    keep = ("rate_of_capacity", "qps", "requests", "served_req_per_s", "p50_ms", "p99_ms", "p50_short_ms",
            "p99_short_ms", "p50_long_ms", "p99_long_ms", "gcups", "same_as_offline")
    return {"workload": lines[0]["workload"], "capacity_req_per_s": lines[0]["capacity_req_per_s"],
            "offline_gcups": lines[0]["offline_gcups"], "saturated_gcups": lines[0]["saturated_gcups"],
            "duration_s_per_rate": duration_s, "host_loop": lines[0]["host_loop"], "graphs": lines[0]["graphs"],
            "latency": "arrival to results visible on the host", "rates": [{k: l[k] for k in keep} for l in lines]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="ont",
                    help="ont (the headline batch, default), longread, mixed or uniform")
    ap.add_argument("--schedule", choices=["persistent", "bucketed"], default="persistent",
                    help="persistent (default) or the plain per-length-bucket launches, for comparison")
    ap.add_argument("--lanes", type=int, default=None,
                    help="streams the class launches spread over (1..4; default: the library's)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default class order instead of the measured one")
    ap.add_argument("--pairs", type=int, default=None, help="fewer pairs (profiling runs only)")
    ap.add_argument("--cpu-sample", type=int, default=8000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-end-to-end", action="store_true",
                    help="skip the end-to-end runs after the timed steps (profiling runs)")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the persistent-vs-bucketed comparison on the 1M-pair mix")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving latency runs")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-captured replays")
    ap.add_argument("--serving-seconds", type=float, default=8.0,
                    help="seconds of Poisson arrivals per serving rate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device copy (scales rocprofv3 byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}): pairs are "
              f"independent and would be split across GPUs with no exchange; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2403_06478_amd as ga
    import seqgen

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)
    wid, wdesc = WORKLOADS[args.workload]
    log(f"generating workload '{args.workload}'")
    batch = seqgen.make_workload(wid, n_pairs=args.pairs)
    ctx = ga.Context(0)
    ctx.set_schedule(args.schedule)
    if args.lanes is not None:
        ctx.set_lanes(args.lanes)
    class_cost = None
    if not args.no_autotune:
        # set-up, outside the timed steps: measure each kernel class, then
        # every pair takes the cheapest class that runs it
        class_cost = ctx.autotune()
        order = sorted(range(len(ga.CLASSES)), key=lambda c: class_cost[c])
        log("autotuned class costs (ns per pair and anti-diagonal): " +
            ", ".join(f"{ga.class_name(c)} {class_cost[c]:.3f}" for c in order))
    packed = ga.pack_batch(ctx, batch)
    out = torch.empty((batch.n_pairs, 7), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    ctx.check()
    stream = torch.cuda.current_stream()
    log(f"packed {batch.n_pairs} pairs, {int(batch.t_len.sum() + batch.q_len.sum())} bases; warmup {args.warmup}")
    for _ in range(args.warmup):
        ga.ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop, out=out, stream=stream)
    torch.cuda.synchronize()
    ctx.check()

    ctx.set_timing(True)
    stage_ms = []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        ga.ga_align_batch(ctx, packed, batch.scoring, batch.w, batch.zdrop, out=out, stream=stream)
        ev[k][1].record(stream)
        stage_ms.append(ctx.timing())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(False)
    ctx.check()
    elapsed = t1 - t0
    ms_per_step = elapsed / args.steps * 1e3
    step_ms = [a.elapsed_time(b) for a, b in ev]
    log(f"{ms_per_step:.2f} ms per step (device time per step: median {np.median(step_ms):.2f} ms; "
        f"steps {[round(x, 2) for x in step_ms]})")

    # the same call captured into one HIP graph and replayed (outside the
    # timed steps above; every replay's results are compared with them)
    graph = None
    if not args.no_graph:
        gs = torch.cuda.Stream()
        gout = torch.empty_like(out)
        torch.cuda.synchronize()
        g = ga.AlignGraph(ctx, packed, batch.scoring, batch.w, batch.zdrop, gout, gs)
        g.launch(gs)
        gs.synchronize()
        gms = []
        for _ in range(args.steps):
            a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(gs)
            g.launch(gs)
            b2.record(gs)
            gs.synchronize()
            gms.append(a.elapsed_time(b2))
        ctx.check()
        same = bool(torch.equal(gout, out))
        g.close()
        if not same:
            raise RuntimeError("graph replays gave results different from the timed steps")
        graph = {"steps": args.steps, "ms_median": round(float(np.median(gms)), 3),
                 "eager_ms_median": round(float(np.median(step_ms)), 3),
                 "saved_ms": round(float(np.median(step_ms) - np.median(gms)), 3), "same_results": same}
        log(f"graph replay: median {graph['ms_median']} ms per call (eager {graph['eager_ms_median']} ms)")

    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 536870912 bytes read + 536870912 bytes written")
        del src, dst

    res = out.cpu().numpy()

    # End to end, outside the timed steps: host ASCII uploaded from pageable
    # memory, packed on the device, aligned, results copied back to the host.
    e2e_ms = []
    for _ in range(0 if args.no_end_to_end else E2E_RUNS):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        pk = ga.pack_batch(ctx, batch, stream)
        host = ga.ga_align_batch(ctx, pk, batch.scoring, batch.w, batch.zdrop, stream=stream).cpu().numpy()
        e2e_ms.append((time.perf_counter() - ta) * 1e3)
        del pk
        if not np.array_equal(host, res):
            raise RuntimeError("end-to-end run gave results different from the timed steps")
    ctx.check()
    if e2e_ms:
        log(f"end to end (upload, pack, align, results to host): median {np.median(e2e_ms):.2f} ms")

    t_len, q_len = batch.t_len, batch.q_len
    cells = ga.count_cells(t_len, q_len, batch.w, res)
    # the class each pair ran in (this context's autotuned order)
    cls = np.array([ctx.pair_class(int(n), int(m), batch.w, batch.n_pairs) for n, m in zip(t_len, q_len)])
    total_cells = int(cells.sum())
    gcups = total_cells / (ms_per_step / 1e3) / 1e9
    e2e_ms_med = float(np.median(e2e_ms)) if e2e_ms else None
    pairs_per_s = batch.n_pairs / (ms_per_step / 1e3)

    stage = np.array(stage_ms)  # [steps, 1 + classes]
    mean_ms = stage.mean(axis=0)
    # the dominant kernel is the class that computed the most cells (the
    # classes' launches overlap on several streams, so an empty launch can
    # span another class's run while it waits for the GPU)
    per_class = np.array([int(cells[cls == c].sum()) for c in range(len(ga.CLASSES))])
    dom = int(np.argmax(per_class))
    dom_cells = int(per_class[dom])
    achieved = OPS_PER_CELL * dom_cells / (mean_ms[1 + dom] / 1e3) / 1e12
    traffic = read_traffic(ga.class_name(dom), args.workload)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / PEAK_TOPS, 4), "traffic": traffic,
                "kernel": ga.class_name(dom),
                "kernel_ms": round(float(mean_ms[1 + dom]), 3),
                "kernel_cells": dom_cells, "ops_per_cell": OPS_PER_CELL}
    log(f"stages ms (prep, then {', '.join(ga.class_name(c) for c in range(len(ga.CLASSES)))}): "
        f"{[round(float(x), 3) for x in mean_ms]}")

    measured_peak = ctx.calibrate_valu(stream) / 1e12
    roofline["peak_measured"] = round(measured_peak, 2)
    roofline["frac_measured"] = round(achieved / measured_peak, 4)
    log(f"measured int32 VALU peak {measured_peak:.2f} T lane-ops/s")

    batching = None
    if not args.no_batching:
        batching = batching_comparison(ctx)
        log(f"batching: persistent {batching['persistent_gcups']} GCUPS, bucketed "
            f"{batching['bucketed_gcups']} GCUPS ({batching['speedup']}x)")
    serving = None
    if not args.no_serving:
        serving = serving_summary(args.serving_seconds)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch, args.cpu_sample)

    line = {
        "metric": "GCUPS",
        "value": round(gcups, 3),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wdesc, "schedule": args.schedule,
                   "class_choice": "autotuned" if class_cost is not None else "default order",
                   "pairs": batch.n_pairs, "w": batch.w, "Z": batch.zdrop,
                   "cells": total_cells, "zdropped": int(res[:, 6].sum())},
        "pairs_per_s": round(pairs_per_s, 1),
        "step_ms_median": round(float(np.median(step_ms)), 3),
        "end_to_end": None if e2e_ms_med is None else {
            "ms_median": round(e2e_ms_med, 3), "runs": E2E_RUNS,
            "gcups": round(total_cells / (e2e_ms_med / 1e3) / 1e9, 3),
            "pairs_per_s": round(batch.n_pairs / (e2e_ms_med / 1e3), 1),
            "includes": "host ASCII upload (pageable), packing kernel, alignment, results to host"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "graph": graph,
        "batching": batching,
        "serving": serving,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
