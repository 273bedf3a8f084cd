#!/usr/bin/env python3
"""Benchmark of the Log(Graph) packed-graph hot path on one MI355X.

One step = encode the graph (validate, widths, scan, pack, offsets; with the
degree relabeling for the Kronecker workloads), BFS from 64 roots
(direction-optimizing, depths and parents; one library call, which runs a few
roots at a time) and 20 PageRank iterations, all on the packed
representation, inputs resident in HBM.  The same step runs on the plain
uint32 CSR (same labeling) for the packed/plain comparison.

Default workload: uniform random (Erdos-Renyi) scale 26, edge factor 16,
seed 1 (n = 2^26, about 2.1e9 stored entries), 26-bit packed IDs and offsets
packed at bl(M) bits -- the largest configuration that fits one GPU.

Throughput is counted in undirected traversed edges (Graph500 convention):
BFS from root r counts half the degree sum of the vertices it reaches; one
PageRank iteration counts every undirected edge once.  `value` = those edges
per second over the whole step (encode included); detail.gteps_traversal
leaves the encode out (BFS and PageRank only), and detail.per_root gives the
Graph500-style per-root rates (one root per call): harmonic mean, median and
its nonparametric 95% confidence interval, p50/p99 latency.

Parity is checked before anything is timed, for both layouts: whole BFS
trees (depths and parents) of two roots against the oracle, the multi-root
call's rows against single-root calls, and the first PageRank iteration
within L1 1e-5 of the FP64 oracle (plus the 20-iteration sum).  The oracle
is also timed on the host's cores (cpu_baseline).  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS & HBM GB/s, Log(Graph)-packed vs plain CSR on GPU; p99 query latency"

WORKLOADS = {
    # name: (generator, scale, encoding)
    "er-s26-global-packed": ("er", 26, dict(ids="global", offsets="packed", relabel=False)),
    "kronecker-s24-dm-local-ef": ("kronecker", 24, dict(ids="local", offsets="succinct", relabel=True)),
    "kronecker-s16-global-packed": ("kronecker", 16, dict(ids="global", offsets="packed", relabel=False)),
    "kronecker-s20-dm-local-ef": ("kronecker", 20, dict(ids="local", offsets="succinct", relabel=True)),
    "er-s22-global-packed": ("er", 22, dict(ids="global", offsets="packed", relabel=False)),
}
DEFAULT_WORKLOAD = "er-s26-global-packed"

# sources whose kernels a committed counter summary describes (a summary
# holds their hash; it no longer applies once they change)
COUNTER_SOURCES = {
    "pr": ["lg_pagerank.hip", "lg_pagerank_pb.hip", "lg_device.hpp", "lg_views.hpp", "lg_heavy.hip",
           "lg_varint.hpp"],
    "bfs": ["lg_bfs.hip", "lg_device.hpp", "lg_views.hpp"],
    "bfsall": ["lg_bfs.hip", "lg_device.hpp", "lg_views.hpp"],
}


# the kernels of one PageRank iteration: the pull (iteration kernel plus the
# sum of cut lists) or propagation blocking (two binning levels and the
# accumulation)
PR_KERNELS = ["pr_iter_kernel", "pr_segmented_kernel", "pb_bin1_kernel", "pb_bin2_kernel", "pb_accum_kernel"]


# counter passes of a counter summary: each runs the same counter-run
# command under rocprofv3 --pmc with these counters (at most 4 TCC counters
# per pass)
COUNTER_PASSES = {
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE"],
    "rdreq": ["TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum"],
    "wrreq": ["TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_WRREQ_DRAM_sum"],
}
COUNTER_KERNEL_REGEX = "sqrt|cos|lg::"


def counters_path(workload: str, layout: str, phase: str) -> str:
    return os.path.join(ROOT, "profiles", f"counters_{workload}_{layout}_{phase}.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(phase: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in COUNTER_SOURCES[phase]:
        with open(os.path.join(ROOT, "paper_2010_15879_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(key: str, workload: str, layout: str, phase: str):
    """A figure of the committed counter summary profiles/counters_<workload>_
    <layout>_<phase>.md (`traffic_bytes_per_launch.<kernel>`: HBM bytes per
    launch, FETCH_SIZE + WRITE_SIZE calibrated; `traffic_bytes_per_phase`),
    or None when there is none or the sources changed since."""
    path = counters_path(workload, layout, phase)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path).read().splitlines():
        if ": " in line and not line.startswith(("#", "|", "`", "-")):
            k, v = line.split(": ", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_hash(phase):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def _kernel_key(name: str) -> str:
    """Base name of a kernel in a trace ("void lg::pb_bin1_kernel<lg::PlainAcc<
    false>, true>(...)" -> "pb_bin1_kernel[count]" for the counting instance)."""
    base = name.split("(")[0]
    tmpl = base[base.find("<"):] if "<" in base else ""
    base = base.split("<")[0].replace("void ", "").strip()
    base = base.split("::")[-1]
    if base == "pb_bin1_kernel" and tmpl.rstrip(">").rstrip().endswith("true"):
        base += "[count]"
    return base


def counter_summary_main(args):
    """Summary of one counter-run under the passes of COUNTER_PASSES: the
    calibration factors (what each counter reads for the elementwise kernel
    of known bytes), each phase kernel's bytes per launch, and the phase's
    total; written as text with the commands that made it."""
    import csv
    import statistics
    d = args.counter_summary
    run = json.loads(open(os.path.join(d, "run.json")).read().strip().splitlines()[-1])
    per = {}   # counter -> list of (dispatch, kernel name, value)
    for pas, ctrs in COUNTER_PASSES.items():
        files = [os.path.join(dp, f) for dp, _, fs in os.walk(os.path.join(d, pas)) for f in fs
                 if f.endswith("counter_collection.csv")]
        if not files:
            raise SystemExit(f"counter summary: no counter_collection.csv under {d}/{pas}")
        rows = list(csv.DictReader(open(files[0])))
        for c in ctrs:
            got = sorted((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]))
                         for r in rows if r["Counter_Name"] == c)
            per[c] = got
    def split(c):
        rows = per[c]
        cal = [v for _, k, v in rows if "sqrt" in k]
        marks = [i for i, (_, k, _) in enumerate(rows) if "cos" in k and "lg::" not in k]
        phase = rows[marks[-1] + 1:] if marks else []
        return cal, phase
    cal_bytes = run["calibration_bytes"] // 2   # read = written = half
    factor, cal_raw = {}, {}
    for c in per:
        cal, _ = split(c)
        cal_raw[c] = statistics.median(cal) if cal else float("nan")
    # bytes each counter set gives for the calibration kernel
    rd_req = lambda x: 32 * x["TCC_EA0_RDREQ_32B_sum"] + 64 * x["TCC_EA0_RDREQ_64B_sum"] + \
        128 * x["TCC_EA0_RDREQ_128B_sum"]  # noqa: E731
    wr_req = lambda x: 64 * x["TCC_EA0_WRREQ_64B_sum"] + 32 * (x["TCC_EA0_WRREQ_sum"] - x["TCC_EA0_WRREQ_64B_sum"])  # noqa: E731
    factor["FETCH_SIZE"] = cal_bytes / (cal_raw["FETCH_SIZE"] * 1024.0)
    factor["WRITE_SIZE"] = cal_bytes / (cal_raw["WRITE_SIZE"] * 1024.0)
    factor["rdreq"] = cal_bytes / rd_req(cal_raw)
    factor["wrreq"] = cal_bytes / wr_req(cal_raw)
    # phase dispatches, kernel by kernel (the passes run the same launches in
    # the same order)
    phase = {c: split(c)[1] for c in per}
    nd = {c: len(v) for c, v in phase.items()}
    if len(set(nd.values())) != 1:
        raise SystemExit(f"counter summary: passes saw different phase dispatch counts {nd}")
    kernels = {}
    for i in range(next(iter(nd.values()))):
        name = phase["FETCH_SIZE"][i][1]
        x = {c: phase[c][i][2] for c in per}
        rec = kernels.setdefault(_kernel_key(name), [])
        rec.append(dict(fetch=x["FETCH_SIZE"] * 1024.0 * factor["FETCH_SIZE"],
                        write=x["WRITE_SIZE"] * 1024.0 * factor["WRITE_SIZE"],
                        rdreq=rd_req(x), wrreq=wr_req(x),
                        r32=x["TCC_EA0_RDREQ_32B_sum"], r64=x["TCC_EA0_RDREQ_64B_sum"],
                        r128=x["TCC_EA0_RDREQ_128B_sum"], rdram=x["TCC_EA0_RDREQ_DRAM_sum"],
                        rtot=x["TCC_EA0_RDREQ_sum"]))
    m = run["stored_edges"]
    phase_name = {"pr": f"one PageRank call of {run['pr_iters']} iterations (with its first-call setup)",
                  "bfs": f"single-root BFS, modes {run.get('bfs_modes')}",
                  "bfsall": f"BFS from all {run.get('roots')} roots in one call (the call the benchmark times)"}[
                      run["phase"]]
    # the passes' directory as given, relative to the repository root
    cdir = os.path.relpath(os.path.abspath(args.counter_summary), ROOT)
    cmd_of = lambda pas: (f"timeout -s KILL 300 rocprofv3 --pmc {' '.join(COUNTER_PASSES[pas])} "  # noqa: E731
                          f"--kernel-include-regex \"{COUNTER_KERNEL_REGEX}\" --output-format csv "
                          f"-d {cdir}/{pas} -o {pas} -- "
                          f"python3 bench.py --workload {args.workload} --counter-run {run['phase']} "
                          f"--layout {args.layout} --pr-iters {run['pr_iters']} --bfs-modes {run.get('bfs_modes')}")
    out = []
    out.append(f"# HBM traffic by kernel: {args.workload}, {args.layout} layout, {phase_name}")
    out.append("")
    out.append("Commands (from the repository root, one MI355X, one pass per counter set; then this summary):")
    out.append("")
    out.append("```")
    out.append("cd /tmp && export TMPDIR=/tmp   # then back in the repository root for the runs")
    for pas in COUNTER_PASSES:
        out.append(cmd_of(pas))
    out.append(f"python3 bench.py --workload {args.workload} --counter-run {run['phase']} --layout {args.layout} "
               f"--pr-iters {run['pr_iters']} --bfs-modes {run.get('bfs_modes')} > {cdir}/run.json")
    out.append(f"python3 bench.py --workload {args.workload} --layout {args.layout} --counter-summary "
               f"{cdir} --summary-out "
               f"profiles/counters_{args.workload}_{args.layout}_{run['phase']}.md")
    out.append("```")
    out.append("")
    out.append(f"n = {run['n']}, stored entries m = {m}; structure bytes {run['structure_bytes']:.0f}.  "
               "The calibration kernel is torch.sqrt over 2^28 floats (reads 1 GiB, writes 1 GiB); "
               "a one-element cos kernel marks where the phase begins.")
    out.append("")
    out.append("| counter set | calibration reads | factor to true bytes |")
    out.append("|---|---:|---:|")
    out.append(f"| FETCH_SIZE (KiB) | {cal_raw['FETCH_SIZE']:.1f} | {factor['FETCH_SIZE']:.4f} |")
    out.append(f"| WRITE_SIZE (KiB) | {cal_raw['WRITE_SIZE']:.1f} | {factor['WRITE_SIZE']:.4f} |")
    out.append(f"| 32/64/128 B read requests (bytes) | {rd_req(cal_raw):.0f} | {factor['rdreq']:.4f} |")
    out.append(f"| 32/64 B write requests (bytes) | {wr_req(cal_raw):.0f} | {factor['wrreq']:.4f} |")
    out.append("")
    out.append("Per kernel (medians over its launches; bytes calibrated; read requests by size as counted):")
    out.append("")
    out.append("| kernel | launches | read B/launch | written B/launch | read B from request sizes | "
               "128 B / 64 B / 32 B read requests (% ) | DRAM share of reads | total B (all launches) |")
    out.append("|---|---:|---:|---:|---:|---|---:|---:|")
    total = 0.0
    med = lambda recs, k: statistics.median(r[k] for r in recs)  # noqa: E731
    for k, recs in sorted(kernels.items(), key=lambda kv: -sum(r["fetch"] + r["write"] for r in kv[1])):
        tot = sum(r["fetch"] + r["write"] for r in recs)
        total += tot
        rq = sum(r["rtot"] for r in recs) or 1.0
        mix = "/".join(f"{100.0 * sum(r[x] for r in recs) / rq:.0f}" for x in ("r128", "r64", "r32"))
        dram = sum(r["rdram"] for r in recs) / rq
        out.append(f"| {k} | {len(recs)} | {med(recs, 'fetch'):.4g} | {med(recs, 'write'):.4g} | "
                   f"{med(recs, 'rdreq'):.4g} | {mix} | {dram:.2f} | {tot:.4g} |")
    out.append("")
    out.append("Machine-readable (bench.py reads these while source_sha256 matches the sources):")
    out.append("")
    for k, recs in sorted(kernels.items()):
        out.append(f"traffic_bytes_per_launch.{k}: {med(recs, 'fetch') + med(recs, 'write'):.0f}")
    out.append(f"traffic_bytes_per_phase: {total:.0f}")
    out.append(f"traffic_bytes_per_stored_entry_per_phase: {total / m:.4f}")
    out.append(f"source_sha256: {run['source_sha256']}")
    out.append("")
    out.append(f"(source_sha256 covers {', '.join(COUNTER_SOURCES[run['phase']])}.)")
    text = "\n".join(out) + "\n"
    if args.summary_out:
        with open(args.summary_out, "w") as fh:
            fh.write(text)
    else:
        sys.stdout.write(text)


def median_ci95(x):
    """Median and the nonparametric 95% confidence interval of the median
    (order statistics of the binomial(n, 1/2) bounds), after dropping the
    first 1% of the samples as warm-up."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    x = x[int(math.ceil(0.01 * x.size)):] if x.size > 1 else x
    s = np.sort(x)
    n = s.size
    lo = int(math.floor((n - 1.96 * math.sqrt(n)) / 2.0))          # 1-based ranks
    hi = int(math.ceil(1 + (n + 1.96 * math.sqrt(n)) / 2.0))
    lo, hi = max(lo, 1), min(hi, n)
    return float(np.median(s)), float(s[lo - 1]), float(s[hi - 1]), n


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    p.add_argument("--roots", type=int, default=64)
    p.add_argument("--pr-iters", type=int, default=20)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="bound on the oracle's timed sample (all-core and one-thread legs together)")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--kernels", action="store_true", help="print the per-kernel time breakdown to stderr")
    p.add_argument("--batch", action="store_true",
                   help="batching configuration: 256 R-MAT graphs (scales 10..18), 16 roots each, one "
                        "persistent graph-captured launch vs one launch per query (own JSON line)")
    p.add_argument("--serve", action="store_true",
                   help="serving configuration: 8 resident graphs (Kronecker and uniform-random scales "
                        "20/22/24/26), Poisson arrivals of 60%% neighbor / 30%% 2-hop / 10%% BFS queries under a "
                        "200 GB budget; saturated queries/s and p50/p99 latency per offered load (own JSON line)")
    p.add_argument("--serve-scales", default="20,22,24,26")
    p.add_argument("--serve-seconds", type=float, default=6.0, help="arrival window per offered load")
    p.add_argument("--relabel-compare", action="store_true",
                   help="the workload's graph under no relabeling, the degree-minimizing relabeling and the greedy "
                        "heuristic (local widths, Elias-Fano offsets): |A|, encode, BFS and PageRank times "
                        "(own JSON line)")
    p.add_argument("--offset-fetch", action="store_true",
                   help="random fetch of 1,000 vertices per worker (256 workers, one call) under each offset "
                        "structure: degrees only and whole lists (own JSON line)")
    p.add_argument("--sssp", action="store_true",
                   help="the workload's graph with uniform integer weights in [1, 255]: SSSP from the roots over "
                        "the weighted plain CSR and the weighted packed encodings, and a sweep of delta "
                        "(own JSON line)")
    p.add_argument("--encoding-compare", action="store_true",
                   help="the workload's graph with local widths, fixed-size gap encoding and Varint lists (full "
                        "labels or differences), with and without the degree-minimizing relabeling (DMf, DMd): "
                        "|A|, encode time, random-vertex list decode, PageRank (own JSON line)")
    p.add_argument("--counter-run", choices=["pr", "bfs", "bfsall"],
                   help="counter-run mode: one elementwise kernel of known traffic (calibration), then one "
                        "PageRank call (pr), one single-root BFS per direction mode in --bfs-modes (bfs) or the "
                        "BFS call from all --roots (bfsall) on --layout, after a one-element cos kernel that marks "
                        "where the phase begins; no timing")
    p.add_argument("--bfs-modes", default="top-down,bottom-up,do",
                   help="counter-run bfs: the direction modes searched, comma separated")
    p.add_argument("--layout", choices=["packed", "plain"], default="packed")
    p.add_argument("--counter-summary", metavar="DIR",
                   help="write the counter summary of --workload, --layout and --counter-run from the rocprofv3 "
                        "CSV output of the passes in DIR/<pass> (passes: " + ", ".join(COUNTER_PASSES) + ") "
                        "and the counter-run's JSON line in DIR/run.json, to --summary-out")
    p.add_argument("--summary-out", default=None, help="counter-summary output file (default: stdout)")
    return p.parse_args()


def calibration_kernel(torch, dev, gib=1):
    """An elementwise kernel that reads and writes `gib` GiB each (square
    root: a kernel the graph generator never launches, so a profiler can pick
    it out by name).  Returns its bytes and time from HIP events."""
    src = torch.ones((gib << 30) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.sqrt(src, out=dst)  # warm
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.sqrt(src, out=dst)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    del src, dst
    torch.cuda.empty_cache()
    ms = sorted(ts)[len(ts) // 2]
    nbytes = 2 * (gib << 30)
    return nbytes, ms


def main():
    args = parse()
    if args.counter_summary:
        return counter_summary_main(args)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              f"(the path runs on a single MI355X and has no multi-GPU sharding)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2010_15879_amd import graphgen as gg
    from paper_2010_15879_amd import lg

    lg.lib()  # fail loudly without the HIP library
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.batch:
        return batch_main(args, np, torch, gg, lg, dev)
    if args.serve:
        return serve_main(args, np, torch, gg, lg, dev)
    gen, scale, enc = WORKLOADS[args.workload]

    t0 = time.time()
    g = (gg.kronecker if gen == "kronecker" else gg.erdos_renyi)(scale, 16, seed=1, device=dev)
    torch.cuda.synchronize()
    roots = gg.pick_roots(g, args.roots, seed=1)
    deg = g.degrees()
    log(f"[bench] graph {args.workload}: n={g.n} M={g.m} isolated={int((deg == 0).sum())} "
        f"maxdeg={int(deg.max())} gen {time.time() - t0:.1f}s")

    n, M = g.n, g.m
    if args.relabel_compare:
        return relabel_main(args, np, torch, lg, g, roots)
    if args.offset_fetch:
        return offset_fetch_main(args, np, torch, lg, g)
    if args.encoding_compare:
        return encoding_main(args, np, torch, lg, g, roots)
    if args.sssp:
        return sssp_main(args, np, torch, gg, lg, g, roots)
    if args.counter_run:
        return counter_main(args, np, torch, lg, g, roots, enc)

    import oracle as orc  # the CPU oracle: test infrastructure, timed below as the CPU baseline

    stream = torch.cuda.current_stream()
    degf = deg.to(torch.float64)
    t0 = time.time()
    off_h = g.row_offsets.cpu().numpy().view(np.uint64)
    col_h = g.col.cpu().numpy().view(np.uint32)
    # the oracle's parent rule needs the stored label of every vertex: the
    # degree permutation's inverse when the graph is relabeled (computed once,
    # outside every timed region)
    labels = orc.dm_permutation(off_h)[1] if enc["relabel"] else None
    threads = orc.max_threads()
    log(f"[bench] host copy {time.time() - t0:.1f}s; oracle threads {threads}")

    # -- the oracle's results every layout is checked against -------------
    t0 = time.time()
    check_roots = [roots[0], roots[-1]]
    orc_trees = [orc.bfs_levels(off_h, col_h, r, labels=labels) for r in check_roots]
    pr1_orc = orc.pagerank_par(off_h, col_h, 0.85, 1)
    log(f"[bench] oracle BFS x{len(check_roots)} + 1 PageRank iteration on {threads} threads: "
        f"{time.time() - t0:.1f}s")

    all_depth = torch.empty((len(roots), n), dtype=torch.int32, device=dev)
    all_parent = torch.empty((len(roots), n), dtype=torch.int32, device=dev)

    def run_step(layout, opts):
        """One step; returns (handle, timings dict, scores).  Times come from
        HIP events on the stream the library launches on."""
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        e0, e1, b1, p1 = ev(), ev(), ev(), ev()
        e0.record(stream)
        h = lg.encode(g.row_offsets, g.col, n, layout=layout, **opts)
        e1.record(stream)
        lg.bfs(h, roots, depth_out=all_depth, parent_out=all_parent)  # all roots in one call
        b1.record(stream)
        pr = lg.pagerank(h, 0.85, args.pr_iters)
        p1.record(stream)
        torch.cuda.synchronize()
        return h, dict(encode=e0.elapsed_time(e1), bfs=e1.elapsed_time(b1), pr=b1.elapsed_time(p1)), pr

    def per_root_ms(h):
        """Graph500-style per-root times: one root per call, one after another."""
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        out = []
        for i, r in enumerate(roots):
            a, b = ev(), ev()
            a.record(stream)
            lg.bfs(h, [r], depth_out=all_depth[i:i + 1], parent_out=all_parent[i:i + 1])
            b.record(stream)
            out.append((a, b))
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) for a, b in out])

    def parity(layout, h, pr20):
        ok = True
        for r, (d0, p0) in zip(check_roots, orc_trees):
            i = roots.index(r)
            d1, p1 = lg.bfs(h, [r])
            torch.cuda.synchronize()
            same = bool(np.array_equal(d1[0].cpu().numpy(), d0) and np.array_equal(p1[0].cpu().numpy(), p0))
            # the multi-root call gives every root the result of a call alone
            rows = bool(torch.equal(all_depth[i], d1[0]) and torch.equal(all_parent[i], p1[0]))
            log(f"[bench] {layout} parity root {r}: tree {'ok' if same else 'FAILED'}, "
                f"multi-root row {'ok' if rows else 'FAILED'}")
            ok = ok and same and rows
        pr1 = lg.pagerank(h, 0.85, 1).cpu().numpy().astype(np.float64)
        l1 = float(np.abs(pr1 - pr1_orc).sum())
        s20 = float(pr20.double().sum())
        log(f"[bench] {layout} PageRank: iteration-1 L1 {l1:.3e}, {args.pr_iters}-iteration sum {s20:.8f}")
        return ok and l1 <= 1e-5 and abs(s20 - 1.0) <= 1e-5, l1

    def kernel_breakdown(layout, opts):
        lg.prof_reset()
        lg.prof_filter("")
        lg.prof_enable(True)
        h, _, _ = run_step(layout, opts)
        h.free()
        torch.cuda.synchronize()
        lg.prof_enable(False)
        km = {}
        for name in lg.prof_names():
            base = name.lstrip("(").split("<")[0].rstrip(")")
            if base not in km:
                km[base] = lg.prof_query(base)
        return km

    def measure(layout, opts):
        """Parity, per-root times, warm-up, timed steps, kernel breakdown."""
        h, _, pr20 = run_step(layout, opts)
        ok, l1 = parity(layout, h, pr20)
        if not ok:
            print(json.dumps({"error": f"parity check failed before timing ({layout})"}), flush=True)
            sys.exit(1)
        reached_edges = [float(degf[all_depth[i] >= 0].sum()) / 2.0 for i in range(len(roots))]
        root_ms = per_root_ms(h)
        info = h.info()
        h.free()
        for _ in range(args.warmup):
            h, _, _ = run_step(layout, opts)
            h.free()
        # in the timed steps only the PageRank iteration's kernels are timed
        # (HIP events on the stream they run on); timing every launch would
        # add two events to each of the BFS lanes' many small launches
        lg.prof_reset()
        lg.prof_filter("|".join(PR_KERNELS))
        lg.prof_enable(True)
        torch.cuda.synchronize()
        t_begin = time.perf_counter()
        timings = []
        for _ in range(args.steps):
            h, tt, _ = run_step(layout, opts)
            timings.append(tt)
            h.free()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_begin
        log(f"[bench] {layout} timed steps (encode / BFS / PageRank ms): " +
            "; ".join(f"{t['encode']:.0f}/{t['bfs']:.0f}/{t['pr']:.0f}" for t in timings))
        lg.prof_enable(False)
        pr_k = {k: lg.prof_query(k) for k in PR_KERNELS}
        pr_k = {k: v for k, v in pr_k.items() if v[0]}
        km = kernel_breakdown(layout, opts)
        return dict(info=info, l1=l1, edges_root=reached_edges, root_ms=root_ms, timings=timings,
                    ms_per_step=wall * 1000.0 / args.steps, pr_kernels=pr_k, kernels=km)

    def summarize(layout, r):
        tm = r["timings"]
        bfs_ms = float(np.mean([t["bfs"] for t in tm]))
        pr_ms = float(np.mean([t["pr"] for t in tm]))
        step_ms = np.array([t["encode"] + t["bfs"] + t["pr"] for t in tm])
        enc_ms = float(np.mean([t["encode"] for t in tm]))
        edges_root = r["edges_root"]
        pr_edges = args.pr_iters * (M / 2.0)
        step_edges = sum(edges_root) + pr_edges
        teps = np.array(edges_root) / (r["root_ms"] / 1000.0)
        med, lo, hi, used = median_ci95(teps / 1e9)
        ms_med, ms_lo, ms_hi, _ = median_ci95(r["root_ms"])
        info = r["info"]
        # algorithmic bytes of one PageRank iteration launch: the lists, the
        # offset structure and width table (packed) or offsets (plain), 4 B of
        # contribution gathered per stored entry, 4 B written per vertex
        if layout == "packed":
            struct_bytes = info["adj_bits"] / 8.0 + info["bytes_offsets"] + info["bytes_widths"]
        else:
            struct_bytes = info["bytes_adj"] + info["bytes_offsets"]
        pr_bytes = struct_bytes + 4.0 * M + 4.0 * n
        iters_timed = args.steps * args.pr_iters
        pr_avg_ms = sum(v[1] for v in r["pr_kernels"].values()) / max(iters_timed, 1)  # per iteration
        pr_gbs = pr_bytes / (pr_avg_ms / 1000.0) / 1e9 if pr_avg_ms > 0 else 0.0
        km = r["kernels"]
        largest = max(km.items(), key=lambda kv: kv[1][1])[0] if km else None
        return dict(
            value=step_edges / (r["ms_per_step"] / 1000.0) / 1e9, ms_per_step=r["ms_per_step"],
            step_ms_events={"p50": float(np.percentile(step_ms, 50)), "p90": float(np.percentile(step_ms, 90)),
                            "min": float(step_ms.min()), "max": float(step_ms.max())},
            gteps_traversal=step_edges / ((bfs_ms + pr_ms) / 1000.0) / 1e9,
            encode_ms=enc_ms, encode_gedges_s=M / (enc_ms / 1000.0) / 1e9,
            bfs_all_roots_ms=bfs_ms, bfs_gteps_all_roots=sum(edges_root) / (bfs_ms / 1000.0) / 1e9,
            pr_ms=pr_ms, pr_gteps_directed=args.pr_iters * M / (pr_ms / 1000.0) / 1e9,
            per_root={"gteps_hmean": float(len(teps) / np.sum(1.0 / teps)) / 1e9,
                      "gteps_median": med, "gteps_median_ci95": [lo, hi], "samples": used,
                      "ms_median": ms_med, "ms_median_ci95": [ms_lo, ms_hi],
                      "ms_p50": float(np.percentile(r["root_ms"], 50)),
                      "ms_p99": float(np.percentile(r["root_ms"], 99))},
            pr_kernel={"name": "+".join(r["pr_kernels"]), "kernels": list(r["pr_kernels"]),
                       "avg_launch_ms": pr_avg_ms,
                       "per_kernel_avg_ms": {k: v[1] / max(v[0], 1) for k, v in r["pr_kernels"].items()},
                       "launches": {k: v[0] for k, v in r["pr_kernels"].items()},
                       "bytes_per_launch": pr_bytes, "achieved_gbs": pr_gbs,
                       "bytes_per_edge_algorithmic": pr_bytes / M},
            bytes={k: info[k] for k in ("bytes_adj", "bytes_offsets", "bytes_widths", "bytes_perm")},
            structure_bytes=struct_bytes,
            adj_bits=info["adj_bits"], parity_pr_iter1_l1=r["l1"],
            kernels_ms_profiled_step={k: round(v[1], 3) for k, v in km.items()},
            largest_summed_kernel=largest)

    res = {"packed": measure("packed", enc)}
    if not args.no_plain:
        res["plain"] = measure("plain", dict(relabel=enc["relabel"]))
    summ = {k: summarize(k, v) for k, v in res.items()}
    if args.kernels:
        for layout, r in res.items():
            tot = sum(v[1] for v in r["kernels"].values())
            for k, (c, ms) in sorted(r["kernels"].items(), key=lambda kv: -kv[1][1])[:16]:
                log(f"[kernel {layout}] {k:32s} launches={c:7d} total={ms:10.3f} ms "
                    f"({100 * ms / max(tot, 1e-9):5.1f}%) avg={ms / max(c, 1) * 1000:9.2f} us")

    # -- achievable bandwidth on this GPU: an elementwise kernel -----------
    cal_bytes, cal_ms = calibration_kernel(torch, dev)
    copy_gbs = cal_bytes / (cal_ms / 1000.0) / 1e9
    log(f"[bench] elementwise 1 GiB read + 1 GiB write: {cal_ms:.3f} ms = {copy_gbs:.0f} GB/s")

    # -- CPU baseline: the oracle on the host's cores, bounded sample -------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, np, orc, off_h, col_h, labels, roots, degf.cpu().numpy(), M, threads)

    P = summ["packed"]
    rooflines = {}
    for layout, s in summ.items():
        k = s["pr_kernel"]
        # counter bytes of the iteration: the sum over its kernels, when every
        # one has a current summary
        parts = [measured_counters(f"traffic_bytes_per_launch.{name}", args.workload, layout, "pr")
                 for name in k["kernels"]]
        traffic = sum(parts) if parts and all(p is not None for p in parts) else None
        rooflines[layout] = {
            "bound": "hbm", "kernel": k["name"], "achieved": round(k["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(k["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "frac_of_achievable_copy": round(k["achieved_gbs"] / copy_gbs, 4),
            "traffic": traffic,
            "bytes_per_launch": k["bytes_per_launch"], "avg_launch_ms": k["avg_launch_ms"],
            "launch_unit": "one PageRank iteration (every kernel it launches)",
            "per_kernel_avg_ms": k["per_kernel_avg_ms"],
            "bytes_per_edge_algorithmic": round(k["bytes_per_edge_algorithmic"], 4)}
        if rooflines[layout]["traffic"]:
            rooflines[layout]["bytes_per_edge_measured"] = round(rooflines[layout]["traffic"] / M, 4)
        if "pb_bin1_kernel" in k["kernels"]:
            # propagation blocking streams more than the algorithmic bytes by
            # design: level 1 reads the structure and the contributions and
            # writes 8 B per entry, level 2 reads 8 B and writes 6 B per entry,
            # the accumulation reads 6 B per entry and writes 4 B per vertex
            design = s["structure_bytes"] + 4.0 * n + 28.0 * M + 4.0 * n
            rooflines[layout]["design_bytes_per_launch"] = design
            rooflines[layout]["design_frac"] = round(design / (k["avg_launch_ms"] / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)
        tb = measured_counters("traffic_bytes_per_phase", args.workload, layout, "bfs")
        if tb:
            rooflines[layout]["bfs_traffic_bytes_per_search"] = tb
            rooflines[layout]["bfs_bytes_per_stored_entry_measured"] = round(tb / M, 4)
            rooflines[layout]["bfs_achieved_gbs_median_root"] = round(
                tb / (s["per_root"]["ms_median"] / 1000.0) / 1e9, 1)
        ta = measured_counters("traffic_bytes_per_phase", args.workload, layout, "bfsall")
        if ta:
            # the BFS phase as timed: all roots in one call
            rooflines[layout]["bfs_all_roots_traffic_bytes"] = ta
            rooflines[layout]["bfs_all_roots_achieved_gbs"] = round(ta / (s["bfs_all_roots_ms"] / 1000.0) / 1e9, 1)
    pr_share = P["pr_kernel"]["avg_launch_ms"] * args.pr_iters
    dominant = P["pr_kernel"]["name"] if pr_share >= max(P["bfs_all_roots_ms"], P["encode_ms"]) else \
        P["largest_summed_kernel"]
    roof = dict(rooflines["packed"])
    roof["dominant_kernel"] = dominant
    roof["dominant_by"] = ("wall-time share: the PageRank iteration kernels' time per step vs the BFS and encode "
                           "phases' wall times, which bound every kernel inside them")
    ratio = None
    if "plain" in summ:
        Q = summ["plain"]
        ratio = {"step": round(P["value"] / Q["value"], 4),
                 "traversal": round(P["gteps_traversal"] / Q["gteps_traversal"], 4),
                 "bfs": round(P["bfs_gteps_all_roots"] / Q["bfs_gteps_all_roots"], 4),
                 "bfs_per_root_hmean": round(P["per_root"]["gteps_hmean"] / Q["per_root"]["gteps_hmean"], 4),
                 "pr": round(Q["pr_ms"] / P["pr_ms"], 4),
                 "encode": round(Q["encode_ms"] / P["encode_ms"], 4),
                 "pr_bytes_per_edge_algorithmic": round(P["pr_kernel"]["bytes_per_edge_algorithmic"]
                                                        / Q["pr_kernel"]["bytes_per_edge_algorithmic"], 4)}
    out = {
        "metric": METRIC,
        "value": round(P["value"], 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(P["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "stored_edges": M, "roots": len(roots),
                   "pagerank_iters": args.pr_iters, "encoding": enc, "seed": 1, "edge_factor": 16,
                   "step": "encode + BFS from every root (one call) + PageRank iterations, packed layout"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": {
            "packed": P,
            "plain_csr": summ.get("plain"),
            "packed_over_plain": ratio,
            "roofline_plain": rooflines.get("plain"),
            "achievable_copy": {"kernel": "elementwise sqrt, 1 GiB read + 1 GiB write", "ms": round(cal_ms, 4),
                                "gbs": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4)},
            "p99_query_latency_ms": round(P["per_root"]["ms_p99"], 4),
            "p99_note": "per-root BFS latency (one root per call); the serving mix's p50/p99 come from --serve",
        },
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(args, np, orc, off_h, col_h, labels, roots, degs, M, threads):
    """The oracle on the host: level-synchronous BFS and PageRank on every
    core (the oracle's all-core functions), then the one-thread FIFO BFS and
    PageRank, each over as many roots / iterations as fit the time bound
    (at least one of each).  Labels for the parent rule were computed before
    (no permutation inside the timed calls).  Rates in the same units as the
    GPU's (undirected edges per second)."""
    budget = args.cpu_seconds

    def sample(bfs_fn, pr_fn, share):
        t_end = time.perf_counter() + budget * share
        bfs_t, bfs_e = [], []
        for r in roots:
            t0 = time.perf_counter()
            d, _ = bfs_fn(r)
            bfs_t.append(time.perf_counter() - t0)
            bfs_e.append(float(degs[d >= 0].sum()) / 2.0)
            if time.perf_counter() > t_end - budget * share / 2:
                break
        pr_t, iters = 0.0, 0
        while True:
            t0 = time.perf_counter()
            pr_fn(1)
            pr_t += time.perf_counter() - t0
            iters += 1
            if iters >= args.pr_iters or time.perf_counter() + pr_t / iters > t_end:
                break
        edges = sum(bfs_e) + iters * M / 2.0
        return {"gteps": edges / (sum(bfs_t) + pr_t) / 1e9, "bfs_roots": len(bfs_t), "bfs_s": sum(bfs_t),
                "bfs_gteps": sum(bfs_e) / sum(bfs_t) / 1e9, "pr_iters": iters, "pr_s": pr_t,
                "pr_gteps": iters * M / 2.0 / pr_t / 1e9}

    allc = sample(lambda r: orc.bfs_levels(off_h, col_h, r, labels=labels, threads=threads),
                  lambda it: orc.pagerank_par(off_h, col_h, 0.85, it, threads=threads), 0.6)
    one = sample(lambda r: orc.bfs(off_h, col_h, r, labels=labels),
                 lambda it: orc.pagerank(off_h, col_h, 0.85, it), 0.4)
    hi = host_info()
    log(f"[bench] oracle all-core ({threads} threads): {allc}; one thread: {one}; host {hi}")
    return {"value": allc["gteps"], "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": (f"oracle on {threads} threads: level-synchronous BFS from the first {allc['bfs_roots']} "
                       f"roots ({allc['bfs_s']:.1f}s) + {allc['pr_iters']} PageRank iteration(s) "
                       f"({allc['pr_s']:.1f}s); parent labels precomputed, not timed"),
            "one_thread": one, "all_core": allc, "host": hi}


def counter_main(args, np, torch, lg, g, roots, enc):
    """Counter runs: the calibration kernel (1 GiB read + 1 GiB write), then
    the phase under study on --layout, so that a profiler collecting one
    counter per pass sees each kernel's traffic per launch."""
    nbytes, ms = calibration_kernel(torch, g.col.device)
    log(f"[counter-run] calibration done ({nbytes} bytes, {ms:.3f} ms); encoding {args.layout}")
    opts = enc if args.layout == "packed" else dict(relabel=enc["relabel"])
    h = lg.encode(g.row_offsets, g.col, g.n, layout=args.layout, **opts)
    info = h.info()
    torch.cuda.synchronize()
    torch.cos(torch.zeros(1, device=g.col.device))  # marks where the phase begins
    torch.cuda.synchronize()
    if args.counter_run == "pr":
        log("[counter-run] PageRank")
        lg.pagerank(h, 0.85, args.pr_iters)
    elif args.counter_run == "bfs":
        for mode in args.bfs_modes.split(","):
            log(f"[counter-run] BFS {mode} from root {roots[0]}")
            lg.bfs(h, [roots[0]], mode=mode)
    else:
        log(f"[counter-run] BFS from all {len(roots)} roots in one call")
        lg.bfs(h, roots)
    torch.cuda.synchronize()
    struct = (info["adj_bits"] / 8.0 + info["bytes_offsets"] + info["bytes_widths"]) if args.layout == "packed" \
        else (info["bytes_adj"] + info["bytes_offsets"])
    print(json.dumps({"mode": "counter-run", "phase": args.counter_run, "layout": args.layout,
                      "workload": args.workload, "calibration_bytes": nbytes, "pr_iters": args.pr_iters,
                      "bfs_modes": args.bfs_modes, "roots": len(roots),
                      "n": g.n, "stored_edges": g.m, "structure_bytes": struct,
                      "pr_algorithmic_bytes_per_iteration": struct + 4.0 * g.m + 4.0 * g.n,
                      "source_sha256": source_hash(args.counter_run)}), flush=True)
    h.free()


def _time_ms(torch, fn, reps=3):
    """Median of `reps` timed calls after one untimed call, HIP events on the
    current stream."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sorted(ts)[len(ts) // 2]


def relabel_main(args, np, torch, lg, g, roots):
    """The workload's graph under each relabeling, local widths and
    Elias-Fano offsets: bytes of the packed lists |A|, of the offsets and of
    the width table; encode time; BFS from the roots (one call) and 20
    PageRank iterations.  The same graph and roots for every relabeling."""
    n = g.n
    depth = torch.empty((len(roots), n), dtype=torch.int32, device=g.col.device)
    parent = torch.empty_like(depth)
    res = {}
    for rl, name in [(False, "none"), (True, "degree"), ("greedy", "greedy")]:
        enc = lambda: lg.encode(g.row_offsets, g.col, n, ids="local", offsets="succinct", relabel=rl)  # noqa: E731
        hs = []
        enc_ms = _time_ms(torch, lambda: hs.append(enc()))
        for h in hs[:-1]:
            h.free()
        h = hs[-1]
        info = h.info()
        bfs_ms = _time_ms(torch, lambda: lg.bfs(h, roots, depth_out=depth, parent_out=parent))
        pr = lg.pagerank(h, 0.85, 20)
        pr_ms = _time_ms(torch, lambda: lg.pagerank(h, 0.85, 20, out=pr))
        res[name] = {"adj_bytes": info["adj_bits"] / 8.0, "offsets_bytes": info["bytes_offsets"],
                     "widths_bytes": info["bytes_widths"], "encode_ms": round(enc_ms, 3),
                     "bfs_all_roots_ms": round(bfs_ms, 3), "pagerank_20_ms": round(pr_ms, 3)}
        log(f"[relabel] {name}: {res[name]}")
        h.free()
    base = res["none"]["adj_bytes"]
    for name in res:
        res[name]["adj_vs_none"] = round(res[name]["adj_bytes"] / base, 4)
    print(json.dumps({"mode": "relabel-compare", "workload": args.workload, "n": n, "stored_edges": g.m,
                      "roots": len(roots), "encoding": {"ids": "local", "offsets": "succinct"},
                      "data": "synthetic", "results": res}), flush=True)


def offset_fetch_main(args, np, torch, lg, g):
    """Random fetch under each offset structure (the random-offset-fetch test
    of the offset-structure comparison: 1,000 random vertices per worker;
    here 256 workers, one per compute unit, in one call), no relabeling,
    global widths, so that every structure indexes elements of the lists as
    in the paper's comparison: degrees only (one offset pair per vertex: the
    structure's random access) and whole lists."""
    import ctypes as C
    n = g.n
    k = 1000 * 256
    rng = np.random.default_rng(7)
    vt = torch.from_numpy(rng.integers(0, n, size=k).astype(np.int32)).to(g.col.device)
    off = torch.empty(k + 1, dtype=torch.int64, device=g.col.device)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {}
    # ptr32: plain 32-bit element offsets; ptrW: offsets at bl(M) bits
    # (logarithmized single offsets); bvPL: the plain bit vector with a
    # rank/select directory; bvIL: the bit vector with interleaved 64-bit
    # counts; bvSD: the Elias-Fano sparse bit vector
    for name, kw in [("ptr32", dict(layout="plain")), ("ptrW", dict(ids="global", offsets="packed")),
                     ("bvPL", dict(ids="global", offsets="plain-bv")),
                     ("bvIL", dict(ids="global", offsets="interleaved-bv")),
                     ("bvSD", dict(ids="global", offsets="succinct"))]:
        h = lg.encode(g.row_offsets, g.col, n, **kw)
        info = h.info()

        def degrees_only():
            # no output array: only the offsets are fetched (the call reports
            # the capacity it would need)
            lg.lib().lg_decode_neighbors(h.handle, C.c_void_p(vt.data_ptr()), k, C.c_void_p(off.data_ptr()), None, 0,
                                         2, s)
        deg_ms = _time_ms(torch, degrees_only, reps=5)
        total = int(off[-1].item())
        # parity before the numbers count: every structure gives the input's
        # degrees for the fetched vertices
        want = (g.row_offsets[vt.long() + 1] - g.row_offsets[vt.long()]).cumsum(0)
        if not (int(off[0].item()) == 0 and torch.equal(off[1:], want)):
            print(json.dumps({"error": f"offset fetch parity failed ({name})"}), flush=True)
            sys.exit(1)
        ids = torch.empty(max(total, 1), dtype=torch.int32, device=g.col.device)

        def lists():
            st = lg.lib().lg_decode_neighbors(h.handle, C.c_void_p(vt.data_ptr()), k, C.c_void_p(off.data_ptr()),
                                              C.c_void_p(ids.data_ptr()), total, 2, s)
            assert st == 0, lg.lib().lg_last_error()
        lists_ms = _time_ms(torch, lists, reps=5)
        if name == "ptr32":
            ref_ids = ids.clone()
        elif not torch.equal(ids, ref_ids):
            print(json.dumps({"error": f"offset fetch list parity failed ({name})"}), flush=True)
            sys.exit(1)
        res[name] = {"offsets_bytes": info["bytes_offsets"], "degrees_only_ms": round(deg_ms, 4),
                     "ns_per_offset_fetch": round(deg_ms * 1e6 / k, 3), "lists_ms": round(lists_ms, 4),
                     "entries": total, "gentries_per_s": round(total / (lists_ms * 1e-3) / 1e9, 3)}
        log(f"[offsets] {name}: {res[name]}")
        h.free()
    print(json.dumps({"mode": "offset-fetch", "workload": args.workload, "n": n, "stored_edges": g.m,
                      "vertices_per_call": k, "data": "synthetic", "results": res}), flush=True)


def sssp_main(args, np, torch, gg, lg, g, roots):
    """Weighted SSSP (delta-stepping) on the workload's graph, weights uniform
    integers in [1, 255] (the same for both directions of an edge): the
    weighted plain CSR against the packed weighted encodings (ID then weight
    per entry, global or local IDs, Elias-Fano offsets; local IDs also after
    the degree-minimizing relabeling), bytes of the lists and the time of one
    SSSP per root (median over the roots), then delta swept on the local
    encoding.  Edges per second count the stored entries
    of the vertices a root reaches, halved (as the BFS rate)."""
    n = g.n
    wt = gg.edge_weights(g, 255, seed=1)
    deg = g.degrees().to(torch.float64)
    res = {}
    encs = [("plain", dict(layout="plain")), ("packed-global", dict(ids="global", offsets="succinct")),
            ("packed-local", dict(ids="local", offsets="succinct")),
            ("packed-local-dm", dict(ids="local", offsets="succinct", relabel=True))]
    sweep = {}
    timed_roots = roots[:8]
    # parity before timing: the oracle's Dijkstra for the first root, then
    # every encoding's distances for every timed root equal the plain CSR's
    import oracle as orc  # the CPU oracle: test infrastructure
    off_h = g.row_offsets.cpu().numpy().view(np.uint64)
    col_h = g.col.cpu().numpy().view(np.uint32)
    t0 = time.time()
    want0 = orc.sssp(off_h, col_h, wt.cpu().numpy().view(np.uint32), timed_roots[0])
    log(f"[sssp] oracle Dijkstra from root {timed_roots[0]}: {time.time() - t0:.1f}s")
    plain_dist = None
    for name, kw in encs:
        h = lg.encode(g.row_offsets, g.col, n, weights=wt, **kw)
        info = h.info()
        dists = [lg.sssp(h, r) for r in timed_roots]
        ok = bool(np.array_equal(dists[0].cpu().numpy(), want0))
        if plain_dist is None:
            plain_dist = dists
        else:
            ok = ok and all(bool(torch.equal(a, b)) for a, b in zip(dists, plain_dist))
        log(f"[sssp] {name}: parity {'ok' if ok else 'FAILED'} (root {timed_roots[0]} against the oracle, "
            f"{len(timed_roots)} roots against the plain CSR)")
        if not ok:
            print(json.dumps({"error": f"SSSP parity failed before timing ({name})"}), flush=True)
            sys.exit(1)
        times, edges = [], []
        for r, d in zip(timed_roots, dists):
            edges.append(float(deg[d >= 0].sum()) / 2.0)
            times.append(_time_ms(torch, lambda: lg.sssp(h, r), reps=1))
        med = sorted(times)[len(times) // 2]
        res[name] = {"adj_bytes": info["adj_bits"] / 8.0 if kw.get("layout") != "plain" else 4.0 * g.m,
                     "weight_bytes": info["bytes_weights"], "weight_bits": info["weight_bits"],
                     "sssp_ms_median": round(med, 3),
                     "gteps_median": round(sorted(e / t * 1e-6 for e, t in zip(edges, times))[len(times) // 2], 3)}
        log(f"[sssp] {name}: {res[name]}")
        if name == "packed-local":
            for delta in (16, 64, 128, 256, 512, 1024, 4096):
                sweep[delta] = round(_time_ms(torch, lambda: lg.sssp(h, roots[0], delta), reps=1), 3)
            log(f"[sssp] delta sweep (root {roots[0]}): {sweep}")
        h.free()
    print(json.dumps({"mode": "sssp", "workload": args.workload, "n": n, "stored_edges": g.m,
                      "roots": len(timed_roots), "max_weight": 255, "data": "synthetic", "results": res,
                      "parity": "root 0 equal to the oracle's Dijkstra; every root equal across encodings",
                      "delta_sweep_ms": sweep}), flush=True)


def encoding_main(args, np, torch, lg, g, roots):
    """List encodings side by side, Elias-Fano offsets, without and with the
    degree-minimizing relabeling: local widths (LG-l), fixed-size gap
    encoding (LG-l-gap), and Varint lists of full labels or of differences
    (with the relabeling: DMf and DMd).  Bytes of the lists |A|, of the width
    tables and of the offsets, encode time, the decode of the lists of
    256,000 random vertices (one call, stored labels), a BFS from every root
    (one call), and 20 PageRank iterations where the encoding supports
    them."""
    import ctypes as C
    n = g.n
    k = 1000 * 256
    rng = np.random.default_rng(7)
    vt = torch.from_numpy(rng.integers(0, n, size=k).astype(np.int32)).to(g.col.device)
    off = torch.empty(k + 1, dtype=torch.int64, device=g.col.device)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {}
    names = {"local": "LG-l", "local-gap": "LG-l-gap", "varint-full": "Varint-full", "varint-diff": "Varint-diff"}
    for rl in (False, True):
        for ids in ("local", "local-gap", "varint-full", "varint-diff"):
            name = f"{names[ids]}{'+DM' if rl else ''}"
            hs = []
            enc_ms = _time_ms(torch, lambda: hs.append(lg.encode(g.row_offsets, g.col, n, ids=ids,
                                                                 offsets="succinct", relabel=rl)))
            for h in hs[:-1]:
                h.free()
            h = hs[-1]
            info = h.info()
            lg.lib().lg_decode_neighbors(h.handle, C.c_void_p(vt.data_ptr()), k, C.c_void_p(off.data_ptr()), None,
                                         0, 2, s)
            total = int(off[-1].item())
            ids_buf = torch.empty(max(total, 1), dtype=torch.int32, device=g.col.device)

            def lists():
                st = lg.lib().lg_decode_neighbors(h.handle, C.c_void_p(vt.data_ptr()), k, C.c_void_p(off.data_ptr()),
                                                  C.c_void_p(ids_buf.data_ptr()), total, 2, s)
                assert st == 0, lg.lib().lg_last_error()
            dec_ms = _time_ms(torch, lists, reps=5)
            pr_ms = _time_ms(torch, lambda: lg.pagerank(h, 0.85, 20))
            bfs_ms = _time_ms(torch, lambda: lg.bfs(h, roots))
            res[name] = {"adj_bytes": info["adj_bits"] / 8.0, "widths_bytes": info["bytes_widths"],
                         "offsets_bytes": info["bytes_offsets"], "encode_ms": round(enc_ms, 3),
                         "decode_ms": round(dec_ms, 4), "decoded_entries": total,
                         "decode_gentries_per_s": round(total / (dec_ms * 1e-3) / 1e9, 3),
                         "pagerank20_ms": None if pr_ms is None else round(pr_ms, 3),
                         "bfs_all_roots_ms": None if bfs_ms is None else round(bfs_ms, 3)}
            log(f"[encodings] {name}: {res[name]}")
            h.free()
    for rl in ("", "+DM"):
        a = res["LG-l" + rl]
        for other in ("LG-l-gap", "Varint-full", "Varint-diff"):
            b = res[other + rl]
            b["adj_vs_local"] = round(b["adj_bytes"] / a["adj_bytes"], 4)
            b["total_vs_local"] = round((b["adj_bytes"] + b["widths_bytes"] + b["offsets_bytes"])
                                        / (a["adj_bytes"] + a["widths_bytes"] + a["offsets_bytes"]), 4)
    print(json.dumps({"mode": "encoding-compare", "workload": args.workload, "n": n, "stored_edges": g.m,
                      "vertices_per_call": k, "data": "synthetic", "results": res}), flush=True)


def batch_main(args, np, torch, gg, lg, dev):
    """256 independent R-MAT graphs, scale ~ U{10..18} (seed 1), graph g with
    seed 1000 + g, edge factor 16, global widths + packed offsets; 16 roots per
    graph; all 4,096 BFS queries in one persistent graph-captured launch."""
    t0 = time.time()
    rng = np.random.default_rng(1)
    scales = rng.integers(10, 19, size=256)
    graphs, hs, jobs, edges = [], [], [], []
    for gi, sc in enumerate(scales):
        g = gg.kronecker(int(sc), 16, seed=1000 + gi, device=dev)
        graphs.append(g)
        hs.append(lg.encode(g.row_offsets, g.col, g.n))
        for r in gg.pick_roots(g, 16, seed=gi):
            jobs.append((gi, r))
    torch.cuda.synchronize()
    log(f"[batch] {len(graphs)} graphs, {len(jobs)} queries, "
        f"{sum(g.m for g in graphs) / 1e6:.1f} M stored edges; built in {time.time() - t0:.1f}s")
    plan = lg.BatchPlan(hs, jobs, autotune=True)
    info = plan.info()
    log(f"[batch] autotuned: {info}")
    # Graph500 edges per query (from the batch's own depths)
    degs = [g.degrees().to(torch.float64) for g in graphs]
    edges = [float(degs[gi][plan.depth(i) >= 0].sum()) / 2.0 for i, (gi, _) in enumerate(jobs)]
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(args.steps):
        plan.run()
    ev[1].record()
    torch.cuda.synchronize()
    batch_ms = ev[0].elapsed_time(ev[1]) / args.steps
    # the batch's own rows, kept to compare with one launch per query
    dflat, pflat = plan.depth_flat, plan.parent_flat
    torch.cuda.synchronize()
    batch_d, batch_p = dflat.clone(), pflat.clone()
    # one launch per query, same graphs and roots, results written to the same rows
    ev[0].record()
    for i, (gi, r) in enumerate(jobs):
        lg.bfs(hs[gi], [r], depth_out=dflat[plan.offsets[i]:plan.offsets[i + 1]].view(1, -1),
               parent_out=pflat[plan.offsets[i]:plan.offsets[i + 1]].view(1, -1))
    ev[1].record()
    torch.cuda.synchronize()
    single_ms = ev[0].elapsed_time(ev[1])
    # parity: every batch row equals the single-query call's, and a sample of
    # 32 queries equals the oracle's tree
    same = bool(torch.equal(batch_d, dflat) and torch.equal(batch_p, pflat))
    import oracle as orc  # the CPU oracle: test infrastructure
    rng = np.random.default_rng(3)
    sample = sorted(rng.choice(len(jobs), size=min(32, len(jobs)), replace=False).tolist())
    for i in sample:
        gi, r = jobs[i]
        off_h, col_h = graphs[gi].numpy()
        d0, p0 = orc.bfs(off_h, col_h, r)
        same = same and bool(np.array_equal(plan.depth(i).cpu().numpy(), d0)
                             and np.array_equal(plan.parent(i).cpu().numpy(), p0))
    log(f"[batch] parity: {len(jobs)} rows against one launch per query, {len(sample)} against the oracle: "
        f"{'ok' if same else 'FAILED'}")
    if not same:
        print(json.dumps({"error": "batch parity failed"}), flush=True)
        sys.exit(1)
    total_edges = sum(edges)
    out = {"metric": "GTEPS & HBM GB/s, Log(Graph)-packed vs plain CSR on GPU; p99 query latency",
           "value": round(total_edges / (batch_ms / 1000.0) / 1e9, 4), "unit": "GTEPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(batch_ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "batch-rmat256-s10-18", "graphs": len(graphs), "queries": len(jobs),
                      "encoding": {"ids": "global", "offsets": "packed"}},
           "detail": {"one_launch_per_query_ms": round(single_ms, 3),
                      "speedup_vs_one_launch_per_query": round(single_ms / batch_ms, 2),
                      "parity": "every row equal to one launch per query; 32 rows equal to the oracle",
                      "autotune": info}}
    print(json.dumps(out), flush=True)
    plan.free()
    for h in hs:
        h.free()


def serve_main(args, np, torch, gg, lg, dev):
    """8 resident graphs: Kronecker and uniform-random at each scale of
    --serve-scales (edge factor 16, seed 1), global widths + packed offsets.
    Queries: graph uniform, vertex uniform over the graph's non-isolated
    vertices, kind 60% neighbor fetch / 30% 2-hop / 10% full BFS.  First the
    saturated throughput (a closed batch submitted at once), then Poisson
    arrivals at 0.25/0.5/0.75/0.9 of it; latency runs from the scheduled
    arrival to the result on the host."""
    import threading
    scales = [int(x) for x in args.serve_scales.split(",")]
    t0 = time.time()
    hs, cands, names = [], [], []
    for gen in ["kronecker", "er"]:
        for sc in scales:
            g = (gg.kronecker if gen == "kronecker" else gg.erdos_renyi)(sc, 16, seed=1, device=dev)
            hs.append(lg.encode(g.row_offsets, g.col, g.n))
            cands.append(torch.nonzero(g.degrees() > 0).flatten().cpu().numpy())
            names.append(f"{gen}-s{sc}")
            log(f"[serve] {names[-1]}: n={g.n} M={g.m} packed {hs[-1].info()['device_bytes'] / 1e9:.2f} GB "
                f"({time.time() - t0:.0f}s)")
            del g
            torch.cuda.empty_cache()
    torch.cuda.synchronize()
    lg.trim()  # the encoder's cached temporaries are not part of the served state
    torch.cuda.empty_cache()
    budget = 200 * 10**9
    srv = lg.Server(hs, budget_bytes=budget, workers=8, max_batch=64)
    kinds = ["neighbors", "khop", "bfs"]

    def draw(count, seed):
        rng = np.random.default_rng(seed)
        gi = rng.integers(len(hs), size=count)
        r = rng.random(count)
        kind = np.where(r < 0.6, 0, np.where(r < 0.9, 1, 2))
        vs = [int(cands[g][rng.integers(cands[g].size)]) for g in gi]
        return [(kinds[k], int(g), v) for k, g, v in zip(kind, gi, vs)]

    def closed(qs):
        t = time.perf_counter()
        tickets = [srv.submit(k, g, v, k=2) for k, g, v in qs]
        res = [srv.wait(x, arrays=False) for x in tickets]
        return time.perf_counter() - t, res

    # warm every worker's buffers on every graph and kind
    warm = [(k, g, int(cands[g][0])) for g in range(len(hs)) for k in kinds for _ in range(2)]
    closed(warm)
    qs_sat = draw(4000, seed=1)
    wall, res = closed(qs_sat)
    assert all(r["status"] == 0 for r in res), "a query failed"
    sat_qps = len(res) / wall
    # parity: 300 queries of the saturated mix again, served one at a time
    # (alone on the device), must return the same results: the same sorted
    # IDs for neighbor and k-hop queries, the same reach, depth and digest of
    # (depth, parent) for BFS
    rng = np.random.default_rng(9)
    pick = sorted(rng.choice(len(qs_sat), size=300, replace=False).tolist())
    tickets = [srv.submit(k, g, v, k=2) for k, g, v in (qs_sat[i] for i in pick)]
    mixed = [srv.wait(t) for t in tickets]
    mismatch = 0
    for i, m in zip(pick, mixed):
        k, gsel, v = qs_sat[i]
        alone = srv.wait(srv.submit(k, gsel, v, k=2))
        same = m["status"] == alone["status"] == 0 and m["count"] == alone["count"]
        if k == "bfs":
            same = same and m["digest"] == alone["digest"] and m["max_depth"] == alone["max_depth"]
        else:
            same = same and np.array_equal(m["ids"], alone["ids"])
        mismatch += 0 if same else 1
    log(f"[serve] parity: {len(pick)} queries served in a mix and alone: {mismatch} mismatches")
    if mismatch:
        print(json.dumps({"error": f"serving parity failed ({mismatch} queries)"}), flush=True)
        sys.exit(1)
    log(f"[serve] saturated: {len(res)} queries in {wall:.2f}s = {sat_qps:.1f} q/s")

    loads = {}
    for li, f in enumerate([0.25, 0.5, 0.75, 0.9]):
        lam = f * sat_qps
        count = max(200, int(lam * args.serve_seconds))
        qs = draw(count, seed=100 + li)
        rng = np.random.default_rng(200 + li)
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=count))
        tickets, lag = [None] * count, [0.0] * count
        out = [None] * count
        submitted = threading.Semaphore(0)

        def collect():
            for i in range(count):
                submitted.acquire()
                out[i] = srv.wait(tickets[i], arrays=False)

        th = threading.Thread(target=collect)
        th.start()
        start = time.perf_counter()
        for i, (k, g, v) in enumerate(qs):
            due = start + arrivals[i]
            while True:
                d = due - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 0.002) if d > 0.0005 else 0)
            lag[i] = (time.perf_counter() - due) * 1e3
            tickets[i] = srv.submit(k, g, v, k=2)
            submitted.release()
        th.join()
        end = max(lag[i] / 1e3 + arrivals[i] + out[i]["latency_ms"] / 1e3 for i in range(count))
        lat = np.array([lag[i] + out[i]["latency_ms"] for i in range(count)])
        assert all(r["status"] == 0 for r in out), "a query failed"
        per_kind = {}
        for kname in kinds:
            sel = np.array([q[0] == kname for q in qs])
            if sel.any():
                per_kind[kname] = {"p50_ms": round(float(np.percentile(lat[sel], 50)), 3),
                                   "p99_ms": round(float(np.percentile(lat[sel], 99)), 3), "count": int(sel.sum())}
        loads[str(f)] = {"offered_qps": round(lam, 1), "achieved_qps": round(float(count / end), 1), "queries": count,
                         "p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "mean_batch": round(float(np.mean([r["batch"] for r in out])), 2),
                         "submit_lag_p99_ms": round(float(np.percentile(lag, 99)), 3), "per_kind": per_kind}
        log(f"[serve] load {f}: {loads[str(f)]}")
    st = srv.stats()
    srv.free()
    assert st["peak_bytes"] <= budget and st["overruns"] == 0
    out = {"metric": "GTEPS & HBM GB/s, Log(Graph)-packed vs plain CSR on GPU; p99 query latency",
           "value": round(sat_qps, 2), "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": round(1000.0 / sat_qps, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "serve-8graphs-kron-er-s" + "-".join(map(str, scales)), "graphs": names,
                      "mix": {"neighbors": 0.6, "khop2": 0.3, "bfs": 0.1}, "budget_bytes": budget,
                      "workers": st["workers"], "encoding": {"ids": "global", "offsets": "packed"}},
           "detail": {"loads": loads, "resident_bytes": st["resident_bytes"], "peak_bytes": st["peak_bytes"],
                      "parity": "300 queries of the saturated mix equal to the same queries served alone",
                      "batches": st["batches"], "completed": st["completed"]}}
    print(json.dumps(out), flush=True)
    for h in hs:
        h.free()


if __name__ == "__main__":
    main()
