#!/usr/bin/env python3
"""Benchmark of the partition-centric scatter/gather iteration on one MI355X.

Default workload: BFS (levels) from 8 sources plus min-label connected
components on the symmetrised RMAT graph of scale 22, edge factor 16
(4,194,304 vertices, 134,217,728 directed CSR entries). One step = the 8
BFS runs + 1 CC run, each from a fresh initial state, on inputs already
resident in HBM. Prints one JSON line.

Throughput is traversed edges per second: each BFS counts the out-degrees of
the vertices it reaches (directed CSR entries), CC counts every entry once.
`roofline` reports the kernel with the largest share of device time: its
algorithmic bytes per launch (the byte model below) over its mean launch
duration, from HIP events recorded around every launch on the stream the
kernel runs on, against the 8 TB/s HBM peak.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- byte model
def kernel_bytes(rec, next_va, q, k, weighted, sum_prog):
    """Algorithmic bytes of each kernel for one iteration record, with the
    element sizes the kernels use: 2-byte ids, 4-byte values and state,
    1-byte weights, 4-byte CSR entries and offsets."""
    s_id, s_v, s_w = 2, 4, (1 if weighted else 0)
    s_part = 8 if sum_prog else 4
    state_in = 0 if sum_prog else 4 * q
    plan = 25 * k
    sc = (rec["sc_active_vertices"] * (2 + 4 + 8 + 4) + rec["sc_active_edges"] * (4 + s_w)
          + rec["sc_ids"] * (s_id + s_w) + rec["sc_msgs"] * s_v + rec["sc_parts"] * 8 * k)
    pc = (rec["pc_vertices"] * (4 + 0.125 + (8 if sum_prog else 0))
          + rec["pc_msgs"] * (2 + s_v))
    whole = rec["gather_parts"]
    part = rec["split_tasks"]
    merged = rec["merged_parts"]
    gather = ((rec["sc_ids"] + rec["pc_ids"]) * (s_id + s_w) + (rec["sc_msgs"] + rec["pc_msgs"]) * s_v
              + whole * (24 * k + state_in + 4 * q + 4 * q + q / 8) + part * s_part * q
              + next_va * (2 + 4))
    merge = merged * (state_in + 4 * q + 4 * q + q / 8) + part * s_part * q
    return {"plan": plan, "scatter_sc": sc, "scatter_pc": pc, "gather": gather, "merge": merge}


def run_bytes(stats, q, k, weighted, sum_prog):
    tot = {"plan": 0.0, "scatter_sc": 0.0, "scatter_pc": 0.0, "gather": 0.0, "merge": 0.0}
    for i, rec in enumerate(stats):
        nva = stats[i + 1]["active_vertices"] if i + 1 < len(stats) else 0
        for kname, b in kernel_bytes(rec, nva, q, k, weighted, sum_prog).items():
            tot[kname] += b
    return tot


# ----------------------------------------------------------------- workloads
KERNEL_SOURCES = {
    "plan": ["scatter.hip", "gpop_dev.h"],
    "scatter_sc": ["scatter.hip", "gpop_dev.h"],
    "scatter_pc": ["scatter.hip", "gpop_dev.h"],
    "gather": ["gather.hip", "gpop_dev.h"],
    "merge": ["gather.hip", "gpop_dev.h"],
}


def kernel_source_hash(kname):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kname]:
        with open(os.path.join(ROOT, "paper_1806_08092_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kname, workload):
    """HBM bytes per launch of one kernel family from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, scaled by the copy-kernel calibration.
    None when there is no summary or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kname, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash(kname):
        return None
    return float(kv["traffic_bytes_per_launch"])


def load_workload(name):
    import graphgen as gg
    if name == "bfs_cc_rmat22":
        g = gg.workload_bfs_cc_rmat22()
        runs = [("bfs", int(s)) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED, 8)] + [("cc", 0)]
        return g, runs, 14, "BFS levels from 8 sources + min-label CC, RMAT scale 22 ef16 symmetrised"
    if name == "pagerank_rmat16":
        g = gg.workload_pagerank_rmat16()
        return g, [("pagerank", 0)], 13, "PageRank 10 iterations d=0.85, RMAT scale 16 ef16 directed"
    if name == "sssp_rmat24":
        g = gg.workload_sssp_rmat24()
        runs = [("sssp", int(s)) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED, 8)]
        return g, runs, 14, "SSSP u8 weights [1,255] from 8 sources, RMAT scale 24 ef16 directed"
    if name == "sssp_er24":
        g = gg.workload_sssp_er24()
        runs = [("sssp", int(s)) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED, 8)]
        return g, runs, 14, "SSSP u8 weights [1,255] from 8 sources, Erdos-Renyi 2^24 vertices deg 16"
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(g, runs, budget_s):
    """The oracle (single-threaded C) on the same graph: runs of the step in
    order until the time budget is spent. Returns GTEPS and the sample."""
    import numpy as np
    import oracle
    deg = g.degrees()
    edges = 0
    done = []
    t0 = time.perf_counter()
    for prog, root in runs:
        if prog == "bfs":
            lv = oracle.bfs_levels(g, root)
            edges += int(deg[lv != 0xFFFFFFFF].sum())
        elif prog == "cc":
            oracle.cc_minlabel(g)
            edges += g.m
        elif prog == "sssp":
            d = oracle.sssp(g, root)
            edges += int(deg[d != 0xFFFFFFFF].sum())
        elif prog == "pagerank":
            oracle.pagerank(g, 0.85, 10)
            edges += 10 * g.m
        done.append("%s(%d)" % (prog, root))
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return edges / dt / 1e9, "oracle " + " ".join(done) + " in %.1f s" % dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bfs_cc_rmat22")
    ap.add_argument("--selector", default="analytical")
    ap.add_argument("--bw-ratio", type=float, default=2.0)
    ap.add_argument("--log2-part", type=int, default=0)
    ap.add_argument("--gather-task-ids", type=int, default=0,
                    help="ids per gather task (0: library default)")
    ap.add_argument("--sc-task-log2", type=int, default=0,
                    help="log2 of active edges per source-centric task (0: library default)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the device copy used as the practical bandwidth ceiling")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1806_08092_amd as gp

    t = time.perf_counter()
    g, runs, lp, desc = load_workload(args.workload)
    if args.log2_part:
        lp = args.log2_part
    log("workload %s: V=%d E=%d generated in %.1f s" % (args.workload, g.n, g.m, time.perf_counter() - t))
    off, cols, w = gp.upload_csr(g)
    torch.cuda.synchronize()
    t = time.perf_counter()
    G = gp.Graph(off, cols, w, log2_part=lp, sc_task_log2=args.sc_task_log2,
                 gather_task_ids=args.gather_task_ids)
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - t) * 1e3
    info = G.info()
    log("preprocessed in %.1f ms: q=%d k=%d M=%d bins=%d" % (prep_ms, info.q, info.k, info.num_messages,
                                                             info.nonempty_bins))
    G.set_selector(args.selector, args.bw_ratio)
    st = torch.empty(g.n, dtype=torch.int32, device="cuda")
    roots = {r: torch.tensor([r], dtype=torch.int32, device="cuda") for _, r in runs}
    max_iter = {"pagerank": 10, "ppr": 20}

    def do_run(prog, root):
        G.state_init(prog, st, root=root)
        if prog in ("cc", "pagerank"):
            G.set_frontier_all()
        else:
            G.set_frontier(roots[root])
        return G.run(max_iter.get(prog, 1 << 30))

    def step():
        for prog, root in runs:
            do_run(prog, root)

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)

    G.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = G.profile_read()
    G.profile_enable(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log("timed %d steps: %.3f ms/step" % (args.steps, ms_per_step))

    # one untimed pass for the deterministic per-iteration statistics
    deg = (off[1:] - off[:-1]).to(torch.int64)
    edges_per_step = 0
    bytes_step = {"plan": 0.0, "scatter_sc": 0.0, "scatter_pc": 0.0, "gather": 0.0, "merge": 0.0}
    iters_per_run = []
    for prog, root in runs:
        iters = do_run(prog, root)
        iters_per_run.append(iters)
        stats = G.iter_stats()
        b = run_bytes(stats, info.q, info.k, prog == "sssp", prog in ("pagerank", "ppr"))
        for kname in bytes_step:
            bytes_step[kname] += b[kname]
        if prog in ("bfs", "sssp"):
            reached = st != -1
            edges_per_step += int(deg[reached].sum().item())
        elif prog == "pagerank":
            edges_per_step += 10 * g.m
        else:
            edges_per_step += g.m
    G.check()

    per_kernel = {}
    for kname, (ms, n) in prof.items():
        if n == 0:
            continue
        gbytes = bytes_step[kname] * args.steps
        per_kernel[kname] = {
            "ms_per_step": ms / args.steps,
            "launches_per_step": n / args.steps,
            "mean_launch_us": ms * 1e3 / n,
            "alg_GB_per_step": bytes_step[kname] / 1e9,
            "achieved_GBps": gbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0,
        }
    dom = max(per_kernel, key=lambda kn: per_kernel[kn]["ms_per_step"])
    ach = per_kernel[dom]["achieved_GBps"]
    traffic = measured_traffic(dom, args.workload)
    gteps = edges_per_step / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "GTEPS (traversed directed CSR edges per second) and % of HBM peak per kernel",
        "value": gteps,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if all(p in ("bfs", "cc", "sssp") for p, _ in runs) else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "vertices": g.n, "edges": g.m, "q": info.q, "k": info.k,
                   "selector": args.selector, "bw_ratio": args.bw_ratio,
                   "gather_task_ids": args.gather_task_ids, "sc_task_log2": args.sc_task_log2,
                   "runs_per_step": len(runs), "iterations_per_run": iters_per_run,
                   "edges_traversed_per_step": edges_per_step, "preprocess_ms": prep_ms},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS, "traffic": traffic,
                     "alg_bytes_per_launch": bytes_step[dom] / per_kernel[dom]["launches_per_step"]},
        "per_kernel": per_kernel,
    }
    if args.copy_mib:
        # a plain elementwise copy kernel of known size (reads and writes
        # 4n bytes): the measured ceiling, and the reference that scales
        # rocprofv3 FETCH_SIZE / WRITE_SIZE
        n = args.copy_mib << 18
        a = torch.empty(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.bitwise_not(a, out=b)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.bitwise_not(a, out=b)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        out["copy_ceiling"] = {"bytes": 2 * 4 * n, "GBps": 2 * 4 * n / (ms * 1e-3) / 1e9}
        out["roofline"]["frac_of_copy"] = ach / out["copy_ceiling"]["GBps"]
        del a, b
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        v, sample = cpu_baseline(g, runs, args.cpu_budget)
        out["cpu_baseline"] = {"value": v, "unit": "GTEPS", "cores": 1, "kind": "oracle",
                               "sample": sample}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
