"""Benchmark: k-bisimulation to the fixed point (cap k=10) of a 10M-node /
100M-edge power-law graph on one MI355X.

A step is one whole job on the graph, with the edge table already resident in
device memory: kbisim_create (validation, pId_0, edge-label ranks, CSR build)
+ kbisim_refine(k) (rounds to the fixed point or k) + kbisim_result (ids to a
device buffer) + destroy. value = |E| * rounds / seconds per step.

Prints one JSON line (rank 0). Options:
  --gpus N        only N=1 is supported (one GPU per box)
  --steps K       timed steps (default 3)
  --warmup W      untimed steps first (default 1)
  --workload W    synth.CONFIGS name (default powerlaw-10M-100M)
  --k K           round cap (default: the workload's, 10)
  --no-early-stop run all K rounds even past the fixed point
  --no-cpu-baseline   skip timing the oracle on the host
  --form F        plain (default), batched or served: the two system forms
                  print their own JSON line (see bench_batched / bench_served)
  --host-io M     plain job with host inputs and result (pinned or pageable):
                  the PCIe-inclusive rate, on its own JSON line
  --copy-probe    only a 1 GiB device-to-device copy (1 GiB read, 1 GiB
                  written): the calibration run for rocprofv3 FETCH_SIZE /
                  WRITE_SIZE readings of the library's kernels
  --form update   maintenance (Section 5.3): m random edges of the graph are
                  left out, the partition of the rest is computed with the
                  history kept, then kbisim_update adds the m edges back;
                  its time against a rebuild of the whole job, for
                  m = 1, 10, ..., --max-batch (one JSON line)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per unit of the signature launch: each edge of an active
# node reads its (label, dst) table entry (4 + 4 B in a plain table layout)
# and gathers pid_prev[dst] (4 B); each active node reads row_ptr (4 B) and
# pid_prev (4 B) and its id write is 4 B.
BYTES_PER_EDGE = 12
BYTES_PER_NODE = 12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1210_0748_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1210_0748_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_class, workload, early_stop, k_cap):
    """HBM bytes per launch measured with rocprofv3 counters, if the committed
    measurement was taken on the current kernel sources and on this same job
    (workload, early stop, k), else None: the average over a job's launches
    depends on its rounds."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_digest") != kernel_source_digest():
        return None
    # entries are named "<class>" or "<class>@<workload>"; the one read on this job counts
    for name, k in t.get("kernels", {}).items():
        if name.split("@")[0] != kernel_class:
            continue
        if (k.get("workload"), k.get("early_stop"), k.get("k_cap")) == (workload, early_stop, k_cap):
            return k.get("bytes_per_launch")
    return None


# Workloads up to this many edges: the oracle runs the whole job itself.
WHOLE_JOB_ORACLE_EDGES = 1_000_000
# Larger ones: a sample with about this many out-edges (about 16 s of oracle work).
SAMPLE_EDGES = 25_000_000


def cpu_baseline(seed=1, g=None, k=None, early_stop=True):
    """The oracle (single thread) on the measured workload `g`. Small
    workloads (at most WHOLE_JOB_ORACLE_EDGES edges): the whole job (k rounds,
    the same stop rule). Larger ones: a bounded sample of the same graph,
    the oracle's round 1 over a seeded uniform sample of its nodes (a
    quarter, or fewer so that the sample has about SAMPLE_EDGES out-edges)
    with all their out-edges (signatures from pId_0, one ordered
    dictionary), rated per edge of the sample; its scan of the whole edge
    table is charged to the sample."""
    import numpy as np
    import oracle
    oracle.build()
    if g.num_edges <= WHOLE_JOB_ORACLE_EDGES:
        t0 = time.perf_counter()
        r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k, early_stop=early_stop)
        dt = time.perf_counter() - t0
        return {"value": g.num_edges * r.rounds_done / dt, "unit": "edge-rounds/s", "cores": 1,
                "kind": "oracle", "seconds": dt, "rounds": r.rounds_done,
                "sample": "the whole job (%s, k=%d, %s); %.3f s" % (
                    g.name, k, "early stop" if early_stop else "no early stop", dt)}
    rng = np.random.Generator(np.random.PCG64(seed))
    frac = min(0.25, SAMPLE_EDGES / g.num_edges)
    size = max(1, int(g.num_nodes * frac))
    sample = np.sort(rng.choice(g.num_nodes, size=size, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    _, edges = oracle.round_sample(g.num_nodes, g.node_label, g.src, g.elab, g.dst, sample)
    dt = time.perf_counter() - t0
    return {"value": edges / dt, "unit": "edge-rounds/s", "cores": 1, "kind": "oracle", "seconds": dt,
            "sample": "oracle round 1 of the measured graph (%s) over a seeded uniform sample of %.1f%% of its "
                      "nodes (%d nodes, %d out-edges, seed %d); %.1f s" % (g.name, 100 * frac, size, edges, seed,
                                                                           dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="powerlaw-10M-100M")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-early-stop", action="store_true",
                    help="plain form: run all k rounds even past the fixed point")
    ap.add_argument("--medium-cap", type=int, default=None)
    ap.add_argument("--radix-tile", type=int, default=0, help="items per radix-sort tile (0 = library default)")
    ap.add_argument("--form", choices=["plain", "batched", "served", "update"], default="plain")
    ap.add_argument("--max-batch", type=int, default=1_000_000, help="update: largest batch of added edges")
    ap.add_argument("--graphs", type=int, default=512, help="batched: number of graphs")
    ap.add_argument("--requests", type=int, default=300, help="served: number of requests")
    ap.add_argument("--max-nodes", type=int, default=10_000_000, help="served: largest request")
    ap.add_argument("--slots", type=int, default=4, help="served: concurrent slots")
    ap.add_argument("--host-io", choices=["pinned", "pageable"], default=None,
                    help="plain form: inputs and result in host memory (PCIe included; its own JSON line)")
    ap.add_argument("--edge-window", type=int, default=0,
                    help="with --host-io: keep the edge table in host memory, streamed through device windows "
                         "of this many bytes in all")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1210_0748_amd as kb
    kb.load_library()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.copy_probe:
        return copy_probe(torch, dev)
    if args.form == "batched":
        return bench_batched(args, torch, kb, dev)
    if args.form == "served":
        return bench_served(args, torch, kb, dev)
    if args.form == "update":
        return bench_update(args, torch, kb, dev)
    if args.host_io:
        return bench_host_io(args, torch, kb)

    t0 = time.perf_counter()
    g, k_default = synth.make_config(args.workload, seed=args.seed, progress=log)
    k = args.k if args.k is not None else k_default
    log("generated %s: N=%d E=%d in %.1f s" % (args.workload, g.num_nodes, g.num_edges,
                                                time.perf_counter() - t0))
    arrs = [torch.from_numpy(a).to(dev) for a in (g.node_label, g.src, g.elab, g.dst)]
    out = torch.empty(g.num_nodes, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    early_stop = not args.no_early_stop
    torch.cuda.synchronize()

    def step(profile):
        h = kb.kbisim_create(g.num_nodes, *arrs, stream=stream, profile=profile,
                             medium_cap=args.medium_cap, radix_tile=args.radix_tile, early_stop=early_stop)
        try:
            rd = kb.kbisim_refine(h, k)
            nb, counts = kb.kbisim_result(h, out, counts_cap=k + 1)
            prof = kb.kbisim_profile(h) if profile else None
            work = (kb.kbisim_work(h), kb.kbisim_round_profile(h)) if profile else None
        finally:
            kb.kbisim_destroy(h)
        return rd, counts, prof, work

    for w in range(args.warmup):
        rd, counts, _, _ = step(False)
        log("warmup %d: rounds=%d counts=%s" % (w, rd, counts))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        rd, counts, _, _ = step(False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / max(args.steps, 1)
    value = g.num_edges * rd / (ms_per_step / 1e3)
    log("timed %d steps: %.2f ms/step, rounds=%d" % (args.steps, ms_per_step, rd))

    # Phases of one more (untimed) step, each closed by a device sync.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = kb.kbisim_create(g.num_nodes, *arrs, stream=stream, medium_cap=args.medium_cap,
                         radix_tile=args.radix_tile, early_stop=early_stop)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kb.kbisim_refine(h, k)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kb.kbisim_result(h, out, counts_cap=k + 1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    kb.kbisim_destroy(h)
    phases = {"create_ms": (t1 - t0) * 1e3, "refine_ms": (t2 - t1) * 1e3, "result_ms": (t3 - t2) * 1e3}
    log("phases: " + json.dumps(phases))

    # One extra profiled step (HIP events on the library's stream around each
    # launch) for the per-kernel roofline; not part of the timed region.
    rd_p, counts_p, prof, (work, per_round) = step(True)
    assert counts_p == counts
    log("profile: " + json.dumps(prof))
    log("work: " + json.dumps(work))
    # dominant kernel: the signature launch (one per round, all degree buckets)
    dom = "signature"
    ms_total, launches = prof[dom]
    nodes = sum(v[0] for v in work.values())
    edges = sum(v[1] for v in work.values())
    algo_bytes_per_launch = (BYTES_PER_EDGE * edges + BYTES_PER_NODE * nodes) / max(launches, 1)
    avg_ms = ms_total / max(launches, 1)
    achieved = algo_bytes_per_launch / (avg_ms / 1e3) / 1e9
    traffic = load_traffic(dom, args.workload, early_stop, k)
    line = {
        "metric": ("edge-rounds/s (|E|*rounds/time), %s %s" % (
            "10M-node/100M-edge power-law graph" if args.workload == "powerlaw-10M-100M" else args.workload,
            ("to fixed point" if args.workload == "powerlaw-10M-100M" else "to fixed point (cap k)")
            if early_stop else "all k rounds, no early stop")),
        "value": value,
        "unit": "edge-rounds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "num_nodes": g.num_nodes, "num_edges": g.num_edges,
                   "k_cap": k, "early_stop": early_stop, "rounds": rd, "counts": counts, "seed": args.seed,
                   **({"radix_tile": args.radix_tile} if args.radix_tile else {})},
        "phases": dict(phases, note="one untimed step, each phase closed by a device sync"),
        "roofline": {"bound": "hbm", "kernel": "signature_k", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "launch_avg_ms": avg_ms, "algo_bytes_per_launch": algo_bytes_per_launch},
        "kernel_ms": {c: prof[c][0] for c in prof},
        # round by round: the signature launch's algorithmic GB/s and the round's time
        # (max_sig_ints: the longest signature as integers, the old id plus a (label, id) pair per key)
        "rounds": [{"round": r + 1, "blocks": counts[r + 1] if r + 1 < len(counts) else None,
                    "max_sig_ints": 1 + 2 * x["max_keys"],
                    "active_nodes": x["active_nodes"], "active_edges": x["active_edges"],
                    "signature_ms": x["signature_ms"], "round_ms": x["round_ms"],
                    "signature_gbs": (BYTES_PER_EDGE * x["active_edges"] + BYTES_PER_NODE * x["active_nodes"])
                    / max(x["signature_ms"], 1e-9) / 1e6}
                   for r, x in enumerate(per_round)],
    }
    # edges whose signature was actually built (active nodes' out-edges),
    # per second of the step: the rate of work done, beside the headline's
    # |E| * rounds
    processed = sum(x["active_edges"] for x in per_round)
    line["processed_edges"] = {"per_step": processed, "per_s": processed / (ms_per_step / 1e3)}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        line["cpu_baseline"] = cpu_baseline(args.seed, g, k, early_stop)
        full = recorded_full_job(args.workload, args.seed, early_stop, k)
        if full:
            line["cpu_baseline"]["full_job_recorded"] = full
    print(json.dumps(line), flush=True)


def recorded_full_job(workload, seed, early_stop, k):
    """The oracle's whole run on this workload as recorded when its golden
    file was written (tests/golden/make_fullsize.py, one thread), if any."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "%s%s.json" % (
        workload, "" if early_stop else "_k%d-no-early-stop" % k))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("seed") != seed or d.get("k") != k or "oracle_seconds" not in d:
        return None
    return {"seconds": d["oracle_seconds"], "value": d["oracle_edge_rounds_per_s"], "unit": "edge-rounds/s",
            "rounds": d["rounds_done"], "cores": 1, "host": d.get("oracle_host"), "source": os.path.relpath(path)}


def copy_probe(torch, dev):
    """A device copy of known size (1 GiB read, 1 GiB written). Run under the
    same rocprofv3 counter collection as the library, its FETCH_SIZE and
    WRITE_SIZE readings turn the library's readings into bytes."""
    n = 1 << 28  # int32 elements: 1 GiB
    a = torch.ones(n, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log("copied %d bytes" % (4 * n))


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def bench_batched(args, torch, kb, dev):
    """Batched form: many graphs of log-normal size (median 20k nodes, sigma
    1, 1k..1M nodes, mean out-degree 8, 16 node and 16 edge labels), k = 5,
    refined as one batch (medium_cap and radix_tile from the autotuner) vs the per-graph
    plain refine loop on the same GPU; results must be identical."""
    import numpy as np
    import synth
    from paper_1210_0748_amd import autotune
    k = 5
    t0 = time.perf_counter()
    graphs = synth.batch_graphs(args.graphs, seed=args.seed, progress=log)
    noff = np.zeros(len(graphs) + 1, np.int64)
    eoff = np.zeros(len(graphs) + 1, np.int64)
    for i, g in enumerate(graphs):
        noff[i + 1] = noff[i] + g.num_nodes
        eoff[i + 1] = eoff[i] + g.num_edges
    cat = lambda name: np.concatenate([getattr(g, name) for g in graphs])
    arrs = [torch.from_numpy(cat(nm)).to(dev) for nm in ("node_label", "src", "elab", "dst")]
    log("generated %d graphs: N=%d E=%d in %.1f s" % (len(graphs), noff[-1], eoff[-1], time.perf_counter() - t0))
    (cap, tile), tune_report = autotune.tune(graphs, k, use_cache=False)
    log("autotuned medium_cap=%d radix_tile=%d %s" % (cap, tile, json.dumps(tune_report)))
    out = torch.empty(int(noff[-1]), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def batched():
        h, G = kb.kbisim_batch_create(noff, eoff, *arrs, stream=stream, medium_cap=cap, radix_tile=tile)
        try:
            rd = kb.kbisim_batch_refine(h, [k] * G)
            kb.kbisim_batch_result(h, G, out)
        finally:
            kb.kbisim_batch_destroy(h)
        return rd

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rd = batched()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / max(args.steps, 1)
    edge_rounds = float(np.sum((eoff[1:] - eoff[:-1]) * rd))
    got = out.cpu().numpy()

    # per-graph plain refine loop (same device-resident inputs, one pass)
    loop_out = torch.empty_like(out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, g in enumerate(graphs):
        a, b = int(noff[i]), int(noff[i + 1])
        c, d = int(eoff[i]), int(eoff[i + 1])
        h = kb.kbisim_create(b - a, arrs[0][a:b], arrs[1][c:d], arrs[2][c:d], arrs[3][c:d], stream=stream,
                             medium_cap=cap, radix_tile=tile)
        try:
            kb.kbisim_refine(h, k)
            kb.kbisim_result(h, loop_out[a:b])
        finally:
            kb.kbisim_destroy(h)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    same = bool(np.array_equal(got, loop_out.cpu().numpy()))
    line = {
        "metric": "batched edge-rounds/s (sum over graphs of |E|*rounds / time)",
        "value": edge_rounds / t_batch, "unit": "edge-rounds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batched-%d-graphs" % len(graphs), "graphs": len(graphs),
                   "total_nodes": int(noff[-1]), "total_edges": int(eoff[-1]), "k": k,
                   "median_nodes": 20000, "sigma": 1.0, "avg_degree": 8, "labels": 16},
        "medium_cap": cap, "radix_tile": tile, "tune": tune_report,
        "per_graph_loop": {"ms": t_loop * 1e3, "edge_rounds_per_s": edge_rounds / t_loop},
        "speedup_vs_loop": t_loop / t_batch, "identical_to_loop": same,
    }
    print(json.dumps(line), flush=True)


def bench_update_extreme(args, torch, kb, dev):
    """The two extreme cases of Section 5.3 at about 100M edges, one edge
    added, k = 10: Dbest, a full 10-ary tree of height 8 (one node and one
    edge label) and an edge from a parent of leaves to a leaf of another
    parent (no signature changes); Dworst, the complete graph on 10,000
    nodes (edges labelled x) and an edge labelled y from node 0 to a new
    isolated node (every signature changes). The update against a rebuild
    of the updated graph (plain job), ids compared bit for bit."""
    import numpy as np
    import synth
    k = 10
    if args.workload == "dbest-100M":
        g = synth.tree_graph(10, 8)
        n = g.num_nodes
        leaves0 = n - 10 ** 8
        upd = dict(add=(np.array([(leaves0 - 1) // 10], np.int32), np.array([0], np.int32),
                        np.array([n - 1], np.int32)))
        new_labels = None
    else:
        g = synth.complete_graph(10_000)
        n = g.num_nodes
        upd = dict(new_labels=np.array([0], np.int32),
                   add=(np.array([0], np.int32), np.array([1], np.int32), np.array([n], np.int32)))
        new_labels = upd["new_labels"]
    log("%s: N=%d E=%d" % (args.workload, g.num_nodes, g.num_edges))
    arrs = [torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(dev) for a in (g.node_label, g.src, g.elab, g.dst)]
    stream = torch.cuda.current_stream()
    # the updated graph, for the rebuild
    lab2 = np.concatenate([g.node_label, new_labels]) if new_labels is not None else g.node_label
    n2 = lab2.shape[0]
    up = [torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(dev) for a in upd["add"]]
    arrs2 = [torch.from_numpy(np.ascontiguousarray(lab2, np.int32)).to(dev)] + \
        [torch.cat([a, b]) for a, b in zip(arrs[1:], up)]
    out_r = torch.empty(n2, dtype=torch.int32, device=dev)
    out_u = torch.empty(n2, dtype=torch.int32, device=dev)

    def rebuild():
        h = kb.kbisim_create(n2, *arrs2, stream=stream)
        try:
            rd = kb.kbisim_refine(h, k)
            kb.kbisim_result(h, out_r)
        finally:
            kb.kbisim_destroy(h)
        return rd

    rebuild()
    torch.cuda.synchronize()
    ts = []
    for _ in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        rd_r = rebuild()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    t_rebuild = float(np.median(ts))
    rows = []
    nl_dev = torch.from_numpy(upd["new_labels"]).to(dev) if "new_labels" in upd else None
    for mode in (0, 1, 2):
        tu = []
        for rep in range(max(args.steps, 1) + 1):
            h = kb.kbisim_create(n, *arrs, stream=stream, history=True, update_mode=mode)
            try:
                rd0 = kb.kbisim_refine(h, k)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rd1 = kb.kbisim_update(h, new_labels=nl_dev, add=tuple(up))
                torch.cuda.synchronize()
                if rep:
                    tu.append((time.perf_counter() - t0) * 1e3)
                stats = kb.kbisim_update_stats(h)
                kb.kbisim_result(h, out_u)
            finally:
                kb.kbisim_destroy(h)
        same = bool(torch.equal(out_u, out_r)) and rd1 == rd_r
        rows.append({"update_mode": ["by cost", "level by level", "full rounds"][mode],
                     "update_ms": float(np.median(tu)), "speedup_vs_rebuild": t_rebuild / float(np.median(tu)),
                     "rounds": rd1, "levels": stats[0], "full_rounds_from": stats[1], "rechecked": stats[2],
                     "recomputed": stats[3], "changed": stats[4], "identical_to_rebuild": same})
        log("%s mode %d: update %.2f ms vs rebuild %.2f ms, stats %s, identical %s" % (
            args.workload, mode, rows[-1]["update_ms"], t_rebuild, stats, same))
    line = {
        "metric": "Add_Edges time vs rebuild (ms), %s, one edge added" % args.workload,
        "value": rows[0]["update_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": rows[0]["update_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "num_nodes": g.num_nodes, "num_edges": g.num_edges, "k": k,
                   "rounds": rd_r},
        "rebuild_ms": t_rebuild, "modes": rows,
        "identical_to_rebuild": all(r["identical_to_rebuild"] for r in rows),
    }
    print(json.dumps(line), flush=True)


def bench_update(args, torch, kb, dev):
    """Add_Edges against a rebuild (the paper's multiple-edge experiment,
    Section 5.3): for each batch size m, m edges drawn at random from the
    graph are left out, the job runs on the rest with the history kept, and
    kbisim_update adds the m edges back. The updated ids must equal those of
    the whole graph's job bit for bit. The rebuild is the plain job (create,
    refine, result) on the whole graph, with and without the history."""
    import numpy as np
    import synth
    if args.workload in ("dbest-100M", "dworst-100M"):
        return bench_update_extreme(args, torch, kb, dev)
    g, k_default = synth.make_config(args.workload, seed=args.seed, progress=log)
    k = args.k if args.k is not None else k_default
    arrs = [torch.from_numpy(a).to(dev) for a in (g.node_label, g.src, g.elab, g.dst)]
    stream = torch.cuda.current_stream()
    ref = torch.empty(g.num_nodes, dtype=torch.int32, device=dev)

    def job(history):
        h = kb.kbisim_create(g.num_nodes, *arrs, stream=stream, history=history)
        try:
            rd = kb.kbisim_refine(h, k)
            kb.kbisim_result(h, ref)
        finally:
            kb.kbisim_destroy(h)
        return rd

    rebuild = {}
    for history in (False, True):
        job(history)
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(args.steps, 1)):
            t0 = time.perf_counter()
            rd = job(history)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        rebuild["history" if history else "plain"] = float(np.median(ts))
    want = ref.cpu().numpy()
    log("rebuild: %s ms, rounds=%d" % (rebuild, rd))
    rng = np.random.Generator(np.random.PCG64(args.seed + 17))
    rows = []
    m = 1
    out = torch.empty(g.num_nodes, dtype=torch.int32, device=dev)
    while m <= min(args.max_batch, g.num_edges):
        pick = np.sort(rng.choice(g.num_edges, size=m, replace=False))
        keep = np.ones(g.num_edges, bool)
        keep[pick] = False
        keep_t = torch.from_numpy(keep).to(dev)
        base = [arrs[0]] + [a[keep_t].contiguous() for a in arrs[1:]]
        added = [a[torch.from_numpy(pick).to(dev)].contiguous() for a in arrs[1:]]
        h = kb.kbisim_create(g.num_nodes, *base, stream=stream, history=True)
        try:
            rd0 = kb.kbisim_refine(h, k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rd1 = kb.kbisim_update(h, add=tuple(added))
            torch.cuda.synchronize()
            t_upd = (time.perf_counter() - t0) * 1e3
            levels, full_from, rechecked, recomputed, changed = kb.kbisim_update_stats(h)
            kb.kbisim_result(h, out)
        finally:
            kb.kbisim_destroy(h)
        same = bool(np.array_equal(out.cpu().numpy(), want)) and rd1 == rd
        rows.append({"edges": m, "update_ms": t_upd, "speedup_vs_rebuild": rebuild["plain"] / t_upd,
                     "rounds_before": rd0, "rounds_after": rd1, "full_rounds_from": full_from,
                     "rechecked": rechecked, "recomputed": recomputed,
                     "changed": changed, "identical_to_rebuild": same})
        log("m=%d: update %.2f ms (rebuild %.2f ms), full rounds from %d, rechecked %d, recomputed %d, "
            "identical %s" % (m, t_upd, rebuild["plain"], full_from, rechecked, recomputed, same))
        del base, added, keep_t
        m *= 10
    line = {
        "metric": "Add_Edges time vs rebuild (ms), %s, m random edges added back" % args.workload,
        "value": rows[0]["update_ms"] if rows else None, "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rows[0]["update_ms"] if rows else None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "num_nodes": g.num_nodes, "num_edges": g.num_edges, "k_cap": k,
                   "rounds": rd},
        "rebuild_ms": rebuild, "batches": rows,
        "identical_to_rebuild": all(r["identical_to_rebuild"] for r in rows),
    }
    print(json.dumps(line), flush=True)


def bench_host_io(args, torch, kb):
    """The plain job with the edge table and labels in host memory and the
    ids returned to host memory: create copies the inputs over PCIe, the
    result copies the ids back. Pinned buffers come from torch's pinned
    allocator; pageable ones are plain numpy arrays."""
    import numpy as np
    import synth
    g, k_default = synth.make_config(args.workload, seed=args.seed, progress=log)
    k = args.k if args.k is not None else k_default
    if args.host_io == "pinned":
        keep = [torch.from_numpy(a).pin_memory() for a in (g.node_label, g.src, g.elab, g.dst)]
        inputs = [t.numpy() for t in keep]
        keep.append(torch.empty(g.num_nodes, dtype=torch.int32).pin_memory())
        out = keep[-1].numpy()
    else:
        inputs = [g.node_label, g.src, g.elab, g.dst]
        out = np.empty(g.num_nodes, np.int32)

    stats = {}

    def job():
        h = kb.kbisim_create(g.num_nodes, *inputs, early_stop=not args.no_early_stop,
                             edge_window_bytes=args.edge_window)
        try:
            rd = kb.kbisim_refine(h, k)
            _, counts = kb.kbisim_result(h, out, counts_cap=k + 1)
            if args.edge_window:
                stats["partitions"], stats["bytes_moved_by_rounds"], stats["rounds_in_place"] = \
                    kb.kbisim_stream_stats(h)
        finally:
            kb.kbisim_destroy(h)
        return rd, counts

    # device memory one job holds: the library's cache after a job run from
    # an empty cache (its blocks are reused within the job, so this is about
    # the job's peak)
    kb.kbisim_release_cached()
    job()
    device_bytes = kb.kbisim_release_cached()
    for _ in range(args.warmup):
        job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rd, counts = job()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    in_bytes = 4 * (g.num_nodes + 3 * g.num_edges)
    what = ("edge table kept in %s host memory and streamed through %d-byte device windows every round" % (
        args.host_io, args.edge_window) if args.edge_window else "including the host-device copies (%s host memory)"
            % args.host_io)
    line = {
        "metric": "edge-rounds/s %s, %s" % (what, args.workload),
        "value": g.num_edges * rd / (ms / 1e3), "unit": "edge-rounds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "num_nodes": g.num_nodes, "num_edges": g.num_edges, "k_cap": k,
                   "rounds": rd, "counts": counts, "host_io": args.host_io,
                   "bytes_in": in_bytes, "bytes_out": 4 * g.num_nodes, "edge_window_bytes": args.edge_window},
        "device_bytes": device_bytes,
        "device_bytes_per_edge": device_bytes / max(g.num_edges, 1),
    }
    if stats:
        line["streamed"] = stats
    print(json.dumps(line), flush=True)


def bench_served(args, torch, kb, dev):
    """Served form: Poisson arrivals (rate 200/s) of k-bisimulation requests;
    sizes log-uniform between 10k nodes and --max-nodes, |E| = 10 |N| with a
    power-law out-degree, 32 edge labels, k uniform in 2..10. Requests refer
    to a device-resident pool of graphs (24 sizes, generated and uploaded
    once). The server (HBM budget 200 GB) runs them concurrently; the
    baseline solves them one after another in arrival order on one stream.
    Latency = completion - arrival."""
    import numpy as np
    import synth
    rng = np.random.Generator(np.random.PCG64(args.seed))
    sizes = np.unique(np.round(np.geomspace(10_000, args.max_nodes, 24)).astype(np.int64))
    t0 = time.perf_counter()
    pool = []
    for i, n in enumerate(sizes):
        g = synth.powerlaw_graph(int(n), int(10 * n), seed=(args.seed, 1000 + i), deg_cap=max(64, int(n) // 10))
        pool.append((g.num_nodes, [torch.from_numpy(a).to(dev) for a in (g.node_label, g.src, g.elab, g.dst)],
                     g.num_edges))
        log("request pool: graph %d of %d (%d nodes) after %.1f s" % (i + 1, len(sizes), n, time.perf_counter() - t0))
    log("request pool: %d graphs, %d..%d nodes, %.1f s" % (len(pool), sizes[0], sizes[-1], time.perf_counter() - t0))
    reqs = synth.serving_stream(args.requests, seed=args.seed, rate=200.0, max_nodes=args.max_nodes)
    logs = np.log(sizes)
    for r in reqs:
        r["pool"] = int(np.argmin(np.abs(logs - np.log(r["num_nodes"]))))
    torch.cuda.synchronize()

    # served: submit each request at its arrival time
    lat, results = [], {}
    with kb.Server(200 << 30, max_slots=args.slots) as srv:
        ids = []
        t_start = time.perf_counter()
        for r in reqs:
            now = time.perf_counter() - t_start
            if r["arrival"] > now:
                time.sleep(r["arrival"] - now)
            n, a, _ = pool[r["pool"]]
            ids.append((srv.submit(n, *a, r["k"]), time.perf_counter() - t_start))
        done_at = []
        for (rid, t_sub), r in zip(ids, reqs):
            pid, nb, rd = srv.wait(rid, timeout_s=600)
            q, tot = srv.timing(rid)
            done_at.append(t_sub + tot)
            lat.append(t_sub + tot - r["arrival"])
            results[rid] = (pid, rd)
            srv.release(rid)
        makespan = max(done_at) if done_at else 0.0

    # serial plain solves in arrival order on one stream
    lat_s, same = [], True
    stream = torch.cuda.current_stream()
    t_start = time.perf_counter()
    for (rid, _), r in zip(ids, reqs):
        now = time.perf_counter() - t_start
        if r["arrival"] > now:
            time.sleep(r["arrival"] - now)
        n, a, _ = pool[r["pool"]]
        with kb.Graph(n, *a, stream=stream) as h:
            rd = h.refine(r["k"])
            pid, nb, counts = h.result()
        lat_s.append(time.perf_counter() - t_start - r["arrival"])
        same = same and rd == results[rid][1] and np.array_equal(pid, results[rid][0])
    makespan_s = time.perf_counter() - t_start
    er = float(sum(pool[r["pool"]][2] * results[rid][1] for (rid, _), r in zip(ids, reqs)))
    line = {
        "metric": "served requests/s with p50/p99 latency (Poisson arrivals, 200/s)",
        "value": len(reqs) / makespan, "unit": "req/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": makespan * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "served-poisson-200", "requests": len(reqs), "min_nodes": 10000,
                   "max_nodes": args.max_nodes, "avg_degree": 10, "edge_labels": 32, "k": "uniform 2..10",
                   "hbm_budget_gb": 200, "slots": args.slots, "pool_graphs": len(pool)},
        "latency_s": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat) if lat else None},
        "edge_rounds_per_s": er / makespan,
        "serial_baseline": {"req_per_s": len(reqs) / makespan_s, "p50": pct(lat_s, 50), "p99": pct(lat_s, 99),
                            "edge_rounds_per_s": er / makespan_s},
        "identical_to_serial": bool(same),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
