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
  --no-cpu-baseline   skip timing the oracle on the host
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
# Algorithmic bytes per unit of the signature kernels: each processed edge
# reads its (label, dst) table entry (4 + 4 B in a plain table layout) and
# gathers pid_prev[dst] (4 B); each processed node reads row_ptr (4 B) and
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


def load_traffic(kernel_class):
    """HBM bytes per launch measured with rocprofv3 counters, if the committed
    measurement was taken on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_digest") != kernel_source_digest():
        return None
    return t.get("kernels", {}).get(kernel_class)


def cpu_baseline(seed=1):
    """The oracle (single thread) on a bounded sample: the first two rounds of
    a 1M-node / 10M-edge graph drawn from the same power-law recipe."""
    import oracle
    import synth
    g = synth.powerlaw_graph(1_000_000, 10_000_000, seed=seed, name="powerlaw-1M-10M")
    oracle.build()
    t0 = time.perf_counter()
    r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 2, early_stop=False)
    dt = time.perf_counter() - t0
    return {"value": g.num_edges * r.rounds_done / dt, "unit": "edge-rounds/s", "cores": 1,
            "kind": "oracle",
            "sample": "oracle rounds 1-2 (plus its adjacency build) of a 1M-node / 10M-edge graph "
                      "from the same power-law recipe, seed %d; %.1f s" % (seed, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="powerlaw-10M-100M")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--medium-cap", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
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

    t0 = time.perf_counter()
    g, k_default = synth.make_config(args.workload, seed=args.seed)
    k = args.k if args.k is not None else k_default
    log("generated %s: N=%d E=%d in %.1f s" % (args.workload, g.num_nodes, g.num_edges,
                                                time.perf_counter() - t0))
    arrs = [torch.from_numpy(a).to(dev) for a in (g.node_label, g.src, g.elab, g.dst)]
    out = torch.empty(g.num_nodes, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(profile):
        h = kb.kbisim_create(g.num_nodes, *arrs, stream=stream, profile=profile,
                             medium_cap=args.medium_cap)
        try:
            rd = kb.kbisim_refine(h, k)
            nb, counts = kb.kbisim_result(h, out, counts_cap=k + 1)
            prof = kb.kbisim_profile(h) if profile else None
            work = kb.kbisim_work(h) if profile else None
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

    # One extra profiled step (HIP events on the library's stream around each
    # launch) for the per-kernel roofline; not part of the timed region.
    rd_p, counts_p, prof, work = step(True)
    assert counts_p == counts
    log("profile: " + json.dumps(prof))
    log("work: " + json.dumps(work))
    classes = ["sig_thread", "sig_wave", "sig_block", "sig_hub"]
    dom = max(classes, key=lambda c: prof[c][0])
    ms_total, launches = prof[dom]
    nodes, edges = work[dom]
    # the thread-per-node kernel also reads row_ptr and pid of every node
    scanned_nodes = g.num_nodes * launches if dom == "sig_thread" else nodes
    algo_bytes_per_launch = (BYTES_PER_EDGE * edges + BYTES_PER_NODE * scanned_nodes) / max(launches, 1)
    avg_ms = ms_total / max(launches, 1)
    achieved = algo_bytes_per_launch / (avg_ms / 1e3) / 1e9
    traffic = load_traffic(dom)
    rounds_only_ms = prof["round"][0]
    line = {
        "metric": "edge-rounds/s (|E|*rounds/time), 10M-node/100M-edge power-law graph to fixed point",
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
                   "k_cap": k, "rounds": rd, "counts": counts, "seed": args.seed},
        "rounds_only": {"ms": rounds_only_ms,
                        "edge_rounds_per_s": g.num_edges * rd / (rounds_only_ms / 1e3),
                        "note": "sum of per-round event times of the profiled step (no create)"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "launch_avg_ms": avg_ms, "algo_bytes_per_launch": algo_bytes_per_launch},
        "kernel_ms": {c: prof[c][0] for c in prof},
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        line["cpu_baseline"] = cpu_baseline(args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
