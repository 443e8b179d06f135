"""Writes the oracle's whole result on a large seeded workload as a compact
golden file: per round a SHA-256 digest of the id array (int32, little
endian, node order), the block counts, rounds_done, the longest signature per
round, and the ids of a fixed sample of nodes (to locate a mismatch).

Only the oracle (``oracle/``) and the seeded generators (``synth/``) are
called; nothing here touches the GPU library. The GPU parity test recomputes
the same digests from the library's per-round ids and compares them, which is
an element-by-element comparison of every node in every round.

usage: python tests/golden/make_fullsize.py [workload] [--no-early-stop] [--k K]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLE_SEED = 7
SAMPLE_NODES = 2000


def digest(ids: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(ids, dtype="<i4").tobytes()).hexdigest()


def sample_of(n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return np.sort(rng.choice(n, size=min(n, SAMPLE_NODES), replace=False)).astype(np.int64)


def golden_path(workload: str, early_stop: bool, k: int) -> str:
    tag = "" if early_stop else "_k%d-no-early-stop" % k
    return os.path.join(HERE, "%s%s.json" % (workload, tag))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", nargs="?", default="powerlaw-10M-100M")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--no-early-stop", action="store_true")
    args = ap.parse_args()
    t0 = time.perf_counter()
    g, k_default = synth.make_config(args.workload, seed=args.seed,
                                     progress=lambda m: print(m, flush=True))
    k = args.k if args.k is not None else k_default
    early_stop = not args.no_early_stop
    t_gen = time.perf_counter() - t0
    print("generated %s N=%d E=%d in %.1f s" % (args.workload, g.num_nodes, g.num_edges, t_gen), flush=True)
    oracle.build()
    t0 = time.perf_counter()
    r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k, history=True,
                      early_stop=early_stop)
    t_oracle = time.perf_counter() - t0
    print("oracle: rounds=%d counts=%s in %.1f s" % (r.rounds_done, r.counts, t_oracle), flush=True)
    sample = sample_of(g.num_nodes)
    rows = r.history[: r.rounds_done + 1]
    # longest signature per round among nodes of classes with two or more
    # members in the previous round (the nodes a round can still split)
    multi = [1]
    for j in range(1, r.rounds_done + 1):
        lengths = oracle.signature_lengths(g.num_nodes, g.src, g.elab, g.dst, rows[j - 1])
        multi.append(oracle.longest_multi_member(lengths, rows[j - 1]))
        print("round %d: longest signature in a class of two or more: %d ints" % (j, multi[-1]), flush=True)
    out = {
        "source": "oracle/kbisim_oracle.cpp (Algorithm 1 with an ordered-dictionary S) on the seeded "
                  "synthetic workload; written by tests/golden/make_fullsize.py",
        "workload": args.workload, "seed": args.seed, "num_nodes": g.num_nodes, "num_edges": g.num_edges,
        "k": k, "early_stop": early_stop,
        "rounds_done": r.rounds_done, "counts": r.counts, "max_sig_ints": r.max_sig_ints,
        "max_sig_ints_multi": multi,
        "digest": "sha256 of the int32 little-endian id array of each round, node order",
        "round_digests": [digest(rows[j]) for j in range(r.rounds_done + 1)],
        "sample_seed": SAMPLE_SEED, "sample_nodes": sample.tolist(),
        "sample_ids": [rows[j][sample].tolist() for j in range(r.rounds_done + 1)],
        "oracle_seconds": t_oracle,
        "oracle_edge_rounds_per_s": g.num_edges * r.rounds_done / t_oracle,
        "oracle_host": {"machine": platform.machine(), "processor": platform.processor() or None,
                        "threads": 1, "numpy": np.__version__},
    }
    path = golden_path(args.workload, early_stop, k)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print("wrote %s" % path, flush=True)


if __name__ == "__main__":
    main()
