"""Autotuner for the ordering kernels' size split (medium_cap).

Groups of up to 64 members are ordered by one wave, groups of up to
`medium_cap` members by one workgroup in LDS, larger groups by global radix
passes. The best split depends on the workload's block-size distribution, so
the tuner times a refinement of a sample of the workload with every
candidate and keeps the fastest. Results are cached in a JSON file keyed by
GPU architecture and a coarse workload class; ids never depend on the choice.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATES = (64, 512, 1024, 4096)


def _cache_path():
    base = os.environ.get("KBISIM_TUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "kbisim", "tuned.json")


def _arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name)


def workload_class(graphs):
    """Coarse key: log2 of the mean node count and of the mean degree."""
    n = sum(int(g.num_nodes) for g in graphs)
    e = sum(int(len(g.src)) for g in graphs)
    mean_n = max(n / max(len(graphs), 1), 1.0)
    deg = e / max(n, 1)
    return "n%d_d%d" % (int(math.log2(mean_n)), int(math.log2(max(deg, 1.0))))


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(table):
    p = _cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p + ".tmp", "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(p + ".tmp", p)
    except OSError:
        pass  # a read-only cache location only costs re-tuning


def tune_medium_cap(graphs, k, sample_edges=20_000_000, repeats=2, device="cuda:0", use_cache=True):
    """Returns (best medium_cap, {candidate: seconds}) for refining `graphs`
    as one batch with k rounds; times a prefix of the graphs holding about
    `sample_edges` edges."""
    from . import refine_batch
    key = "%s/%s/k%d" % (_arch(), workload_class(graphs), int(k))
    table = _load() if use_cache else {}
    if key in table:
        return int(table[key]["best"]), table[key]["times"]
    sample, acc = [], 0
    for g in graphs:
        sample.append(g)
        acc += len(g.src)
        if acc >= sample_edges:
            break
    times = {}
    for cap in CANDIDATES:
        best = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            refine_batch(sample, k, device=device, medium_cap=cap)
            best = min(best, time.perf_counter() - t0)
        times[str(cap)] = best
    choice = int(min(times, key=times.get))
    table[key] = {"best": choice, "times": times}
    if use_cache:
        _store(table)
    return choice, times
