"""Autotuner for the ordering's LDS sort tile (medium_cap) and the radix
sort tile (radix_tile).

Groups of up to 64 members are ordered by one wave, groups of up to
`medium_cap` members by one workgroup sorting them in an LDS tile, larger
groups by device-wide radix passes; every radix pass (the edge table's sort
by source at create, the ordering's passes) works on tiles of `radix_tile`
items (2048, 3072 or 4096 compiled). The best pair depends on the workload's
sizes and block-size distribution, so the tuner times create + refinement
of a sample of the workload (inputs already on the device) with every
candidate pair, several times, interleaved (so drift hits all candidates
alike), and compares medians. A candidate replaces the library's default
only when its median beats the default's by more than the noise (the larger
of MIN_GAIN and twice the default's relative spread); otherwise the default
stays. Results are cached in a JSON file keyed by GPU architecture and a
coarse workload class; ids never depend on the choice.
"""
from __future__ import annotations

import json
import math
import os
import statistics
import time

CAPS = (64, 512, 1024, 4096)
TILES = (2048, 3072, 4096)
CANDIDATES = tuple((c, t) for c in CAPS for t in TILES)
DEFAULT = (4096, 3072)
MIN_GAIN = 0.03


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


def cache_key(arch, graphs, k, candidates):
    """Cache entry of one tuning: architecture, workload class, k and the
    candidate set (a search over fewer pairs is not reused for a larger one)."""
    cand_id = ",".join("%d:%d" % tuple(c) for c in candidates)
    return "%s/%s/k%d/%s" % (arch, workload_class(graphs), int(k), cand_id)


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


def choose(runs, default=DEFAULT):
    """runs: {candidate: [seconds, ...]}. The fastest candidate by median if
    it beats the default's median by more than the noise (the larger of
    MIN_GAIN and twice the default's median absolute deviation, relative),
    else the default. Returns (choice, report)."""
    med = {c: statistics.median(v) for c, v in runs.items()}
    mad = {c: statistics.median(abs(x - med[c]) for x in v) for c, v in runs.items()}
    noise = max(MIN_GAIN, 2.0 * mad[default] / med[default])
    best = min(med, key=med.get)
    choice = best if med[best] < med[default] * (1.0 - noise) else default
    report = {"median_s": {str(c): med[c] for c in runs}, "spread_s": {str(c): mad[c] for c in runs},
              "noise": noise, "fastest": best, "kept_default": choice == default}
    return choice, report


def tune(graphs, k, sample_edges=20_000_000, repeats=5, device="cuda:0", use_cache=True,
         candidates=CANDIDATES, default=DEFAULT):
    """Returns ((medium_cap, radix_tile), report) for refining `graphs` as one
    batch with k rounds. A prefix of the graphs holding about `sample_edges`
    edges is concatenated and moved to the device once; per run a batch handle
    is created from those device arrays and refined (kbisim_batch_create +
    kbisim_batch_refine, synchronised before and after: device work and the
    library's own host steps, no host copies of the inputs), then destroyed
    outside the timed region. report: per candidate the median and spread
    (median absolute deviation) in seconds, the noise threshold and whether
    the default was kept."""
    import numpy as np
    import torch
    from . import kbisim_batch_create, kbisim_batch_refine, kbisim_batch_destroy
    key = cache_key(_arch(), graphs, k, candidates)
    table = _load() if use_cache else {}
    if key in table and "best_pair" in table[key]:
        return tuple(table[key]["best_pair"]), table[key]["report"]
    sample, acc = [], 0
    for g in graphs:
        sample.append(g)
        acc += len(g.src)
        if acc >= sample_edges:
            break
    noff = np.zeros(len(sample) + 1, np.int64)
    eoff = np.zeros(len(sample) + 1, np.int64)
    for i, g in enumerate(sample):
        noff[i + 1] = noff[i] + int(g.num_nodes)
        eoff[i + 1] = eoff[i] + len(g.src)
    arrs = [torch.from_numpy(np.concatenate([np.asarray(getattr(g, nm), np.int32) for g in sample])).to(device)
            for nm in ("node_label", "src", "elab", "dst")]
    ks = [int(k)] * len(sample)
    stream = torch.cuda.current_stream()

    def job_seconds(pair):
        cap, tile = pair
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, _ = kbisim_batch_create(noff, eoff, *arrs, stream=stream, medium_cap=cap, radix_tile=tile)
        try:
            kbisim_batch_refine(h, ks)
            torch.cuda.synchronize()
            return time.perf_counter() - t0
        finally:
            kbisim_batch_destroy(h)

    for pair in candidates:  # warm the allocator and every compiled variant
        job_seconds(pair)
    runs = {c: [] for c in candidates}
    for _ in range(repeats):
        for pair in candidates:
            runs[pair].append(job_seconds(pair))
    choice, report = choose(runs, default)
    report.update(repeats=repeats, sample_graphs=len(sample), sample_edges=acc,
                  timed="kbisim_batch_create + kbisim_batch_refine from device inputs",
                  candidates="(medium_cap, radix_tile)")
    table[key] = {"best_pair": list(choice), "report": report}
    if use_cache:
        _store(table)
    return choice, report

