"""Parity at full size: the 10M-node / 100M-edge power-law graph that the
bench times, with the bench's options, refined to the fixed point on the GPU.
The whole oracle run is too slow for a test at this size, so every round is
checked on sampled nodes against the oracle's signatures (computed from the
GPU's previous-round ids, one sampled node at a time) and by properties that
hold at any size: pId_0 is the label rank, ids are dense, every round refines
the previous one with ids monotone in the previous ids, counts grow until the
first repeated count, where the run stops."""
import time

import numpy as np
import pytest

import oracle
from oracle import checks
import synth
from gpu_util import gpu_rounds, need_gpu, say

pytestmark = pytest.mark.gpu


def sample_nodes(rng, prev, n_random=1500, n_pairs=300):
    """Random nodes plus neighbours in the previous order (members of one old
    class, so the ordering inside classes is compared as well)."""
    n = prev.shape[0]
    picks = rng.choice(n, size=min(n, n_random), replace=False)
    order = np.argsort(prev, kind="stable")
    pos = rng.integers(0, max(n - 1, 1), size=n_pairs)
    pairs = np.concatenate([order[pos], order[np.minimum(pos + 1, n - 1)]])
    return np.unique(np.concatenate([picks, pairs])).astype(np.int32)


def test_powerlaw_10M_100M_sampled():
    torch, kb = need_gpu()
    t0 = time.perf_counter()
    g, k = synth.make_config("powerlaw-10M-100M")
    say("generated %s N=%d E=%d in %.1f s" % (g.name, g.num_nodes, g.num_edges, time.perf_counter() - t0))
    hist, counts, rd = gpu_rounds(torch, kb, g, k)
    say("GPU: rounds=%d counts=%s" % (rd, counts[: rd + 1]))
    n = g.num_nodes
    # stop rule: counts strictly increase until the first repeat, at round rd
    c = counts[: rd + 1]
    checks.check_counts(c, n)
    assert rd >= 1 and c[rd] == c[rd - 1], "stopped before the fixed point"
    assert all(c[i] < c[i + 1] for i in range(rd - 1)), "a repeated count did not stop the run"
    checks.check_label_rank(g.node_label, hist[0])
    rng = np.random.default_rng(2024)
    for j in range(1, rd + 1):
        prev, cur = hist[j - 1], hist[j]
        checks.check_dense(cur, c[j])
        checks.check_refines_monotone(prev, cur)
        sample = sample_nodes(rng, prev)
        sigs = oracle.signatures(n, g.src, g.elab, g.dst, prev, sample)
        checks.check_lex_order(sigs, cur[sample].tolist())
        say("round %d: %d blocks, %d sampled nodes agree with the oracle's signatures" % (j, c[j], sample.size))
