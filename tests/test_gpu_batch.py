"""Batched form: every graph of a batch gets exactly the ids, block count and
rounds of refining it alone (oracle and plain GPU refine)."""
import os
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def mixed_graphs():
    rng = np.random.default_rng(77)
    gs = [synth.worked_example(),
          synth.Graph(0, *(np.zeros(0, np.int32),) * 4, name="empty"),
          synth.Graph(1, np.array([5], np.int32), *(np.zeros(0, np.int32),) * 3, name="single"),
          synth.Graph(4, np.array([1, 0, 1, 2], np.int32), *(np.zeros(0, np.int32),) * 3, name="noedges"),
          synth.path_graph(7), synth.cycle_graph(5), synth.tree_graph(2, 4), synth.complete_graph(5, 1)]
    for i in range(8):
        n = int(rng.integers(2, 40))
        gs.append(synth.random_small_graph(rng, n, int(rng.integers(0, 3 * n)), 3, 3))
    gs.append(synth.uniform_graph(2000, 8000, seed=3, name="u2k"))
    gs.append(synth.powerlaw_graph(6000, 50000, seed=4, deg_cap=3000, num_node_labels=8,
                                   num_edge_labels=4, name="pl6k"))
    gs.append(synth.powerlaw_graph(20000, 150000, seed=5, deg_cap=9000, name="pl20k"))
    return gs


@pytest.mark.parametrize("device", [True, False])
def test_batch_matches_oracle(device):
    torch, kb = need_gpu()
    gs = mixed_graphs()
    ks = [(i * 3) % 11 for i in range(len(gs))]
    say("batch of %d graphs, device=%s" % (len(gs), device))
    pids, blocks, rounds = kb.refine_batch(gs, ks, device="cuda:0" if device else None)
    for g, k, pid, b, rd in zip(gs, ks, pids, blocks, rounds):
        r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k)
        assert rd == r.rounds_done, (g.name, k, rd, r.rounds_done)
        assert b == r.counts[-1], (g.name, b, r.counts)
        assert np.array_equal(pid, r.pid), g.name


def test_batch_no_early_stop_equals_plain():
    torch, kb = need_gpu()
    gs = mixed_graphs()[:12]
    pids, blocks, rounds = kb.refine_batch(gs, 6, early_stop=False)
    for g, pid, rd in zip(gs, pids, rounds):
        assert rd == 6
        p2, counts, _ = kb.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 6, early_stop=False)
        assert np.array_equal(pid, p2), g.name


@pytest.mark.parametrize("radix_tile", [2048, 4096])
def test_batch_radix_tiles(radix_tile):
    """The batch's union build and ordering on the other compiled radix tile
    sizes (the tuner's second knob): ids equal the oracle's per graph."""
    torch, kb = need_gpu()
    gs = mixed_graphs()
    ks = [(i * 5) % 9 for i in range(len(gs))]
    pids, blocks, rounds = kb.refine_batch(gs, ks, device="cuda:0", radix_tile=radix_tile)
    for g, k, pid, b, rd in zip(gs, ks, pids, blocks, rounds):
        r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k)
        assert rd == r.rounds_done and b == r.counts[-1] and np.array_equal(pid, r.pid), (g.name, radix_tile)


def test_batch_many_small():
    """A few hundred graphs of log-normal size (the batched workload's shape,
    scaled down) against per-graph oracle runs."""
    torch, kb = need_gpu()
    gs = synth.batch_graphs(300, seed=2, median_nodes=300, min_nodes=20, max_nodes=5000)
    pids, blocks, rounds = kb.refine_batch(gs, 5, device="cuda:0")
    for g, pid, b, rd in zip(gs, pids, blocks, rounds):
        r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 5)
        assert rd == r.rounds_done and b == r.counts[-1] and np.array_equal(pid, r.pid), g.name


def test_batch_invalid_endpoint():
    torch, kb = need_gpu()
    a = synth.worked_example()
    b = synth.path_graph(3)
    bad = synth.Graph(b.num_nodes, b.node_label, b.src, b.elab, b.dst + 1)  # dst == N_b
    with pytest.raises(kb.KbisimError) as e:
        kb.refine_batch([a, bad], 3)
    assert e.value.status == -1


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("KBISIM_FULL_BATCH") != "1", reason="about three minutes; set KBISIM_FULL_BATCH=1")
def test_full_batch_4096_sampled():
    """The batched configuration itself (4,096 graphs, 136M nodes, 1.09B
    edges, k = 5, the bench's seed) refined as one batch on the GPU; 48
    seeded random graphs and the largest one checked against the oracle run
    on each graph alone (ids, block count, rounds)."""
    torch, kb = need_gpu()
    t0 = time.perf_counter()
    gs = synth.batch_graphs(4096, seed=1, progress=say)
    say("generated %d graphs, %d edges, in %.1f s" % (len(gs), sum(g.num_edges for g in gs), time.perf_counter() - t0))
    pids, blocks, rounds = kb.refine_batch(gs, 5, device="cuda:0")
    rng = np.random.default_rng(4096)
    pick = sorted(set(rng.choice(len(gs), 48, replace=False).tolist()) | {int(np.argmax([g.num_nodes for g in gs]))})
    for i in pick:
        g = gs[i]
        r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 5)
        assert rounds[i] == r.rounds_done and blocks[i] == r.counts[-1], (g.name, rounds[i], blocks[i], r.counts)
        assert np.array_equal(pids[i], r.pid), g.name
    say("%d graphs of the batch agree with the oracle (largest: %d nodes)" % (len(pick), max(gs[i].num_nodes for i in pick)))
