"""Invariants of the oracle on seeded graphs of a few thousand nodes and on the
10k-node / 50k-edge uniform workload."""
import numpy as np
import pytest

import oracle
from oracle import checks
import synth


def graphs():
    yield synth.uniform_graph(10_000, 50_000, seed=1, name="uniform-10k-50k")
    yield synth.powerlaw_graph(3_000, 30_000, seed=3, deg_cap=1_500, name="powerlaw-3k")
    yield synth.uniform_graph(2_000, 2_500, num_node_labels=2, num_edge_labels=1, seed=5,
                              name="sparse-1label")


@pytest.mark.parametrize("g", list(graphs()), ids=lambda g: g.name)
def test_invariants(g):
    k = 8
    r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k, history=True,
                      early_stop=False)
    h = r.history
    checks.check_label_rank(g.node_label, h[0])
    checks.check_counts(r.counts, g.num_nodes)
    for j in range(k + 1):
        checks.check_dense(h[j], r.counts[j])
    for j in range(1, k + 1):
        checks.check_refines_monotone(h[j - 1], h[j])
    # fixed point stability: after the first repeated count ids never change
    first = next((j for j in range(1, k + 1) if r.counts[j] == r.counts[j - 1]), None)
    if first is not None:
        for j in range(first, k + 1):
            assert np.array_equal(h[j], h[first - 1])
    # early-stop run returns the same final ids
    r2 = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k)
    assert np.array_equal(r2.pid, h[k])
    assert r2.rounds_done <= g.num_nodes


@pytest.mark.parametrize("g", list(graphs())[:2], ids=lambda g: g.name)
def test_lex_order_of_ids(g):
    """Ids of round j order the signatures lexicographically (checked with
    Python tuple comparison on signatures rebuilt from round j-1 ids)."""
    r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 4, history=True,
                      early_stop=False)
    allv = np.arange(g.num_nodes, dtype=np.int32)
    for j in range(1, 5):
        sigs = oracle.signatures(g.num_nodes, g.src, g.elab, g.dst, r.history[j - 1], allv)
        checks.check_lex_order(sigs, r.history[j].tolist())
        assert len(set(sigs)) == r.counts[j]


def test_relabel_invariance():
    """Renaming nodes by a permutation permutes the ids and nothing else."""
    g = synth.powerlaw_graph(4_000, 40_000, seed=11, deg_cap=2_000)
    rng = np.random.default_rng(3)
    perm = rng.permutation(g.num_nodes).astype(np.int32)
    lab2 = np.empty_like(g.node_label)
    lab2[perm] = g.node_label
    eperm = rng.permutation(g.num_edges)
    a = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 6)
    b = oracle.refine(g.num_nodes, lab2, perm[g.src][eperm], g.elab[eperm], perm[g.dst][eperm], 6)
    assert a.counts == b.counts
    assert np.array_equal(b.pid[perm], a.pid)


def test_label_values_only_matter_by_order():
    """Shifting labels by an order-preserving map changes no id."""
    g = synth.uniform_graph(1_000, 4_000, seed=2)
    a = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 5)
    b = oracle.refine(g.num_nodes, g.node_label * 7 + 100, g.src, g.elab * 1000 + 3, g.dst, 5)
    assert np.array_equal(a.pid, b.pid) and a.counts == b.counts
