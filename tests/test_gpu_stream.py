"""Streamed edge tables (edge_window_bytes > 0): the graph's edge table stays
in host memory and every round moves it through device windows, one
partition of consecutive source nodes at a time, or reads the rows of the
round's active nodes in place (the paper's setting of a graph larger than the
fast memory, Section 2.2). Every round's ids are compared with the oracle's,
element by element, on graphs cut into many partitions."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import need_gpu, gpu_rounds, oracle_rounds, say

pytestmark = pytest.mark.gpu


def longest_row(g):
    return int(np.bincount(g.src, minlength=max(g.num_nodes, 1)).max(initial=0))


def check_streamed(g, k, window, word=4, expect_parts=None):
    torch, kb = need_gpu()
    say("streamed case %s N=%d E=%d k=%d window=%d" % (g.name, g.num_nodes, g.num_edges, k, window))
    hist, counts, rd = gpu_rounds(torch, kb, g, k, device_inputs=False, edge_window_bytes=window)
    r = oracle_rounds(g, k)
    assert rd == r.rounds_done and counts == r.counts, (rd, r.rounds_done, counts, r.counts)
    for j, row in enumerate(hist):
        bad = np.flatnonzero(row != r.history[j])
        assert bad.size == 0, "round %d: %d ids differ, first at node %d" % (j, bad.size, bad[0])
    with kb.Graph(g.num_nodes, g.node_label, g.src, g.elab, g.dst, edge_window_bytes=window) as h:
        h.refine(k)
        parts, moved, direct = kb.kbisim_stream_stats(h._h)
    say("  partitions=%d bytes moved=%d rounds in place=%d" % (parts, moved, direct))
    if expect_parts is not None:
        assert parts >= expect_parts
    return parts, moved, direct


def test_figure1_one_row_per_window():
    """Windows of exactly twice the longest row (two edge words each): the
    six nodes of Figure 1 fall into several partitions."""
    from golden_io import graph_of, load
    g = graph_of(load("figure1.json"), "figure1")
    check_streamed(g, 6, window=2 * 4 * longest_row(g), expect_parts=3)


@pytest.mark.parametrize("seed", range(4))
def test_uniform_many_partitions(seed):
    g = synth.uniform_graph(3000, 15000, num_node_labels=4, num_edge_labels=8, seed=seed)
    g.name = "uniform-3k-15k-s%d" % seed
    w = 2 * 4 * max(longest_row(g), 64)
    parts, moved, _ = check_streamed(g, 10, window=w, expect_parts=20)
    assert moved > 0


def test_powerlaw_partitions_and_rows_in_place():
    """A power-law graph with hubs: the first rounds move every partition,
    later rounds with few active nodes read their rows in place."""
    g = synth.powerlaw_graph(200_000, 2_000_000, seed=3, name="powerlaw-200k-2M")
    w = max(1 << 20, 2 * 4 * longest_row(g))
    parts, moved, direct = check_streamed(g, 10, window=w, expect_parts=8)
    assert moved >= g.num_edges * 4 and direct >= 1


def test_wide_edge_words_and_label_table():
    """Edge labels above 255 (ranks through a table from a second read of the
    labels) and label rank + target id wider than 32 bits (8-byte edge
    words in the windows)."""
    rng = np.random.default_rng(7)
    n, e = 100_000, 300_000
    g = synth.Graph(n, rng.integers(0, 3, n).astype(np.int32), rng.integers(0, n, e).astype(np.int32),
                    rng.integers(0, 70_000, e).astype(np.int32), rng.integers(0, n, e).astype(np.int32),
                    name="wide-100k-300k")
    check_streamed(g, 4, window=2 * 8 * max(longest_row(g), 1024), expect_parts=10)


def test_isolated_nodes_and_empty():
    g = synth.Graph(50, np.zeros(50, np.int32), np.array([3, 3, 40], np.int32), np.array([0, 1, 0], np.int32),
                    np.array([4, 5, 3], np.int32), name="mostly-isolated")
    check_streamed(g, 5, window=16)
    e = np.zeros(0, np.int32)
    check_streamed(synth.Graph(7, np.arange(7, dtype=np.int32) % 2, e, e, e, name="no-edges"), 3, window=64)


def test_streamed_rejections():
    torch, kb = need_gpu()
    g = synth.uniform_graph(1000, 5000, seed=2)
    with pytest.raises(kb.KbisimError, match="longest row"):
        kb.Graph(g.num_nodes, g.node_label, g.src, g.elab, g.dst, edge_window_bytes=8)
    dev = [torch.from_numpy(a).cuda() for a in (g.node_label, g.src, g.elab, g.dst)]
    with pytest.raises(kb.KbisimError, match="host memory"):
        kb.Graph(g.num_nodes, *dev, edge_window_bytes=1 << 20)
    with pytest.raises(kb.KbisimError, match="history"):
        kb.Graph(g.num_nodes, g.node_label, g.src, g.elab, g.dst, edge_window_bytes=1 << 20, history=True)
    big = g.elab.copy()
    big[0] = 1 << 24
    with pytest.raises(kb.KbisimError, match="2\\^24"):
        kb.Graph(g.num_nodes, g.node_label, g.src, big, g.dst, edge_window_bytes=1 << 20)
    bad = g.dst.copy()
    bad[5] = g.num_nodes
    with pytest.raises(kb.KbisimError, match="outside"):
        kb.Graph(g.num_nodes, g.node_label, g.src, g.elab, bad, edge_window_bytes=1 << 20)
