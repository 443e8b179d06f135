"""Pins of the CPU oracle against values printed in the paper and closed forms.

Each test names the passage it follows. These run without a GPU.
"""
import numpy as np
import pytest

import oracle
from oracle import checks
import synth
from golden_io import graph_of, load


def run(g, k, **kw):
    return oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k, **kw)


# --- Figure 1 / Table 1 / Table 2 -------------------------------------------------

def test_table1_paper_numbering():
    """Table 1: pId_0..pId_2 with one global counter, head pId_0 (Definition 3)."""
    fx = load("figure1.json")
    g = graph_of(fx)
    r = run(g, 2, paper_numbering=True, head_pid0=True, history=True, early_stop=False)
    assert r.history.tolist() == fx["paper_numbering"]["pid"]


def test_table1_signatures():
    """Table 1's sig_1 and sig_2 columns (head pId_0, pairs of the previous ids)."""
    fx = load("figure1.json")
    g = graph_of(fx)
    pn = fx["paper_numbering"]
    pid0, pid1 = pn["pid"][0], pn["pid"][1]
    allv = list(range(g.num_nodes))
    # the head of Definition 3 is pId_0; oracle.signatures uses the given array
    # as both head and pair source, so replace the head afterwards
    s1 = oracle.signatures(g.num_nodes, g.src, g.elab, g.dst, pid0, allv)
    s2 = oracle.signatures(g.num_nodes, g.src, g.elab, g.dst, pid1, allv)
    s2 = [(pid0[v],) + s[1:] for v, s in enumerate(s2)]
    assert [list(s) for s in s1] == pn["sig1"]
    assert [list(s) for s in s2] == pn["sig2"]


def test_table2_edge_table():
    """Table 2: after k=2 the edge table's pId_old(tId) column holds pId_1 of the
    target (paper numbering)."""
    fx = load("figure1.json")
    g = graph_of(fx)
    r = run(g, 2, paper_numbering=True, head_pid0=True, history=True, early_stop=False)
    pid1 = r.history[1]
    rows = fx["paper_numbering"]["table2_edge_pid_old_of_target"]["rows"]
    for s, lab, t, p_old in rows:
        # the row is an edge of the graph and carries pId_1(t)
        assert any(a == s - 1 and b == lab and c == t - 1 for a, b, c in zip(g.src, g.elab, g.dst))
        assert pid1[t - 1] == p_old


def test_figure1_canonical_ids():
    """Canonical ids (lexicographic ranks, head pId_{i-1}) of the example graph,
    derived by hand from Definition 3; fixed point at round 4."""
    fx = load("figure1.json")
    g = graph_of(fx)
    can = fx["canonical"]
    r = run(g, 10, history=True)
    assert r.counts == can["counts"]
    assert r.rounds_done == can["rounds_done"]
    for i, row in enumerate(can["pid"]):
        assert r.history[i].tolist() == row
    assert r.pid.tolist() == can["pid"][-1]


def test_figure1_prose():
    """Section 2.1: nodes 1 and 2 are 0- and 1-bisimilar but not 2-bisimilar."""
    g = graph_of(load("figure1.json"))
    r = run(g, 2, history=True, early_stop=False)
    h = r.history
    assert h[0][0] == h[0][1] and h[1][0] == h[1][1] and h[2][0] != h[2][1]


@pytest.mark.parametrize("table", ["table4", "table5"])
def test_update_tables_as_partitions(table):
    """Tables 4 and 5 (Section 4.2): a from-scratch run on the updated graph gives
    the same partitions (block structure) the update algorithm printed."""
    fx = load("updates.json")[table]
    g = graph_of(fx, table)
    r = run(g, 2, history=True, early_stop=False)
    for i, row in enumerate(fx["pid_paper"]):
        assert checks.canon(r.history[i]).tolist() == checks.canon(row).tolist()


def test_table5_fixed_point():
    """Table 5: pId_1 and pId_2 induce the same partition, so the run stops at 2."""
    g = graph_of(load("updates.json")["table5"])
    r = run(g, 10)
    assert r.counts == [2, 3, 3] and r.rounds_done == 2


def test_table4_paper_numbering_exact():
    """Table 4's ids are what a from-scratch run with Table 1's numbering gives."""
    fx = load("updates.json")["table4"]
    g = graph_of(fx)
    r = run(g, 2, paper_numbering=True, head_pid0=True, history=True, early_stop=False)
    assert r.history.tolist() == fx["pid_paper"]


# --- closed forms ------------------------------------------------------------------

@pytest.mark.parametrize("arity,height", [(2, 3), (3, 2), (2, 6), (1, 5)])
def test_full_tree(arity, height):
    """Dbest shape (Section 5.3): a full tree with one node and one edge label
    has B_j = min(j, H) + 1, the blocks being node heights."""
    g = synth.tree_graph(arity, height)
    r = run(g, height + 3, history=True, early_stop=False)
    for j in range(height + 4):
        assert r.counts[j] == min(j, height) + 1
    # height of node v: leaves are the last arity^height nodes
    n = g.num_nodes
    depth = np.zeros(n, np.int64)
    for v in range(1, n):
        depth[v] = depth[(v - 1) // arity] + 1
    hgt = height - depth
    assert checks.canon(r.pid).tolist() == checks.canon(hgt).tolist()


def test_dbest_instance():
    """Dbest example (Section 5.3 figure): binary tree a..g with x edges from the
    root and y edges below it; adding c -y-> e changes no id."""
    node_label = np.zeros(7, np.int32)
    edges = [(0, 0, 1), (0, 0, 2), (1, 1, 3), (1, 1, 4), (2, 1, 5), (2, 1, 6)]
    s, l, d = (np.array(c, np.int32) for c in zip(*edges))
    g = synth.Graph(7, node_label, s, l, d)
    r0 = run(g, 5)
    assert r0.counts == [1, 3, 3]
    s2, l2, d2 = np.append(s, 2), np.append(l, 1), np.append(d, 4)
    r1 = oracle.refine(7, node_label, s2, l2, d2, 5)
    assert r1.counts == [1, 3, 3] and r1.pid.tolist() == r0.pid.tolist()


@pytest.mark.parametrize("n", [3, 4, 5, 9])
def test_dworst(n):
    """Dworst (Section 5.3): a complete graph with all edges x is one block at
    every k; adding a y edge a -> f to a new isolated node f gives three
    blocks: f, the other clique nodes, and a (ranked f < others < a)."""
    g = synth.complete_graph(n)
    r = run(g, 6, early_stop=False)
    assert r.counts == [1] * 7
    g2 = synth.complete_graph(n, extra_isolated=1)
    f = n
    src = np.append(g2.src, 0).astype(np.int32)
    lab = np.append(g2.elab, 1).astype(np.int32)
    dst = np.append(g2.dst, f).astype(np.int32)
    r2 = oracle.refine(n + 1, g2.node_label, src, lab, dst, 6, history=True)
    assert r2.counts == [1, 3, 3] and r2.rounds_done == 2
    expect = [2] + [1] * (n - 1) + [0]
    assert r2.history[1].tolist() == expect and r2.history[2].tolist() == expect


@pytest.mark.parametrize("n", [1, 2, 7])
def test_cycle_one_block(n):
    g = synth.cycle_graph(n)
    r = run(g, 5)
    assert r.counts == [1, 1] and r.pid.tolist() == [0] * n


@pytest.mark.parametrize("length", [1, 2, 5, 11])
def test_path(length):
    """A directed path v0 -> ... -> vL: blocks are the distances to the end,
    capped at j, so B_j = min(j, L) + 1."""
    g = synth.path_graph(length)
    r = run(g, length + 3, history=True, early_stop=False)
    for j in range(length + 4):
        assert r.counts[j] == min(j, length) + 1
    dist = length - np.arange(length + 1)
    assert r.pid.tolist() == dist.tolist()  # lex rank: (d, ...) ordered by distance


def test_no_edges():
    """E empty: every signature is (head, {}), so pId_i == pId_0 and the first
    round already repeats the count."""
    g = synth.Graph(5, np.array([3, 1, 3, 0, 1], np.int32), *(np.zeros(0, np.int32),) * 3)
    r = run(g, 4)
    assert r.counts == [3, 3] and r.rounds_done == 1
    assert r.pid.tolist() == [2, 1, 2, 0, 1]


def test_k0_and_empty_graph():
    g = synth.worked_example()
    r = run(g, 0)
    assert r.rounds_done == 0 and r.counts == [2] and r.pid.tolist() == [0, 0, 1, 1, 1, 1]
    z = np.zeros(0, np.int32)
    r = oracle.refine(0, z, z, z, z, 3)
    assert r.counts == [0, 0] and r.rounds_done == 1 and r.pid.size == 0


def test_pair_order_inside_signature():
    """Section 3.1 builds the signature as a string with the set elements in
    sorted order; read as ascending (label, id). Nodes a=2 with pairs
    {(0,1),(1,0)} and b=3 with {(0,0),(1,1)} share the head, and b's string
    [2,0,0,1,1] precedes a's [2,0,1,1,0]: ids x=0, y=1, b=2, a=3."""
    g = synth.Graph(4, np.array([0, 1, 2, 2], np.int32), np.array([2, 2, 3, 3], np.int32),
                    np.array([0, 1, 0, 1], np.int32), np.array([1, 0, 0, 1], np.int32))
    r = run(g, 1)
    assert r.pid.tolist() == [0, 1, 3, 2]


def test_rounds_match_python_lex_ranking():
    """Every round of the oracle equals a pure-Python ranking of signatures
    rebuilt from the previous round (Definition 3, tuple order)."""
    from oracle import bruteforce as bf
    rng = np.random.default_rng(2024)
    for _ in range(30):
        g = synth.random_small_graph(rng, 12, 20, 2, 3)
        tri = list(zip(g.src.tolist(), g.elab.tolist(), g.dst.tolist()))
        r = run(g, 6, history=True, early_stop=False)
        for j in range(1, 7):
            assert r.history[j].tolist() == bf.lex_rank_round(12, tri, r.history[j - 1],
                                                              r.history[j - 1])
        r0 = run(g, 6, history=True, early_stop=False, head_pid0=True)
        for j in range(1, 7):
            assert r0.history[j].tolist() == bf.lex_rank_round(12, tri, r0.history[0],
                                                               r0.history[j - 1])


def test_duplicate_and_parallel_edges():
    """Set semantics of Definition 3: repeating an edge changes nothing; a
    second label on the same node pair is a distinct pair."""
    g = synth.worked_example()
    base = run(g, 6, history=True)
    s = np.concatenate([g.src, g.src]); l = np.concatenate([g.elab, g.elab])
    d = np.concatenate([g.dst, g.dst])
    dup = oracle.refine(6, g.node_label, s, l, d, 6, history=True)
    assert np.array_equal(dup.history, base.history)
    s2 = np.append(g.src, 4); l2 = np.append(g.elab, 0); d2 = np.append(g.dst, 1)
    par = oracle.refine(6, g.node_label, s2, l2, d2, 6)
    assert par.pid[2] != par.pid[4]  # 5 now differs from 3 already at round 1


def test_invalid_input_rejected():
    z = np.zeros(0, np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.refine(2, [0, 0], [0], [0], [2], 1)  # dst out of range
    with pytest.raises(oracle.OracleError):
        oracle.refine(2, [0, -1], z, z, z, 1)  # negative label
    with pytest.raises(oracle.OracleError):
        oracle.refine(2, [0, 0], [0], [-1], [1], 1)  # negative edge label
    with pytest.raises(oracle.OracleError):
        oracle.refine(2, [0, 0], z, z, z, -1)


def test_signature_lengths_table1():
    """Lengths of Table 1's signatures (sig_1 and sig_2 as printed) from the
    previous round's ids; and the longest among nodes of non-singleton
    classes (all of round 1's classes have two or more members)."""
    fx = load("figure1.json")
    g = graph_of(fx)
    pn = fx["paper_numbering"]
    for j, key in ((1, "sig1"), (2, "sig2")):
        lengths = oracle.signature_lengths(g.num_nodes, g.src, g.elab, g.dst, pn["pid"][j - 1])
        assert lengths.tolist() == [len(s) for s in pn[key]]
    lengths = oracle.signature_lengths(g.num_nodes, g.src, g.elab, g.dst, pn["pid"][0])
    assert oracle.longest_multi_member(lengths, np.asarray(pn["pid"][0]) - 1) == 5
    # round 2: classes of pId_1 {1,2}, {3,5} have two members; 4 and 6 are alone
    lengths = oracle.signature_lengths(g.num_nodes, g.src, g.elab, g.dst, pn["pid"][1])
    assert oracle.longest_multi_member(lengths, np.asarray(pn["pid"][1]) - 3) == 5
    assert oracle.longest_multi_member(np.array([7, 3, 5]), np.array([0, 1, 2])) == 1


def test_round_sample_figure1_and_subsets():
    """The oracle's round restricted to a node sample (the timed sample of the
    bench's CPU baseline). On Figure 1 with every node it gives round 1's
    canonical ids (Appendix A of the survey: [0,0,2,3,2,1]); on a subset the
    ranks are round 1's ids renumbered densely within the subset, since the
    lexicographic order of signatures does not depend on which other nodes
    are present; the edge count is the subset's out-degree sum."""
    fx = load("figure1.json")
    g = graph_of(fx)
    rank, edges = oracle.round_sample(g.num_nodes, g.node_label, g.src, g.elab, g.dst, np.arange(6))
    assert rank.tolist() == [0, 0, 2, 3, 2, 1] and edges == 7
    rng = np.random.default_rng(5)
    h = synth.uniform_graph(300, 1500, num_node_labels=3, num_edge_labels=4, seed=3)
    full = run(h, 1, early_stop=False).pid
    outdeg = np.bincount(h.src, minlength=h.num_nodes)
    for _ in range(5):
        sample = rng.choice(h.num_nodes, size=int(rng.integers(1, 200)), replace=False).astype(np.int32)
        rank, edges = oracle.round_sample(h.num_nodes, h.node_label, h.src, h.elab, h.dst, sample)
        _, dense = np.unique(full[sample], return_inverse=True)
        assert rank.tolist() == dense.tolist()
        assert edges == int(outdeg[sample].sum())
