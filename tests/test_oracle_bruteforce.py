"""The oracle's partitions against brute-force bisimilarity on tiny graphs.

Definition 1, Kaushik's definition and the Paige-Tarjan stability definition
(Appendix) are evaluated pairwise, independently of the signature method.
"""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from oracle import checks
import synth


def oracle_history(n, labels, triples, k, **kw):
    if triples:
        s, l, d = (np.array(c, np.int32) for c in zip(*triples))
    else:
        s = l = d = np.zeros(0, np.int32)
    return oracle.refine(n, np.array(labels, np.int32), s, l, d, k, history=True,
                         early_stop=False, **kw)


def triples_of(g):
    return list(zip(g.src.tolist(), g.elab.tolist(), g.dst.tolist()))


CASES = []
_rng = np.random.default_rng(12345)
for _i in range(60):
    n = int(_rng.integers(1, 9))
    e = int(_rng.integers(0, 3 * n + 1))
    CASES.append(dict(n=n, e=e, nl=int(_rng.integers(1, 3)), el=int(_rng.integers(1, 4)),
                      dag=bool(_rng.integers(0, 4) == 0), seed=int(_rng.integers(0, 2**31))))


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_e%d_s%d" % (c["n"], c["e"], c["seed"]))
def test_def1_and_kaushik(case):
    rng = np.random.default_rng(case["seed"])
    g = synth.random_small_graph(rng, case["n"], case["e"], case["nl"], case["el"], dag=case["dag"])
    tri = triples_of(g)
    k = g.num_nodes + 1
    r = oracle_history(g.num_nodes, g.node_label.tolist(), tri, k)
    r0 = oracle_history(g.num_nodes, g.node_label.tolist(), tri, k, head_pid0=True)
    d1 = bf.def1_relations(g.num_nodes, g.node_label.tolist(), tri, k)
    ka = bf.kaushik_relations(g.num_nodes, g.node_label.tolist(), tri, k)
    for j in range(k + 1):
        assert bf.relation_of_ids(r.history[j]) == d1[j], "round %d vs Definition 1" % j
        assert d1[j] == ka[j]
        # head pId_0 (Definition 3 as printed) gives the same partition
        assert checks.canon(r0.history[j]).tolist() == checks.canon(r.history[j]).tolist()
    # the fixed point is the greatest bisimulation
    full = bf.greatest_bisimulation(g.num_nodes, g.node_label.tolist(), tri)
    assert bf.relation_of_ids(r.history[k]) == full


@pytest.mark.parametrize("case", CASES[:25], ids=lambda c: "n%d_s%d" % (c["n"], c["seed"]))
def test_paige_tarjan(case):
    if case["n"] > 6:
        pytest.skip("set-partition enumeration limited to n <= 6")
    rng = np.random.default_rng(case["seed"])
    g = synth.random_small_graph(rng, case["n"], case["e"], case["nl"], case["el"])
    tri = triples_of(g)
    k = 3
    r = oracle_history(g.num_nodes, g.node_label.tolist(), tri, k)
    parts = bf.paige_tarjan_partitions(g.num_nodes, g.node_label.tolist(), tri, k)
    for j in range(k + 1):
        assert bf.partition_of_ids(r.history[j]) == parts[j]


@pytest.mark.parametrize("n,nl,el", [(1, 2, 2), (2, 2, 2), (3, 2, 1)])
def test_exhaustive_tiny(n, nl, el):
    """Every graph on n <= 3 nodes (given label alphabets) vs Definition 1."""
    count = 0
    for labels, tri in bf.all_graphs(n, nl, el):
        k = n + 1
        r = oracle_history(n, labels, tri, k)
        d1 = bf.def1_relations(n, labels, tri, k)
        for j in range(k + 1):
            assert bf.relation_of_ids(r.history[j]) == d1[j]
        count += 1
    assert count == nl ** n * 2 ** (n * n * el)


def test_early_stop_equals_full_run():
    """Stop rule (Section 3.2): stopping at the first repeated count returns
    the same ids as running all k rounds."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        g = synth.random_small_graph(rng, 30, 40, 2, 2)
        a = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 40)
        b = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 40, early_stop=False)
        assert np.array_equal(a.pid, b.pid)
        assert a.rounds_done <= g.num_nodes
