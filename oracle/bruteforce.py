"""Brute-force bisimilarity for tiny graphs (test infrastructure).

Each function works on a graph given as (n, node_label, triples) where
``triples`` is an iterable of (src, label, dst); duplicates collapse (the
relation E of the data model is a set; several labels on one node pair are
read as several labelled edges).

* ``def1_relations``      -- Definition 1 (k-bisimilar), level by level.
* ``kaushik_relations``   -- Kaushik k-bisimilarity (Appendix, "Alternative
                             definitions for localized bisimulation"), which
                             adds the conjunct u ~^{k-1} v.
* ``paige_tarjan_partitions`` -- the k-partition as the least-cardinality
                             refinement of the (k-1)-partition that is stable
                             with respect to it (same appendix), found by
                             enumerating every set partition (n <= 6).
* ``greatest_bisimulation`` -- full bisimulation (Appendix, "Connection
                             between localized bisimulation and full
                             bisimulation"), as the greatest fixed point.

All relations are returned as n x n lists of booleans.
"""
from __future__ import annotations

from itertools import product


def _edges(triples):
    out = {}
    for s, l, d in set((int(a), int(b), int(c)) for a, b, c in triples):
        out.setdefault(s, set()).add((l, d))
    return out


def _step(n, labels, out, prev, with_prev):
    cur = [[False] * n for _ in range(n)]
    for u in range(n):
        for v in range(n):
            if labels[u] != labels[v]:
                continue
            if with_prev and not prev[u][v]:
                continue
            ou, ov = out.get(u, set()), out.get(v, set())
            ok = all(any(lb == la and prev[up][vp] for (lb, vp) in ov) for (la, up) in ou) and \
                all(any(la == lb and prev[vp][up] for (la, up) in ou) for (lb, vp) in ov)
            cur[u][v] = ok
    return cur


def def1_relations(n, labels, triples, k):
    """[R_0, ..., R_k] with R_j[u][v] == (u ~^j v) by Definition 1."""
    out = _edges(triples)
    rel = [[labels[u] == labels[v] for v in range(n)] for u in range(n)]
    rels = [rel]
    for _ in range(k):
        rel = _step(n, labels, out, rel, with_prev=False)
        rels.append(rel)
    return rels


def kaushik_relations(n, labels, triples, k):
    """[R_0, ..., R_k] by Kaushik's definition (extra conjunct u ~^{j-1} v)."""
    out = _edges(triples)
    rel = [[labels[u] == labels[v] for v in range(n)] for u in range(n)]
    rels = [rel]
    for _ in range(k):
        rel = _step(n, labels, out, rel, with_prev=True)
        rels.append(rel)
    return rels


def greatest_bisimulation(n, labels, triples):
    """Full bisimilarity: iterate the Definition 1 step from label equality to
    its greatest fixed point (at most n steps are needed)."""
    out = _edges(triples)
    rel = [[labels[u] == labels[v] for v in range(n)] for u in range(n)]
    while True:
        nxt = _step(n, labels, out, rel, with_prev=False)
        if nxt == rel:
            return rel
        rel = nxt


def relation_of_ids(ids):
    n = len(ids)
    return [[ids[u] == ids[v] for v in range(n)] for u in range(n)]


# ---------------------------------------------------------------------------
# Paige-Tarjan style definition via stability, by enumeration of partitions.

def _set_partitions(items):
    """All set partitions of ``items`` (restricted growth strings)."""
    items = list(items)
    n = len(items)
    if n == 0:
        yield []
        return

    def rec(i, assign, nblocks):
        if i == n:
            blocks = [[] for _ in range(nblocks)]
            for it, b in zip(items, assign):
                blocks[b].append(it)
            yield [frozenset(b) for b in blocks]
            return
        for b in range(nblocks + 1):
            assign.append(b)
            yield from rec(i + 1, assign, max(nblocks, b + 1))
            assign.pop()

    yield from rec(0, [], 0)


def _refines(fine, coarse):
    return all(any(b <= c for c in coarse) for b in fine)


def _stable(fine, coarse, triples, edge_labels):
    tri = set((int(a), int(b), int(c)) for a, b, c in triples)
    for block_j in coarse:
        for lab in edge_labels:
            parents = {s for (s, l, d) in tri if l == lab and d in block_j}
            for block_i in fine:
                if not (block_i <= parents or not (block_i & parents)):
                    return False
    return True


def paige_tarjan_partitions(n, labels, triples, k):
    """[P_0, ..., P_k], each a set of frozensets. P_0 groups by node label; P_j
    is the unique least-cardinality partition that refines P_{j-1} and is
    stable w.r.t. it (asserted unique)."""
    by_label = {}
    for v in range(n):
        by_label.setdefault(labels[v], set()).add(v)
    cur = frozenset(frozenset(b) for b in by_label.values())
    parts = [cur]
    edge_labels = sorted(set(int(l) for _, l, _ in triples))
    all_parts = [frozenset(p) for p in _set_partitions(range(n))]
    for _ in range(k):
        good = [p for p in all_parts if _refines(p, cur) and _stable(p, cur, triples, edge_labels)]
        least = min(len(p) for p in good)
        best = [p for p in good if len(p) == least]
        assert len(best) == 1, "least stable refinement is not unique"
        cur = best[0]
        parts.append(cur)
    return parts


def partition_of_ids(ids):
    blocks = {}
    for v, b in enumerate(ids):
        blocks.setdefault(int(b), set()).add(v)
    return frozenset(frozenset(b) for b in blocks.values())


def all_graphs(n, num_node_labels, num_edge_labels):
    """Every labelled graph on n nodes (node labels from range(num_node_labels),
    edge sets over range(num_edge_labels)); yields (labels, triples)."""
    cand = [(s, l, d) for s in range(n) for l in range(num_edge_labels) for d in range(n)]
    for labels in product(range(num_node_labels), repeat=n):
        for mask in range(1 << len(cand)):
            yield list(labels), [cand[i] for i in range(len(cand)) if mask >> i & 1]


def lex_rank_round(n, triples, head, pid_prev):
    """One round of canonical numbering written directly from Definition 3:
    the signature of u is the tuple (head[u], l1, p1, l2, p2, ...) with the set
    {(label, pid_prev[target])} listed in ascending order; ids are the ranks of
    the distinct signatures in Python's tuple order (a prefix is smaller)."""
    pairs = [set() for _ in range(n)]
    for s, l, d in triples:
        pairs[int(s)].add((int(l), int(pid_prev[int(d)])))
    sigs = []
    for u in range(n):
        flat = [int(head[u])]
        for l, p in sorted(pairs[u]):
            flat += [l, p]
        sigs.append(tuple(flat))
    rank = {s: i for i, s in enumerate(sorted(set(sigs)))}
    return [rank[s] for s in sigs]
