"""Invariants of k-bisimulation refinement that hold at any size (test
infrastructure). Each check raises AssertionError with a message on failure.

They restate properties proved in the paper's appendix:
* Proposition 1 (each round refines the previous one),
* the stop-condition propositions (a round with an unchanged block count is a
  fixed point; it is reached within |N| rounds),
plus the properties of the canonical numbering used here (dense
0-based lexicographic ranks whose first key is the previous id).
"""
from __future__ import annotations

import numpy as np


def check_label_rank(node_label, pid0):
    """k = 0 ids are the ascending rank of the node label (textbook unique)."""
    expect = np.unique(np.asarray(node_label), return_inverse=True)[1].astype(np.int64)
    got = np.asarray(pid0).astype(np.int64)
    assert np.array_equal(expect.ravel(), got), "pId_0 differs from the label rank"


def check_dense(pid, blocks):
    pid = np.asarray(pid)
    if pid.size == 0:
        assert blocks == 0
        return
    assert pid.min() >= 0 and pid.max() == blocks - 1, "ids not in [0, B)"
    assert np.unique(pid).size == blocks, "ids are not dense"


def check_refines_monotone(pid_prev, pid_next):
    """pid_prev must be a non-decreasing function of pid_next: equal new ids
    imply equal old ids (refinement, Proposition 1) and smaller old ids give
    smaller new ids (the previous id leads the signature)."""
    a = np.asarray(pid_prev, np.int64)
    b = np.asarray(pid_next, np.int64)
    if a.size == 0:
        return
    order = np.argsort(b, kind="stable")
    bs, as_ = b[order], a[order]
    same = bs[1:] == bs[:-1]
    assert np.all(as_[1:][same] == as_[:-1][same]), "a new block spans two old blocks"
    assert np.all(as_[1:] >= as_[:-1]), "new ids are not monotone in old ids"


def check_counts(counts, n):
    c = list(counts)
    assert all(c[i] <= c[i + 1] for i in range(len(c) - 1)), "block count decreased"
    assert all(x <= max(n, 0) for x in c), "more blocks than nodes"


def check_lex_order(sigs, ids):
    """For signatures given as tuples and the ids assigned to them: equal ids
    iff equal signatures, smaller id iff lexicographically smaller signature
    (Python tuple order: element-wise, a proper prefix is smaller)."""
    pairs = sorted(zip(sigs, ids))
    for (s0, i0), (s1, i1) in zip(pairs, pairs[1:]):
        if s0 == s1:
            assert i0 == i1, "equal signatures got different ids"
        else:
            assert i0 < i1, "id order differs from signature order"


def canon(ids):
    """Renumber ids by first occurrence (0, 1, ...) -- compares partitions."""
    seen = {}
    out = np.empty(len(ids), np.int64)
    for v, b in enumerate(ids):
        out[v] = seen.setdefault(int(b), len(seen))
    return out
