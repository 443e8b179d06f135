"""Maintenance of a k-bisimulation partition (Section 4), test infrastructure.

* ``State``          -- the paper's maintenance state (node table with the
                        history pId_0..pId_k, edge table by source and by
                        target, signature store S) in the paper's numbering;
                        methods run Add_Nodes (Algorithm 2), Add_Edges
                        (Algorithm 3) and the deletions of Section 4 in the
                        C++ oracle (maintain_oracle.cpp).
* ``updated_graph``  -- the graph after an update, by definition: new nodes
                        appended, every copy of each deleted triple removed,
                        deleted nodes removed with their edges (the others
                        keep their order), added edges appended. Refining it
                        from scratch gives the partition any maintenance
                        algorithm must reach.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _i32, _load, _ptr, OracleError


class State:
    def __init__(self, num_nodes, node_label, src, elab, dst, k):
        self._lib = _load()
        node_label, src, elab, dst = _i32(node_label), _i32(src), _i32(elab), _i32(dst)
        self.k = int(k)
        self._h = self._lib.oracle_state_create(int(num_nodes), _ptr(node_label), int(src.shape[0]), _ptr(src),
                                                _ptr(elab), _ptr(dst), self.k)
        if not self._h:
            raise OracleError("invalid input")

    @property
    def num_nodes(self):
        return int(self._lib.oracle_state_num_nodes(self._h))

    def history(self):
        """[(k+1), N] int32: pId_0..pId_k (paper numbering)."""
        out = np.empty((self.k + 1, self.num_nodes), np.int32)
        self._lib.oracle_state_history(self._h, _ptr(out))
        return out

    def work(self):
        """(signatures checked, ids changed) by the last update."""
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        self._lib.oracle_state_work(self._h, ctypes.byref(a), ctypes.byref(b))
        return int(a.value), int(b.value)

    def add_nodes(self, labels):
        labels = _i32(labels)
        if self._lib.oracle_state_add_nodes(self._h, int(labels.shape[0]), _ptr(labels)) != 0:
            raise OracleError("invalid node labels")

    def _edges(self, fn, src, elab, dst):
        src, elab, dst = _i32(src), _i32(elab), _i32(dst)
        if fn(self._h, int(src.shape[0]), _ptr(src), _ptr(elab), _ptr(dst)) != 0:
            raise OracleError("invalid edges")

    def add_edges(self, src, elab, dst):
        self._edges(self._lib.oracle_state_add_edges, src, elab, dst)

    def delete_edges(self, src, elab, dst):
        self._edges(self._lib.oracle_state_delete_edges, src, elab, dst)

    def delete_nodes(self, nodes):
        nodes = _i32(nodes)
        if self._lib.oracle_state_delete_nodes(self._h, int(nodes.shape[0]), _ptr(nodes)) != 0:
            raise OracleError("invalid node ids")

    def close(self):
        if self._h:
            self._lib.oracle_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def updated_graph(num_nodes, node_label, src, elab, dst, *, new_labels=(), add=None, delete=None,
                  delete_nodes=()):
    """The graph after an update, in this order: new nodes appended (ids
    N..), edges deleted (every copy of each given triple), nodes deleted
    (with all their edges; remaining nodes renumbered in order), edges
    added. add / delete: (src, label, dst) arrays or None. Endpoints of
    added edges refer to ids after the node deletions. Returns (N', labels,
    src, elab, dst) as int32 arrays."""
    labels = np.concatenate([_i32(node_label), _i32(new_labels)])
    n = int(num_nodes) + len(new_labels)
    s, l, d = _i32(src), _i32(elab), _i32(dst)
    if delete is not None and len(delete[0]):
        gone = set(zip(*(np.asarray(x).tolist() for x in delete)))
        keep = np.array([(a, b, c) not in gone for a, b, c in zip(s.tolist(), l.tolist(), d.tolist())], bool)
        s, l, d = s[keep], l[keep], d[keep]
    if len(delete_nodes):
        dead = np.zeros(n, bool)
        dead[np.asarray(delete_nodes, np.int64)] = True
        keep = ~(dead[s] | dead[d])
        s, l, d = s[keep], l[keep], d[keep]
        newid = np.cumsum(~dead) - 1
        s, d = newid[s].astype(np.int32), newid[d].astype(np.int32)
        labels = labels[~dead]
        n = int((~dead).sum())
    if add is not None and len(add[0]):
        s = np.concatenate([s, _i32(add[0])])
        l = np.concatenate([l, _i32(add[1])])
        d = np.concatenate([d, _i32(add[2])])
    return n, labels, s, l, d
