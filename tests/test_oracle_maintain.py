"""Pins of the maintenance oracle (Section 4: Add_Nodes, Add_Edges,
deletions, change of k) and of the updated-graph definition.

* Tables 4 and 5 (the example run of Add_Edges on Figure 3): the exact ids
  the paper prints, from the Figure 1 state plus the update.
* The example run's prose: for (2,l,7) the two queued pairs are checked and
  nothing changes; for (6,l,5) node 6 changes at level 1, then nodes 2 and 6
  are checked and both change at level 2.
* Random graphs and random update sequences: the partition the maintained
  state holds at every level equals a from-scratch Build_Bisim of the
  updated graph (Theorem 2, correctness of Add_Edges), which is itself
  pinned against brute-force bisimilarity.
* A planted mistake in the maintenance oracle breaks one of these pins.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import checks
from oracle import maintain as M
import synth
from golden_io import graph_of, load

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fig1():
    return graph_of(load("figure1.json"))


def state_of(g, k):
    return M.State(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k)


def test_build_matches_table1():
    fx = load("figure1.json")
    st = state_of(fig1(), 2)
    assert st.history().tolist() == fx["paper_numbering"]["pid"]


def test_table4_add_node_then_edge():
    """Node 7 (label P) is added, then edge (2, l, 7): Table 4's ids."""
    fx = load("updates.json")["table4"]
    st = state_of(fig1(), 2)
    st.add_nodes([1])
    assert st.work() == (0, 0)
    st.add_edges([1], [1], [6])
    assert st.history().tolist() == fx["pid_paper"]
    assert st.work() == (2, 0)  # (1, 2) and (2, 2) checked, no change


def test_table5_add_edge():
    """Edge (6, l, 5): Table 5's ids, with node 6 changing at level 1 and
    nodes 2 and 6 checked and changed at level 2."""
    fx = load("updates.json")["table5"]
    st = state_of(fig1(), 2)
    st.add_edges([5], [1], [4])
    assert st.history().tolist() == fx["pid_paper"]
    assert st.work() == (3, 3)


@pytest.mark.parametrize("table,upd", [
    ("table4", dict(new_labels=[1], add=([1], [1], [6]))),
    ("table5", dict(add=([5], [1], [4]))),
])
def test_updated_graph_definition(table, upd):
    """The updated-graph definition gives Figure 3's graphs (as written in
    the fixture, edge multiset compared as sorted triples)."""
    g = fig1()
    n, lab, s, l, d = M.updated_graph(g.num_nodes, g.node_label, g.src, g.elab, g.dst, **upd)
    want = graph_of(load("updates.json")[table])
    assert n == want.num_nodes and lab.tolist() == want.node_label.tolist()
    got = sorted(zip(s.tolist(), l.tolist(), d.tolist()))
    assert got == sorted(zip(want.src.tolist(), want.elab.tolist(), want.dst.tolist()))


def test_updated_graph_deletions():
    g = fig1()
    # delete (1, w, 1) (both copies if duplicated) and node 3 (paper node 4)
    s = np.concatenate([g.src, [1]])
    l = np.concatenate([g.elab, [0]])
    d = np.concatenate([g.dst, [1]])
    n, lab, s2, l2, d2 = M.updated_graph(6, g.node_label, s, l, d, delete=([1], [0], [1]), delete_nodes=[3])
    assert n == 5 and lab.tolist() == [0, 0, 1, 1, 1]
    # remaining edges of Figure 1 without (2,w,2) and those of node 4,
    # renumbered (paper node 5 -> index 3, node 6 -> index 4)
    assert sorted(zip(s2.tolist(), l2.tolist(), d2.tolist())) == \
        sorted([(0, 0, 1), (1, 1, 4), (2, 1, 0), (3, 1, 1)])


def partitions_equal(hist_a, hist_b):
    for a, b in zip(hist_a, hist_b):
        if checks.canon(a).tolist() != checks.canon(b).tolist():
            return False
    return True


def random_update(rng, n, k_labels, e_labels, cur):
    """One random update: which kinds and their payloads."""
    kind = rng.integers(0, 4)
    if kind == 0:
        return "nodes", rng.integers(0, k_labels + 1, size=rng.integers(1, 3))
    m = rng.integers(1, 4)
    if kind == 1 or cur[2].shape[0] == 0:
        return "add", (rng.integers(0, n, m), rng.integers(0, e_labels, m), rng.integers(0, n, m))
    if kind == 2:
        pick = rng.integers(0, cur[2].shape[0], m)
        return "delete", (cur[2][pick], cur[3][pick], cur[4][pick])
    return "delete_nodes", np.unique(rng.integers(0, n, rng.integers(1, 3)))


def apply_both(st, cur, upd):
    n, lab, s, l, d = cur
    kind, payload = upd
    if kind == "nodes":
        st.add_nodes(payload)
        return M.updated_graph(n, lab, s, l, d, new_labels=payload)
    if kind == "add":
        st.add_edges(*payload)
        return M.updated_graph(n, lab, s, l, d, add=payload)
    if kind == "delete":
        st.delete_edges(*payload)
        return M.updated_graph(n, lab, s, l, d, delete=payload)
    st.delete_nodes(payload)
    return M.updated_graph(n, lab, s, l, d, delete_nodes=payload)


def maintained_equals_scratch(seed, steps=6, k=4, lib_state=None):
    rng = np.random.default_rng(seed)
    n0 = int(rng.integers(3, 9))
    g = synth.random_small_graph(rng, n0, int(rng.integers(0, 14)), 2, 2)
    st = (lib_state or M.State)(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k)
    cur = (g.num_nodes, g.node_label, g.src, g.elab, g.dst)
    for _ in range(steps):
        if cur[0] == 0:
            break
        cur = apply_both(st, cur, random_update(rng, cur[0], 2, 2, cur))
        r = oracle.refine(cur[0], cur[1], cur[2], cur[3], cur[4], k, history=True, early_stop=False)
        if not partitions_equal(st.history(), r.history):
            return False
    return True


@pytest.mark.parametrize("seed", range(40))
def test_random_updates_equal_scratch(seed):
    assert maintained_equals_scratch(seed)


def test_change_k_from_history():
    """Change k (Section 4): a smaller k is read from the stored history; the
    rows equal a from-scratch run with that k."""
    rng = np.random.default_rng(5)
    g = synth.random_small_graph(rng, 12, 30, 2, 3)
    st = state_of(g, 5)
    h = st.history()
    for k in range(6):
        r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k, history=True, early_stop=False,
                          paper_numbering=True, head_pid0=True)
        assert checks.canon(h[k]).tolist() == checks.canon(r.pid).tolist()


# --- planted mistakes in the maintenance oracle --------------------------------

SRC = os.path.join(ROOT, "oracle", "maintain_oracle.cpp")
MUTANTS = {
    "no_propagation": ("for (const Pair& e : st.in[u]) pq.emplace(j + 1, e.second);", ";"),
    "propagate_to_targets": ("for (const Pair& e : st.in[u]) pq.emplace(j + 1, e.second);",
                             "for (const Pair& e : st.out[u]) pq.emplace(j + 1, e.second);"),
    "only_level1_queued": ("for (int32_t j = 1; j <= st.k; ++j) pq.emplace(j, src[e]);\n  for (int64_t e = 0",
                           "pq.emplace(1, src[e]);\n  for (int64_t e = 0"),
    "add_without_propagation": ("  propagate(st, std::move(pq));\n  return 0;\n}\n\n// Deletions",
                           "  return 0;\n}\n\n// Deletions"),
    "new_label_reuses_id": ("for (int32_t v : fresh) st.label_id[v] = int32_t(st.counter++);",
                            "for (int32_t v : fresh) st.label_id[v] = 1;"),
    "delete_one_copy": ("o.erase(std::remove(o.begin(), o.end(), Pair(l, t)), o.end());",
                        "{ auto it = std::find(o.begin(), o.end(), Pair(l, t)); if (it != o.end()) o.erase(it); }"),
}


def compile_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor for %s not unique" % name
    cpp = tmp_path / ("%s.cpp" % name)
    cpp.write_text(src.replace(old, new))
    so = tmp_path / ("%s.so" % name)
    base = os.path.join(ROOT, "oracle", "kbisim_oracle.cpp")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-o", str(so), str(cpp), base])
    return str(so)


class MutantState(M.State):
    lib_path = None

    def __init__(self, *a):
        lib = ctypes.CDLL(self.lib_path)
        p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.oracle_state_create.restype = p
        lib.oracle_state_create.argtypes = [i64, p, i64, p, p, p, i32]
        lib.oracle_state_num_nodes.restype = i64
        lib.oracle_state_num_nodes.argtypes = [p]
        lib.oracle_state_history.argtypes = [p, p]
        lib.oracle_state_work.argtypes = [p, p, p]
        lib.oracle_state_destroy.argtypes = [p]
        lib.oracle_state_add_nodes.argtypes = [p, i64, p]
        lib.oracle_state_delete_nodes.argtypes = [p, i64, p]
        for f in ("oracle_state_add_edges", "oracle_state_delete_edges"):
            getattr(lib, f).argtypes = [p, i64, p, p, p]
        node_label, src, elab, dst = (M._i32(x) for x in a[1:5])
        self._lib = lib
        self.k = int(a[5])
        self._h = lib.oracle_state_create(int(a[0]), M._ptr(node_label), int(src.shape[0]), M._ptr(src),
                                          M._ptr(elab), M._ptr(dst), self.k)


def mutant_fails_a_pin(so):
    MutantState.lib_path = so
    fx4, fx5 = load("updates.json")["table4"], load("updates.json")["table5"]
    g = fig1()
    st = MutantState(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 2)
    st.add_nodes([1])
    st.add_edges([1], [1], [6])
    if st.history().tolist() != fx4["pid_paper"]:
        return True
    st = MutantState(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 2)
    st.add_edges([5], [1], [4])
    if st.history().tolist() != fx5["pid_paper"] or st.work() != (3, 3):
        return True
    return not all(maintained_equals_scratch(seed, lib_state=MutantState) for seed in range(40))


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    return tmp_path_factory.mktemp("maintain_mutants")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_maintenance_mutant_is_caught(mutant_dir, name):
    assert mutant_fails_a_pin(compile_mutant(mutant_dir, name)), "planted mistake %s passed every pin" % name
