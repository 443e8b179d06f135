"""The pins are strong enough: each plausible mistake planted in a copy of the
oracle (on the CPU, in a temporary directory) makes at least one pin fail.

A mutant is the oracle source with one textual substitution; it is compiled
with g++ and driven through the same C entry point.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import checks
import synth
from golden_io import graph_of, load

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "kbisim_oracle.cpp")

MUTANTS = {
    "no_dedup": ("pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());", ""),
    "no_head": ("s.push_back(head);", ""),
    "pair_transposed": ("pairs.emplace_back(le.first, pid_prev[le.second]);",
                        "pairs.emplace_back(pid_prev[le.second], le.first);"),
    "target_id_not_pid": ("pairs.emplace_back(le.first, pid_prev[le.second]);",
                          "pairs.emplace_back(le.first, le.second);"),
    "label_dropped": ("pairs.emplace_back(le.first, pid_prev[le.second]);",
                      "pairs.emplace_back(0, pid_prev[le.second]);"),
    "descending_pairs": ("std::sort(pairs.begin(), pairs.end());",
                         "std::sort(pairs.rbegin(), pairs.rend());"),
    "descending_ranks": ("std::map<Sig, int32_t> store;\n      for (int64_t v = 0; v < n; ++v) store.emplace",
                         "std::map<Sig, int32_t, std::greater<Sig>> store;\n      for (int64_t v = 0; v < n; ++v) store.emplace"),
    "edges_reversed": ("out[src[e]].emplace_back(elab[e], dst[e]);",
                       "out[dst[e]].emplace_back(elab[e], src[e]);"),
    "stop_too_early": ("const bool fixed = (blocks == blocks_prev);",
                       "const bool fixed = (blocks >= blocks_prev);"),
    "head_is_label_rank_always": ("const int32_t head = head_pid0 ? pid0[v] : pid[v];",
                                  "const int32_t head = pid0[v];"),
    "paper_counter_restarts": ("next_global = 1 + int64_t(labels.size());",
                               "next_global = 1;"),
    "k0_descending": ("std::sort(labels.begin(), labels.end());",
                      "std::sort(labels.rbegin(), labels.rend());"),
}


def compile_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor for %s not unique" % name
    mut = src.replace(old, new)
    if "std::greater" in mut:
        mut = "#include <functional>\n" + mut
    cpp = tmp_path / ("%s.cpp" % name)
    cpp.write_text(mut)
    so = tmp_path / ("%s.so" % name)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-o", str(so), str(cpp)])
    lib = ctypes.CDLL(str(so))
    p = ctypes.c_void_p
    lib.oracle_refine.restype = ctypes.c_int32
    lib.oracle_refine.argtypes = [ctypes.c_int64, ctypes.c_int64, p, p, p, p, ctypes.c_int32,
                                  ctypes.c_int32, p, p, p, p, p]
    return lib


def refine_with(lib, g, k, flags=0):
    """Returns (history[(k+1), N], counts, rounds_done)."""
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    n = g.num_nodes
    lab, s, l, d = (np.ascontiguousarray(a, np.int32) for a in (g.node_label, g.src, g.elab, g.dst))
    pid = np.empty(n, np.int32)
    counts = np.empty(k + 1, np.int64)
    msi = np.empty(k + 1, np.int64)
    hist = np.empty((k + 1, n), np.int32)
    rd = np.zeros(1, np.int32)
    st = lib.oracle_refine(n, s.shape[0], ptr(lab), ptr(s), ptr(l), ptr(d), k, flags, ptr(pid),
                           ptr(counts), ptr(msi), ptr(hist), ptr(rd))
    assert st == 0
    return hist, [int(c) for c in counts[: rd[0] + 1]], int(rd[0])


def pin_suite(lib):
    """Runs the pins; returns the names of those that fail."""
    failed = []
    fx = load("figure1.json")
    g = graph_of(fx)
    h, counts, rd = refine_with(lib, g, 10)
    can = fx["canonical"]
    if counts != can["counts"] or rd != can["rounds_done"] or \
            any(h[i].tolist() != row for i, row in enumerate(can["pid"])):
        failed.append("figure1_canonical")
    h, _, _ = refine_with(lib, g, 2, flags=1 | 2 | 4)
    if h.tolist() != fx["paper_numbering"]["pid"]:
        failed.append("table1")
    t = synth.tree_graph(2, 4)
    _, counts, _ = refine_with(lib, t, 7, flags=4)
    if counts != [min(j, 4) + 1 for j in range(8)]:
        failed.append("tree_closed_form")
    # pair order inside a signature decides the rank (hand-derived)
    po = synth.Graph(4, np.array([0, 1, 2, 2], np.int32), np.array([2, 2, 3, 3], np.int32),
                     np.array([0, 1, 0, 1], np.int32), np.array([1, 0, 0, 1], np.int32))
    h, _, _ = refine_with(lib, po, 1, flags=4)
    if h[1].tolist() != [0, 1, 3, 2]:
        failed.append("pair_order")
    # duplicate edges change nothing
    dup = synth.Graph(6, g.node_label, np.concatenate([g.src, g.src]),
                      np.concatenate([g.elab, g.elab]), np.concatenate([g.dst, g.dst]))
    h1, _, _ = refine_with(lib, g, 6, flags=4)
    h2, _, _ = refine_with(lib, dup, 6, flags=4)
    if not np.array_equal(h1, h2):
        failed.append("duplicates")
    rng = np.random.default_rng(99)
    for _ in range(12):
        gg = synth.random_small_graph(rng, 6, 9, 2, 2)
        tri = list(zip(gg.src.tolist(), gg.elab.tolist(), gg.dst.tolist()))
        hh, _, _ = refine_with(lib, gg, 5, flags=4)
        rel = bf.def1_relations(6, gg.node_label.tolist(), tri, 5)
        try:
            for j in range(1, 6):
                assert hh[j].tolist() == bf.lex_rank_round(6, tri, hh[j - 1], hh[j - 1])
            checks.check_label_rank(gg.node_label, hh[0])
            for j in range(6):
                checks.check_dense(hh[j], len(set(hh[j].tolist())))
                if j:
                    checks.check_refines_monotone(hh[j - 1], hh[j])
            ok = all(bf.relation_of_ids(hh[j]) == rel[j] for j in range(6))
        except AssertionError:
            ok = False
        if not ok:
            failed.append("bruteforce_or_invariants")
            break
    return failed


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    return tmp_path_factory.mktemp("mutants")


def test_unmutated_passes(tmp_path):
    lib = ctypes.CDLL(__import__("oracle").build())
    lib.oracle_refine.restype = ctypes.c_int32
    p = ctypes.c_void_p
    lib.oracle_refine.argtypes = [ctypes.c_int64, ctypes.c_int64, p, p, p, p, ctypes.c_int32,
                                  ctypes.c_int32, p, p, p, p, p]
    assert pin_suite(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(mutant_dir, name):
    lib = compile_mutant(mutant_dir, name)
    assert pin_suite(lib), "planted mistake %s passed every pin" % name
