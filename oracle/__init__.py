"""CPU oracle for k-bisimulation partition refinement (test infrastructure).

This package is the checker, not the product: only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it. It shares no code with the GPU library ``paper_1210_0748_amd``
and never imports it.

Contents
--------
* ``refine``      -- Build_Bisim (Algorithm 1, Section 3) in plain C++17 with
                     S as an ordered dictionary; canonical ids are per-round
                     lexicographic signature ranks.
* ``signature_lengths`` -- lengths of all signatures from given previous ids.
* ``signatures``  -- Definition 3 signatures of sampled nodes from a given
                     previous-round id array (one-round checks at full size).
* ``maintain``    -- the maintenance algorithms of Section 4 (Add_Nodes,
                     Add_Edges, deletions) on a stored history, in the
                     paper's numbering, and the updated graph by definition.
* ``bruteforce``  -- pairwise bisimilarity from Definition 1, Kaushik's
                     definition and the Paige-Tarjan stable-partition
                     definition (Appendix, "Alternative definitions"), plus the
                     greatest bisimulation (Appendix, "Connection between
                     localized bisimulation and full bisimulation").
* ``checks``      -- invariants of the method (refinement, density, monotone
                     ids, lexicographic order of ids vs signatures).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kbisim_oracle.cpp")
_SRCS = [_SRC, os.path.join(_HERE, "maintain_oracle.cpp")]
_LIB = os.path.join(_HERE, "liboracle.so")

HEAD_PID0 = 1
PAPER_NUMBERING = 2
NO_EARLY_STOP = 4


def build(force: bool = False) -> str:
    """Compile the C++ oracle with g++ (one thread, -O2). Returns the .so path."""
    newest = max(os.path.getmtime(f) for f in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        p = ctypes.c_void_p
        lib.oracle_refine.restype = i32
        lib.oracle_refine.argtypes = [i64, i64, p, p, p, p, i32, i32, p, p, p, p, p]
        lib.oracle_signatures.restype = i32
        lib.oracle_signatures.argtypes = [i64, i64, p, p, p, p, i64, p, p, p]
        lib.oracle_signature_lengths.restype = i32
        lib.oracle_signature_lengths.argtypes = [i64, i64, p, p, p, p, p]
        lib.oracle_round_sample.restype = i32
        lib.oracle_round_sample.argtypes = [i64, i64, p, p, p, p, i64, p, p, p]
        lib.oracle_state_create.restype = p
        lib.oracle_state_create.argtypes = [i64, p, i64, p, p, p, i32]
        lib.oracle_state_destroy.restype = None
        lib.oracle_state_destroy.argtypes = [p]
        lib.oracle_state_num_nodes.restype = i64
        lib.oracle_state_num_nodes.argtypes = [p]
        lib.oracle_state_history.restype = None
        lib.oracle_state_history.argtypes = [p, p]
        lib.oracle_state_work.restype = None
        lib.oracle_state_work.argtypes = [p, p, p]
        lib.oracle_state_add_nodes.restype = i32
        lib.oracle_state_add_nodes.argtypes = [p, i64, p]
        for f in ("oracle_state_add_edges", "oracle_state_delete_edges"):
            getattr(lib, f).restype = i32
            getattr(lib, f).argtypes = [p, i64, p, p, p]
        lib.oracle_state_delete_nodes.restype = i32
        lib.oracle_state_delete_nodes.argtypes = [p, i64, p]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


@dataclass
class Result:
    pid: np.ndarray            # [N] int32, ids of round rounds_done (== pId_k)
    counts: list               # B_0 .. B_rounds_done
    max_sig_ints: list         # longest signature per round (ints)
    rounds_done: int
    history: np.ndarray | None  # [(k+1), N] when requested


class OracleError(ValueError):
    pass


def refine(num_nodes, node_label, src, elab, dst, k, *, head_pid0=False,
           paper_numbering=False, early_stop=True, history=False) -> Result:
    """Run Build_Bisim for up to k rounds on the graph; see module docstring."""
    lib = _load()
    n = int(num_nodes)
    node_label = _i32(node_label)
    src, elab, dst = _i32(src), _i32(elab), _i32(dst)
    m = int(src.shape[0])
    if node_label.shape[0] != n or elab.shape[0] != m or dst.shape[0] != m:
        raise OracleError("array lengths do not match N / E")
    k = int(k)
    if k < 0:
        raise OracleError("k must be >= 0")
    flags = (HEAD_PID0 if head_pid0 else 0) | (PAPER_NUMBERING if paper_numbering else 0) | \
            (0 if early_stop else NO_EARLY_STOP)
    pid = np.empty(n, np.int32)
    counts = np.empty(k + 1, np.int64)
    msi = np.empty(k + 1, np.int64)
    hist = np.empty((k + 1, n), np.int32) if history else None
    rd = np.zeros(1, np.int32)
    st = lib.oracle_refine(n, m, _ptr(node_label), _ptr(src), _ptr(elab), _ptr(dst), k, flags,
                           _ptr(pid), _ptr(counts), _ptr(msi), _ptr(hist), _ptr(rd))
    if st != 0:
        raise OracleError("invalid input (status %d)" % st)
    r = int(rd[0])
    return Result(pid=pid, counts=[int(c) for c in counts[: r + 1]],
                  max_sig_ints=[int(c) for c in msi[: r + 1]], rounds_done=r, history=hist)


def signature_lengths(num_nodes, src, elab, dst, pid_prev):
    """[N] int64: length (ints) of every node's signature from pid_prev."""
    lib = _load()
    n = int(num_nodes)
    src, elab, dst, pid_prev = _i32(src), _i32(elab), _i32(dst), _i32(pid_prev)
    out = np.empty(n, np.int64)
    if lib.oracle_signature_lengths(n, int(src.shape[0]), _ptr(src), _ptr(elab), _ptr(dst), _ptr(pid_prev),
                                    _ptr(out)) != 0:
        raise OracleError("invalid input")
    return out


def longest_multi_member(lengths, pid_prev):
    """Longest signature among the nodes whose class in the previous round
    has two or more members (1 when there is none): nodes alone in their
    class keep it in every later round whatever their signature."""
    pid_prev = np.asarray(pid_prev)
    if pid_prev.size == 0:
        return 1
    sizes = np.bincount(pid_prev)
    multi = sizes[pid_prev] >= 2
    return int(max(1, lengths[multi].max())) if multi.any() else 1


def round_sample(num_nodes, node_label, src, elab, dst, sample):
    """Round 1 of Build_Bisim restricted to the sampled nodes (their
    signatures from pId_0 inserted into one ordered dictionary). Returns
    (ranks of the sampled nodes' signatures among the sample's distinct
    signatures, number of out-edges of the sampled nodes)."""
    lib = _load()
    n = int(num_nodes)
    node_label = _i32(node_label)
    src, elab, dst = _i32(src), _i32(elab), _i32(dst)
    sample = _i32(sample)
    rank = np.empty(sample.shape[0], np.int32)
    edges = np.zeros(1, np.int64)
    st = lib.oracle_round_sample(n, int(src.shape[0]), _ptr(node_label), _ptr(src), _ptr(elab), _ptr(dst),
                                 int(sample.shape[0]), _ptr(sample), _ptr(rank), _ptr(edges))
    if st != 0:
        raise OracleError("invalid input (status %d)" % st)
    return rank, int(edges[0])


def signatures(num_nodes, src, elab, dst, pid_prev, sample):
    """Flattened signatures [pid_prev[v], l1, p1, ...] of the sampled nodes.

    Returns a list of tuples (one per sampled node, in sample order).
    """
    lib = _load()
    n = int(num_nodes)
    src, elab, dst = _i32(src), _i32(elab), _i32(dst)
    pid_prev = _i32(pid_prev)
    sample = _i32(sample)
    m = int(src.shape[0])
    off = np.empty(sample.shape[0] + 1, np.int64)
    st = lib.oracle_signatures(n, m, _ptr(src), _ptr(elab), _ptr(dst), _ptr(pid_prev),
                               int(sample.shape[0]), _ptr(sample), _ptr(off), None)
    if st != 0:
        raise OracleError("invalid input (status %d)" % st)
    buf = np.empty(int(off[-1]), np.int32)
    st = lib.oracle_signatures(n, m, _ptr(src), _ptr(elab), _ptr(dst), _ptr(pid_prev),
                               int(sample.shape[0]), _ptr(sample), _ptr(off), _ptr(buf))
    if st != 0:
        raise OracleError("invalid input (status %d)" % st)
    return [tuple(int(x) for x in buf[off[j]:off[j + 1]]) for j in range(sample.shape[0])]
