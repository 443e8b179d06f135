"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np
import pytest

import oracle


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_0748_amd as kb
    kb.load_library()  # raises if the HIP library is not built: no fallback
    return torch, kb


def to_dev(torch, g):
    d = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(d)
    return t(g.node_label), t(g.src), t(g.elab), t(g.dst)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_rounds(torch, kb, g, k, device_inputs=True, **kw):
    """Runs the GPU refine one round at a time; returns (history rows, counts, rounds_done)."""
    if device_inputs:
        arrs = to_dev(torch, g)
    else:
        arrs = (g.node_label, g.src, g.elab, g.dst)
    hist = []
    with kb.Graph(g.num_nodes, *arrs, **kw) as h:
        pid, nb, counts = h.result()
        hist.append(pid.copy())
        for j in range(1, k + 1):
            rd = h.refine(j)
            pid, nb, counts = h.result()
            if rd < j:
                break
            hist.append(pid.copy())
        return hist, counts, h.rounds_done


def oracle_rounds(g, k, early_stop=True):
    r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k, history=True,
                      early_stop=early_stop)
    return r
