"""The allocation-free entry point (kbisim_refine_static, static scratch
region) against the ordinary entry points (kbisim_create / kbisim_refine /
kbisim_result) on the same inputs, bit-exact, on two calls in a row (the
second on a smaller graph, so the region holds the first call's contents),
and against the oracle; a graph too large for the region is rejected."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def ordinary(kb, g, arrs, k, stream):
    h = kb.kbisim_create(g.num_nodes, *arrs, stream=stream)
    try:
        rd = kb.kbisim_refine(h, k)
        out = np.empty(g.num_nodes, np.int32)
        nb, _ = kb.kbisim_result(h, out)
    finally:
        kb.kbisim_destroy(h)
    return out, nb, rd


def test_static_matches_ordinary_two_calls():
    torch, kb = need_gpu()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    big = synth.powerlaw_graph(100_000, 1_000_000, seed=21, num_node_labels=12, num_edge_labels=6)
    small = synth.uniform_graph(10_000, 50_000, seed=22)
    for g, k in ((big, 10), (small, 5)):
        arrs = to_dev(torch, g)
        want, nb_w, rd_w = ordinary(kb, g, arrs, k, stream)
        out = torch.full((g.num_nodes,), -7, dtype=torch.int32, device=dev)
        nb, rd = kb.kbisim_refine_static(g.num_nodes, *arrs, k, out, stream=stream)
        got = out.cpu().numpy()
        say("%s: static call rounds=%d blocks=%d" % (g.name, rd, nb))
        assert (nb, rd) == (nb_w, rd_w)
        assert np.array_equal(got, want)
        r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k)
        assert np.array_equal(got, r.pid) and rd == r.rounds_done
        # host inputs and a host result give the same
        host_out = np.empty(g.num_nodes, np.int32)
        nb2, rd2 = kb.kbisim_refine_static(g.num_nodes, g.node_label, g.src, g.elab, g.dst, k, host_out)
        assert (nb2, rd2) == (nb, rd) and np.array_equal(host_out, want)
        # the smallest radix tile (most tiles, largest histograms) fits the region too
        out.fill_(-7)
        nb3, rd3 = kb.kbisim_refine_static(g.num_nodes, *arrs, k, out, stream=stream, radix_tile=2048)
        assert (nb3, rd3) == (nb, rd) and np.array_equal(out.cpu().numpy(), want)


def test_static_rejects_oversize_and_bad_input():
    torch, kb = need_gpu()
    g = synth.uniform_graph(1_000_000, 4_000_000, seed=3)
    out = np.empty(g.num_nodes, np.int32)
    with pytest.raises(kb.KbisimError) as e:
        kb.kbisim_refine_static(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 3, out)
    assert e.value.status == -2
    bad = synth.uniform_graph(100, 300, seed=4)
    bad.dst = bad.dst.copy()
    bad.dst[3] = 100
    with pytest.raises(kb.KbisimError) as e:
        kb.kbisim_refine_static(bad.num_nodes, bad.node_label, bad.src, bad.elab, bad.dst, 3,
                                np.empty(100, np.int32))
    assert e.value.status == -1
    # the region is usable again afterwards
    ok = synth.uniform_graph(2_000, 9_000, seed=5)
    o2 = np.empty(ok.num_nodes, np.int32)
    kb.kbisim_refine_static(ok.num_nodes, ok.node_label, ok.src, ok.elab, ok.dst, 4, o2)
    r = oracle.refine(ok.num_nodes, ok.node_label, ok.src, ok.elab, ok.dst, 4)
    assert np.array_equal(o2, r.pid)
