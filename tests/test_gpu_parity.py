"""Parity of the HIP path (through the C ABI) with the CPU oracle: ids of
every round bit-exact, block counts and rounds_done equal."""
import numpy as np
import pytest

import oracle
import synth
from golden_io import graph_of, load
from gpu_util import need_gpu, gpu_rounds, oracle_rounds, say, to_dev

pytestmark = pytest.mark.gpu


def check_parity(g, k, **kw):
    torch, kb = need_gpu()
    say("parity case %s N=%d E=%d k=%d %s" % (g.name, g.num_nodes, g.num_edges, k, kw))
    hist, counts, rd = gpu_rounds(torch, kb, g, k, **kw)
    r = oracle_rounds(g, k, early_stop=kw.get("early_stop", True))
    assert rd == r.rounds_done, (rd, r.rounds_done)
    assert counts == r.counts, (counts, r.counts)
    for j, row in enumerate(hist):
        bad = np.flatnonzero(row != r.history[j])
        assert bad.size == 0, "round %d: %d ids differ, first at node %d (gpu %d, oracle %d)" % (
            j, bad.size, bad[0], row[bad[0]], r.history[j][bad[0]])


def test_worked_example():
    check_parity(graph_of(load("figure1.json"), "figure1"), 6)


def test_worked_example_golden_values():
    """The GPU reproduces the hand-derived canonical ids of Figure 1 directly."""
    torch, kb = need_gpu()
    fx = load("figure1.json")
    g = graph_of(fx, "figure1")
    hist, counts, rd = gpu_rounds(torch, kb, g, 10)
    assert counts == fx["canonical"]["counts"] and rd == fx["canonical"]["rounds_done"]
    for j, row in enumerate(fx["canonical"]["pid"]):
        assert hist[j].tolist() == row


@pytest.mark.parametrize("table", ["table4", "table5"])
def test_update_tables(table):
    check_parity(graph_of(load("updates.json")[table], table), 4)


@pytest.mark.parametrize("seed", range(12))
def test_random_small(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 60))
    e = int(rng.integers(0, 4 * n))
    g = synth.random_small_graph(rng, n, e, int(rng.integers(1, 4)), int(rng.integers(1, 5)),
                                 dag=seed % 3 == 0)
    g.name = "small%d" % seed
    check_parity(g, n + 1)


def test_uniform_10k_50k_k5():
    g, k = synth.make_config("uniform-10k-50k")
    check_parity(g, k)


def test_uniform_no_early_stop():
    g = synth.uniform_graph(3000, 6000, num_node_labels=2, num_edge_labels=2, seed=4, name="u3k")
    check_parity(g, 9, early_stop=False)


def test_host_inputs():
    g = synth.uniform_graph(2000, 9000, seed=6, name="host-inputs")
    check_parity(g, 6, device_inputs=False)


def test_degree_buckets():
    """Out-degrees at every bucket edge: 0, 1, 15..17, 63..65, 128/129,
    256/257, 512/513, 4095..4097 and a 20k hub, among 3k low-degree nodes."""
    degs = [0, 1, 15, 16, 17, 63, 64, 65, 128, 129, 256, 257, 512, 513, 4095, 4096, 4097, 20000] * 2
    g = synth.degree_graph(degs + [2] * 3000, num_node_labels=2, num_edge_labels=3, seed=3,
                           name="degrees")
    check_parity(g, 6)


def test_thread_rows_at_list_capacity():
    """Out-degree 16 (the one-thread limit) everywhere: every wave of 64 nodes
    lists exactly 64 x 16 edges, the capacity of its LDS list. Then the same
    with all 16 edges of a node on one (label, target) pair (one unique key
    out of 16), and mixed with rows of 17 edges and empty rows, which the
    thread part leaves to the wave part or writes as empty."""
    g = synth.degree_graph([16] * 4096, num_node_labels=3, num_edge_labels=4, seed=31, name="deg16")
    check_parity(g, 4)
    rng = np.random.default_rng(32)
    n = 2048
    src = np.repeat(np.arange(n, dtype=np.int32), 16)
    dst = np.repeat(rng.integers(0, n, size=n, dtype=np.int32), 16)
    lab = np.repeat(rng.integers(0, 2, size=n, dtype=np.int32), 16)
    perm = rng.permutation(src.shape[0])
    node_label = rng.integers(0, 2, size=n, dtype=np.int32)
    check_parity(synth.Graph(n, node_label, src[perm], lab[perm], dst[perm], name="deg16-copies"), 4)
    g3 = synth.degree_graph([16, 17, 0, 16, 1] * 800, num_node_labels=2, num_edge_labels=3, seed=33,
                            name="deg16-mixed")
    check_parity(g3, 5)


def test_long_runs_without_edges():
    """Sources only at both ends of the id range: the CSR has long runs of
    empty rows (shorter and longer than the row-offset kernel's inline range)."""
    degs = [3] * 10 + [0] * 5000 + [2] * 7 + [0] * 40 + [5] * 4 + [0] * 70 + [1] * 3
    g = synth.degree_graph(degs, num_node_labels=3, num_edge_labels=2, seed=11, name="sparse-rows")
    check_parity(g, 5)
    # all edges from the last node only
    g2 = synth.degree_graph([0] * 3000 + [9], num_node_labels=2, num_edge_labels=2, seed=12, name="one-source")
    check_parity(g2, 3)


@pytest.mark.parametrize("medium_cap", [None, 64, 300, 1000])
def test_powerlaw_mid(medium_cap):
    """Power-law graph with hubs and large blocks; the split between the
    workgroup resolver and the global passes must not change any id."""
    g = synth.powerlaw_graph(200_000, 2_000_000, seed=7, deg_cap=30_000, name="powerlaw-200k")
    check_parity(g, 10, medium_cap=medium_cap)


@pytest.mark.parametrize("radix_tile", [2048, 4096])
def test_radix_tiles(radix_tile):
    """Every radix pass (create's sort by source with its fused first pass,
    the ordering's device-wide passes) on the other compiled tile sizes: the
    power-law graph (hundreds of tiles per pass) and a small graph whose
    passes take the single-launch path (at most 64 tiles)."""
    g = synth.powerlaw_graph(200_000, 2_000_000, seed=7, deg_cap=30_000, name="powerlaw-200k")
    check_parity(g, 10, radix_tile=radix_tile)
    check_parity(synth.uniform_graph(20_000, 100_000, num_node_labels=3, num_edge_labels=5, seed=4,
                                     name="uniform-20k-100k"), 6, radix_tile=radix_tile, medium_cap=64)


def test_radix_tile_rejected():
    torch, kb = need_gpu()
    g = synth.worked_example()
    for bad in (1000, 3000, -1):
        with pytest.raises(kb.KbisimError, match="radix_tile"):
            kb.Graph(6, g.node_label, g.src, g.elab, g.dst, radix_tile=bad)


@pytest.mark.parametrize("members,endings", [(40, 7), (300, 20), (3000, 50)])
def test_deep_common_prefix(members, endings):
    """Blocks (small, medium, large) whose signatures share their first 1000
    keys and differ only after them."""
    width = 1000
    n_t = width + endings
    n = n_t + members
    lab = np.arange(n, dtype=np.int32)
    lab[n_t:] = n_t  # all sources in one block
    src, dst = [], []
    for j in range(members):
        s = n_t + j
        src.append(np.full(width + 1, s))
        dst.append(np.concatenate([np.arange(width), [width + (j * 7919) % endings]]))
    src = np.concatenate(src).astype(np.int32)
    dst = np.concatenate(dst).astype(np.int32)
    g = synth.Graph(n, lab, src, np.zeros(src.shape[0], np.int32), dst,
                    name="prefix%d" % members)
    check_parity(g, 3)
    check_parity(g, 3, medium_cap=64)


def test_identical_hubs():
    """Two hubs with identical long signatures and two that differ only at
    their last key: long verification and a deep split."""
    rng = np.random.default_rng(5)
    n = 12_000
    base = rng.integers(100, n, size=9000)
    src, dst = [], []
    for h in range(4):
        d = base.copy()
        if h == 3:
            d[-1] = 0  # node 0 is unique-labelled: last key differs
        src.append(np.full(d.shape[0], h))
        dst.append(d)
    src.append(rng.integers(100, n, size=20000))
    dst.append(rng.integers(0, n, size=20000))
    src = np.concatenate(src).astype(np.int32)
    dst = np.concatenate(dst).astype(np.int32)
    lab = np.zeros(n, np.int32)
    lab[0] = 1
    g = synth.Graph(n, lab, src, np.zeros(src.shape[0], np.int32), dst, name="hubs")
    check_parity(g, 6)


def test_empty_and_trivial():
    torch, kb = need_gpu()
    z = np.zeros(0, np.int32)
    pid, counts, rd = kb.refine(0, z, z, z, z, 3)
    assert pid.size == 0 and counts == [0, 0] and rd == 1
    g = synth.Graph(5, np.array([3, 1, 3, 0, 1], np.int32), z, z, z, name="noedges")
    check_parity(g, 4)
    check_parity(synth.worked_example(), 0)


def test_resume_and_idempotent():
    torch, kb = need_gpu()
    g = synth.uniform_graph(5000, 20000, seed=12)
    r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 4)
    with kb.Graph(g.num_nodes, *to_dev(torch, g)) as h:
        h.refine(2)
        h.refine(1)  # below the rounds done: no-op
        assert h.refine(4) == r.rounds_done
        pid, nb, counts = h.result()
        assert np.array_equal(pid, r.pid) and counts == r.counts
        out = torch.empty(g.num_nodes, dtype=torch.int32, device="cuda:0")
        pid_d, _, _ = h.result(device="cuda:0")
        assert np.array_equal(pid_d.cpu().numpy(), r.pid)


def test_invalid_inputs():
    torch, kb = need_gpu()
    g = synth.worked_example()
    bad = g.dst.copy()
    bad[0] = 6
    with pytest.raises(kb.KbisimError) as e:
        kb.Graph(6, g.node_label, g.src, g.elab, bad)
    assert e.value.status == -1
    lab = g.node_label.copy()
    lab[2] = -3
    with pytest.raises(kb.KbisimError) as e:
        kb.Graph(6, lab, g.src, g.elab, g.dst)
    assert e.value.status == -1
    with kb.Graph(6, g.node_label, g.src, g.elab, g.dst) as h:
        with pytest.raises(kb.KbisimError):
            h.refine(-1)
        assert h.refine(2) == 2  # the handle still works after an error


def test_profile_mode_same_ids():
    """Profiling (event timers and work counters) leaves the ids unchanged."""
    torch, kb = need_gpu()
    g = synth.powerlaw_graph(30_000, 300_000, seed=21, deg_cap=6_000, name="prof")
    r = oracle.refine(g.num_nodes, g.node_label, g.src, g.elab, g.dst, 6)
    with kb.Graph(g.num_nodes, *to_dev(torch, g), profile=True) as h:
        rd = h.refine(6)
        pid, nb, counts = h.result()
        prof = h.profile()
        work = h.work()
        per_round = h.round_profile()
    assert rd == r.rounds_done and counts == r.counts and np.array_equal(pid, r.pid)
    assert prof["round"][1] == rd and prof["signature"][1] == rd
    assert sum(v[0] for v in work.values()) > 0
    # per round: the same work split by round, times of every round
    assert len(per_round) == rd
    assert sum(x["active_nodes"] for x in per_round) == sum(v[0] for v in work.values())
    assert sum(x["active_edges"] for x in per_round) == sum(v[1] for v in work.values())
    _, lab_rank, lab_count = np.unique(g.node_label, return_inverse=True, return_counts=True)
    assert per_round[0]["active_nodes"] == int(np.sum(lab_count[lab_rank] >= 2))  # round 1: label blocks of 2+
    for x in per_round:
        assert 0 < x["signature_ms"] <= x["round_ms"]
    # round 1: longest signature = most distinct (edge label, label of target) pairs of an active node
    act = lab_count[lab_rank] >= 2
    keep = act[g.src]
    pairs = np.unique(np.stack([g.src[keep].astype(np.int64), g.elab[keep].astype(np.int64),
                                lab_rank[g.dst[keep]].astype(np.int64)]), axis=1)
    assert per_round[0]["max_keys"] == int(np.bincount(pairs[0]).max())
    assert all(0 <= x["max_keys"] <= int(np.bincount(g.src).max()) for x in per_round)
    assert abs(sum(x["round_ms"] for x in per_round) - prof["round"][0]) < 1e-6 * max(1.0, prof["round"][0])


def test_wide_keys():
    """More than 2^22 distinct edge labels on 1000 nodes: label bits + id bits
    exceed 32, so the packed edge words and the keys are 64-bit."""
    rng = np.random.default_rng(17)
    n, e = 1000, (1 << 22) + 5000
    src = rng.integers(0, n, size=e).astype(np.int32)
    dst = rng.integers(0, n, size=e).astype(np.int32)
    lab = rng.permutation(e).astype(np.int32) // 1  # all distinct
    lab[:5000] = lab[5000:10000]                     # some shared labels
    node_label = rng.integers(0, 3, size=n).astype(np.int32)
    g = synth.Graph(n, node_label, src, lab, dst, name="widekeys")
    check_parity(g, 3)


def test_key_width_exactly_32():
    """Label bits + id bits == 32: largest keys use all 32 bits."""
    n = (1 << 21) + 7
    rng = np.random.default_rng(23)
    e = 3 * n
    src = rng.integers(0, n, size=e).astype(np.int32)
    dst = rng.integers(0, n, size=e).astype(np.int32)
    lab = rng.integers(0, 2048, size=e).astype(np.int32)  # 11 label bits + 22 id bits... capped below
    lab = (lab % 1024).astype(np.int32)  # 10 bits + 22 bits = 32
    node_label = rng.integers(0, 4, size=n).astype(np.int32)
    g = synth.Graph(n, node_label, src, lab, dst, name="key32")
    check_parity(g, 2)


@pytest.mark.parametrize("top", [255, 256])
def test_label_values_near_mask_limit(top):
    """Label values around 256: below it the ranks come from the presence
    mask of the validation pass, from 256 on from the marking table."""
    rng = np.random.default_rng(31 + top)
    n, e = 4000, 24000
    nvals = np.array([0, 63, 64, 200, top], np.int32)
    evals = np.array([1, 64, 128, 191, top], np.int32)
    g = synth.Graph(n, nvals[rng.integers(0, 5, size=n)], rng.integers(0, n, size=e).astype(np.int32),
                    evals[rng.integers(0, 5, size=e)], rng.integers(0, n, size=e).astype(np.int32),
                    name="labels%d" % top)
    check_parity(g, 5)


def test_large_label_values():
    """Label values up to 2^31 - 1 (ranked by sorting instead of a table)."""
    rng = np.random.default_rng(29)
    n, e = 5000, 30000
    vals = np.array([0, 7, 1 << 24, (1 << 31) - 1, 123456789], np.int32)
    g = synth.Graph(n, vals[rng.integers(0, 5, size=n)], rng.integers(0, n, size=e).astype(np.int32),
                    vals[rng.integers(0, 5, size=e)], rng.integers(0, n, size=e).astype(np.int32),
                    name="biglabels")
    check_parity(g, 5)
