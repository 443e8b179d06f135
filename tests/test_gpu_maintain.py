"""Maintenance on the GPU (Section 4): the stored history answers a smaller
k (change of k), and updates (new nodes, deleted and added edges) bring every
stored round up to date. After an update the handle must hold exactly what
a from-scratch run on the updated graph gives: every round's ids (bit-exact
against the oracle), the counts and the rounds done."""
import numpy as np
import pytest

import oracle
from oracle import maintain as M
import synth
from golden_io import graph_of, load
from gpu_util import need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def oracle_hist(n, lab, s, l, d, k, early_stop=True):
    return oracle.refine(n, lab, s, l, d, k, history=True, early_stop=early_stop)


def check_against(h, cur, k, early_stop=True, what=""):
    """Every stored round of handle h equals the oracle on graph cur."""
    n, lab, s, l, d = cur
    r = oracle_hist(n, lab, s, l, d, k, early_stop)
    assert h.rounds_done == r.rounds_done, (what, h.rounds_done, r.rounds_done)
    for j in range(r.rounds_done + 1):
        got, nb = h.result_round(j)
        assert nb == r.counts[j], (what, j, nb, r.counts[j])
        assert np.array_equal(got, r.history[j]), (what, "round %d differs" % j)
    pid, nb, counts = h.result()
    assert counts == r.counts and np.array_equal(pid, r.pid), what
    if early_stop and r.rounds_done < k:  # rounds past the fixed point equal it
        got, nb = h.result_round(k)
        assert np.array_equal(got, r.pid)


def cur_of(g):
    return (g.num_nodes, np.asarray(g.node_label, np.int32), np.asarray(g.src, np.int32),
            np.asarray(g.elab, np.int32), np.asarray(g.dst, np.int32))


@pytest.mark.parametrize("name", ["figure1", "powerlaw"])
def test_history_change_k(name):
    """Change k: every round j <= rounds done read back from the history
    equals the oracle's pId_j, and reading them runs no round."""
    torch, kb = need_gpu()
    g = graph_of(load("figure1.json")) if name == "figure1" else \
        synth.powerlaw_graph(200_000, 2_000_000, seed=3, num_node_labels=20, num_edge_labels=8)
    with kb.Graph(g.num_nodes, *to_dev(torch, g), history=True, profile=True) as h:
        h.refine(10)
        before = h.profile()["round"][1]
        check_against(h, cur_of(g), 10)
        assert h.profile()["round"][1] == before, "reading earlier rounds ran a round"
        r = oracle_hist(*cur_of(g), 10)
        # a larger k after a smaller read continues from the stored state
        got, nb = h.result_round(1, device=torch.device("cuda:0"))
        assert np.array_equal(got.cpu().numpy(), r.history[1])
    say("%s: %d rounds checked" % (name, r.rounds_done))


def test_history_needs_option():
    torch, kb = need_gpu()
    g = graph_of(load("figure1.json"))
    with kb.Graph(g.num_nodes, *to_dev(torch, g)) as h:
        h.refine(3)
        with pytest.raises(kb.KbisimError) as e:
            h.result_round(1)
        assert e.value.status == -4
        out, nb = h.result_round(h.rounds_done)  # the current round needs no history
        with pytest.raises(kb.KbisimError) as e:
            h.update(add=([0], [0], [1]))
        assert e.value.status == -4


MODES = [0, 1, 2]  # rounds of an update: by cost, level by level, in full


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("early_stop,k", [(False, 2), (True, 10)])
def test_update_tables_4_and_5(early_stop, k, mode):
    """Section 4's example run: Figure 1 plus node 7 and (2,l,7) (Table 4),
    and plus (6,l,5) (Table 5)."""
    torch, kb = need_gpu()
    g = graph_of(load("figure1.json"))
    for upd in (dict(new_labels=[1], add=([1], [1], [6])), dict(add=([5], [1], [4]))):
        with kb.Graph(g.num_nodes, g.node_label, g.src, g.elab, g.dst, history=True, early_stop=early_stop,
                      update_mode=mode) as h:
            h.refine(k)
            h.update(**upd)
            cur = M.updated_graph(*cur_of(g), **upd)
            check_against(h, cur, k, early_stop, str(upd))


def random_gpu_update(rng, cur, n_labels, e_labels, allow_nodes=True):
    n = cur[0]
    kind = int(rng.integers(0, 6 if allow_nodes else 3))
    m = int(rng.integers(1, 6))
    if kind == 4 and n > 2:  # delete nodes
        return dict(delete_nodes=rng.integers(0, n, size=int(rng.integers(1, 3))).astype(np.int32))
    if kind == 5 and n > 2:  # everything at once
        nn = int(rng.integers(1, 3))
        dn = rng.integers(0, n + nn, size=int(rng.integers(1, 3))).astype(np.int32)
        n_after = n + nn - np.unique(dn).size
        upd = dict(new_labels=rng.integers(0, n_labels + 2, size=nn).astype(np.int32), delete_nodes=dn)
        if cur[2].shape[0]:
            pick = rng.integers(0, cur[2].shape[0], m)
            upd["delete"] = (cur[2][pick], cur[3][pick], cur[4][pick])
        if n_after > 0:
            upd["add"] = tuple(x.astype(np.int32) for x in (rng.integers(0, n_after, m), rng.integers(0, e_labels, m),
                                                           rng.integers(0, n_after, m)))
        return upd
    if kind >= 3:
        return dict(new_labels=rng.integers(0, n_labels + 2, size=int(rng.integers(1, 4))).astype(np.int32))
    if kind == 0 or cur[2].shape[0] == 0:
        return dict(add=tuple(x.astype(np.int32) for x in (rng.integers(0, n, m), rng.integers(0, e_labels + 1, m),
                                                           rng.integers(0, n, m))))
    if kind == 1:
        pick = rng.integers(0, cur[2].shape[0], m)
        return dict(delete=(cur[2][pick], cur[3][pick], cur[4][pick]))
    pick = rng.integers(0, cur[2].shape[0], m)
    return dict(delete=(cur[2][pick], cur[3][pick], cur[4][pick]),
                add=tuple(x.astype(np.int32) for x in (rng.integers(0, n, m), rng.integers(0, e_labels, m),
                                                       rng.integers(0, n, m))))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(12))
def test_update_random_small(seed, mode):
    torch, kb = need_gpu()
    rng = np.random.default_rng(1000 + seed)
    early_stop = bool(seed % 2)
    k = int(rng.integers(1, 7))
    g = synth.random_small_graph(rng, int(rng.integers(4, 40)), int(rng.integers(0, 120)), 3, 3)
    cur = cur_of(g)
    say("seed %d: N=%d E=%d k=%d early_stop=%s" % (seed, cur[0], cur[2].shape[0], k, early_stop))
    with kb.Graph(cur[0], *cur[1:], history=True, early_stop=early_stop, update_mode=mode) as h:
        h.refine(k)
        check_against(h, cur, k, early_stop, "initial")
        for step in range(6):
            upd = random_gpu_update(rng, cur, 3, 3)
            h.update(**upd)
            cur = M.updated_graph(*cur, **upd)
            check_against(h, cur, k, early_stop, "step %d %s" % (step, sorted(upd)))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("m", [1, 100, 10000])
def test_update_powerlaw_200k(m, mode):
    """Edge insertions and deletions on a 200k-node / 2M-edge power-law
    graph (device inputs), every round against the oracle."""
    torch, kb = need_gpu()
    g = synth.powerlaw_graph(200_000, 2_000_000, seed=7, num_node_labels=30, num_edge_labels=8)
    rng = np.random.default_rng(m)
    cur = cur_of(g)
    dev = torch.device("cuda:0")
    with kb.Graph(g.num_nodes, *to_dev(torch, g), history=True, update_mode=mode) as h:
        h.refine(10)
        add = tuple(x.astype(np.int32) for x in (rng.integers(0, g.num_nodes, m), rng.integers(0, 8, m),
                                                 rng.integers(0, g.num_nodes, m)))
        h.update(add=tuple(torch.from_numpy(x).to(dev) for x in add))
        cur = M.updated_graph(*cur, add=add)
        say("m=%d added: stats %s" % (m, h.update_stats()))
        check_against(h, cur, 10, True, "add %d" % m)
        pick = rng.integers(0, cur[2].shape[0], m)
        dele = (cur[2][pick], cur[3][pick], cur[4][pick])
        h.update(delete=dele)
        cur = M.updated_graph(*cur, delete=dele)
        say("m=%d deleted: stats %s" % (m, h.update_stats()))
        check_against(h, cur, 10, True, "delete %d" % m)


@pytest.mark.parametrize("radix_tile", [2048, 4096])
def test_update_radix_tiles(radix_tile):
    """The maintenance sorts (edges by target, merged rows) on the other
    compiled radix tile sizes."""
    torch, kb = need_gpu()
    g = synth.powerlaw_graph(50_000, 400_000, seed=9, num_node_labels=20, num_edge_labels=6)
    rng = np.random.default_rng(radix_tile)
    cur = cur_of(g)
    dev = torch.device("cuda:0")
    with kb.Graph(g.num_nodes, *to_dev(torch, g), history=True, radix_tile=radix_tile) as h:
        h.refine(10)
        m = 5000
        add = tuple(x.astype(np.int32) for x in (rng.integers(0, g.num_nodes, m), rng.integers(0, 6, m),
                                                 rng.integers(0, g.num_nodes, m)))
        h.update(add=tuple(torch.from_numpy(x).to(dev) for x in add))
        cur = M.updated_graph(*cur, add=add)
        check_against(h, cur, 10, True, "add %d, tile %d" % (m, radix_tile))
        pick = rng.integers(0, cur[2].shape[0], m)
        dele = (cur[2][pick], cur[3][pick], cur[4][pick])
        h.update(delete=dele)
        cur = M.updated_graph(*cur, delete=dele)
        check_against(h, cur, 10, True, "delete %d, tile %d" % (m, radix_tile))


@pytest.mark.parametrize("mode", MODES)
def test_update_new_label_values(mode):
    """New node label values below, between and above the old ones, and new
    edge label values: level 0 and the edge encoding are re-ranked."""
    torch, kb = need_gpu()
    rng = np.random.default_rng(4)
    g = synth.random_small_graph(rng, 30, 90, 3, 3)
    lab = (np.asarray(g.node_label) * 10 + 5).astype(np.int32)  # 5, 15, 25
    el = (np.asarray(g.elab) * 10 + 5).astype(np.int32)
    cur = (g.num_nodes, lab, np.asarray(g.src, np.int32), el, np.asarray(g.dst, np.int32))
    with kb.Graph(cur[0], *cur[1:], history=True, update_mode=mode) as h:
        h.refine(8)
        for upd in (dict(new_labels=np.array([0, 10, 40, 15], np.int32)),
                    dict(add=(np.array([0, 31, 2], np.int32), np.array([1, 26, 99], np.int32),
                              np.array([33, 1, 2], np.int32))),
                    dict(new_labels=np.array([2**31 - 1], np.int32),
                         add=(np.array([34], np.int32), np.array([2**31 - 1], np.int32), np.array([0], np.int32)))):
            h.update(**upd)
            cur = M.updated_graph(*cur, **upd)
            check_against(h, cur, 8, True, str(sorted(upd)))


def test_update_invalid_leaves_state():
    torch, kb = need_gpu()
    g = graph_of(load("figure1.json"))
    cur = cur_of(g)
    with kb.Graph(g.num_nodes, g.node_label, g.src, g.elab, g.dst, history=True) as h:
        h.refine(10)
        for bad in (dict(add=([0], [0], [6])), dict(add=([0], [-1], [1])), dict(new_labels=[-3]),
                    dict(delete=([7], [0], [0]))):
            with pytest.raises(kb.KbisimError) as e:
                h.update(**bad)
            assert e.value.status == -1
        check_against(h, cur, 10, True, "after rejected updates")
        h.update(delete=([4], [3], [0]))  # a triple that is not in the graph changes nothing
        check_against(h, cur, 10, True, "absent triple")


@pytest.mark.parametrize("mode", MODES)
def test_update_moves_fixed_point(mode):
    """A path of 3 edges reaches its fixed point at round 4; extending it by
    3 more edges needs rounds 5..7 (up to the k asked before)."""
    torch, kb = need_gpu()
    g = synth.path_graph(3)
    cur = cur_of(g)
    with kb.Graph(g.num_nodes, g.node_label, g.src, g.elab, g.dst, history=True, update_mode=mode) as h:
        h.refine(20)
        assert h.rounds_done == 4
        upd = dict(new_labels=[0, 0, 0], add=([3, 4, 5], [0, 0, 0], [4, 5, 6]))
        h.update(**upd)
        cur = M.updated_graph(*cur, **upd)
        check_against(h, cur, 20, True, "longer path")
        assert h.rounds_done == 7


def test_dbest_no_change():
    """Dbest (Section 5.3): a full tree with one node and one edge label; an
    edge from a parent of leaves to another leaf changes no signature, so no
    id changes, and the update stays level by level (no full round)."""
    torch, kb = need_gpu()
    g = synth.tree_graph(3, 5)
    cur = cur_of(g)
    n = g.num_nodes
    leaves0 = n - 3 ** 5
    parent_of_leaves = (leaves0 - 1) // 3  # the parent of the first leaf
    other_leaf = n - 1  # a leaf under another parent
    with kb.Graph(n, *cur[1:], history=True) as h:
        h.refine(10)
        before = [h.result_round(j)[0] for j in range(h.rounds_done + 1)]
        upd = dict(add=([parent_of_leaves], [0], [other_leaf]))
        h.update(**upd)
        cur = M.updated_graph(*cur, **upd)
        check_against(h, cur, 10, True, "dbest")
        after = [h.result_round(j)[0] for j in range(h.rounds_done + 1)]
        assert all(np.array_equal(a, b) for a, b in zip(before, after))
        levels, full_from, rechecked, recomputed, changed = h.update_stats()
        say("dbest: levels %d full_from %d rechecked %d recomputed %d changed %d" %
            (levels, full_from, rechecked, recomputed, changed))
        assert full_from == 0 and levels == h.rounds_done


def test_dworst_all_change():
    """Dworst (Section 5.3): a complete graph with all edges x plus one
    y-edge to a new isolated node: every node's signature changes; the
    update's result is still exact (B = [1, 3, 3])."""
    torch, kb = need_gpu()
    g = synth.complete_graph(40)
    cur = cur_of(g)
    with kb.Graph(g.num_nodes, *cur[1:], history=True, update_mode=1) as h:
        h.refine(10)
        upd = dict(new_labels=[0], add=([0], [1], [40]))
        h.update(**upd)
        cur = M.updated_graph(*cur, **upd)
        check_against(h, cur, 10, True, "dworst")
        _, _, counts = h.result()
        assert counts == [1, 3, 3]
        say("dworst: stats %s" % (h.update_stats(),))


@pytest.mark.parametrize("mode", MODES)
def test_delete_nodes(mode):
    """Node deletions (with self-loops, a node added and deleted in one
    update, all nodes at once) and a further refine after an update."""
    torch, kb = need_gpu()
    g = graph_of(load("figure1.json"))
    cur = cur_of(g)
    with kb.Graph(g.num_nodes, *cur[1:], history=True, update_mode=mode) as h:
        h.refine(3)
        for upd in (dict(delete_nodes=[1]),  # paper node 2, with its self-loop
                    dict(new_labels=[0, 1], delete_nodes=[5, 0], add=([4, 2], [0, 1], [0, 4])),
                    dict(delete_nodes=[2, 2])):
            h.update(**upd)
            cur = M.updated_graph(*cur, **upd)
            check_against(h, cur, 3, True, str(upd))
        h.refine(10)  # continue after the updates
        check_against(h, cur, 10, True, "refined further")
        h.update(delete_nodes=np.arange(cur[0], dtype=np.int32))
        cur = M.updated_graph(*cur, delete_nodes=np.arange(cur[0]))
        check_against(h, cur, 10, True, "empty")
        h.update(new_labels=[3, 3], add=([0], [2], [1]))
        cur = M.updated_graph(*cur, new_labels=[3, 3], add=([0], [2], [1]))
        check_against(h, cur, 10, True, "after empty")
