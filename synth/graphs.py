"""Seeded graph generators (numpy PCG64).

Every generator returns a ``Graph`` whose arrays are int32: ``node_label[N]``
and the edge table ``src, elab, dst`` of length E in a random order (the
edge table is unsorted, like the paper's input tables before iteration 1).

Workload recipes (the paper's datasets are not available; these stand in):

* uniform  -- src and dst i.i.d. uniform over the nodes (out-degree is
  Binomial(E, 1/N), close to Poisson(E/N)), node and edge labels uniform.
* powerlaw -- Chung-Lu style: node weight w ~ Zipf(a), expected out-degree
  min(c*w, cap') with c chosen so the expected degrees sum to E; the
  out-degrees are one multinomial draw of E over those weights (so the
  total is exactly E, the mean exactly E/N, and degree-0 nodes occur).
  Targets follow static preferential attachment: dst is drawn with
  probability proportional to (out-degree + 1). Node labels follow a
  Zipf-like law p(r) ~ r^-s_n over L_n labels, edge labels p(r) ~ r^-s_e
  over L_e labels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    num_nodes: int
    node_label: np.ndarray
    src: np.ndarray
    elab: np.ndarray
    dst: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_edges(self) -> int:
        return int(self.src.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.bincount(self.src, minlength=self.num_nodes)


def _rng(seed):
    if isinstance(seed, (tuple, list)):
        return np.random.Generator(np.random.PCG64(list(seed)))
    return np.random.Generator(np.random.PCG64(seed))


def _zipf_labels(rng, count, num_labels, s):
    p = np.arange(1, num_labels + 1, dtype=np.float64) ** (-s)
    p /= p.sum()
    return rng.choice(num_labels, size=count, p=p).astype(np.int32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def uniform_graph(n, e, num_node_labels=4, num_edge_labels=8, seed=1, name="uniform"):
    rng = _rng(seed)
    node_label = rng.integers(0, num_node_labels, size=n, dtype=np.int32)
    src = rng.integers(0, n, size=e, dtype=np.int32) if n > 0 else np.zeros(0, np.int32)
    dst = rng.integers(0, n, size=e, dtype=np.int32) if n > 0 else np.zeros(0, np.int32)
    elab = rng.integers(0, num_edge_labels, size=e, dtype=np.int32)
    return Graph(n, node_label, src, elab, dst, name=name,
                 meta=dict(kind="uniform", seed=seed, node_labels=num_node_labels,
                           edge_labels=num_edge_labels))


def _scale_to_total(w, total, cap):
    """c such that sum(min(c*w, cap)) == total (bisection on c); needs
    cap * len(w) >= total."""
    assert cap * w.shape[0] >= total
    lo, hi = 0.0, float(total) / float(w.sum()) * 4.0 + 1.0
    while np.minimum(hi * w, cap).sum() < total:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if np.minimum(mid * w, cap).sum() < total:
            lo = mid
        else:
            hi = mid
    return hi


def powerlaw_graph(n, e, seed=1, zipf_a=2.1, deg_cap=100_000, num_node_labels=100,
                   node_label_exp=1.2, num_edge_labels=32, edge_label_exp=1.1, name="powerlaw",
                   shuffle=True, progress=None):
    """Power-law out-degree graph; see the module docstring for the recipe.
    progress(msg), when given, is called between the generation steps (large
    graphs take minutes)."""
    say = progress or (lambda msg: None)
    rng = _rng(seed)
    w = rng.zipf(zipf_a, size=n).astype(np.float64)
    # expected degrees are held six standard deviations under the cap, so the
    # sampled maximum stays at or below deg_cap (asserted below)
    cap = float(min(deg_cap, max(e, 1)))
    cap_eff = max(cap - 6.0 * np.sqrt(cap), 1.0)
    # the capped expected degrees must be able to add up to e
    cap_eff = max(cap_eff, float(np.ceil(e / max(n, 1))))
    if n == 0 or cap_eff > deg_cap:
        raise ValueError("cannot place %d edges on %d nodes under out-degree cap %d" % (e, n, deg_cap))
    c = _scale_to_total(w, e, cap_eff)
    lam = np.minimum(c * w, cap_eff)
    deg = rng.multinomial(e, lam / lam.sum()).astype(np.int64)
    say("out-degrees drawn")
    assert int(deg.sum()) == e
    assert int(deg.max(initial=0)) <= deg_cap, "out-degree above the cap"
    indeg = rng.multinomial(e, (deg + 1.0) / float((deg + 1).sum())).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int32), deg)
    dst = np.repeat(np.arange(n, dtype=np.int32), indeg)
    dst = rng.permutation(dst)  # i.i.d. draws == multinomial counts in random order
    say("targets drawn")
    elab = _zipf_labels(rng, e, num_edge_labels, edge_label_exp)
    node_label = _zipf_labels(rng, n, num_node_labels, node_label_exp)
    say("labels drawn")
    if shuffle and e > 0:
        perm = rng.permutation(e)
        say("edge order drawn")
        src, dst, elab = src[perm], dst[perm], elab[perm]
        del perm
    return Graph(n, _i32(node_label), _i32(src), _i32(elab), _i32(dst), name=name,
                 meta=dict(kind="powerlaw", seed=seed, zipf_a=zipf_a, deg_cap=deg_cap,
                           node_labels=num_node_labels, edge_labels=num_edge_labels))


def degree_graph(degrees, num_nodes=None, num_node_labels=2, num_edge_labels=3, seed=1,
                 name="degrees"):
    """Graph whose out-degrees are given exactly (segment-size edge cases)."""
    rng = _rng(seed)
    deg = np.asarray(degrees, np.int64)
    n = int(num_nodes if num_nodes is not None else deg.shape[0])
    full = np.zeros(n, np.int64)
    full[: deg.shape[0]] = deg
    e = int(full.sum())
    src = np.repeat(np.arange(n, dtype=np.int32), full)
    dst = rng.integers(0, n, size=e, dtype=np.int32)
    elab = rng.integers(0, num_edge_labels, size=e, dtype=np.int32)
    perm = rng.permutation(e)
    node_label = rng.integers(0, num_node_labels, size=n, dtype=np.int32)
    return Graph(n, node_label, _i32(src[perm]), _i32(elab[perm]), _i32(dst[perm]), name=name)


def random_small_graph(rng, n, e, num_node_labels, num_edge_labels, dag=False, self_loops=True):
    """Tiny random graph for brute-force comparisons (duplicates allowed)."""
    node_label = rng.integers(0, num_node_labels, size=n).astype(np.int32)
    if n == 0:
        z = np.zeros(0, np.int32)
        return Graph(0, node_label, z, z, z, name="tiny")
    src = rng.integers(0, n, size=e)
    dst = rng.integers(0, n, size=e)
    if dag:
        lo, hi = np.minimum(src, dst), np.maximum(src, dst)
        keep = lo != hi
        src, dst = lo[keep], hi[keep]
    elif not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    elab = rng.integers(0, num_edge_labels, size=src.shape[0])
    return Graph(n, node_label, _i32(src), _i32(elab), _i32(dst), name="tiny")


# --- small shapes with closed forms --------------------------------------------

def worked_example():
    """The paper's example graph (Figure 1): nodes 1..6 mapped to 0..5, node
    labels M=0, P=1, edge labels w=0, l=1."""
    node_label = np.array([0, 0, 1, 1, 1, 1], np.int32)
    edges = [(0, 0, 1), (0, 1, 3), (1, 0, 1), (1, 1, 5), (2, 1, 0), (3, 1, 2), (4, 1, 1)]
    s, l, d = (np.array(c, np.int32) for c in zip(*edges))
    return Graph(6, node_label, s, l, d, name="figure1")


def path_graph(length, label=0):
    n = length + 1
    src = np.arange(length, dtype=np.int32)
    return Graph(n, np.full(n, label, np.int32), src, np.zeros(length, np.int32), src + 1,
                 name="path%d" % length)


def cycle_graph(n):
    src = np.arange(n, dtype=np.int32)
    return Graph(n, np.zeros(n, np.int32), src, np.zeros(n, np.int32), (src + 1) % n,
                 name="cycle%d" % n)


def tree_graph(arity, height):
    """Full arity-ary tree, edges parent -> child, one node and one edge label."""
    n = sum(arity ** d for d in range(height + 1))
    parents = np.arange(n, dtype=np.int64)[1:]
    src = ((parents - 1) // arity).astype(np.int32)
    return Graph(n, np.zeros(n, np.int32), src, np.zeros(n - 1, np.int32),
                 parents.astype(np.int32), name="tree%d_%d" % (arity, height))


def complete_graph(n, extra_isolated=0):
    """K_n without self-loops, all edges label 0, plus isolated nodes."""
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s != d
    src, dst = s[keep].astype(np.int32), d[keep].astype(np.int32)
    tot = n + extra_isolated
    return Graph(tot, np.zeros(tot, np.int32), src, np.zeros(src.shape[0], np.int32), dst,
                 name="K%d" % n)


# --- batched and served workloads --------------------------------------------

def batch_graphs(num_graphs, seed=1, median_nodes=20_000, sigma=1.0, min_nodes=1_000,
                 max_nodes=1_000_000, avg_degree=8, num_labels=16, progress=None):
    """Independent graphs of log-normal size; graph g uses seed (seed, g).
    `progress(msg)`, if given, is called every 256 graphs."""
    rng = _rng(seed)
    sizes = np.clip(np.round(median_nodes * np.exp(sigma * rng.standard_normal(num_graphs))),
                    min_nodes, max_nodes).astype(np.int64)
    out = []
    for g in range(num_graphs):
        n = int(sizes[g])
        gr = powerlaw_graph(n, avg_degree * n, seed=(seed, g), deg_cap=max(n, 8 * avg_degree),
                            num_node_labels=num_labels, node_label_exp=0.0,
                            num_edge_labels=num_labels, edge_label_exp=0.0, name="batch%d" % g)
        out.append(gr)
        if progress is not None and (g + 1) % 256 == 0:
            progress("batch graphs: %d of %d" % (g + 1, num_graphs))
    return out


def serving_stream(num_requests, seed=1, rate=200.0, min_nodes=10_000, max_nodes=50_000_000,
                   avg_degree=10, k_lo=2, k_hi=10):
    """Poisson arrivals: list of (arrival_s, num_nodes, k, graph_seed)."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=num_requests)
    t = np.cumsum(gaps)
    lo, hi = np.log(min_nodes), np.log(max_nodes)
    nodes = np.round(np.exp(rng.uniform(lo, hi, size=num_requests))).astype(np.int64)
    ks = rng.integers(k_lo, k_hi + 1, size=num_requests)
    return [dict(arrival=float(t[i]), num_nodes=int(nodes[i]), num_edges=int(avg_degree * nodes[i]),
                 k=int(ks[i]), seed=(seed, i)) for i in range(num_requests)]


# --- named workloads -------------------------------------------------------------

CONFIGS = {
    # 10k nodes, 50k edges, uniform, 4 node labels, 8 edge labels, k=5
    "uniform-10k-50k": dict(maker="uniform", n=10_000, e=50_000, k=5),
    # 10M nodes, 100M edges, power law, fixed point with cap k=10
    "powerlaw-10M-100M": dict(maker="powerlaw", n=10_000_000, e=100_000_000, k=10),
    # 100M nodes, 1B edges, power law, k=10
    "powerlaw-100M-1B": dict(maker="powerlaw", n=100_000_000, e=1_000_000_000, k=10),
}


def make_config(name, seed=1, progress=None):
    cfg = CONFIGS[name]
    if cfg["maker"] == "uniform":
        g = uniform_graph(cfg["n"], cfg["e"], seed=seed, name=name)
    else:
        g = powerlaw_graph(cfg["n"], cfg["e"], seed=seed, name=name, progress=progress)
    return g, cfg["k"]
