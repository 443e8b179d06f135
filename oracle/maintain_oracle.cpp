// CPU oracle for the maintenance of a k-bisimulation partition (Section 4 of
// the paper): Add_Nodes (Algorithm 2), Add_Edges (Algorithm 3) and deletions,
// in the paper's own numbering.
//
// TEST INFRASTRUCTURE ONLY. Like kbisim_oracle.cpp this is the slow, plain
// reference the GPU library is checked against; nothing in the product path
// may include, link or call it, and it shares no code with the GPU library.
//
// State (Section 4, Table 3): the node table with the history pId_0..pId_k of
// every node, the edge table in two copies (by source and by target), and
// the signature store S, kept between updates. Readings taken:
//  * numbering as in the worked example (Table 1): one counter for all ids,
//    starting at 1; S keeps one dictionary per iteration j (the same
//    signature string receives different ids in iterations 1 and 2 there);
//  * the signature head is pId_0(u) (Definition 3 literally), so a node whose
//    pId_{j-1} changed is re-checked at level j only through its targets;
//  * Add_Nodes hands out new level-0 ids to new labels in ascending label
//    order, then inserts (pId_0(u), {}) into S_1..S_k for every new node u in
//    id order (an isolated node's signature is its head alone);
//  * Add_Edges follows Algorithm 3: (j, s) for every new edge's source and
//    every level j enqueued, then level by level the distinct queued nodes
//    have their signature rebuilt from the current table, looked up in S_j,
//    and a changed id is recorded and its sources (edge copy by target)
//    queued at level j + 1;
//  * deletions (Section 4, "Deletions"): removing an edge removes every copy
//    of that (src, label, dst) triple and then propagates exactly as an
//    insertion; removing a node removes its incoming and outgoing edges that
//    way, then its row; the remaining nodes keep their order (ids are
//    renumbered densely, 0-based).
// The partition (not the numbering) this state holds is pinned against a
// from-scratch Build_Bisim of the updated graph in the tests.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace {

using Sig = std::vector<int32_t>;
using Pair = std::pair<int32_t, int32_t>;  // (label, other endpoint)

struct MState {
  int32_t k = 0;
  std::vector<int32_t> label;                   // nLabel per node
  std::vector<std::vector<Pair>> out;           // E_st: (label, target) per source
  std::vector<std::vector<Pair>> in;            // E_ts: (label, source) per target
  std::vector<std::vector<int32_t>> pid;        // pid[j][u], j = 0..k
  std::map<int32_t, int32_t> label_id;          // level 0: label value -> pId_0
  std::vector<std::map<Sig, int32_t>> S;        // S[j] for j = 1..k (S[0] unused)
  int64_t counter = 1;                          // next id
  int64_t checked = 0, changed = 0;             // work of the last update
};

Sig signature(const MState& st, int32_t u, int32_t j) {
  std::vector<Pair> pairs;
  pairs.reserve(st.out[u].size());
  for (const Pair& e : st.out[u]) pairs.emplace_back(e.first, st.pid[j - 1][e.second]);
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  Sig s;
  s.push_back(st.pid[0][u]);
  for (const Pair& p : pairs) {
    s.push_back(p.first);
    s.push_back(p.second);
  }
  return s;
}

int32_t s_insert(MState& st, int32_t j, const Sig& s) {
  auto it = st.S[j].find(s);
  if (it == st.S[j].end()) it = st.S[j].emplace(s, int32_t(st.counter++)).first;
  return it->second;
}

// The propagation loop of Algorithm 3 from a set of (level, node) pairs.
void propagate(MState& st, std::set<std::pair<int32_t, int32_t>> pq) {
  while (!pq.empty()) {
    const int32_t j = pq.begin()->first;
    std::vector<int32_t> M;  // distinct node ids of level j, ascending
    while (!pq.empty() && pq.begin()->first == j) {
      M.push_back(pq.begin()->second);
      pq.erase(pq.begin());
    }
    for (int32_t u : M) {
      const int32_t id = s_insert(st, j, signature(st, u, j));
      ++st.checked;
      if (id != st.pid[j][u]) {
        st.pid[j][u] = id;
        ++st.changed;
        if (j < st.k)
          for (const Pair& e : st.in[u]) pq.emplace(j + 1, e.second);
      }
    }
  }
}

void remove_triple(MState& st, int32_t s, int32_t l, int32_t t) {
  auto& o = st.out[s];
  o.erase(std::remove(o.begin(), o.end(), Pair(l, t)), o.end());
  auto& i = st.in[t];
  i.erase(std::remove(i.begin(), i.end(), Pair(l, s)), i.end());
}

bool valid_edges(const MState& st, int64_t m, const int32_t* src, const int32_t* lab, const int32_t* dst) {
  const int64_t n = int64_t(st.label.size());
  if (m < 0 || (m > 0 && (!src || !lab || !dst))) return false;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n || lab[e] < 0) return false;
  return true;
}

}  // namespace

extern "C" {

// Build_Bisim (Algorithm 1) with all k iterations, keeping the history and S.
void* oracle_state_create(int64_t n, const int32_t* node_label, int64_t m, const int32_t* src,
                          const int32_t* lab, const int32_t* dst, int32_t k) {
  if (n < 0 || k < 0 || (n > 0 && !node_label)) return nullptr;
  for (int64_t v = 0; v < n; ++v)
    if (node_label[v] < 0) return nullptr;
  auto* st = new MState;
  st->k = k;
  st->label.assign(node_label, node_label + n);
  st->out.resize(size_t(n));
  st->in.resize(size_t(n));
  if (!valid_edges(*st, m, src, lab, dst)) {
    delete st;
    return nullptr;
  }
  for (int64_t e = 0; e < m; ++e) {
    st->out[src[e]].emplace_back(lab[e], dst[e]);
    st->in[dst[e]].emplace_back(lab[e], src[e]);
  }
  // iteration 0: one id per distinct label, in ascending label order
  std::set<int32_t> labels(st->label.begin(), st->label.end());
  for (int32_t v : labels) st->label_id[v] = int32_t(st->counter++);
  st->pid.assign(size_t(k) + 1, std::vector<int32_t>(size_t(n)));
  for (int64_t v = 0; v < n; ++v) st->pid[0][v] = st->label_id[st->label[v]];
  st->S.resize(size_t(k) + 1);
  for (int32_t j = 1; j <= k; ++j)
    for (int64_t v = 0; v < n; ++v) st->pid[j][v] = s_insert(*st, j, signature(*st, int32_t(v), j));
  return st;
}

void oracle_state_destroy(void* h) { delete static_cast<MState*>(h); }

int64_t oracle_state_num_nodes(void* h) { return int64_t(static_cast<MState*>(h)->label.size()); }

// history[(k+1) * N]: pId_0..pId_k row by row.
void oracle_state_history(void* h, int32_t* history) {
  const MState& st = *static_cast<MState*>(h);
  const size_t n = st.label.size();
  for (int32_t j = 0; j <= st.k; ++j)
    if (n) std::memcpy(history + size_t(j) * n, st.pid[j].data(), n * sizeof(int32_t));
}

// Signatures checked and ids changed by the last update.
void oracle_state_work(void* h, int64_t* checked, int64_t* changed) {
  const MState& st = *static_cast<MState*>(h);
  *checked = st.checked;
  *changed = st.changed;
}

// Algorithm 2: isolated new nodes with ids N .. N + n_new - 1.
int32_t oracle_state_add_nodes(void* h, int64_t n_new, const int32_t* labels) {
  MState& st = *static_cast<MState*>(h);
  if (n_new < 0 || (n_new > 0 && !labels)) return -1;
  for (int64_t i = 0; i < n_new; ++i)
    if (labels[i] < 0) return -1;
  st.checked = st.changed = 0;
  std::set<int32_t> fresh;
  for (int64_t i = 0; i < n_new; ++i)
    if (!st.label_id.count(labels[i])) fresh.insert(labels[i]);
  for (int32_t v : fresh) st.label_id[v] = int32_t(st.counter++);
  const size_t n0 = st.label.size();
  for (int64_t i = 0; i < n_new; ++i) {
    st.label.push_back(labels[i]);
    st.out.emplace_back();
    st.in.emplace_back();
    st.pid[0].push_back(st.label_id[labels[i]]);
  }
  for (size_t u = n0; u < st.label.size(); ++u)
    for (int32_t j = 1; j <= st.k; ++j) st.pid[j].push_back(s_insert(st, j, Sig{st.pid[0][u]}));
  return 0;
}

// Algorithm 3. Returns 0, or -1 for an invalid edge (nothing changed then).
int32_t oracle_state_add_edges(void* h, int64_t m, const int32_t* src, const int32_t* lab, const int32_t* dst) {
  MState& st = *static_cast<MState*>(h);
  if (!valid_edges(st, m, src, lab, dst)) return -1;
  st.checked = st.changed = 0;
  std::set<std::pair<int32_t, int32_t>> pq;
  for (int64_t e = 0; e < m; ++e)
    for (int32_t j = 1; j <= st.k; ++j) pq.emplace(j, src[e]);
  for (int64_t e = 0; e < m; ++e) {
    st.out[src[e]].emplace_back(lab[e], dst[e]);
    st.in[dst[e]].emplace_back(lab[e], src[e]);
  }
  propagate(st, std::move(pq));
  return 0;
}

// Deletions of edges: every copy of each triple goes, then propagation as
// for an insertion. Triples not in the graph are ignored.
int32_t oracle_state_delete_edges(void* h, int64_t m, const int32_t* src, const int32_t* lab, const int32_t* dst) {
  MState& st = *static_cast<MState*>(h);
  if (!valid_edges(st, m, src, lab, dst)) return -1;
  st.checked = st.changed = 0;
  std::set<std::pair<int32_t, int32_t>> pq;
  for (int64_t e = 0; e < m; ++e) {
    remove_triple(st, src[e], lab[e], dst[e]);
    for (int32_t j = 1; j <= st.k; ++j) pq.emplace(j, src[e]);
  }
  propagate(st, std::move(pq));
  return 0;
}

// Deletion of nodes: their incoming and outgoing edges are deleted as above,
// then their rows; the other nodes keep their order (dense 0-based ids).
int32_t oracle_state_delete_nodes(void* h, int64_t cnt, const int32_t* nodes) {
  MState& st = *static_cast<MState*>(h);
  const int64_t n = int64_t(st.label.size());
  if (cnt < 0 || (cnt > 0 && !nodes)) return -1;
  std::vector<uint8_t> gone(size_t(n), 0);
  for (int64_t i = 0; i < cnt; ++i) {
    if (nodes[i] < 0 || nodes[i] >= n) return -1;
    gone[nodes[i]] = 1;
  }
  std::vector<int32_t> s, l, d;
  for (int32_t u = 0; u < n; ++u) {
    if (!gone[u]) continue;
    for (const Pair& e : st.out[u]) {
      s.push_back(u);
      l.push_back(e.first);
      d.push_back(e.second);
    }
    for (const Pair& e : st.in[u]) {
      s.push_back(e.second);
      l.push_back(e.first);
      d.push_back(u);
    }
  }
  oracle_state_delete_edges(h, int64_t(s.size()), s.data(), l.data(), d.data());
  std::vector<int32_t> newid(size_t(n), -1);
  int32_t next = 0;
  for (int32_t u = 0; u < n; ++u)
    if (!gone[u]) newid[u] = next++;
  auto keep = [&](auto& vec) {
    size_t w = 0;
    for (size_t u = 0; u < size_t(n); ++u) {
      if (gone[u]) continue;
      if (w != u) vec[w] = std::move(vec[u]);  // a vector moved onto itself would be emptied
      ++w;
    }
    vec.resize(w);
  };
  keep(st.label);
  keep(st.out);
  keep(st.in);
  for (auto& row : st.pid) keep(row);
  for (auto& o : st.out)
    for (Pair& e : o) e.second = newid[e.second];
  for (auto& i : st.in)
    for (Pair& e : i) e.second = newid[e.second];
  return 0;
}

}  // extern "C"
