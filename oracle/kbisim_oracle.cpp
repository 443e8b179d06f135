// CPU oracle for k-bisimulation partition refinement.
//
// TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
// GPU library is checked against. Nothing in the product path may include,
// link or call it; it shares no code, header or table with the GPU library.
//
// It follows the construction algorithm of the paper (Build_Bisim, Algorithm 1,
// Section 3) with the signature of Definition 3 and the signature store S of
// Section 2.2 realised as an ordered dictionary (Section 3.2, "Data structures
// for S": a dictionary is one of the admissible set-equality structures).
//
// Readings taken where the paper leaves a choice:
//  * node labels and edge labels are int32 >= 0 and ordered numerically;
//  * the input is any multiset of (src, label, dst) triples; set semantics of
//    the signature (Definition 3) make duplicates irrelevant;
//  * pId_0 is the ascending rank of the node label among the labels present
//    (Section 3.1, "k = 0": sort by label, new id per new label);
//  * canonical ids of round i are the 0-based rank of the node's signature
//    among the distinct signatures of round i, ordered lexicographically as
//    flattened int sequences [head, l1, p1, l2, p2, ...] (a proper prefix is
//    smaller), with the pairs of the set kept in ascending (label, pid) order
//    (Section 3.1: the signature is built as a string with the set elements
//    in sorted order);
//  * the signature head is pId_{i-1}(u) (Kaushik's definition, Appendix,
//    "Alternative definitions", shown there to give the same partition) unless
//    ORACLE_HEAD_PID0 asks for Definition 3's literal pId_0(u) head;
//  * early stop: after round i with B_i == B_{i-1} the partition is the fixed
//    point (Section 3.2 "Early stopping condition"; Appendix propositions on
//    the stop condition), so the loop ends with rounds_done = i.
//
// ORACLE_PAPER_NUMBERING reproduces the numbering of the paper's worked example
// (Table 1): one global counter starting at 1, a fresh S per iteration, ids
// handed out in order of first occurrence while scanning nodes by id.
//
// parity of the canonical id values beyond the worked example is pinned only
// through the invariants (refinement, density, lexicographic order against an
// independent comparison, relabelling invariance); the partitions themselves
// are pinned against brute-force bisimilarity.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

enum : int32_t {
  ORACLE_HEAD_PID0 = 1,        // head = pId_0(u) (Definition 3 literally)
  ORACLE_PAPER_NUMBERING = 2,  // Table 1 numbering (global counter, first occurrence)
  ORACLE_NO_EARLY_STOP = 4,    // run all k rounds
};

enum : int32_t {
  ORACLE_OK = 0,
  ORACLE_EINVAL = -1,
};

using Sig = std::vector<int32_t>;

int32_t validate(int64_t n, int64_t m, const int32_t* node_label, const int32_t* src,
                 const int32_t* elab, const int32_t* dst, int32_t k) {
  if (n < 0 || m < 0 || k < 0) return ORACLE_EINVAL;
  if (n > INT32_MAX) return ORACLE_EINVAL;
  if (n > 0 && node_label == nullptr) return ORACLE_EINVAL;
  if (m > 0 && (src == nullptr || elab == nullptr || dst == nullptr)) return ORACLE_EINVAL;
  for (int64_t v = 0; v < n; ++v)
    if (node_label[v] < 0) return ORACLE_EINVAL;
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n || elab[e] < 0)
      return ORACLE_EINVAL;
  }
  return ORACLE_OK;
}

// Signature of Definition 3 as the paper's string: head, then the sorted,
// de-duplicated pairs (edge label, id of the target in the previous round).
Sig build_signature(int32_t head, const std::vector<std::pair<int32_t, int32_t>>& out_edges,
                    const std::vector<int32_t>& pid_prev) {
  std::vector<std::pair<int32_t, int32_t>> pairs;
  pairs.reserve(out_edges.size());
  for (const auto& le : out_edges) pairs.emplace_back(le.first, pid_prev[le.second]);
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  Sig s;
  s.reserve(1 + 2 * pairs.size());
  s.push_back(head);
  for (const auto& p : pairs) {
    s.push_back(p.first);
    s.push_back(p.second);
  }
  return s;
}

}  // namespace

extern "C" {

// Runs Build_Bisim on the graph (N nodes, E labelled edges) for up to k rounds.
//   pid_out      [N]      ids of the last round computed (pId_k; equal to pId_k
//                         also after an early stop, by the fixed-point property)
//   counts       [k+1]    B_0..B_{rounds_done}; unused tail entries set to -1
//   max_sig_ints [k+1]    longest signature of each round as a count of ints
//                         (1 + 2 * pairs); round 0 reports 1; tail set to -1
//   history      [(k+1)*N] or NULL: pId_0..pId_rounds_done row by row; rows
//                         after an early stop repeat the fixed point
//   rounds_done  number of refinement rounds executed
// Returns 0, or -1 for invalid input (nothing written then).
int32_t oracle_refine(int64_t n, int64_t m, const int32_t* node_label, const int32_t* src,
                      const int32_t* elab, const int32_t* dst, int32_t k, int32_t flags,
                      int32_t* pid_out, int64_t* counts, int64_t* max_sig_ints,
                      int32_t* history, int32_t* rounds_done) {
  int32_t st = validate(n, m, node_label, src, elab, dst, k);
  if (st != ORACLE_OK) return st;
  const bool head_pid0 = (flags & ORACLE_HEAD_PID0) != 0;
  const bool paper_numbering = (flags & ORACLE_PAPER_NUMBERING) != 0;
  const bool early_stop = (flags & ORACLE_NO_EARLY_STOP) == 0;

  for (int32_t i = 0; i <= k; ++i) {
    if (counts) counts[i] = -1;
    if (max_sig_ints) max_sig_ints[i] = -1;
  }

  // Iteration 0: sort the node labels, hand out one id per distinct label.
  std::vector<int32_t> labels(node_label, node_label + n);
  std::sort(labels.begin(), labels.end());
  labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
  std::vector<int32_t> pid(n), pid0(n);
  int64_t next_global = 1;  // paper numbering: one counter for all iterations
  if (paper_numbering) {
    // first occurrence in node-id order among labels sorted ascending is the
    // same as the ascending rank; the counter starts at 1.
    for (int64_t v = 0; v < n; ++v)
      pid[v] = 1 + int32_t(std::lower_bound(labels.begin(), labels.end(), node_label[v]) -
                           labels.begin());
    next_global = 1 + int64_t(labels.size());
  } else {
    for (int64_t v = 0; v < n; ++v)
      pid[v] = int32_t(std::lower_bound(labels.begin(), labels.end(), node_label[v]) -
                       labels.begin());
  }
  pid0 = pid;
  int64_t blocks_prev = int64_t(labels.size());
  if (counts) counts[0] = blocks_prev;
  if (max_sig_ints) max_sig_ints[0] = 1;
  if (history) std::memcpy(history, pid.data(), sizeof(int32_t) * size_t(n));

  // Out-edges of every node as (label, target); order irrelevant.
  std::vector<std::vector<std::pair<int32_t, int32_t>>> out(n);
  for (int64_t e = 0; e < m; ++e) out[src[e]].emplace_back(elab[e], dst[e]);

  int32_t done = 0;
  std::vector<Sig> sig(n);
  for (int32_t i = 1; i <= k; ++i) {
    int64_t longest = 1;
    for (int64_t v = 0; v < n; ++v) {
      const int32_t head = head_pid0 ? pid0[v] : pid[v];
      sig[v] = build_signature(head, out[v], pid);
      longest = std::max<int64_t>(longest, int64_t(sig[v].size()));
    }
    std::vector<int32_t> next(n);
    int64_t blocks = 0;
    if (paper_numbering) {
      std::map<Sig, int32_t> store;  // fresh S for this iteration
      for (int64_t v = 0; v < n; ++v) {
        auto it = store.find(sig[v]);
        if (it == store.end()) it = store.emplace(sig[v], int32_t(next_global++)).first;
        next[v] = it->second;
      }
      blocks = int64_t(store.size());
    } else {
      std::map<Sig, int32_t> store;
      for (int64_t v = 0; v < n; ++v) store.emplace(sig[v], 0);
      int32_t rank = 0;
      for (auto& kv : store) kv.second = rank++;  // in-order: lexicographic rank
      for (int64_t v = 0; v < n; ++v) next[v] = store.find(sig[v])->second;
      blocks = int64_t(store.size());
    }
    pid.swap(next);
    done = i;
    if (counts) counts[i] = blocks;
    if (max_sig_ints) max_sig_ints[i] = longest;
    if (history) std::memcpy(history + size_t(i) * size_t(n), pid.data(), sizeof(int32_t) * size_t(n));
    const bool fixed = (blocks == blocks_prev);
    blocks_prev = blocks;
    if (fixed && early_stop) break;
  }
  if (history) {
    for (int32_t i = done + 1; i <= k; ++i)
      std::memcpy(history + size_t(i) * size_t(n), pid.data(), sizeof(int32_t) * size_t(n));
  }
  if (pid_out) std::memcpy(pid_out, pid.data(), sizeof(int32_t) * size_t(n));
  if (rounds_done) *rounds_done = done;
  return ORACLE_OK;
}

// Signatures of a sample of nodes, built from a given previous-round id
// array (used to check one GPU round at sizes where the whole oracle run is
// too slow). For each sampled node v the flattened signature
// [pid_prev[v], l1, p1, ...] is written to sig_buf starting at sig_off[j];
// sig_off has num_sample+1 entries. If sig_buf is NULL only the offsets are
// computed (so the caller can size the buffer). Returns 0 or -1.
int32_t oracle_signatures(int64_t n, int64_t m, const int32_t* src, const int32_t* elab,
                          const int32_t* dst, const int32_t* pid_prev, int64_t num_sample,
                          const int32_t* sample, int64_t* sig_off, int32_t* sig_buf) {
  if (n < 0 || m < 0 || num_sample < 0) return ORACLE_EINVAL;
  std::vector<int64_t> slot(n, -1);
  for (int64_t j = 0; j < num_sample; ++j) {
    if (sample[j] < 0 || sample[j] >= n) return ORACLE_EINVAL;
    slot[sample[j]] = j;
  }
  std::vector<std::vector<std::pair<int32_t, int32_t>>> out(num_sample);
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORACLE_EINVAL;
    const int64_t j = slot[src[e]];
    if (j >= 0) out[j].emplace_back(elab[e], dst[e]);
  }
  std::vector<int32_t> prev(pid_prev, pid_prev + n);
  sig_off[0] = 0;
  for (int64_t j = 0; j < num_sample; ++j) {
    // a sampled node may appear twice; its out-edges were collected once
    const int64_t owner = slot[sample[j]];
    const Sig s = build_signature(prev[sample[j]], out[owner], prev);
    sig_off[j + 1] = sig_off[j] + int64_t(s.size());
    if (sig_buf) std::memcpy(sig_buf + sig_off[j], s.data(), sizeof(int32_t) * s.size());
  }
  return ORACLE_OK;
}

// One round of Build_Bisim restricted to a sample of nodes (used to time the
// oracle on a bounded part of a large job): iteration 0's ids from the node
// labels, then for every sampled node its out-edges, its signature from
// pId_0 and its insertion into an ordered dictionary S; rank_out[j] is the
// lexicographic rank of sampled node j's signature among the distinct
// signatures of the sample; *sample_edges the out-edges of the sampled
// nodes. Returns 0 or -1.
int32_t oracle_round_sample(int64_t n, int64_t m, const int32_t* node_label, const int32_t* src,
                            const int32_t* elab, const int32_t* dst, int64_t num_sample, const int32_t* sample,
                            int32_t* rank_out, int64_t* sample_edges) {
  int32_t st = validate(n, m, node_label, src, elab, dst, 0);
  if (st != ORACLE_OK || num_sample < 0) return ORACLE_EINVAL;
  // iteration 0: the rank of every node label among the distinct labels
  std::map<int32_t, int32_t> label_rank;
  for (int64_t v = 0; v < n; ++v) label_rank.emplace(node_label[v], 0);
  int32_t r0 = 0;
  for (auto& kv : label_rank) kv.second = r0++;
  std::vector<int32_t> pid(n);
  for (int64_t v = 0; v < n; ++v) pid[v] = label_rank.find(node_label[v])->second;
  std::vector<int64_t> slot(n, -1);
  for (int64_t j = 0; j < num_sample; ++j) {
    if (sample[j] < 0 || sample[j] >= n) return ORACLE_EINVAL;
    if (slot[sample[j]] < 0) slot[sample[j]] = j;
  }
  std::vector<std::vector<std::pair<int32_t, int32_t>>> out(num_sample);
  int64_t edges = 0;
  for (int64_t e = 0; e < m; ++e) {
    const int64_t j = slot[src[e]];
    if (j >= 0) {
      out[j].emplace_back(elab[e], dst[e]);
      ++edges;
    }
  }
  std::vector<Sig> sig(num_sample);
  for (int64_t j = 0; j < num_sample; ++j) sig[j] = build_signature(pid[sample[j]], out[slot[sample[j]]], pid);
  std::map<Sig, int32_t> store;
  for (int64_t j = 0; j < num_sample; ++j) store.emplace(sig[j], 0);
  int32_t rank = 0;
  for (auto& kv : store) kv.second = rank++;
  for (int64_t j = 0; j < num_sample; ++j) rank_out[j] = store.find(sig[j])->second;
  if (sample_edges) *sample_edges = edges;
  return ORACLE_OK;
}

// Length (as a count of ints, 1 + 2 * pairs) of every node's signature built
// from a given previous-round id array; len_out[N]. Returns 0 or -1.
int32_t oracle_signature_lengths(int64_t n, int64_t m, const int32_t* src, const int32_t* elab,
                                 const int32_t* dst, const int32_t* pid_prev, int64_t* len_out) {
  if (n < 0 || m < 0) return ORACLE_EINVAL;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> out(n);
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORACLE_EINVAL;
    out[size_t(src[e])].push_back({elab[e], dst[e]});
  }
  std::vector<int32_t> prev(pid_prev, pid_prev + n);
  for (int64_t v = 0; v < n; ++v) len_out[v] = int64_t(build_signature(prev[v], out[v], prev).size());
  return ORACLE_OK;
}

}  // extern "C"
