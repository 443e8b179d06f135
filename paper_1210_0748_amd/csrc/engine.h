// Host-side round driver for one graph resident in device memory.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "pool.h"

namespace kb {

// Owning device allocation that only grows; memory comes from and returns
// to the caching pool, tagged with the calling thread's current stream.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), s(o.s) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      s = o.s;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) Pool::instance().put(p, bytes, s);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t b) {
    if (b <= bytes && p) return;
    release();
    s = current_stream();
    p = Pool::instance().get(b ? b : 1, s, &bytes);
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    std::swap(s, o.s);
  }
};

// Pinned host words for small device->host readbacks (a slot of the
// process-wide pinned slab; the slot's owner is the only user).
struct HostWords {
  uint64_t* p = nullptr;
  bool pinned = true;
  HostWords() {
    if (active_arena()) {  // allocation-free jobs read back into this thread's own words
      static thread_local uint64_t words[2 * PinnedSlots::kSlotWords];
      p = words;
      pinned = false;
    } else {
      p = PinnedSlots::instance().acquire();
    }
  }
  ~HostWords() {
    if (p && pinned) PinnedSlots::instance().release(p);
  }
  HostWords(const HostWords&) = delete;
  HostWords& operator=(const HostWords&) = delete;
};

constexpr uint32_t kDefaultMediumCap = 4096;

struct Options {
  bool early_stop = true;
  bool profile = false;
  bool history = false;  // keep pId_0..pId_rounds and the maintenance state (reverse CSR, label values)
  int update_mode = 0;   // rounds of an update: 0 chosen by cost, 1 level by level, 2 in full
  uint32_t medium_cap = kDefaultMediumCap;  // groups above this size use the global passes
  uint32_t radix_tile = 0;  // items per radix-sort tile (2048, 3072, 4096); 0 = the default
  uint64_t edge_window = 0;  // > 0: the edge table stays in host memory, streamed through this many bytes
};

// One change to a graph handle's graph (the maintenance of Section 4): new
// isolated nodes appended, then edge triples deleted (every copy), then
// edge triples added. All arrays are device pointers.
struct UpdateArgs {
  int64_t n_new = 0;
  const int32_t* new_label = nullptr;
  int64_t m_del = 0;
  const int32_t *del_src = nullptr, *del_lab = nullptr, *del_dst = nullptr;
  int64_t n_del = 0;  // nodes deleted (ids after the new nodes), with all their edges
  const int32_t* del_nodes = nullptr;
  int64_t m_add = 0;  // endpoints in the numbering after the node deletions
  const int32_t *add_src = nullptr, *add_lab = nullptr, *add_dst = nullptr;
};

// Work of the last update: per level, nodes whose signature was recomputed
// (members of the classes that had to be re-ordered), nodes re-checked
// (the frontier) and nodes found changed.
struct UpdateStat {
  int32_t levels = 0;     // rounds brought up to date level by level
  int32_t full_from = 0;  // first round recomputed in full instead (0: none)
  uint64_t recomputed = 0, rechecked = 0, changed = 0;
};

constexpr int kProfClasses = 4;  // signature launch, ordering, assignment, whole round

// Work lists produced by classifying open segments by size: lane groups
// (four widths), medium and big groups (one workgroup each) and large groups
// (global passes). All lists share one set of arrays; list c is the range
// [off[c], off[c] + cnt[c]).
constexpr int kNumSegLists = 7;
struct SegLists {
  DevBuf start, size, depth;
  DevBuf ioff;               // item offsets of the large groups (exclusive scan of their sizes)
  uint32_t large_items = 0;  // items in the large groups
  uint32_t cnt[kNumSegLists] = {};
  uint32_t off[kNumSegLists] = {};
  uint32_t total() const {
    uint32_t t = 0;
    for (uint32_t c : cnt) t += c;
    return t;
  }
};

class Engine {
 public:
  Engine(int64_t n, int64_t m, hipStream_t s, const Options& o);
  ~Engine();

  // desc arrays: device pointers (copies already made by the caller if host)
  void build(const int32_t* node_label, const int32_t* src, const int32_t* lab, const int32_t* dst);
  // the same with the edge table in host memory, kept there (pinned) and
  // streamed through a device window of opt.edge_window bytes every round
  void build_streamed(const int32_t* node_label_dev, const int32_t* src, const int32_t* lab, const int32_t* dst);
  void stream_stats(int64_t* partitions, int64_t* bytes_moved, int32_t* direct_rounds) const {
    if (partitions) *partitions = streamed_ ? int64_t(part_node_.size()) - 1 : 0;
    if (bytes_moved) *bytes_moved = int64_t(streamed_bytes_);
    if (direct_rounds) *direct_rounds = int32_t(direct_rounds_);
  }
  // Runs rounds until `k` rounds are done or the fixed point is hit.
  void refine(int32_t k);
  // Dense ids of the current partition (pId of the last round done).
  void result(int32_t* pid_out, bool to_device);

  // One refinement round regardless of the fixed point (callers that track
  // several graphs in one union decide when to stop).
  void step_round() {
    StreamScope scope(st_);
    run_round();
  }
  // Ids of an earlier round j <= rounds_done from the stored history (or
  // the current round); dense, written to pid_out (host or device).
  void result_round(int32_t j, int32_t* pid_out, bool to_device, int64_t* blocks);
  // Applies an update (new nodes, deleted and added edges) and brings every
  // stored round up to date, then continues to the round target when the
  // fixed point moved. Needs the history option.
  void update(const UpdateArgs& u);
  void update_core(const UpdateArgs& u);
  const UpdateStat& update_stat() const { return ustat_; }
  bool history() const { return opt_.history; }
  int32_t round_target() const { return k_target_; }
  // Dense ids on the device (computed when the partition changed since the
  // last call) and the cumulative class counts: cls[p] = number of classes
  // starting at positions <= p of ord.
  const int32_t* dense_pid();
  const uint32_t* class_scan();
  const uint32_t* ord_device() const { return ord_.as<uint32_t>(); }
  hipStream_t stream() const { return st_; }
  int64_t num_edges() const { return m_; }
  int64_t num_nodes() const { return n_; }
  int64_t blocks() const { return B_; }
  int32_t rounds_done() const { return rounds_; }
  const std::vector<int64_t>& counts() const { return counts_; }
  bool fixed() const { return fixed_; }
  std::array<double, kProfClasses> prof_ms{};
  std::array<int64_t, kProfClasses> prof_n{};
  // per signature bucket: active nodes and their edges, summed over rounds
  void work_counts(uint64_t* out8);
  void reset_work();
  // per round (profiling): signature and round milliseconds, active nodes
  // and edges; rounds past kRoundSlots share the last slot's counts
  struct RoundStat {
    double sig_ms = 0, round_ms = 0;
    uint64_t nodes = 0, edges = 0, max_keys = 0;
  };
  static constexpr int kRoundSlots = 64;
  static constexpr int kWorkWords = 16;  // per round: 4 buckets x (nodes, edges), longest key list
  std::vector<RoundStat> round_stats();
  void reset_round_stats();
  int adj_bytes() const { return adj64_ ? 8 : 4; }
  int key_bytes() const { return key64_ ? 8 : 4; }
  uint32_t num_edge_labels() const { return n_elab_; }

 private:
  void build_nodes(const int32_t* node_label, uint32_t max_nlab, const unsigned long long* masks,
                   const uint64_t* mask_host);
  void set_edge_layout();
  void finish_build();
  void degree_stats();
  void hub_layout();
  template <typename AdjT>
  void stream_adj(const int32_t* src, const int32_t* lab, const int32_t* dst, const uint32_t* rank_table,
                  uint32_t rank_size);
  template <typename AdjT, typename KeyT>
  void streamed_signature(const void* sig_args, const void* sig_work);
  template <typename AdjT>
  void build_adj(const int32_t* src, const int32_t* lab, const int32_t* dst, const uint32_t* erank,
                 const uint32_t* rank_table, uint32_t* hist0);
  uint32_t label_ranks(const int32_t* val, uint64_t n, uint32_t maxv, const unsigned long long* mask_dev,
                       const uint64_t* mask_host, DevBuf& rank_table, DevBuf& rank,
                       std::vector<int32_t>* values = nullptr);
  template <typename AdjT, typename KeyT>
  void round_impl(bool first);
  template <typename AdjT, typename KeyT, typename CompT>
  void hub_sort(const void* sig_args, const uint32_t* hl, uint32_t nh, int key_bits);
  template <typename KeyT>
  void order_groups(const void* kv);
  template <typename KeyT>
  void resolve_lists(SegLists& L, const void* kv, hipStream_t s_small, hipStream_t s_big);
  hipStream_t side_stream();
  void large_offsets(SegLists& L, const uint32_t* meta, uint32_t* total, uint64_t items);
  void make_lists(const uint32_t* seg_start, const uint32_t* seg_size, const uint32_t* seg_depth,
                  const uint8_t* seg_done, uint32_t nseg, SegLists& out, const uint32_t* nseg_dev = nullptr);
  void assign_round();
  void assign_ids();  // ids of the active positions after ordering (first part of assign_round)
  // maintenance
  void save_level(int32_t j);
  void load_level(int32_t j);
  void build_reverse();
  template <typename AdjT>
  void update_graph(const UpdateArgs& u, uint32_t n_new_total, std::vector<uint32_t>& src_list_host);
  template <typename AdjT, typename KeyT>
  void update_levels();
  void rebuild_active();
  void remove_nodes(const uint32_t* newid, uint32_t n_keep);
  void grow_nodes(uint64_t n_new);
  void graph_stats();
  // mark: set actr[node] = tag for the active nodes (else already done)
  void prepare_active(uint32_t seg_items, uint32_t m_cap, uint32_t tag, bool mark);
  void run_round();
  uint64_t read_word(const void* dev, int bytes);
  template <typename Tin, typename Tout, bool kIncl>
  void scan_dev(const Tin* in, Tout* out, uint64_t n);
  uint32_t* radix_scratch(uint64_t n);
  uint32_t* compact_scratch(uint64_t words);
  uint32_t medium_cap() const;
  int ipt() const { return radix_ipt_of(opt_.radix_tile); }  // radix tile: items per thread

  int ev_begin(int cls);  // returns a slot for ev_end, or -1 when not profiling
  void ev_end(int slot);
  void ev_collect();

  int64_t n_, m_;
  hipStream_t st_;
  Options opt_;
  HostWords hw_;
  uint32_t tag_ = 1;       // marks the active nodes of the coming round in actr_
  int32_t k_target_ = 0;   // largest k asked of refine

  // history (options.history): per round j, ord and class-start position
  // ids of that round's partition
  struct Level {
    DevBuf ord, pid;
  };
  std::vector<Level> hist_;
  // maintenance state: reverse CSR (edges by target, words (label rank <<
  // dst_bits) | source), sorted distinct label values, update scratch
  DevBuf rrowptr_, radj_;
  std::vector<int32_t> nlab_vals_, elab_vals_;
  DevBuf d_nvals_, d_evals_;
  DevBuf rtag_, ctag_, dtag_, cont_;
  uint32_t utag_ = 0;
  DevBuf src_list_, rlist_, clist_, dlist_, dsize_, ufirst_, keep_, kscan_, old_prev_pid_, old_ord_, old_pid_;
  DevBuf fill_, dszpos_, isize_, gw_, inode_, iflag_, w_, wscan_, inu_, kus_, oflag_, ocls_, ofirst_, xpos_, xflag_;
  DevBuf chunk_;
  uint32_t n_src_ = 0;       // sources of changed edges and new nodes, checked at every level
  uint32_t old_n_nodes_ = 0;  // nodes before the update in progress
  UpdateStat ustat_;

  bool adj64_ = false, key64_ = false;
  int dst_bits_ = 1, lab_bits_ = 0;
  uint32_t n_elab_ = 0;
  uint32_t b0_ = 0;  // blocks of pId_0
  int pid0_bytes_ = 4;  // bytes per entry of pid0_

  // graph
  DevBuf rowptr_, adj_, hub_toff_, hub_tmp_;
  // hubs of the round sorted together (rounds with wide keys): offsets of
  // their items, sort space, run ranks; edges of the listed hubs
  DevBuf hub_off_, hub_k0_, hub_k1_, hub_fl_;
  uint32_t hub_edges_act_ = 0;
  uint64_t hub_edges_ = 0;
  uint32_t maxdeg_ = 0;  // largest out-degree
  bool maxdeg_pending_ = false;  // maxdeg_ arrives with the next round summary
  bool hub_toff_valid_ = false;  // hub_toff_ and hub_edges_ match the graph
  // partition state: ord, class-start flags, class-start position ids, and
  // the dense pId_0 used by the first round's keys
  DevBuf pid_, pid0_, ord_, flag_;
  int64_t B_ = 0;
  int32_t rounds_ = 0;
  bool fixed_ = false;
  std::vector<int64_t> counts_;
  std::vector<double> round_secs_;  // host seconds of round j as last computed in full (index j)
  // active set: segments (size classes), their positions and nodes, and the
  // signature work lists (wave, block, hub)
  SegLists act_;
  uint32_t S_act_ = 0, M_act_ = 0;
  DevBuf soff_, apos_, anode_, actr_, blists_, info_;
  bool act_dense_ = false;  // work lists in node order (see prepare_active)
  uint32_t bcnt_[4] = {}, boff_[4] = {};  // per degree bucket: wave, mid, block, hub
  // dense ids
  DevBuf dense_;
  int32_t dense_round_ = -1;
  int32_t cls_round_ = -1;  // round whose class scan cls_ holds (-1: none)
  // round scratch
  DevBuf ukey_, ucnt_, head_, cls_, fl_, first_, scanpart_, radix_, part_, bm_, bmslot_;
  DevBuf scanpart_nodes_, radix_nodes_;  // the node part of create, beside the edge table's sort
  DevBuf bstart_;  // during the build: start position of every k = 0 block (and N)
  // streamed edge table (opt_.edge_window > 0): the CSR edge words in pinned
  // host memory, cut into partitions of consecutive source nodes whose rows
  // fit one of two device windows
  bool streamed_ = false;
  void* host_adj_ = nullptr;
  std::vector<uint32_t> part_node_;  // partition p: nodes [part_node_[p], part_node_[p+1])
  std::vector<uint64_t> part_edge_;  // and edges [part_edge_[p], part_edge_[p+1])
  DevBuf win_[2];
  hipStream_t copy_st_ = nullptr;
  hipEvent_t win_full_[2] = {nullptr, nullptr}, win_free_[2] = {nullptr, nullptr};
  uint64_t streamed_bytes_ = 0;  // host->device bytes of the edge table moved by the rounds
  uint32_t direct_rounds_ = 0;   // rounds that read the rows of their active nodes in place
  DevBuf seg_start_, seg_size_, seg_depth_, seg_done_, cls_meta_;
  SegLists lists_b_[2];  // subgroup lists of alternate global passes
  DevBuf l_fd_, l_long_;
  DevBuf k0_, k1_, k2_, k3_, k4_, v0_, v1_, v2_, v3_, v4_, sflag_, soff2_, ipos_, sub_item_;

  // the resolvers run on two more streams, overlapping the global passes and
  // each other: groups of one workgroup of 1024 threads on side_big_, all
  // smaller ones on side_
  hipStream_t side_ = nullptr, side_big_ = nullptr;
  bool single_stream_ = false;  // all work on st_ (jobs inside a static scratch region)
  int side_dev_ = 0;  // device of the resolver streams
  hipEvent_t ev_side_[2] = {nullptr, nullptr}, ev_big_[2] = {nullptr, nullptr};
  hipEvent_t ev_main_ = nullptr, ev_join_ = nullptr, ev_join_big_ = nullptr;

  // profiling
  struct EvPair {
    hipEvent_t a, b;
    int cls;
    int round;  // round being computed when recorded (1-based)
  };
  std::vector<EvPair> ev_pool_;
  std::vector<RoundStat> round_ms_;  // milliseconds per round (counts come from work_)
  int32_t round_base_ = 0;           // rounds before the last reset of the round stats
  DevBuf work_;                      // kRoundSlots x kWorkWords counters
  size_t ev_used_ = 0;
};

}  // namespace kb
