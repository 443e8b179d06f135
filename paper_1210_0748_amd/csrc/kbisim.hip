// k-bisimulation on one MI355X: host round driver and the C ABI (kbisim.h).
//
// Per round (Algorithm 1, one iteration j > 0):
//   signature kernels  -- join with pId_{j-1}(dst), per-node sort + unique
//   order_groups       -- order the signatures inside every block of pId_{j-1}
//   assign_ids         -- scan of class starts -> pId_j, block starts, B_j
// The graph (CSR by source, packed label|dst words) stays in device memory.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>

#include "active.h"
#include "batch.h"
#include "build.h"
#include "common.h"
#include "engine.h"
#include "maintain.h"
#include "stream.h"
#include "refine.h"
#include "scan_radix.h"
#include "server.h"
#include "signature.h"
#include "../../include/kbisim.h"

namespace kb {

namespace {
constexpr int kNT = 256;
inline uint32_t grid_for(uint64_t n, int nt = kNT) { return n ? ceil_div(n, nt) : 1; }
inline uint32_t grid_stride_blocks(uint64_t n) {
  return std::max<uint32_t>(1, std::min<uint32_t>(ceil_div(n, kNT), 8192));
}
}  // namespace

Engine::Engine(int64_t n, int64_t m, hipStream_t s, const Options& o)
    : n_(n), m_(m), st_(s), opt_(o), single_stream_(active_arena() != nullptr) {}

Engine::~Engine() {
  for (auto& e : ev_pool_) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (hipStream_t q : {side_, side_big_}) {
    if (!q) continue;
    if (hipStreamSynchronize(q) == hipSuccess)
      StreamPool::instance().put(q, side_dev_);
    else
      (void)hipGetLastError();  // a stream in an error state is not reused
  }
  for (hipEvent_t e : {ev_side_[0], ev_side_[1], ev_big_[0], ev_big_[1], ev_main_, ev_join_, ev_join_big_})
    if (e) (void)hipEventDestroy(e);
  if (copy_st_) {
    (void)hipStreamSynchronize(copy_st_);
    (void)hipStreamDestroy(copy_st_);
  }
  for (hipEvent_t e : {win_full_[0], win_full_[1], win_free_[0], win_free_[1]})
    if (e) (void)hipEventDestroy(e);
  if (host_adj_) {
    (void)hipStreamSynchronize(st_);  // launches may still read the table in place
    (void)hipHostFree(host_adj_);
  }
}

// Streams for the resolvers (default priority, not synchronising with the
// null stream; from the process-wide pool) and the events that order them
// against the handle's.
hipStream_t Engine::side_stream() {
  if (!side_) {
    KB_CHECK(hipGetDevice(&side_dev_));
    side_ = StreamPool::instance().get();
    side_big_ = StreamPool::instance().get();
    for (hipEvent_t* e : {&ev_side_[0], &ev_side_[1], &ev_big_[0], &ev_big_[1], &ev_main_, &ev_join_, &ev_join_big_})
      KB_CHECK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  return side_;
}

uint64_t Engine::read_word(const void* dev, int bytes) {
  hw_.p[0] = 0;
  KB_CHECK(hipMemcpyAsync(hw_.p, dev, bytes, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  return hw_.p[0];
}

template <typename Tin, typename Tout, bool kIncl>
void Engine::scan_dev(const Tin* in, Tout* out, uint64_t n) {
  scanpart_.ensure(scan_partials_count(n) * sizeof(uint64_t));
  scan<Tin, Tout, kIncl>(in, out, n, scanpart_.as<Tout>(), st_);
}

uint32_t* Engine::radix_scratch(uint64_t n) {
  radix_.ensure(radix_scratch_words(n) * sizeof(uint32_t));
  return radix_.as<uint32_t>();
}

int Engine::ev_begin(int cls) {
  if (!opt_.profile) return -1;
  if (ev_used_ == ev_pool_.size()) {
    EvPair e;
    KB_CHECK(hipEventCreate(&e.a));
    KB_CHECK(hipEventCreate(&e.b));
    ev_pool_.push_back(e);
  }
  const int slot = int(ev_used_++);
  ev_pool_[slot].cls = cls;
  ev_pool_[slot].round = rounds_ + 1;
  KB_CHECK(hipEventRecord(ev_pool_[slot].a, st_));
  return slot;
}

void Engine::ev_end(int slot) {
  if (slot < 0) return;
  KB_CHECK(hipEventRecord(ev_pool_[size_t(slot)].b, st_));
}

void Engine::ev_collect() {
  if (!opt_.profile) return;
  KB_CHECK(hipStreamSynchronize(st_));
  for (size_t i = 0; i < ev_used_; ++i) {
    float ms = 0.f;
    KB_CHECK(hipEventElapsedTime(&ms, ev_pool_[i].a, ev_pool_[i].b));
    prof_ms[ev_pool_[i].cls] += ms;
    prof_n[ev_pool_[i].cls] += 1;
    const int r = ev_pool_[i].round - round_base_;
    if (r >= 1 && (ev_pool_[i].cls == 0 || ev_pool_[i].cls == 3)) {
      if (round_ms_.size() < size_t(r)) round_ms_.resize(size_t(r));
      (ev_pool_[i].cls == 0 ? round_ms_[size_t(r) - 1].sig_ms : round_ms_[size_t(r) - 1].round_ms) += ms;
    }
  }
  ev_used_ = 0;
}

// ---------------------------------------------------------------------------
// Build: validation, pId_0, edge-label ranks, CSR.

template <typename AdjT>
void Engine::build_adj(const int32_t* src, const int32_t* lab, const int32_t* dst, const uint32_t* erank,
                       const uint32_t* rank_table, uint32_t* hist0) {
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  rowptr_.ensure((N + 1) * sizeof(uint32_t));
  if (E) {
    // sort the packed edges by source (CSR order without atomics); row
    // offsets by binary search in the sorted sources. The first pass reads
    // the edge table itself and packs while it scatters; its per-tile counts
    // came with the validation pass.
    DevBuf ka, kb2, vb;
    ka.ensure(E * 4);
    kb2.ensure(E * 4);
    adj_.ensure(E * sizeof(AdjT));
    vb.ensure(E * sizeof(AdjT));
    const uint32_t nb = radix_blocks(E, ipt());
    const EdgePackLoad<AdjT> load{src, lab, dst, erank, rank_table, dst_bits_};
    if (nb > kRadixFusedTiles) scan_dev<uint32_t, uint32_t, false>(hist0, hist0, uint64_t(nb) * 256);
    with_radix_ipt(ipt(), [&](auto tag) {
      constexpr int I = decltype(tag)::value;
      if (nb <= kRadixFusedTiles)
        pack_scatter_k<AdjT, true, I><<<nb, kRadixNT, 0, st_>>>(load, ka.as<uint32_t>(), adj_.as<AdjT>(), E, hist0, nb);
      else
        pack_scatter_k<AdjT, false, I><<<nb, kRadixNT, 0, st_>>>(load, ka.as<uint32_t>(), adj_.as<AdjT>(), E, hist0,
                                                                 nb);
    });
    KB_LAUNCH_CHECK();
    const bool f = radix_sort<uint32_t, AdjT>(ka.as<uint32_t>(), adj_.as<AdjT>(), kb2.as<uint32_t>(),
                                              vb.as<AdjT>(), E, 8, bits_for(N > 1 ? N - 1 : 1),
                                              radix_scratch(E), st_, ipt());
    if (f) adj_.swap(vb);
    const uint32_t* skey = f ? kb2.as<uint32_t>() : ka.as<uint32_t>();
    // long runs of nodes without edges: at most N / kRowGap + 1 of them
    DevBuf gaps;
    gaps.ensure((3 * (N / kRowGap + 2) + 1) * 4);
    uint32_t* ng = gaps.as<uint32_t>() + 3 * (N / kRowGap + 2);
    KB_CHECK(hipMemsetAsync(ng, 0, 4, st_));
    csr_rowptr_k<<<grid_stride_blocks(E + 1), kNT, 0, st_>>>(skey, E, uint32_t(N), rowptr_.as<uint32_t>(),
                                                            gaps.as<uint32_t>(), ng);
    KB_LAUNCH_CHECK();
    csr_rowptr_gaps_k<<<256, kNT, 0, st_>>>(gaps.as<uint32_t>(), ng, rowptr_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    // the temporaries go back to the pool with an event on this stream: a
    // later user of a block is ordered after this work, no host wait here
  } else {
    adj_.ensure(sizeof(AdjT));
    KB_CHECK(hipMemsetAsync(rowptr_.p, 0, (N + 1) * 4, st_));
  }
  degree_stats();
}

// The largest out-degree, into an info word the next round summary reads
// back (no synchronisation here); the hubs' radix-sort space is laid out by
// hub_layout when a round first needs it.
void Engine::degree_stats() {
  const uint64_t N = uint64_t(n_);
  hub_toff_valid_ = false;
  maxdeg_ = 0;
  if (!N) return;
  uint32_t* w = info_.as<uint32_t>() + kInfoMaxDeg;
  set_u32_k<<<1, 1, 0, st_>>>(w, 0u);
  KB_LAUNCH_CHECK();
  max_degree_k<<<std::min<uint32_t>(grid_for(N), 1024), kNT, 0, st_>>>(rowptr_.as<uint32_t>(), uint32_t(N), w);
  KB_LAUNCH_CHECK();
  maxdeg_pending_ = true;
}

// Offsets of the hubs' items (exclusive scan of the out-degrees above
// kBlockMaxDeg) and their total (synchronises; once per graph).
void Engine::hub_layout() {
  if (hub_toff_valid_) return;
  const uint64_t N = uint64_t(n_);
  hub_toff_.ensure((N + 1) * sizeof(uint32_t));
  hub_edges_ = 0;
  if (N) {
    DevBuf hd;
    hd.ensure((N + 1) * sizeof(uint32_t));
    KB_CHECK(hipMemsetAsync(hd.as<uint32_t>() + N, 0, 4, st_));
    hub_degree_k<<<grid_for(N), kNT, 0, st_>>>(rowptr_.as<uint32_t>(), uint32_t(N), kBlockMaxDeg, hd.as<uint32_t>());
    KB_LAUNCH_CHECK();
    scan_dev<uint32_t, uint32_t, false>(hd.as<uint32_t>(), hub_toff_.as<uint32_t>(), N + 1);
    hub_edges_ = read_word(hub_toff_.as<uint32_t>() + N, 4);  // synchronises: `hd` may be freed
  }
  hub_toff_valid_ = true;
}

// Dense ascending ranks of the label values `val[0..n)` (all >= 0, max
// `maxv`): for small values through a presence table (rank_table[v] = rank
// of value v; below kMaskLabels built from the presence mask of the
// validation pass, else by marking), otherwise through a sort (rank[i] per
// element). Returns the number of distinct values. Exactly one of the two
// outputs is filled.
uint32_t Engine::label_ranks(const int32_t* val, uint64_t n, uint32_t maxv, const unsigned long long* mask_dev,
                             const uint64_t* mask_host, DevBuf& rank_table, DevBuf& rank,
                             std::vector<int32_t>* values) {
  if (values) values->clear();
  if (n == 0) return 0;
  if (maxv < kMaskLabels) {
    // all values are in the presence mask the validation pass collected
    const uint32_t t = maxv + 2;
    rank_table.ensure(uint64_t(t) * 4);
    mask_ranks_k<<<1, 256, 0, st_>>>(mask_dev, t, rank_table.as<uint32_t>());
    KB_LAUNCH_CHECK();
    uint32_t d = 0;
    for (int q = 0; q < 4; ++q) d += uint32_t(__builtin_popcountll(mask_host[q]));
    if (values)
      for (uint32_t v = 0; v < kMaskLabels; ++v)
        if ((mask_host[v / 64] >> (v % 64)) & 1ull) values->push_back(int32_t(v));
    return d;
  }
  if (maxv < kRankTableMax && !single_stream_) {  // (a table of maxv entries may not fit a static region)
    const uint64_t t = uint64_t(maxv) + 2;
    DevBuf present;
    present.ensure(t * 4);
    rank_table.ensure(t * 4);
    KB_CHECK(hipMemsetAsync(present.p, 0, t * 4, st_));
    mark_present_k<<<grid_stride_blocks(n), kNT, 0, st_>>>(val, n, present.as<uint32_t>());
    KB_LAUNCH_CHECK();
    scan_dev<uint32_t, uint32_t, false>(present.as<uint32_t>(), rank_table.as<uint32_t>(), t);
    const uint32_t d = uint32_t(read_word(rank_table.as<uint32_t>() + (t - 1), 4));
    if (values) {  // value v is present where the exclusive scan steps
      std::vector<uint32_t> tab(t);
      KB_CHECK(hipMemcpyAsync(tab.data(), rank_table.p, uint64_t(t) * 4, hipMemcpyDeviceToHost, st_));
      KB_CHECK(hipStreamSynchronize(st_));
      for (uint32_t v = 0; v + 1 < t; ++v)
        if (tab[v + 1] != tab[v]) values->push_back(int32_t(v));
    }
    return d;  // synchronised: `present` may be freed
  }
  DevBuf ka, kb2, va, vb;
  for (DevBuf* b : {&ka, &kb2, &va, &vb}) b->ensure(n * 4);
  to_u32_iota_k<<<grid_for(n), kNT, 0, st_>>>(val, ka.as<uint32_t>(), va.as<uint32_t>(), uint32_t(n));
  KB_LAUNCH_CHECK();
  const bool f = radix_sort<uint32_t>(ka.as<uint32_t>(), va.as<uint32_t>(), kb2.as<uint32_t>(), vb.as<uint32_t>(),
                                      n, 0, bits_for(maxv), radix_scratch(n), st_, ipt());
  uint32_t* keys = f ? kb2.as<uint32_t>() : ka.as<uint32_t>();
  uint32_t* vals = f ? vb.as<uint32_t>() : va.as<uint32_t>();
  uint32_t* fl = f ? ka.as<uint32_t>() : kb2.as<uint32_t>();   // the free key buffer
  uint32_t* cl = f ? va.as<uint32_t>() : vb.as<uint32_t>();    // the free value buffer
  run_start_flags_k<<<grid_for(n), kNT, 0, st_>>>(keys, uint32_t(n), nullptr, fl);
  KB_LAUNCH_CHECK();
  scan_dev<uint32_t, uint32_t, true>(fl, cl, n);
  rank.ensure(n * 4);
  rank_scatter_k<<<grid_for(n), kNT, 0, st_>>>(vals, cl, uint32_t(n), rank.as<uint32_t>());
  KB_LAUNCH_CHECK();
  const uint32_t d = uint32_t(read_word(cl + (n - 1), 4));
  if (values && d) {
    DevBuf dv;
    dv.ensure(uint64_t(d) * 4);
    distinct_values_k<<<grid_for(n), kNT, 0, st_>>>(keys, fl, cl, uint32_t(n), dv.as<int32_t>());
    KB_LAUNCH_CHECK();
    values->resize(d);
    KB_CHECK(hipMemcpyAsync(values->data(), dv.p, uint64_t(d) * 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
  }
  return d;
}

void Engine::build(const int32_t* node_label, const int32_t* src, const int32_t* lab, const int32_t* dst) {
  StreamScope scope(st_);
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  // error word, label maxima, and the presence masks of node and edge labels
  // below kMaskLabels (4 words each, from byte 16)
  constexpr size_t kErrBytes = 16 + 8 * sizeof(uint64_t);
  DevBuf errb;
  errb.ensure(kErrBytes);
  KB_CHECK(hipMemsetAsync(errb.p, 0, kErrBytes, st_));
  uint32_t* err = errb.as<uint32_t>();
  unsigned long long* masks = reinterpret_cast<unsigned long long*>(errb.as<uint8_t>() + 16);
  DevBuf hist0;  // per-tile source counts for the first pass of the sort by source
  const uint32_t enb = E ? radix_blocks(E, ipt()) : 0u;
  if (N) {
    validate_nodes_k<<<validate_blocks(N), kRadixNT, 0, st_>>>(node_label, N, err, err + 1, masks);
    KB_LAUNCH_CHECK();
  }
  if (E) {
    hist0.ensure(uint64_t(enb) * 256 * 4);
    with_radix_ipt(ipt(), [&](auto tag) {
      edge_scan_k<decltype(tag)::value><<<std::min<uint32_t>(enb, 2048), kRadixNT, 0, st_>>>(
          src, lab, dst, E, n_, err, err + 2, masks + 4, hist0.as<uint32_t>(), enb);
    });
    KB_LAUNCH_CHECK();
  }
  KB_CHECK(hipMemcpyAsync(hw_.p, errb.p, kErrBytes, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  uint32_t words[3];
  uint64_t mask_host[8];
  std::memcpy(words, hw_.p, sizeof(words));
  std::memcpy(mask_host, hw_.p + 2, sizeof(mask_host));
  if (words[0] & 1u) throw InvalidInput("edge endpoint outside [0, num_nodes)");
  if (words[0] & 2u) throw InvalidInput("negative edge label");
  if (words[0] & 4u) throw InvalidInput("negative node label");
  const uint32_t max_nlab = words[1], max_elab = words[2];
  info_.ensure(kInfoWords * 4);

  // The node part (pId_0, the order by label, the blocks) does not read the
  // edge table: unless the handle must stay on one stream, it runs on the
  // side stream beside the edge table's sort, with scratch of its own, and
  // the handle's stream waits for it before the first round's set-up. The
  // edge part is queued first, so its long passes start at once.
  const bool split = !single_stream_ && N > 0 && E > 0;
  hipStream_t ns = st_;
  if (split) {
    ns = side_stream();
    KB_CHECK(hipEventRecord(ev_main_, st_));  // the validation pass is done
    KB_CHECK(hipStreamWaitEvent(ns, ev_main_, 0));
  }

  // edge labels: dense ascending ranks
  DevBuf etable, erank;
  n_elab_ = label_ranks(lab, E, max_elab, masks + 4, mask_host + 4, etable, erank,
                        opt_.history ? &elab_vals_ : nullptr);
  set_edge_layout();
  const uint32_t* er = erank.p ? erank.as<uint32_t>() : nullptr;
  const uint32_t* et = etable.p ? etable.as<uint32_t>() : nullptr;
  if (adj64_)
    build_adj<uint64_t>(src, lab, dst, er, et, hist0.as<uint32_t>());
  else
    build_adj<uint32_t>(src, lab, dst, er, et, hist0.as<uint32_t>());

  if (split) {
    // this thread's launches, scans, sorts, read-backs and pool traffic go
    // to the side stream and its scratch until the node part is queued
    struct Swap {
      Engine* e;
      hipStream_t st;
      Swap(Engine* eng, hipStream_t s) : e(eng), st(s) { flip(); }
      ~Swap() { flip(); }
      void flip() {
        std::swap(e->st_, st);
        e->scanpart_.swap(e->scanpart_nodes_);
        e->radix_.swap(e->radix_nodes_);
      }
    };
    {
      StreamScope scope(ns);
      Swap on_side(this, ns);
      build_nodes(node_label, max_nlab, masks, mask_host);
    }
    KB_CHECK(hipEventRecord(ev_join_, ns));
    KB_CHECK(hipStreamWaitEvent(st_, ev_join_, 0));
    // the node part's lasting buffers are used on the handle's stream from
    // here on: their release must be ordered there (the pool records the
    // release on a buffer's stream)
    for (DevBuf* b : {&pid_, &ord_, &flag_, &cls_, &act_.start, &act_.size, &act_.depth, &soff_, &apos_, &anode_,
                      &blists_, &fl_, &first_, &actr_, &pid0_, &bstart_})
      b->s = st_;
  } else {
    build_nodes(node_label, max_nlab, masks, mask_host);
  }
  finish_build();
}

void Engine::set_edge_layout() {
  const uint64_t N = uint64_t(n_);
  lab_bits_ = n_elab_ > 1 ? bits_for(n_elab_ - 1) : 0;
  dst_bits_ = bits_for(N > 1 ? N - 1 : 1);
  adj64_ = dst_bits_ + lab_bits_ > 32;
  key64_ = lab_bits_ + bits_for(N > 1 ? N - 1 : 1) > 32;
}

// Per-node state and the k = 0 partition from the node labels (validated,
// largest label max_nlab, presence mask of labels below kMaskLabels on the
// device and the host).
void Engine::build_nodes(const int32_t* node_label, uint32_t max_nlab, const unsigned long long* masks,
                         const uint64_t* mask_host) {
  const uint64_t N = uint64_t(n_);
  const uint64_t N1 = std::max<uint64_t>(N, 1);
  pid_.ensure(N1 * 4);
  ord_.ensure(N1 * 4);
  flag_.ensure(N1);
  cls_.ensure(N1 * 4);
  info_.ensure(kInfoWords * 4);
  for (DevBuf* b : {&act_.start, &act_.size, &act_.depth, &soff_}) b->ensure((N + 1) * 4);
  for (DevBuf* b : {&apos_, &anode_, &blists_, &fl_, &first_, &actr_}) b->ensure(N1 * 4);

  // pId_0: the rank of the node label; nodes sorted by it give `ord` and the
  // blocks (Section 3.1, k = 0: sort by label, a new id per new label).
  // pId_0 is kept in the narrowest type that holds it (the first round
  // gathers it for every edge); ids and the first round's active marks are
  // written in node order.
  DevBuf bstart;
  bstart.ensure((N + 1) * 4);
  B_ = 0;
  pid0_bytes_ = 4;
  if (N) {
    DevBuf table, rank, ka, kb2, va, vb;
    const uint32_t nl = label_ranks(node_label, N, max_nlab, masks, mask_host, table, rank,
                                    opt_.history ? &nlab_vals_ : nullptr);
    pid0_bytes_ = nl <= 256 ? 1 : nl <= 65536 ? 2 : 4;
    pid0_.ensure(N * pid0_bytes_);
    for (DevBuf* b : {&ka, &kb2, &va, &vb}) b->ensure(N * 4);
    const uint32_t n32 = uint32_t(N);
    if (table.p) {
      const uint32_t* t = table.as<uint32_t>();
      if (pid0_bytes_ == 1)
        lookup_rank_k<uint8_t><<<grid_for(N), kNT, 0, st_>>>(node_label, t, n32, ka.as<uint32_t>(),
                                                             va.as<uint32_t>(), pid0_.as<uint8_t>());
      else if (pid0_bytes_ == 2)
        lookup_rank_k<uint16_t><<<grid_for(N), kNT, 0, st_>>>(node_label, t, n32, ka.as<uint32_t>(),
                                                              va.as<uint32_t>(), pid0_.as<uint16_t>());
      else
        lookup_rank_k<uint32_t><<<grid_for(N), kNT, 0, st_>>>(node_label, t, n32, ka.as<uint32_t>(),
                                                              va.as<uint32_t>(), pid0_.as<uint32_t>());
    } else {
      KB_CHECK(hipMemcpyAsync(ka.p, rank.p, N * 4, hipMemcpyDeviceToDevice, st_));
      iota_k<<<grid_for(N), kNT, 0, st_>>>(va.as<uint32_t>(), n32);
      if (pid0_bytes_ == 1)
        narrow_ids_k<uint8_t><<<grid_for(N), kNT, 0, st_>>>(rank.as<uint32_t>(), n32, pid0_.as<uint8_t>());
      else if (pid0_bytes_ == 2)
        narrow_ids_k<uint16_t><<<grid_for(N), kNT, 0, st_>>>(rank.as<uint32_t>(), n32, pid0_.as<uint16_t>());
      else
        KB_CHECK(hipMemcpyAsync(pid0_.p, rank.p, N * 4, hipMemcpyDeviceToDevice, st_));
    }
    KB_LAUNCH_CHECK();
    const bool f = radix_sort<uint32_t>(ka.as<uint32_t>(), va.as<uint32_t>(), kb2.as<uint32_t>(),
                                        vb.as<uint32_t>(), N, 0, bits_for(nl > 1 ? nl - 1 : 1),
                                        radix_scratch(N), st_, ipt());
    const uint32_t* keys = f ? kb2.as<uint32_t>() : ka.as<uint32_t>();
    const uint32_t* vals = f ? vb.as<uint32_t>() : va.as<uint32_t>();
    KB_CHECK(hipMemcpyAsync(ord_.p, vals, N * 4, hipMemcpyDeviceToDevice, st_));
    run_start_flags_k<<<grid_for(N), kNT, 0, st_>>>(keys, n32, flag_.as<uint8_t>(), nullptr);
    KB_LAUNCH_CHECK();
    // block starts (the ranks are dense: nl blocks), then per node its
    // block's start position and whether the block has two or more members
    scan_dev<uint8_t, uint32_t, true>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), N);
    block_starts_k<<<grid_for(N), kNT, 0, st_>>>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), n32,
                                                 bstart.as<uint32_t>());
    KB_LAUNCH_CHECK();
    B_ = int64_t(nl);
    set_u32_k<<<1, 1, 0, st_>>>(bstart.as<uint32_t>() + B_, n32);
    KB_LAUNCH_CHECK();
    if (pid0_bytes_ == 1)
      node_ids0_k<uint8_t><<<grid_for(N), kNT, 0, st_>>>(pid0_.as<uint8_t>(), bstart.as<uint32_t>(), n32,
                                                         pid_.as<int32_t>(), actr_.as<uint32_t>(), 1u);
    else if (pid0_bytes_ == 2)
      node_ids0_k<uint16_t><<<grid_for(N), kNT, 0, st_>>>(pid0_.as<uint16_t>(), bstart.as<uint32_t>(), n32,
                                                          pid_.as<int32_t>(), actr_.as<uint32_t>(), 1u);
    else
      node_ids0_k<uint32_t><<<grid_for(N), kNT, 0, st_>>>(pid0_.as<uint32_t>(), bstart.as<uint32_t>(), n32,
                                                          pid_.as<int32_t>(), actr_.as<uint32_t>(), 1u);
    KB_LAUNCH_CHECK();
  }
  b0_ = uint32_t(B_);
  counts_.assign(1, B_);
  rounds_ = 0;
  fixed_ = false;
  dense_round_ = -1;
  cls_round_ = -1;
  bstart_.swap(bstart);
}

// Per-round buffers and the first round's active set, once the CSR, the
// degree statistics and the k = 0 blocks (bstart_) are in place.
void Engine::finish_build() {
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  const uint64_t N1 = std::max<uint64_t>(N, 1);
  // per-round buffers
  hub_off_.ensure((E / (uint64_t(kBlockMaxDeg) + 1) + 2) * 4);
  ukey_.ensure(std::max<uint64_t>(E, 1) * (key64_ ? 8 : 4));
  ucnt_.ensure(N1 * 4);
  head_.ensure(N1 * 8);

  // the first round's segments: the blocks of pId_0 with two or more members
  if (N) {
    const uint32_t med = std::min(medium_cap(), kMediumCapSmall), big = medium_cap();
    KB_CHECK(hipMemsetAsync(act_.size.p, 0, (uint64_t(B_) + 1) * 4, st_));
    compact<kSegClasses>(BlockSegOf{bstart_.as<uint32_t>(), med, big},
                         BlockSegWrite{bstart_.as<uint32_t>(), act_.start.as<uint32_t>(), act_.size.as<uint32_t>(),
                                       act_.depth.as<uint32_t>()},
                         uint32_t(B_), nullptr, compact_scratch(compact_part_words<kSegClasses>(B_)),
                         info_.as<uint32_t>() + kInfoSeg, st_);
    large_offsets(act_, info_.as<uint32_t>() + kInfoSeg, info_.as<uint32_t>() + kInfoLargeItems, N);
    prepare_active(uint32_t(B_), uint32_t(N), 1u, false);  // active marks written above
  }
  if (opt_.history) {
    hist_.clear();
    save_level(0);
    build_reverse();
  }
  KB_CHECK(hipStreamSynchronize(st_));
  bstart_.release();
}

uint32_t Engine::medium_cap() const { return opt_.medium_cap; }

uint32_t* Engine::compact_scratch(uint64_t words) {
  part_.ensure(std::max<uint64_t>(words, 1) * 4);
  return part_.as<uint32_t>();
}

// After the segment lists of the coming round are in act_ (their summary in
// info_): item offsets of the segments, the active positions and nodes, the
// signature work lists, and one read-back of the summary. seg_items bounds the
// number of segments (act_.size must be zero from the last segment up to
// seg_items), m_cap the number of active positions, tag the number of the
// round being prepared (1 for the first), which marks its nodes in actr_.
void Engine::prepare_active(uint32_t seg_items, uint32_t m_cap, uint32_t tag, bool mark) {
  tag_ = tag;
  uint32_t* info = info_.as<uint32_t>();
  scan_dev<uint32_t, uint32_t, false>(act_.size.as<uint32_t>(), soff_.as<uint32_t>(), uint64_t(seg_items) + 1);
  expand_k<<<std::max<uint32_t>(1, ceil_div(m_cap, kExpandTile)), 256, 0, st_>>>(act_.start.as<uint32_t>(), soff_.as<uint32_t>(),
                                             info + kInfoSeg + 2 * kSegClasses, m_cap, ord_.as<uint32_t>(),
                                             apos_.as<uint32_t>(), anode_.as<uint32_t>(),
                                             mark ? actr_.as<uint32_t>() : nullptr, tag, info);
  KB_LAUNCH_CHECK();
  // when many nodes are active, the work lists and the thread part go over
  // node ids in order (neighbouring rows), else over the active list; when
  // the bound m_cap leaves it open, the real count decides (one read-back
  // costs less than a pass over every node id)
  act_dense_ = uint64_t(m_cap) * 8 >= uint64_t(n_);
  if (act_dense_ && uint64_t(m_cap) * 2 < uint64_t(n_))
    act_dense_ = read_word(info + kInfoItems, 4) * 8 >= uint64_t(n_);
  if (act_dense_) {
    compact<kNumBuckets>(NodeBucketDenseOf{actr_.as<uint32_t>(), tag, rowptr_.as<uint32_t>()},
                         NodeWriteDense{blists_.as<uint32_t>()}, uint32_t(n_), nullptr,
                         compact_scratch(compact_part_words<kNumBuckets>(uint64_t(n_))), info + kInfoBucket, st_);
  } else {
    compact<kNumBuckets>(NodeBucketOf{anode_.as<uint32_t>(), rowptr_.as<uint32_t>()},
                         NodeWrite{anode_.as<uint32_t>(), blists_.as<uint32_t>()}, m_cap, info + kInfoItems,
                         compact_scratch(compact_part_words<kNumBuckets>(m_cap)), info + kInfoBucket, st_);
  }
  // offsets of the hubs' items for the device-wide hub sort
  hub_offsets_k<<<1, 1024, 0, st_>>>(rowptr_.as<uint32_t>(), blists_.as<uint32_t>(), info + kInfoBucket + kBucketHub,
                                     info + kInfoBucket + kNumBuckets + kBucketHub, hub_off_.as<uint32_t>(),
                                     info + kInfoHubEdges);
  KB_LAUNCH_CHECK();
  uint32_t* h = reinterpret_cast<uint32_t*>(hw_.p);
  static_assert(kInfoWords <= 2 * PinnedSlots::kSlotWords, "read-back slot too small");
  for (int i = 0; i < kInfoWords; ++i) h[i] = 0;  // before the copy is queued
  KB_CHECK(hipMemcpyAsync(h, info, kInfoWords * 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  for (int c = 0; c < kSegClasses; ++c) {
    act_.cnt[c] = h[kInfoSeg + c];
    act_.off[c] = h[kInfoSeg + kSegClasses + c];
  }
  if (maxdeg_pending_) {
    maxdeg_ = h[kInfoMaxDeg];
    maxdeg_pending_ = false;
  }
  S_act_ = h[kInfoSeg + 2 * kSegClasses];
  M_act_ = h[kInfoItems];
  hub_edges_act_ = h[kInfoHubEdges];
  act_.large_items = h[kInfoLargeItems];
  for (int c = 0; c < kNumBuckets; ++c) {
    bcnt_[c] = h[kInfoBucket + c];
    boff_[c] = h[kInfoBucket + kNumBuckets + c];
  }
}

// Ids for the active positions after ordering: every class of the round gets
// the position of its first member as id; classes with two or more members
// become the next round's segments. Returns with the next active set ready.
void Engine::assign_ids() {
  const uint32_t M = M_act_;
  uint32_t* info = info_.as<uint32_t>();
  act_flags_k<<<grid_for(M), kNT, 0, st_>>>(apos_.as<uint32_t>(), flag_.as<uint8_t>(), M, fl_.as<uint32_t>());
  KB_LAUNCH_CHECK();
  cls_round_ = -1;  // cls_ holds the scan over the active positions from here on
  scan_dev<uint32_t, uint32_t, true>(fl_.as<uint32_t>(), cls_.as<uint32_t>(), M);
  class_first_k<<<grid_for(M), kNT, 0, st_>>>(fl_.as<uint32_t>(), cls_.as<uint32_t>(), M, first_.as<uint32_t>(),
                                              info);
  KB_LAUNCH_CHECK();
  assign_pos_k<<<grid_for(M), kNT, 0, st_>>>(apos_.as<uint32_t>(), cls_.as<uint32_t>(), first_.as<uint32_t>(),
                                             ord_.as<uint32_t>(), M, pid_.as<int32_t>());
  KB_LAUNCH_CHECK();
}

void Engine::assign_round() {
  const uint32_t M = M_act_;
  uint32_t* info = info_.as<uint32_t>();
  assign_ids();
  const uint32_t med = std::min(medium_cap(), kMediumCapSmall), big = medium_cap();
  KB_CHECK(hipMemsetAsync(act_.size.p, 0, (uint64_t(M) + 1) * 4, st_));
  NextSegOf of{first_.as<uint32_t>(), info + kInfoClasses, M, med, big, apos_.as<uint32_t>(), ord_.as<uint32_t>(),
               ucnt_.as<uint32_t>()};
  compact<kSegClasses>(of, NextSegWrite{of, apos_.as<uint32_t>(), act_.start.as<uint32_t>(),
                                        act_.size.as<uint32_t>(), act_.depth.as<uint32_t>()},
                       M, info + kInfoClasses, compact_scratch(compact_part_words<kSegClasses>(M)),
                       info + kInfoSeg, st_);
  large_offsets(act_, info + kInfoSeg, info + kInfoLargeItems, M);
  prepare_active(M, M, tag_ + 1, true);  // runs inside round rounds_ + 1
}

// ---------------------------------------------------------------------------
// Group ordering.

void Engine::make_lists(const uint32_t* seg_start, const uint32_t* seg_size, const uint32_t* seg_depth,
                        const uint8_t* seg_done, uint32_t nseg, SegLists& out, const uint32_t* nseg_dev) {
  static_assert(kNumSegLists == kSegClasses, "list count");
  for (int c = 0; c < kNumSegLists; ++c) out.cnt[c] = out.off[c] = 0;
  out.large_items = 0;
  if (nseg == 0) return;
  const uint32_t med = std::min(medium_cap(), kMediumCapSmall), big = medium_cap();
  cls_meta_.ensure((2 * kSegClasses + 2) * 4);
  for (DevBuf* b : {&out.start, &out.size, &out.depth}) b->ensure(uint64_t(nseg) * 4);
  compact<kSegClasses>(SegClassOf{seg_size, seg_done, med, big},
                       SegCopy{seg_start, seg_size, seg_depth, out.start.as<uint32_t>(), out.size.as<uint32_t>(),
                               out.depth.as<uint32_t>()},
                       nseg, nseg_dev, compact_scratch(compact_part_words<kSegClasses>(nseg)),
                       cls_meta_.as<uint32_t>(), st_);
  large_offsets(out, cls_meta_.as<uint32_t>(), cls_meta_.as<uint32_t>() + 2 * kSegClasses + 1, nseg);
  uint32_t* hw32 = reinterpret_cast<uint32_t*>(hw_.p);
  for (int c = 0; c < 2 * kSegClasses + 2; ++c) hw32[c] = 0;  // before the copy is queued
  KB_CHECK(hipMemcpyAsync(hw32, cls_meta_.p, (2 * kSegClasses + 2) * 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  for (int c = 0; c < kSegClasses; ++c) {
    out.cnt[c] = hw32[c];
    out.off[c] = hw32[kSegClasses + c];
  }
  out.large_items = hw32[2 * kSegClasses + 1];
}

// Item offsets of the large groups of a list just classified (meta on the
// device), and their total into *total; `items` bounds the list's items.
// Large groups have more than 64 members, so at most items / 65 + 1 of them.
void Engine::large_offsets(SegLists& L, const uint32_t* meta, uint32_t* total, uint64_t items) {
  L.ioff.ensure((items / 65 + 2) * 4);
  large_offsets_k<<<1, 1024, 0, st_>>>(L.size.as<uint32_t>(), meta, L.ioff.as<uint32_t>(), total);
  KB_LAUNCH_CHECK();
}

template <int W, typename KeyT>
static void launch_lanes(const SegLists& L, int c, uint32_t* ord, uint8_t* flag, const KeyView<KeyT>& kv,
                         hipStream_t st) {
  const uint32_t n = L.cnt[c];
  if (!n) return;
  const uint32_t o = L.off[c];
  const uint32_t per_block = 256 / W;
  resolve_lanes_k<W, KeyT><<<ceil_div(n, per_block), 256, 0, st>>>(
      L.start.as<uint32_t>() + o, L.size.as<uint32_t>() + o, L.depth.as<uint32_t>() + o, n, ord, flag, kv);
  KB_LAUNCH_CHECK();
}

template <typename KeyT>
void Engine::resolve_lists(SegLists& L, const void* kvp, hipStream_t st, hipStream_t st_big) {
  const KeyView<KeyT>& kv = *static_cast<const KeyView<KeyT>*>(kvp);
  uint32_t* ord = ord_.as<uint32_t>();
  uint8_t* flag = flag_.as<uint8_t>();
  launch_lanes<8, KeyT>(L, 0, ord, flag, kv, st);
  launch_lanes<16, KeyT>(L, 1, ord, flag, kv, st);
  launch_lanes<32, KeyT>(L, 2, ord, flag, kv, st);
  launch_lanes<64, KeyT>(L, 3, ord, flag, kv, st);
  const uint32_t nm = L.cnt[kMediumClass];
  if (nm) {
    const uint32_t o = L.off[kMediumClass];
    resolve_k<kMediumNT, kMediumCapSmall, KeyT><<<nm, kMediumNT, 0, st>>>(
        L.start.as<uint32_t>() + o, L.size.as<uint32_t>() + o, L.depth.as<uint32_t>() + o, ord, flag, kv);
    KB_LAUNCH_CHECK();
  }
  const uint32_t nbig = L.cnt[kBigClass];
  if (nbig) {
    const uint32_t o = L.off[kBigClass];
    resolve_k<kBigNT, kBigCap, KeyT><<<nbig, kBigNT, 0, st_big>>>(
        L.start.as<uint32_t>() + o, L.size.as<uint32_t>() + o, L.depth.as<uint32_t>() + o, ord, flag, kv);
    KB_LAUNCH_CHECK();
  }
}

template <typename KeyT>
void Engine::order_groups(const void* kvp) {
  // The round's segments are already classified by size (act_). Groups small
  // enough for one workgroup are resolved on the side stream while the main
  // stream runs the global passes over the large ones: they touch disjoint
  // ranges of ord and flag, and both only read the signatures.
  const bool one = single_stream_;  // everything in stream order on st_, no events
  hipStream_t side = one ? st_ : side_stream();
  hipStream_t big = one ? st_ : side_big_;
  if (!one) {
    KB_CHECK(hipEventRecord(ev_main_, st_));
    KB_CHECK(hipStreamWaitEvent(side, ev_main_, 0));
    KB_CHECK(hipStreamWaitEvent(big, ev_main_, 0));
  }
  resolve_lists<KeyT>(act_, kvp, side, big);
  bool side_pending[2] = {false, false};

  // Large groups: global passes. The first sorts whole classes by their
  // leading digits; later ones split every group around its pivot.
  const KeyView<KeyT>& kv = *static_cast<const KeyView<KeyT>*>(kvp);
  uint32_t nl = act_.cnt[kLargeClass];
  const uint32_t* Ls = act_.start.as<uint32_t>() + act_.off[kLargeClass];
  const uint32_t* Ld = act_.depth.as<uint32_t>() + act_.off[kLargeClass];
  uint32_t M = act_.large_items;         // items of the large groups
  const uint32_t* gio = act_.ioff.as<uint32_t>();  // and their offsets
  int nx = 0;
  bool first_pass = true;
  const int dbits = kv.dbits;
  const uint64_t last_mask = dbits >= 64 ? ~0ull : ((1ull << dbits) - 1);
  const uint32_t head_w = dbits >= 64 ? 1u : uint32_t(64 / dbits);
  const int fd_bits = bits_for(maxdeg_ > 0 ? maxdeg_ : 1);  // first differences are below the longest sequence
  while (nl > 0) {

    // pivot passes: every item's first difference with its group's pivot
    if (!first_pass) {
      l_fd_.ensure(uint64_t(M) * 4);
      l_long_.ensure((uint64_t(M) + 1) * 4);
      KB_CHECK(hipMemsetAsync(l_long_.as<uint32_t>() + M, 0, 4, st_));
      large_fd_k<KeyT><<<grid_for(M), kNT, 0, st_>>>(Ls, Ld, gio, nl, M, ord_.as<uint32_t>(), l_fd_.as<uint32_t>(),
                                                    l_long_.as<uint32_t>(), l_long_.as<uint32_t>() + M, kv);
      KB_LAUNCH_CHECK();
      large_fd_wave_k<KeyT><<<std::min<uint32_t>(grid_for(uint64_t(M) * kWave), 4096), kNT, 0, st_>>>(
          Ls, Ld, gio, nl, ord_.as<uint32_t>(), l_fd_.as<uint32_t>(), l_long_.as<uint32_t>(),
          l_long_.as<uint32_t>() + M, kv);
      KB_LAUNCH_CHECK();
    }
    const uint64_t* head = first_pass ? head_.as<uint64_t>() : nullptr;
    const uint32_t* fdv = first_pass ? nullptr : l_fd_.as<uint32_t>();

    // sort key layout: one word when (high part, >= 1 digit) fit
    const int g_bits = nl > 1 ? bits_for(nl - 1) : 0;
    LargeKey lk;
    lk.fd_bits = first_pass ? 0 : fd_bits;
    const int hi_bits = first_pass ? g_bits : g_bits + 2 + fd_bits;
    if (hi_bits + dbits <= 64) {
      lk.packed = true;
      lk.width = std::min<uint32_t>(uint32_t((64 - hi_bits) / dbits), head_w);
    } else {
      lk.packed = false;
      lk.width = head_w;
    }
    lk.dig_bits = int(lk.width) * dbits;
    for (DevBuf* b : {&k0_, &k1_}) b->ensure(uint64_t(M) * 8);
    for (DevBuf* b : {&v0_, &v1_, &ipos_, &sub_item_}) b->ensure(uint64_t(M) * 4);
    for (DevBuf* b : {&sflag_, &soff2_}) b->ensure((uint64_t(M) + 1) * 4);
    const uint64_t* KA;
    const uint64_t* KB = nullptr;
    const uint32_t* V;
    if (lk.packed) {
      large_gather_k<KeyT><<<grid_for(M), kNT, 0, st_>>>(Ls, Ld, gio, nl, M, ord_.as<uint32_t>(), fdv, lk,
                                                        k0_.as<uint64_t>(), nullptr, v0_.as<uint32_t>(), kv, head,
                                                        head_w);
      KB_LAUNCH_CHECK();
      const bool f = radix_sort<uint64_t>(k0_.as<uint64_t>(), v0_.as<uint32_t>(), k1_.as<uint64_t>(),
                                          v1_.as<uint32_t>(), M, 0, hi_bits + lk.dig_bits, radix_scratch(M), st_, ipt());
      KA = f ? k1_.as<uint64_t>() : k0_.as<uint64_t>();
      V = f ? v1_.as<uint32_t>() : v0_.as<uint32_t>();
    } else {
      // two words: sort by lo (digits) carrying the item index, then stably
      // by hi; the final order follows the second permutation
      for (DevBuf* b : {&k2_, &k3_, &k4_}) b->ensure(uint64_t(M) * 8);
      for (DevBuf* b : {&v2_, &v3_, &v4_}) b->ensure(uint64_t(M) * 4);
      large_gather_k<KeyT><<<grid_for(M), kNT, 0, st_>>>(Ls, Ld, gio, nl, M, ord_.as<uint32_t>(), fdv, lk,
                                                        k2_.as<uint64_t>(), k0_.as<uint64_t>(), v4_.as<uint32_t>(),
                                                        kv, head, head_w);
      iota_k<<<grid_for(M), kNT, 0, st_>>>(v0_.as<uint32_t>(), M);
      KB_LAUNCH_CHECK();
      const bool f1 = radix_sort<uint64_t>(k0_.as<uint64_t>(), v0_.as<uint32_t>(), k1_.as<uint64_t>(),
                                           v1_.as<uint32_t>(), M, 0, lk.dig_bits, radix_scratch(M), st_, ipt());
      const uint64_t* L1 = f1 ? k1_.as<uint64_t>() : k0_.as<uint64_t>();
      const uint32_t* I1 = f1 ? v1_.as<uint32_t>() : v0_.as<uint32_t>();
      gather_u64_k<<<grid_for(M), kNT, 0, st_>>>(k2_.as<uint64_t>(), I1, M, k3_.as<uint64_t>());
      iota_k<<<grid_for(M), kNT, 0, st_>>>(v2_.as<uint32_t>(), M);
      KB_LAUNCH_CHECK();
      const bool f2 = radix_sort<uint64_t>(k3_.as<uint64_t>(), v2_.as<uint32_t>(), k4_.as<uint64_t>(),
                                           v3_.as<uint32_t>(), M, 0, std::max(hi_bits, 1), radix_scratch(M), st_, ipt());
      KA = f2 ? k4_.as<uint64_t>() : k3_.as<uint64_t>();
      const uint32_t* PS = f2 ? v3_.as<uint32_t>() : v2_.as<uint32_t>();
      uint64_t* lo_out = (L1 == k0_.as<uint64_t>()) ? k1_.as<uint64_t>() : k0_.as<uint64_t>();
      uint32_t* val_out = (I1 == v0_.as<uint32_t>()) ? v1_.as<uint32_t>() : v0_.as<uint32_t>();
      two_word_finish_k<<<grid_for(M), kNT, 0, st_>>>(L1, I1, PS, v4_.as<uint32_t>(), M, lo_out, val_out);
      KB_LAUNCH_CHECK();
      KB = lo_out;
      V = val_out;
    }
    large_write_k<<<grid_for(M), kNT, 0, st_>>>(Ls, gio, M, KA, KB, V, lk, ord_.as<uint32_t>(), flag_.as<uint8_t>(),
                                                sflag_.as<uint32_t>(), ipos_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemsetAsync(sflag_.as<uint32_t>() + M, 0, 4, st_));
    scan_dev<uint32_t, uint32_t, false>(sflag_.as<uint32_t>(), soff2_.as<uint32_t>(), uint64_t(M) + 1);
    const uint32_t* ns_dev = soff2_.as<uint32_t>() + M;  // number of subgroups, kept on the device
    seg_start_.ensure(uint64_t(M) * 4 + 4);
    seg_size_.ensure(uint64_t(M) * 4 + 4);
    seg_depth_.ensure(uint64_t(M) * 4 + 4);
    seg_done_.ensure(uint64_t(M) + 1);
    large_subgroups_k<<<grid_for(M), kNT, 0, st_>>>(sflag_.as<uint32_t>(), soff2_.as<uint32_t>(), M,
                                                    ipos_.as<uint32_t>(), KA, KB, lk, last_mask, Ld,
                                                    sub_item_.as<uint32_t>(),
                                                    seg_start_.as<uint32_t>(), seg_depth_.as<uint32_t>(),
                                                    seg_done_.as<uint8_t>());
    subgroup_sizes_k<<<grid_for(M), kNT, 0, st_>>>(sub_item_.as<uint32_t>(), ns_dev, M, seg_size_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    // subgroup lists alternate between two buffers: the one written now was
    // last read by the resolvers of two passes ago (side stream) and by the
    // global pass before this one (this stream)
    SegLists& out = lists_b_[nx];
    if (side_pending[nx] && !one) {
      KB_CHECK(hipStreamWaitEvent(st_, ev_side_[nx], 0));
      KB_CHECK(hipStreamWaitEvent(st_, ev_big_[nx], 0));
    }
    make_lists(seg_start_.as<uint32_t>(), seg_size_.as<uint32_t>(), seg_depth_.as<uint32_t>(),
               seg_done_.as<uint8_t>(), M, out, ns_dev);
    if (!one) {
      KB_CHECK(hipEventRecord(ev_main_, st_));
      KB_CHECK(hipStreamWaitEvent(side, ev_main_, 0));
      KB_CHECK(hipStreamWaitEvent(big, ev_main_, 0));
    }
    resolve_lists<KeyT>(out, kvp, side, big);
    if (!one) {
      KB_CHECK(hipEventRecord(ev_side_[nx], side));
      KB_CHECK(hipEventRecord(ev_big_[nx], big));
    }
    side_pending[nx] = true;
    // the next pass works on the large subgroups, read from `out`
    nl = out.cnt[kLargeClass];
    Ls = out.start.as<uint32_t>() + out.off[kLargeClass];
    Ld = out.depth.as<uint32_t>() + out.off[kLargeClass];
    M = out.large_items;
    gio = out.ioff.as<uint32_t>();
    nx ^= 1;
    first_pass = false;
  }
  // everything the resolver streams did comes before what follows on this one
  if (!one) {
    KB_CHECK(hipEventRecord(ev_join_, side));
    KB_CHECK(hipEventRecord(ev_join_big_, big));
    KB_CHECK(hipStreamWaitEvent(st_, ev_join_, 0));
    KB_CHECK(hipStreamWaitEvent(st_, ev_join_big_, 0));
  }
}

// The round's hubs (list hl, nh entries, item offsets in hub_off_) sorted
// together by (hub, key): unique keys, counts and head words of every hub.
template <typename AdjT, typename KeyT, typename CompT>
void Engine::hub_sort(const void* sig_args, const uint32_t* hl, uint32_t nh, int key_bits) {
  const SigArgs<AdjT, KeyT>& a = *static_cast<const SigArgs<AdjT, KeyT>*>(sig_args);
  const uint32_t H = hub_edges_act_;
  const int hub_bits = bits_for(nh > 1 ? nh - 1 : 1);
  const uint32_t* hoff = hub_off_.as<uint32_t>();
  hub_k0_.ensure(uint64_t(H) * sizeof(CompT));
  hub_k1_.ensure(uint64_t(H) * sizeof(CompT));
  hub_fl_.ensure((uint64_t(H) + 1) * 4);
  CompT* k0 = hub_k0_.as<CompT>();
  CompT* k1 = hub_k1_.as<CompT>();
  uint32_t* fl = hub_fl_.as<uint32_t>();
  hub_keys_k<AdjT, KeyT, CompT><<<ceil_div(H, kHubKeyTile), 256, 0, st_>>>(a, hl, hoff, nh, H, key_bits, k0);
  KB_LAUNCH_CHECK();
  const bool f = radix_sort<CompT>(k0, static_cast<uint32_t*>(nullptr), k1, static_cast<uint32_t*>(nullptr), H, 0,
                                   hub_bits + key_bits, radix_scratch(H), st_, ipt());
  const CompT* c = f ? k1 : k0;
  hub_flags_k<CompT><<<grid_for(uint64_t(H) + 1), kNT, 0, st_>>>(c, H, fl);
  KB_LAUNCH_CHECK();
  scan_dev<uint32_t, uint32_t, false>(fl, fl, uint64_t(H) + 1);
  hub_write_k<AdjT, KeyT, CompT><<<grid_for(H), kNT, 0, st_>>>(a, hl, hoff, c, fl, H, key_bits);
  KB_LAUNCH_CHECK();
  hub_finish_k<AdjT, KeyT><<<ceil_div(nh, kNT), kNT, 0, st_>>>(a, hl, hoff, fl, nh);
  KB_LAUNCH_CHECK();
}

template <typename AdjT, typename KeyT>
void Engine::round_impl(bool first) {
  const uint32_t N = uint32_t(n_);
  // round 1 keys use the dense pId_0 (narrow when there are few labels);
  // later rounds (and the rounds of an update) use class-start positions
  const uint64_t id_max = first ? (b0_ > 1 ? b0_ - 1 : 1) : (N > 1 ? N - 1 : 1);
  const int pid_bits = bits_for(id_max);
  const int key_bits = lab_bits_ + pid_bits;
  // a digit is key + 1 (0 marks the end of a sequence): as many bits as the
  // largest key + 1 needs
  const uint64_t max_key = (uint64_t(n_elab_ > 0 ? n_elab_ - 1 : 0) << pid_bits) | id_max;
  const int digit_bits = bits_for(max_key + 1);
  SigArgs<AdjT, KeyT> a;
  a.rowptr = rowptr_.as<uint32_t>();
  a.adj = adj_.as<AdjT>();
  if (first) {
    a.pid = pid0_.p;
    a.pid_bytes = pid0_bytes_;
  } else {
    a.pid = pid_.p;
    a.pid_bytes = 4;
  }
  a.ukey = ukey_.as<KeyT>();
  a.ucnt = ucnt_.as<uint32_t>();
  a.head = head_.as<uint64_t>();
  a.dst_bits = dst_bits_;
  a.pid_bits = pid_bits;
  a.hdbits = digit_bits;
  a.hw = a.hdbits >= 64 ? 1u : uint32_t(64 / a.hdbits);

  SigWork w{};
  const uint32_t* lists = blists_.as<uint32_t>();
  w.anode = anode_.as<uint32_t>();
  w.nact = M_act_;
  w.actr = actr_.as<uint32_t>();
  w.tag = tag_;
  w.n_nodes = N;
  // the work lists were built in node order when many nodes could have been
  // active; the thread part goes over all node ids only when many are
  w.dense = act_dense_ && uint64_t(M_act_) * 8 >= uint64_t(n_);
  w.wl = lists + boff_[kBucketWave];
  w.nw = bcnt_[kBucketWave];
  w.ml = lists + boff_[kBucketMid];
  w.nm = bcnt_[kBucketMid];
  w.bl = lists + boff_[kBucketBlock];
  w.nb = bcnt_[kBucketBlock];
  w.hl = lists + boff_[kBucketHub];
  w.nh = bcnt_[kBucketHub];
  w.key_bits = key_bits;
  // small key universe: workgroup nodes de-duplicate through bitmaps, which
  // the ordering then uses for first-difference searches
  const bool use_bm = key_bits <= kBmKeyBits && (w.nm + w.nb + w.nh) > 0;
  w.hub_units = 1;
  w.hub_chunk = 0;
  if (use_bm) {
    w.words = std::max<uint32_t>((1u << key_bits) / 32u, 4u);
    bm_.ensure(uint64_t(w.nm + w.nb + w.nh) * w.words * 4);
    bmslot_.ensure(std::max<uint64_t>(N, 1) * 4);
    w.bm = bm_.as<uint32_t>();
    w.bmslot = bmslot_.as<uint32_t>();
    if (w.nh) {
      // hubs in units of at least kHubChunk edges, at most kHubUnits per hub;
      // their bitmaps start at zero
      w.hub_chunk = std::max<uint32_t>(kHubChunk, ceil_div(maxdeg_, kHubUnits));
      w.hub_units = std::max<uint32_t>(1, ceil_div(maxdeg_, w.hub_chunk));
      if (w.hub_units > 1)
        KB_CHECK(hipMemsetAsync(w.bm + uint64_t(w.hub_slot0()) * w.words, 0, uint64_t(w.nh) * w.words * 4, st_));
    }
  } else if (w.nh) {
    // wide keys: all hubs in one device-wide sort by (hub, key) when that
    // fits 64 bits, else one workgroup per hub
    const int hub_bits = bits_for(w.nh > 1 ? w.nh - 1 : 1);
    if (hub_bits + key_bits <= 64 && !streamed_) {  // (the device-wide sort reads every hub's row at once)
      if (hub_bits + key_bits <= 32)
        hub_sort<AdjT, KeyT, uint32_t>(&a, w.hl, w.nh, key_bits);
      else
        hub_sort<AdjT, KeyT, uint64_t>(&a, w.hl, w.nh, key_bits);
      w.nh = 0;
    } else {
      hub_layout();
      hub_tmp_.ensure(std::max<uint64_t>(hub_edges_, 1) * sizeof(KeyT));
      w.hub_tmp = hub_tmp_.p;
      w.hub_toff = hub_toff_.as<uint32_t>();
    }
  }
  if (opt_.profile) {
    if (!work_.p) {
      work_.ensure(kRoundSlots * kWorkWords * sizeof(unsigned long long));
      KB_CHECK(hipMemsetAsync(work_.p, 0, kRoundSlots * kWorkWords * sizeof(unsigned long long), st_));
    }
    const int slot = std::min<int>(rounds_ - round_base_, kRoundSlots - 1);
    work_count_k<<<std::min<uint32_t>(grid_for(M_act_), kProfGrid), kSigNT, 0, st_>>>(
        w.anode, a.rowptr, M_act_, work_.as<unsigned long long>() + kWorkWords * std::max(slot, 0));
    KB_LAUNCH_CHECK();
  }
  const int ev = ev_begin(0);
  if (streamed_) {
    streamed_signature<AdjT, KeyT>(&a, &w);
  } else {
    signature_k<AdjT, KeyT><<<w.grid(), kSigNT, 0, st_>>>(a, w);
    KB_LAUNCH_CHECK();
  }
  if (w.bm && w.nh && w.hub_units > 1) {
    sig_hub_list_k<AdjT, KeyT><<<w.nh, kSigNT, 0, st_>>>(a, w);
    KB_LAUNCH_CHECK();
  }
  ev_end(ev);
  if (opt_.profile) {  // longest signature of the round (unique keys)
    const int slot = std::min<int>(rounds_ - round_base_, kRoundSlots - 1);
    max_ucnt_k<<<std::min<uint32_t>(grid_for(M_act_), kProfGrid), kSigNT, 0, st_>>>(
        w.anode, a.ucnt, M_act_, work_.as<unsigned long long>() + kWorkWords * std::max(slot, 0) + 8);
    KB_LAUNCH_CHECK();
  }

  KeyView<KeyT> kv{rowptr_.as<uint32_t>(), ukey_.as<KeyT>(), ucnt_.as<uint32_t>(), digit_bits};
  if (use_bm) {
    kv.bm = bm_.as<uint64_t>();
    kv.bmslot = bmslot_.as<uint32_t>();
    kv.bm_words64 = w.words / 2;
    kv.bm_min_deg = kWaveMaxDeg;
  }
  const int evo = ev_begin(1);
  order_groups<KeyT>(&kv);
  ev_end(evo);
}

void Engine::run_round() {
  const int64_t B_old = B_;
  const auto t0 = std::chrono::steady_clock::now();
  const int evr = ev_begin(3);
  if (M_act_ > 0) {
    const bool first = rounds_ == 0;
    if (adj64_) {
      if (key64_) round_impl<uint64_t, uint64_t>(first); else round_impl<uint64_t, uint32_t>(first);
    } else {
      if (key64_) round_impl<uint32_t, uint64_t>(first); else round_impl<uint32_t, uint32_t>(first);
    }
    const uint32_t S_old = S_act_;
    const int eva = ev_begin(2);
    assign_round();  // reads back the classes of this round and the next active set
    ev_end(eva);
    const uint32_t C = reinterpret_cast<const uint32_t*>(hw_.p)[kInfoClasses];
    B_ = B_old + int64_t(C) - int64_t(S_old);
  }
  ev_end(evr);
  ++rounds_;
  counts_.push_back(B_);
  fixed_ = (B_ == B_old);
  if (opt_.history) save_level(rounds_);
  ev_collect();
  // host time of the round (it ended with a read-back), for the update's
  // choice between level by level and full rounds
  if (round_secs_.size() <= size_t(rounds_)) round_secs_.resize(size_t(rounds_) + 1, 0.0);
  round_secs_[size_t(rounds_)] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void Engine::work_counts(uint64_t* out8) {
  StreamScope scope(st_);
  for (int i = 0; i < 8; ++i) out8[i] = 0;
  if (!work_.p) return;
  std::vector<uint64_t> all(size_t(kRoundSlots) * kWorkWords);
  KB_CHECK(hipMemcpyAsync(all.data(), work_.p, all.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  for (size_t r = 0; r < size_t(kRoundSlots); ++r)
    for (int i = 0; i < 8; ++i) out8[i] += all[r * kWorkWords + size_t(i)];
}

void Engine::reset_work() {
  if (work_.p) KB_CHECK(hipMemsetAsync(work_.p, 0, kRoundSlots * kWorkWords * sizeof(unsigned long long), st_));
}

std::vector<Engine::RoundStat> Engine::round_stats() {
  StreamScope scope(st_);
  std::vector<RoundStat> out(round_ms_);
  if (out.empty() || !work_.p) return out;
  std::vector<uint64_t> all(size_t(kRoundSlots) * kWorkWords);
  KB_CHECK(hipMemcpyAsync(all.data(), work_.p, all.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  for (size_t r = 0; r < out.size(); ++r) {
    const size_t slot = std::min<size_t>(r, size_t(kRoundSlots) - 1);
    for (int c = 0; c < 4; ++c) {
      out[r].nodes += all[slot * kWorkWords + size_t(2 * c)];
      out[r].edges += all[slot * kWorkWords + size_t(2 * c + 1)];
    }
    out[r].max_keys = all[slot * kWorkWords + 8];
  }
  return out;
}

// The per-round counters restart at the next round (shared with kbisim_work).
void Engine::reset_round_stats() {
  round_ms_.clear();
  round_base_ = rounds_;
  reset_work();
}

void Engine::refine(int32_t k) {
  StreamScope scope(st_);
  k_target_ = std::max(k_target_, k);
  while (rounds_ < k) {
    if (fixed_ && opt_.early_stop) break;
    run_round();
  }
  KB_CHECK(hipStreamSynchronize(st_));
}

const uint32_t* Engine::class_scan() {
  StreamScope scope(st_);
  if (n_ && cls_round_ != rounds_) {
    scan_dev<uint8_t, uint32_t, true>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), uint64_t(n_));
    cls_round_ = rounds_;
  }
  return cls_.as<uint32_t>();
}

const int32_t* Engine::dense_pid() {
  StreamScope scope(st_);
  const uint64_t N = uint64_t(n_);
  dense_.ensure(std::max<uint64_t>(N, 1) * 4);
  if (N && dense_round_ != rounds_) {
    class_scan();
    dense_ids_k<<<grid_for(N), kNT, 0, st_>>>(pid_.as<int32_t>(), cls_.as<uint32_t>(), uint32_t(N),
                                              dense_.as<int32_t>());
    KB_LAUNCH_CHECK();
    dense_round_ = rounds_;
  }
  return dense_.as<int32_t>();
}

void Engine::result(int32_t* pid_out, bool to_device) {
  if (n_ == 0) return;
  const int32_t* d = dense_pid();
  KB_CHECK(hipMemcpyAsync(pid_out, d, uint64_t(n_) * 4, to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          st_));
  KB_CHECK(hipStreamSynchronize(st_));
}


#include "maintain_engine.h"
#include "stream_engine.h"

// ---------------------------------------------------------------------------
// Batched form.

Batch::Batch(int32_t G, const int64_t* node_off, const int64_t* edge_off, const int32_t* label, const int32_t* src,
             const int32_t* lab, const int32_t* dst, bool host_mem, hipStream_t s, const Options& o)
    : G_(G), st_(s), opt_(o) {
  StreamScope scope(s);
  if (G < 1) throw InvalidInput("num_graphs < 1");
  node_off_.assign(node_off, node_off + G + 1);
  edge_off_.assign(edge_off, edge_off + G + 1);
  if (node_off_[0] != 0 || edge_off_[0] != 0) throw InvalidInput("offsets must start at 0");
  for (int32_t g = 0; g < G; ++g)
    if (node_off_[g + 1] < node_off_[g] || edge_off_[g + 1] < edge_off_[g])
      throw InvalidInput("offsets must be non-decreasing");
  ntot_ = node_off_[G];
  etot_ = edge_off_[G];
  if (ntot_ >= (int64_t(1) << 31)) throw InvalidInput("total nodes >= 2^31");
  if (etot_ >= int64_t(0xffffffffll)) throw InvalidInput("total edges >= 2^32 - 1");
  const uint64_t N = uint64_t(ntot_), E = uint64_t(etot_);
  d_node_off_.ensure((G + 1) * 8);
  d_edge_off_.ensure((G + 1) * 8);
  KB_CHECK(hipMemcpyAsync(d_node_off_.p, node_off_.data(), (G + 1) * 8, hipMemcpyHostToDevice, s));
  KB_CHECK(hipMemcpyAsync(d_edge_off_.p, edge_off_.data(), (G + 1) * 8, hipMemcpyHostToDevice, s));
  DevBuf hl, hs, hb, hd;
  if (host_mem) {
    hl.ensure(std::max<uint64_t>(N, 1) * 4);
    hs.ensure(std::max<uint64_t>(E, 1) * 4);
    hb.ensure(std::max<uint64_t>(E, 1) * 4);
    hd.ensure(std::max<uint64_t>(E, 1) * 4);
    if (N) KB_CHECK(hipMemcpyAsync(hl.p, label, N * 4, hipMemcpyHostToDevice, s));
    if (E) {
      KB_CHECK(hipMemcpyAsync(hs.p, src, E * 4, hipMemcpyHostToDevice, s));
      KB_CHECK(hipMemcpyAsync(hb.p, lab, E * 4, hipMemcpyHostToDevice, s));
      KB_CHECK(hipMemcpyAsync(hd.p, dst, E * 4, hipMemcpyHostToDevice, s));
    }
    label = hl.as<int32_t>();
    src = hs.as<int32_t>();
    lab = hb.as<int32_t>();
    dst = hd.as<int32_t>();
  }
  // union endpoints and graph-major node labels
  DevBuf usrc, udst, glabel, err;
  usrc.ensure(std::max<uint64_t>(E, 1) * 4);
  udst.ensure(std::max<uint64_t>(E, 1) * 4);
  glabel.ensure(std::max<uint64_t>(N, 1) * 4);
  // err word, largest node label, label mask (unused here)
  constexpr size_t kErrBytes = 16 + 4 * sizeof(uint64_t);
  err.ensure(kErrBytes);
  KB_CHECK(hipMemsetAsync(err.p, 0, kErrBytes, s));
  uint32_t* errw = err.as<uint32_t>();
  if (E) {
    union_edges_k<<<ceil_div(E, kUnionTile), 256, 0, s>>>(src, dst, E, d_node_off_.as<int64_t>(),
                                                          d_edge_off_.as<int64_t>(), uint32_t(G), usrc.as<int32_t>(),
                                                          udst.as<int32_t>(), errw);
    KB_LAUNCH_CHECK();
  }
  if (N) {
    validate_nodes_k<<<std::max<uint32_t>(1, std::min<uint32_t>(ceil_div(N, 256), 2048)), kRadixNT, 0, s>>>(
        label, N, errw, errw + 1, reinterpret_cast<unsigned long long*>(err.as<uint8_t>() + 16));
    KB_LAUNCH_CHECK();
  }
  uint32_t ew[2] = {0, 0};
  KB_CHECK(hipMemcpyAsync(ew, err.p, 8, hipMemcpyDeviceToHost, s));
  KB_CHECK(hipStreamSynchronize(s));
  if (ew[0] & 1u) throw InvalidInput("edge endpoint outside its graph's node range");
  if (ew[0] & 4u) throw InvalidInput("negative node label");
  if (N) {
    // union label (g << lbits) | label when that stays below 2^31; else the
    // dense rank of (graph, label) through a sort
    const int lbits = bits_for(ew[1] > 0 ? ew[1] : 1);
    const int gbits = bits_for(G > 1 ? uint64_t(G - 1) : 1);
    if (lbits + gbits <= 31) {
      union_labels_k<<<ceil_div(N, kUnionTile), 256, 0, s>>>(label, N, d_node_off_.as<int64_t>(), uint32_t(G), lbits,
                                                             glabel.as<int32_t>());
      KB_LAUNCH_CHECK();
    } else {
      DevBuf k0, k1, i0, i1, fl, cl, scratch, part;
      k0.ensure(N * 8);
      k1.ensure(N * 8);
      for (DevBuf* b : {&i0, &i1, &fl, &cl}) b->ensure(N * 4);
      union_node_keys_k<<<ceil_div(N, 256), 256, 0, s>>>(label, N, d_node_off_.as<int64_t>(), uint32_t(G),
                                                          k0.as<uint64_t>(), i0.as<uint32_t>());
      KB_LAUNCH_CHECK();
      scratch.ensure(radix_scratch_words(N) * 4);
      const bool f = radix_sort<uint64_t>(k0.as<uint64_t>(), i0.as<uint32_t>(), k1.as<uint64_t>(), i1.as<uint32_t>(),
                                          N, 0, 31 + gbits, scratch.as<uint32_t>(), s);
      const uint64_t* K = f ? k1.as<uint64_t>() : k0.as<uint64_t>();
      const uint32_t* I = f ? i1.as<uint32_t>() : i0.as<uint32_t>();
      u64_run_flags_k<<<ceil_div(N, 256), 256, 0, s>>>(K, uint32_t(N), fl.as<uint32_t>());
      KB_LAUNCH_CHECK();
      part.ensure(scan_partials_count(N) * 4);
      scan<uint32_t, uint32_t, true>(fl.as<uint32_t>(), cl.as<uint32_t>(), N, part.as<uint32_t>(), s);
      scatter_rank_k<<<ceil_div(N, 256), 256, 0, s>>>(I, cl.as<uint32_t>(), uint32_t(N), glabel.as<int32_t>());
      KB_LAUNCH_CHECK();
    }
  }
  eng_ = new Engine(ntot_, etot_, s, o);
  try {
    eng_->build(glabel.as<int32_t>(), usrc.as<int32_t>(), lab, udst.as<int32_t>());
  } catch (...) {
    delete eng_;
    eng_ = nullptr;
    throw;
  }
  out_.ensure(std::max<uint64_t>(N, 1) * 4);
  base_.ensure(uint64_t(G) * 4);
  cnt_.ensure(uint64_t(G) * 4);
  take_.ensure(uint64_t(G));
  read_counts(prev_);
  blocks_ = prev_;
  rounds_.assign(G, 0);
  done_.assign(G, 0);
}

Batch::~Batch() { delete eng_; }

void Batch::read_counts(std::vector<int32_t>& cnt) {
  cnt.assign(G_, 0);
  graph_id_range_k<<<ceil_div(uint64_t(G_), 256), 256, 0, st_>>>(eng_->class_scan(), d_node_off_.as<int64_t>(),
                                                                 uint32_t(G_), base_.as<int32_t>(),
                                                                 cnt_.as<int32_t>());
  KB_LAUNCH_CHECK();
  KB_CHECK(hipMemcpyAsync(cnt.data(), cnt_.p, uint64_t(G_) * 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
}

void Batch::take_snapshot(const std::vector<uint8_t>& take) {
  if (ntot_ == 0) return;
  KB_CHECK(hipMemcpyAsync(take_.p, take.data(), uint64_t(G_), hipMemcpyHostToDevice, st_));
  snapshot_k<<<ceil_div(uint64_t(ntot_), kUnionTile), 256, 0, st_>>>(eng_->dense_pid(), uint64_t(ntot_), d_node_off_.as<int64_t>(), uint32_t(G_),
                                   base_.as<int32_t>(), take_.as<uint8_t>(), out_.as<int32_t>());
  KB_LAUNCH_CHECK();
  KB_CHECK(hipStreamSynchronize(st_));  // `take` is a host vector the caller may change
}

void Batch::refine(const std::vector<int32_t>& k) {
  StreamScope scope(st_);
  if (refined_) throw StateError("batch already refined");
  k_ = k;
  std::vector<uint8_t> take(G_, 0);
  bool any = false, open = false;
  for (int32_t g = 0; g < G_; ++g) {
    if (k_[g] == 0) {
      take[g] = 1;
      done_[g] = 1;
      any = true;
    } else {
      open = true;
    }
  }
  if (any) take_snapshot(take);
  std::vector<int32_t> cur;
  for (int32_t i = 1; open; ++i) {
    eng_->step_round();
    read_counts(cur);
    std::fill(take.begin(), take.end(), 0);
    any = false;
    open = false;
    for (int32_t g = 0; g < G_; ++g) {
      if (done_[g]) continue;
      blocks_[g] = cur[g];
      if ((opt_.early_stop && cur[g] == prev_[g]) || i == k_[g]) {
        rounds_[g] = i;
        done_[g] = 1;
        take[g] = 1;
        any = true;
      } else {
        open = true;
      }
    }
    prev_ = cur;
    if (any) take_snapshot(take);
  }
  refined_ = true;
}

void Batch::result(int32_t* pid_out, bool to_device, int64_t* blocks, int32_t* rounds) const {
  if (!refined_) throw StateError("batch not refined yet");
  if (pid_out && ntot_) {
    KB_CHECK(hipMemcpyAsync(pid_out, out_.p, uint64_t(ntot_) * 4,
                            to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
  }
  for (int32_t g = 0; g < G_; ++g) {
    if (blocks) blocks[g] = blocks_[g];
    if (rounds) rounds[g] = rounds_[g];
  }
}


// ---------------------------------------------------------------------------
// Served form.

struct Cancelled : std::runtime_error {
  Cancelled() : std::runtime_error("cancelled") {}
};

Server::Server(uint64_t budget, int32_t slots, const Options& o) : budget_(budget), slots_(slots), opt_(o) {
  KB_CHECK(hipGetDevice(&device_));
  for (int32_t i = 0; i < slots; ++i) {
    hipStream_t s = nullptr;
    KB_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));  // default priority
    streams_.push_back(s);
  }
  for (int32_t i = 0; i < slots; ++i) threads_.emplace_back(&Server::worker, this, int(i));
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
    for (auto& r : queue_) {
      r->state = Request::kCancelled;
      if (r->ready) (void)hipEventDestroy(r->ready);
      r->ready = nullptr;
    }
    queue_.clear();
    for (auto& kv : all_)
      if (kv.second->state == Request::kRunning) kv.second->cancel = true;
  }
  cv_work_.notify_all();
  cv_done_.notify_all();
  for (auto& t : threads_) t.join();
  for (auto s : streams_) (void)hipStreamDestroy(s);
}

uint64_t Server::submit(const int32_t* label, const int32_t* src, const int32_t* lab, const int32_t* dst, int64_t n,
                        int64_t m, bool device_inputs, int32_t k, hipStream_t caller) {
  auto r = std::make_shared<Request>();
  r->k = k;
  r->n = n;
  r->m = m;
  r->device_inputs = device_inputs;
  r->footprint = job_footprint(uint64_t(n), uint64_t(m));
  if (r->footprint > budget_)
    throw OutOfMemory("request needs about " + std::to_string(r->footprint) + " device bytes; budget is " +
                      std::to_string(budget_));
  if (device_inputs) {
    r->dev[0] = label;
    r->dev[1] = src;
    r->dev[2] = lab;
    r->dev[3] = dst;
    // the caller's kernels that write the inputs may still be in flight:
    // the worker's stream waits for this point of the caller's stream
    KB_CHECK(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
    const hipError_t e = hipEventRecord(r->ready, caller);
    if (e != hipSuccess) {
      (void)hipEventDestroy(r->ready);
      r->ready = nullptr;
      KB_CHECK(e);
    }
  } else {
    r->host[0].assign(label, label + n);
    r->host[1].assign(src, src + m);
    r->host[2].assign(lab, lab + m);
    r->host[3].assign(dst, dst + m);
  }
  r->t_submit = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> lk(mu_);
  if (stop_) {
    if (r->ready) (void)hipEventDestroy(r->ready);
    throw StateError("server is shutting down");
  }
  r->id = next_id_++;
  all_[r->id] = r;
  queue_.push_back(r);
  cv_work_.notify_all();
  return r->id;
}

void Server::worker(int slot) {
  (void)hipSetDevice(device_);
  hipStream_t s = streams_[size_t(slot)];
  for (;;) {
    std::vector<std::shared_ptr<Request>> group;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] {
        return stop_ || (!queue_.empty() && in_use_ + queue_.front()->footprint <= budget_);
      });
      if (stop_) return;
      group.push_back(queue_.front());
      queue_.pop_front();
      in_use_ += group[0]->footprint;
      // small requests right behind a small head join it
      int64_t edges = group[0]->m;
      while (group[0]->m <= kServeSmallEdges && !queue_.empty() && group.size() < kServeGroupMax) {
        const std::shared_ptr<Request>& q = queue_.front();
        if (q->m > kServeSmallEdges || edges + q->m > kServeGroupEdges || in_use_ + q->footprint > budget_) break;
        edges += q->m;
        in_use_ += q->footprint;
        group.push_back(q);
        queue_.pop_front();
      }
      const auto now = std::chrono::steady_clock::now();
      for (auto& r : group) {
        r->state = Request::kRunning;
        r->t_start = now;
      }
    }
    bool alone = group.size() == 1;
    if (!alone) {
      try {
        alone = !run_group(group, s);
      } catch (const std::exception& e) {
        for (auto& r : group) finish(*r, KBISIM_EDEVICE, e.what(), false);
        continue;
      }
      if (!alone) continue;
    }
    for (auto& r : group) {  // one at a time (also after a rejected union)
      int status = 0;
      std::string err;
      bool cancelled = false;
      try {
        run(*r, s);
      } catch (const Cancelled&) {
        cancelled = true;
      } catch (const InvalidInput& e) {
        status = KBISIM_EINVAL;
        err = e.what();
      } catch (const OutOfMemory& e) {
        status = KBISIM_ENOMEM;
        err = e.what();
      } catch (const std::exception& e) {
        status = KBISIM_EDEVICE;
        err = e.what();
      }
      finish(*r, status, err, cancelled);
    }
  }
}

void Server::finish(Request& r, int status, const std::string& err, bool cancelled) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    in_use_ -= r.footprint;
    r.t_end = std::chrono::steady_clock::now();
    r.status = status;
    r.error = err;
    r.state = cancelled ? Request::kCancelled : status ? Request::kFailed : Request::kDone;
    for (auto& h : r.host) std::vector<int32_t>().swap(h);  // inputs no longer needed
    if (r.ready) {
      (void)hipEventDestroy(r.ready);
      r.ready = nullptr;
    }
  }
  cv_done_.notify_all();
  cv_work_.notify_all();  // memory came back: the queue head may fit now
}

bool Server::run_group(std::vector<std::shared_ptr<Request>>& group, hipStream_t s) {
  StreamScope scope(s);
  const int32_t G = int32_t(group.size());
  std::vector<int64_t> noff(G + 1, 0), eoff(G + 1, 0);
  std::vector<int32_t> ks(G);
  for (int32_t g = 0; g < G; ++g) {
    noff[g + 1] = noff[g] + group[g]->n;
    eoff[g + 1] = eoff[g] + group[g]->m;
    ks[g] = group[g]->k;
  }
  const uint64_t N = uint64_t(noff[G]), E = uint64_t(eoff[G]);
  // the requests' inputs, concatenated in device memory (graph-local ids)
  DevBuf cat[4];
  const uint64_t tot[4] = {N, E, E, E};
  for (int i = 0; i < 4; ++i) cat[i].ensure(std::max<uint64_t>(tot[i], 1) * 4);
  for (int32_t g = 0; g < G; ++g) {
    Request& r = *group[g];
    const uint64_t len[4] = {uint64_t(r.n), uint64_t(r.m), uint64_t(r.m), uint64_t(r.m)};
    const uint64_t at[4] = {uint64_t(noff[g]), uint64_t(eoff[g]), uint64_t(eoff[g]), uint64_t(eoff[g])};
    if (r.device_inputs) KB_CHECK(hipStreamWaitEvent(s, r.ready, 0));
    for (int i = 0; i < 4; ++i) {
      if (!len[i]) continue;
      int32_t* to = cat[i].as<int32_t>() + at[i];
      if (r.device_inputs)
        KB_CHECK(hipMemcpyAsync(to, r.dev[i], len[i] * 4, hipMemcpyDeviceToDevice, s));
      else
        KB_CHECK(hipMemcpyAsync(to, r.host[i].data(), len[i] * 4, hipMemcpyHostToDevice, s));
    }
  }
  std::unique_ptr<Batch> b;
  try {
    b.reset(new Batch(G, noff.data(), eoff.data(), cat[0].as<int32_t>(), cat[1].as<int32_t>(),
                      cat[2].as<int32_t>(), cat[3].as<int32_t>(), false, s, opt_));
  } catch (const InvalidInput&) {
    KB_CHECK(hipStreamSynchronize(s));  // the copies out of the requests' inputs are done
    return false;
  }
  b->refine(ks);
  std::vector<int32_t> pid(std::max<uint64_t>(N, 1));
  std::vector<int64_t> blocks(G);
  std::vector<int32_t> rounds(G);
  b->result(N ? pid.data() : nullptr, false, blocks.data(), rounds.data());
  for (int32_t g = 0; g < G; ++g) {
    Request& r = *group[g];
    r.pid.assign(pid.begin() + noff[g], pid.begin() + noff[g + 1]);
    r.counts.assign(1, blocks[g]);
    r.rounds = rounds[g];
    bool cancelled;
    {
      std::lock_guard<std::mutex> lk(mu_);
      cancelled = r.cancel;
    }
    finish(r, 0, std::string(), cancelled);
  }
  return true;
}

void Server::run(Request& r, hipStream_t s) {
  StreamScope scope(s);
  Engine eng(r.n, r.m, s, opt_);
  if (r.device_inputs) {
    KB_CHECK(hipStreamWaitEvent(s, r.ready, 0));
    eng.build(r.dev[0], r.dev[1], r.dev[2], r.dev[3]);
  } else {
    DevBuf b[4];
    const uint64_t len[4] = {uint64_t(r.n), uint64_t(r.m), uint64_t(r.m), uint64_t(r.m)};
    const int32_t* p[4];
    for (int i = 0; i < 4; ++i) {
      b[i].ensure(std::max<uint64_t>(len[i], 1) * 4);
      if (len[i]) KB_CHECK(hipMemcpyAsync(b[i].p, r.host[i].data(), len[i] * 4, hipMemcpyHostToDevice, s));
      p[i] = b[i].as<int32_t>();
    }
    eng.build(p[0], p[1], p[2], p[3]);
  }
  while (eng.rounds_done() < r.k && !(eng.fixed() && opt_.early_stop)) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (r.cancel) throw Cancelled();
    }
    eng.step_round();
  }
  r.pid.resize(size_t(r.n));
  if (r.n) eng.result(r.pid.data(), false);
  r.counts = eng.counts();
  r.rounds = eng.rounds_done();
}

int Server::wait(uint64_t id, int32_t* pid_out, bool to_device, int64_t* num_blocks, int32_t* rounds,
                 double timeout_s, std::string* err) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end()) return KBISIM_EINVAL;
  std::shared_ptr<Request> r = it->second;
  auto finished = [&] {
    return r->state == Request::kDone || r->state == Request::kFailed || r->state == Request::kCancelled;
  };
  if (timeout_s < 0) {
    cv_done_.wait(lk, finished);
  } else if (!cv_done_.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
    return KBISIM_ETIMEDOUT;
  }
  if (r->state == Request::kCancelled) return KBISIM_ECANCELED;
  if (r->state == Request::kFailed) {
    if (err) *err = r->error;
    return r->status;
  }
  lk.unlock();  // a done request is not modified any more
  if (pid_out && r->n) {
    if (to_device)
      KB_CHECK(hipMemcpy(pid_out, r->pid.data(), size_t(r->n) * 4, hipMemcpyHostToDevice));
    else
      std::memcpy(pid_out, r->pid.data(), size_t(r->n) * 4);
  }
  if (num_blocks) *num_blocks = r->counts.empty() ? 0 : r->counts.back();
  if (rounds) *rounds = r->rounds;
  return KBISIM_OK;
}

int Server::cancel(uint64_t id) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end()) return KBISIM_EINVAL;
  Request& r = *it->second;
  if (r.state == Request::kQueued) {
    for (auto q = queue_.begin(); q != queue_.end(); ++q)
      if ((*q)->id == id) {
        queue_.erase(q);
        break;
      }
    r.state = Request::kCancelled;
    if (r.ready) (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
    cv_done_.notify_all();
    cv_work_.notify_all();
    return KBISIM_OK;
  }
  if (r.state == Request::kRunning) {
    r.cancel = true;
    return KBISIM_OK;
  }
  return KBISIM_ESTATE;  // already finished
}

int Server::state(uint64_t id, int32_t* st) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end()) return KBISIM_EINVAL;
  switch (it->second->state) {
    case Request::kQueued: *st = KBISIM_REQ_QUEUED; break;
    case Request::kRunning: *st = KBISIM_REQ_RUNNING; break;
    case Request::kDone: *st = KBISIM_REQ_DONE; break;
    case Request::kFailed: *st = KBISIM_REQ_FAILED; break;
    case Request::kCancelled: *st = KBISIM_REQ_CANCELLED; break;
  }
  return KBISIM_OK;
}

bool Server::timing(uint64_t id, double* queued_s, double* total_s) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end() || it->second->state != Request::kDone) return false;
  const Request& r = *it->second;
  if (queued_s) *queued_s = std::chrono::duration<double>(r.t_start - r.t_submit).count();
  if (total_s) *total_s = std::chrono::duration<double>(r.t_end - r.t_submit).count();
  return true;
}

void Server::release(uint64_t id) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end()) return;
  const auto st = it->second->state;
  if (st == Request::kDone || st == Request::kFailed || st == Request::kCancelled) all_.erase(it);
}

}  // namespace kb

// ===========================================================================
// C ABI

// The static scratch region of the allocation-free entry point: one copy per
// GPU the library runs on, held until the process ends. Host code never uses
// the symbol itself (a host-side stand-in): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[KBISIM_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_busy[kMaxDevices];  // one job at a time per device uses the region

int current_device() {
  int dev = 0;
  KB_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw kb::DeviceError(hipErrorInvalidDevice, "device index out of range");
  return dev;
}

// Device address of this device's scratch region (looked up on first use).
void* scratch_region(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    KB_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw kb::DeviceError(hipErrorInvalidSymbol, "no device address for the scratch region");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Upper bound on the region a job of n nodes and m edges may need (all its
// buffers at their peak, with room for the first-fit arena's fragmentation).
uint64_t static_footprint(uint64_t n, uint64_t m) { return 48 * m + 256 * n + (uint64_t(1) << 20); }
}  // namespace

struct kbisim_graph {
  kb::Engine* eng = nullptr;
};

struct kbisim_batch {
  kb::Batch* b = nullptr;
};

struct kbisim_server {
  kb::Server* s = nullptr;
};

namespace {
thread_local std::string g_last_error;

template <typename F>
kbisim_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const kb::InvalidInput& e) {
    g_last_error = e.what();
    return KBISIM_EINVAL;
  } catch (const kb::StateError& e) {
    g_last_error = e.what();
    return KBISIM_ESTATE;
  } catch (const kb::OutOfMemory& e) {
    g_last_error = e.what();
    return KBISIM_ENOMEM;
  } catch (const kb::DeviceError& e) {
    g_last_error = e.what();
    return KBISIM_EDEVICE;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return KBISIM_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return KBISIM_EDEVICE;
  }
}

kbisim_status fail(kbisim_status s, const char* msg) {
  g_last_error = msg;
  return s;
}
}  // namespace

extern "C" {

void kbisim_options_default(kbisim_options* opt) {
  if (!opt) return;
  opt->early_stop = 1;
  opt->profile = 0;
  opt->medium_cap = int32_t(kb::kDefaultMediumCap);
  opt->history = 0;
  opt->update_mode = 0;
  opt->radix_tile = 0;
  opt->edge_window_bytes = 0;
}

static kbisim_status parse_options(const kbisim_options* opt, kb::Options* o) {
  if (!opt) return KBISIM_OK;
  o->early_stop = opt->early_stop != 0;
  o->profile = opt->profile != 0;
  if (opt->medium_cap < 0 || opt->medium_cap > int32_t(kb::kBigCap))
    return fail(KBISIM_EINVAL, "medium_cap outside [0, 4096]");
  if (opt->medium_cap > 0) o->medium_cap = uint32_t(opt->medium_cap);
  if (opt->radix_tile < 0 || !kb::radix_tile_valid(uint32_t(opt->radix_tile)))
    return fail(KBISIM_EINVAL, "radix_tile not 0, 2048, 3072 or 4096");
  o->radix_tile = uint32_t(opt->radix_tile);
  o->history = opt->history != 0;
  if (opt->update_mode < 0 || opt->update_mode > 2) return fail(KBISIM_EINVAL, "update_mode outside [0, 2]");
  o->update_mode = opt->update_mode;
  if (opt->edge_window_bytes < 0) return fail(KBISIM_EINVAL, "edge_window_bytes < 0");
  o->edge_window = uint64_t(opt->edge_window_bytes);
  return KBISIM_OK;
}

kbisim_status kbisim_create(const kbisim_graph_desc* d, const kbisim_options* opt, kbisim_graph** out) {
  if (!d || !out) return fail(KBISIM_EINVAL, "null desc or out");
  if (d->num_nodes < 0 || d->num_edges < 0) return fail(KBISIM_EINVAL, "negative size");
  if (d->num_nodes >= (int64_t(1) << 31)) return fail(KBISIM_EINVAL, "num_nodes >= 2^31");
  if (d->num_edges >= int64_t(0xffffffffll)) return fail(KBISIM_EINVAL, "num_edges >= 2^32 - 1");
  if (d->num_nodes > 0 && !d->node_label) return fail(KBISIM_EINVAL, "null node_label");
  if (d->num_edges > 0 && (!d->edge_src || !d->edge_label || !d->edge_dst))
    return fail(KBISIM_EINVAL, "null edge array");
  if (d->mem != KBISIM_MEM_HOST && d->mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  kb::Options o;
  if (parse_options(opt, &o) != KBISIM_OK) return KBISIM_EINVAL;
  if (o.edge_window > 0 && d->mem != KBISIM_MEM_HOST)
    return fail(KBISIM_EINVAL, "edge_window_bytes needs the edge table in host memory (KBISIM_MEM_HOST)");
  if (o.edge_window > 0 && o.history) return fail(KBISIM_EINVAL, "edge_window_bytes with history = 1");
  return guarded([&]() {
    hipStream_t s = static_cast<hipStream_t>(d->stream);
    kb::StreamScope scope(s);
    auto* eng = new kb::Engine(d->num_nodes, d->num_edges, s, o);
    try {
      const uint64_t N = uint64_t(d->num_nodes), E = uint64_t(d->num_edges);
      if (o.edge_window > 0) {
        kb::DevBuf nl;
        nl.ensure(std::max<uint64_t>(N, 1) * 4);
        if (N) KB_CHECK(hipMemcpyAsync(nl.p, d->node_label, N * 4, hipMemcpyHostToDevice, s));
        eng->build_streamed(nl.as<int32_t>(), d->edge_src, d->edge_label, d->edge_dst);
      } else if (d->mem == KBISIM_MEM_HOST) {
        kb::DevBuf nl, sr, lb, ds;
        nl.ensure(std::max<uint64_t>(N, 1) * 4);
        sr.ensure(std::max<uint64_t>(E, 1) * 4);
        lb.ensure(std::max<uint64_t>(E, 1) * 4);
        ds.ensure(std::max<uint64_t>(E, 1) * 4);
        if (N) KB_CHECK(hipMemcpyAsync(nl.p, d->node_label, N * 4, hipMemcpyHostToDevice, s));
        if (E) {
          KB_CHECK(hipMemcpyAsync(sr.p, d->edge_src, E * 4, hipMemcpyHostToDevice, s));
          KB_CHECK(hipMemcpyAsync(lb.p, d->edge_label, E * 4, hipMemcpyHostToDevice, s));
          KB_CHECK(hipMemcpyAsync(ds.p, d->edge_dst, E * 4, hipMemcpyHostToDevice, s));
        }
        eng->build(nl.as<int32_t>(), sr.as<int32_t>(), lb.as<int32_t>(), ds.as<int32_t>());
      } else {
        eng->build(d->node_label, d->edge_src, d->edge_label, d->edge_dst);
      }
    } catch (...) {
      delete eng;
      throw;
    }
    auto* h = new kbisim_graph;
    h->eng = eng;
    *out = h;
    return KBISIM_OK;
  });
}

kbisim_status kbisim_refine_static(const kbisim_graph_desc* d, int32_t k, const kbisim_options* opt,
                                   int32_t* pid_out, kbisim_mem out_mem, int64_t* num_blocks,
                                   int32_t* rounds_done) {
  if (!d) return fail(KBISIM_EINVAL, "null desc");
  if (d->num_nodes < 0 || d->num_edges < 0) return fail(KBISIM_EINVAL, "negative size");
  if (k < 0) return fail(KBISIM_EINVAL, "k < 0");
  if (d->num_nodes > 0 && !d->node_label) return fail(KBISIM_EINVAL, "null node_label");
  if (d->num_edges > 0 && (!d->edge_src || !d->edge_label || !d->edge_dst))
    return fail(KBISIM_EINVAL, "null edge array");
  if (d->num_nodes > 0 && !pid_out) return fail(KBISIM_EINVAL, "null pid_out");
  if (d->mem != KBISIM_MEM_HOST && d->mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  if (out_mem != KBISIM_MEM_HOST && out_mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad output mem kind");
  if (d->num_nodes >= (int64_t(1) << 31) || d->num_edges >= int64_t(0xffffffffll) ||
      static_footprint(uint64_t(d->num_nodes), uint64_t(d->num_edges)) > uint64_t(KBISIM_STATIC_SCRATCH_BYTES))
    return fail(KBISIM_ENOMEM, "graph too large for the static scratch region (KBISIM_STATIC_SCRATCH_BYTES)");
  kb::Options o;
  if (parse_options(opt, &o) != KBISIM_OK) return KBISIM_EINVAL;
  if (o.edge_window > 0) return fail(KBISIM_EINVAL, "edge_window_bytes applies to kbisim_create only");
  o.profile = false;
  o.history = false;
  return guarded([&]() {
    const int dev = current_device();
    void* region = scratch_region(dev);
    std::lock_guard<std::mutex> busy(g_scratch_busy[dev]);
    hipStream_t s = static_cast<hipStream_t>(d->stream);
    kb::Arena arena(region, KBISIM_STATIC_SCRATCH_BYTES);
    kb::ArenaScope as(&arena);
    kb::StreamScope scope(s);
    const uint64_t N = uint64_t(d->num_nodes), E = uint64_t(d->num_edges);
    kb::Engine eng(d->num_nodes, d->num_edges, s, o);
    if (d->mem == KBISIM_MEM_HOST) {
      kb::DevBuf b[4];
      const uint64_t len[4] = {N, E, E, E};
      const int32_t* src[4] = {d->node_label, d->edge_src, d->edge_label, d->edge_dst};
      for (int i = 0; i < 4; ++i) {
        b[i].ensure(std::max<uint64_t>(len[i], 1) * 4);
        if (len[i]) KB_CHECK(hipMemcpyAsync(b[i].p, src[i], len[i] * 4, hipMemcpyHostToDevice, s));
      }
      eng.build(b[0].as<int32_t>(), b[1].as<int32_t>(), b[2].as<int32_t>(), b[3].as<int32_t>());
    } else {
      eng.build(d->node_label, d->edge_src, d->edge_label, d->edge_dst);
    }
    eng.refine(k);
    if (N) eng.result(pid_out, out_mem == KBISIM_MEM_DEVICE);
    if (num_blocks) *num_blocks = eng.blocks();
    if (rounds_done) *rounds_done = eng.rounds_done();
    return KBISIM_OK;
  });
}

kbisim_status kbisim_refine(kbisim_graph* g, int32_t k, int32_t* rounds_done) {
  if (!g || !g->eng) return fail(KBISIM_EINVAL, "null handle");
  if (k < 0) return fail(KBISIM_EINVAL, "k < 0");
  return guarded([&]() {
    g->eng->refine(k);
    if (rounds_done) *rounds_done = g->eng->rounds_done();
    return KBISIM_OK;
  });
}

kbisim_status kbisim_result(const kbisim_graph* g, int32_t* pid_out, kbisim_mem mem, int64_t* num_blocks,
                            int64_t* counts, int32_t counts_cap) {
  if (!g || !g->eng) return fail(KBISIM_EINVAL, "null handle");
  if (mem != KBISIM_MEM_HOST && mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  if (counts && counts_cap < 0) return fail(KBISIM_EINVAL, "negative counts_cap");
  return guarded([&]() {
    if (pid_out) g->eng->result(pid_out, mem == KBISIM_MEM_DEVICE);
    if (num_blocks) *num_blocks = g->eng->blocks();
    if (counts) {
      const auto& c = g->eng->counts();
      const size_t nc = std::min<size_t>(c.size(), size_t(counts_cap));
      for (size_t i = 0; i < nc; ++i) counts[i] = c[i];
    }
    return KBISIM_OK;
  });
}

kbisim_status kbisim_result_round(const kbisim_graph* g, int32_t round, int32_t* pid_out, kbisim_mem mem,
                                  int64_t* num_blocks) {
  if (!g || !g->eng) return fail(KBISIM_EINVAL, "null handle");
  if (mem != KBISIM_MEM_HOST && mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  if (round < 0) return fail(KBISIM_EINVAL, "round < 0");
  return guarded([&]() {
    int64_t b = 0;
    g->eng->result_round(round, pid_out, mem == KBISIM_MEM_DEVICE, &b);
    if (num_blocks) *num_blocks = b;
    return KBISIM_OK;
  });
}

kbisim_status kbisim_update(kbisim_graph* g, const kbisim_update_desc* u, int32_t* rounds_done) {
  if (!g || !g->eng || !u) return fail(KBISIM_EINVAL, "null argument");
  if (u->num_new_nodes < 0 || u->num_del_edges < 0 || u->num_add_edges < 0 || u->num_del_nodes < 0)
    return fail(KBISIM_EINVAL, "negative size");
  if (u->num_del_nodes > 0 && !u->del_nodes) return fail(KBISIM_EINVAL, "null del_nodes");
  if (u->num_new_nodes > 0 && !u->new_node_label) return fail(KBISIM_EINVAL, "null new_node_label");
  if (u->num_del_edges > 0 && (!u->del_src || !u->del_label || !u->del_dst))
    return fail(KBISIM_EINVAL, "null deleted edge array");
  if (u->num_add_edges > 0 && (!u->add_src || !u->add_label || !u->add_dst))
    return fail(KBISIM_EINVAL, "null added edge array");
  if (u->mem != KBISIM_MEM_HOST && u->mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  if (u->num_new_nodes >= (int64_t(1) << 31) || u->num_add_edges >= int64_t(0xffffffffll) ||
      u->num_del_edges >= int64_t(0xffffffffll))
    return fail(KBISIM_EINVAL, "update too large");
  if (!g->eng->history()) return fail(KBISIM_ESTATE, "updates need options.history = 1");
  return guarded([&]() {
    kb::StreamScope scope(g->eng->stream());
    kb::UpdateArgs a;
    a.n_new = u->num_new_nodes;
    a.m_del = u->num_del_edges;
    a.m_add = u->num_add_edges;
    a.n_del = u->num_del_nodes;
    kb::DevBuf b[8];
    if (u->mem == KBISIM_MEM_HOST) {
      const int32_t* src[8] = {u->new_node_label, u->del_src, u->del_label, u->del_dst,
                               u->add_src, u->add_label, u->add_dst, u->del_nodes};
      const uint64_t len[8] = {uint64_t(a.n_new), uint64_t(a.m_del), uint64_t(a.m_del), uint64_t(a.m_del),
                               uint64_t(a.m_add), uint64_t(a.m_add), uint64_t(a.m_add), uint64_t(a.n_del)};
      const int32_t* dev[8];
      for (int i = 0; i < 8; ++i) {
        b[i].ensure(std::max<uint64_t>(len[i], 1) * 4);
        if (len[i])
          KB_CHECK(hipMemcpyAsync(b[i].p, src[i], len[i] * 4, hipMemcpyHostToDevice, g->eng->stream()));
        dev[i] = b[i].as<int32_t>();
      }
      a.new_label = dev[0];
      a.del_src = dev[1];
      a.del_lab = dev[2];
      a.del_dst = dev[3];
      a.add_src = dev[4];
      a.add_lab = dev[5];
      a.add_dst = dev[6];
      a.del_nodes = dev[7];
    } else {
      a.del_nodes = u->del_nodes;
      a.new_label = u->new_node_label;
      a.del_src = u->del_src;
      a.del_lab = u->del_label;
      a.del_dst = u->del_dst;
      a.add_src = u->add_src;
      a.add_lab = u->add_label;
      a.add_dst = u->add_dst;
    }
    g->eng->update(a);
    if (rounds_done) *rounds_done = g->eng->rounds_done();
    return KBISIM_OK;
  });
}

kbisim_status kbisim_stream_stats(const kbisim_graph* g, int64_t* partitions, int64_t* bytes_moved,
                                  int32_t* direct_rounds) {
  if (!g) return fail(KBISIM_EINVAL, "null handle");
  g->eng->stream_stats(partitions, bytes_moved, direct_rounds);
  return KBISIM_OK;
}

kbisim_status kbisim_update_stats(const kbisim_graph* g, int64_t* levels, int64_t* full_from, int64_t* rechecked,
                                  int64_t* recomputed, int64_t* changed) {
  if (!g || !g->eng) return fail(KBISIM_EINVAL, "null handle");
  const kb::UpdateStat& s = g->eng->update_stat();
  if (levels) *levels = s.levels;
  if (full_from) *full_from = s.full_from;
  if (rechecked) *rechecked = int64_t(s.rechecked);
  if (recomputed) *recomputed = int64_t(s.recomputed);
  if (changed) *changed = int64_t(s.changed);
  return KBISIM_OK;
}

kbisim_status kbisim_profile(const kbisim_graph* g, double* ms, int64_t* launches, int32_t cap,
                             int32_t reset) {
  if (!g || !g->eng) return fail(KBISIM_EINVAL, "null handle");
  if (cap < 0) return fail(KBISIM_EINVAL, "negative cap");
  const int n = std::min<int>(cap, kb::kProfClasses);
  for (int i = 0; i < n; ++i) {
    if (ms) ms[i] = g->eng->prof_ms[i];
    if (launches) launches[i] = g->eng->prof_n[i];
  }
  if (reset) {
    g->eng->prof_ms.fill(0.0);
    g->eng->prof_n.fill(0);
  }
  return KBISIM_OK;
}

kbisim_status kbisim_round_profile(const kbisim_graph* g, kbisim_round_stat* stats, int32_t cap, int32_t* n,
                                   int32_t reset) {
  if (!g || !g->eng) return fail(KBISIM_EINVAL, "null handle");
  if (cap < 0 || (cap > 0 && !stats)) return fail(KBISIM_EINVAL, "bad stats buffer");
  return guarded([&]() {
    const std::vector<kb::Engine::RoundStat> rs = g->eng->round_stats();
    if (n) *n = int32_t(rs.size());
    for (size_t r = 0; r < std::min<size_t>(rs.size(), size_t(cap)); ++r) {
      stats[r].signature_ms = rs[r].sig_ms;
      stats[r].round_ms = rs[r].round_ms;
      stats[r].active_nodes = int64_t(rs[r].nodes);
      stats[r].active_edges = int64_t(rs[r].edges);
      stats[r].max_keys = int64_t(rs[r].max_keys);
    }
    if (reset) g->eng->reset_round_stats();
    return KBISIM_OK;
  });
}

kbisim_status kbisim_work(const kbisim_graph* g, int64_t* nodes_edges, int32_t cap, int32_t reset) {
  if (!g || !g->eng) return fail(KBISIM_EINVAL, "null handle");
  if (cap < 0) return fail(KBISIM_EINVAL, "negative cap");
  return guarded([&]() {
    uint64_t w[8];
    g->eng->work_counts(w);
    for (int i = 0; i < std::min(cap, 8); ++i) nodes_edges[i] = int64_t(w[i]);
    if (reset) g->eng->reset_work();
    return KBISIM_OK;
  });
}


kbisim_status kbisim_batch_create(int32_t num_graphs, const int64_t* node_off, const int64_t* edge_off,
                                  const kbisim_graph_desc* d, const kbisim_options* opt, kbisim_batch** out) {
  if (!d || !out || !node_off || !edge_off) return fail(KBISIM_EINVAL, "null argument");
  if (num_graphs < 1) return fail(KBISIM_EINVAL, "num_graphs < 1");
  if (d->num_nodes != node_off[num_graphs] || d->num_edges != edge_off[num_graphs])
    return fail(KBISIM_EINVAL, "desc sizes differ from the offsets' totals");
  if (d->num_nodes > 0 && !d->node_label) return fail(KBISIM_EINVAL, "null node_label");
  if (d->num_edges > 0 && (!d->edge_src || !d->edge_label || !d->edge_dst))
    return fail(KBISIM_EINVAL, "null edge array");
  if (d->mem != KBISIM_MEM_HOST && d->mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  kb::Options o;
  if (parse_options(opt, &o) != KBISIM_OK) return KBISIM_EINVAL;
  if (o.edge_window > 0) return fail(KBISIM_EINVAL, "edge_window_bytes applies to kbisim_create only");
  return guarded([&]() {
    hipStream_t s = static_cast<hipStream_t>(d->stream);
    auto* b = new kb::Batch(num_graphs, node_off, edge_off, d->node_label, d->edge_src, d->edge_label, d->edge_dst,
                            d->mem == KBISIM_MEM_HOST, s, o);
    auto* h = new kbisim_batch;
    h->b = b;
    *out = h;
    return KBISIM_OK;
  });
}

kbisim_status kbisim_batch_refine(kbisim_batch* h, const int32_t* k_per_graph, int32_t* rounds_done) {
  if (!h || !h->b || !k_per_graph) return fail(KBISIM_EINVAL, "null argument");
  const int32_t G = h->b->num_graphs();
  for (int32_t g = 0; g < G; ++g)
    if (k_per_graph[g] < 0) return fail(KBISIM_EINVAL, "k < 0");
  return guarded([&]() {
    h->b->refine(std::vector<int32_t>(k_per_graph, k_per_graph + G));
    if (rounds_done) h->b->result(nullptr, false, nullptr, rounds_done);
    return KBISIM_OK;
  });
}

kbisim_status kbisim_batch_result(const kbisim_batch* h, int32_t* pid_out, kbisim_mem mem, int64_t* num_blocks) {
  if (!h || !h->b) return fail(KBISIM_EINVAL, "null handle");
  if (mem != KBISIM_MEM_HOST && mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  return guarded([&]() {
    h->b->result(pid_out, mem == KBISIM_MEM_DEVICE, num_blocks, nullptr);
    return KBISIM_OK;
  });
}

void kbisim_batch_destroy(kbisim_batch* h) {
  if (!h) return;
  delete h->b;
  delete h;
}


kbisim_status kbisim_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, const kbisim_options* opt,
                                   kbisim_server** out) {
  if (!out) return fail(KBISIM_EINVAL, "null out");
  if (max_slots < 1 || max_slots > 64) return fail(KBISIM_EINVAL, "max_slots outside [1, 64]");
  if (hbm_budget_bytes == 0) return fail(KBISIM_EINVAL, "zero budget");
  kb::Options o;
  if (parse_options(opt, &o) != KBISIM_OK) return KBISIM_EINVAL;
  if (o.edge_window > 0) return fail(KBISIM_EINVAL, "edge_window_bytes applies to kbisim_create only");
  o.profile = false;
  return guarded([&]() {
    auto* h = new kbisim_server;
    h->s = new kb::Server(hbm_budget_bytes, max_slots, o);
    *out = h;
    return KBISIM_OK;
  });
}

kbisim_status kbisim_server_submit(kbisim_server* h, const kbisim_graph_desc* d, int32_t k, uint64_t* req_id) {
  if (!h || !h->s || !d || !req_id) return fail(KBISIM_EINVAL, "null argument");
  if (k < 0) return fail(KBISIM_EINVAL, "k < 0");
  if (d->num_nodes < 0 || d->num_edges < 0) return fail(KBISIM_EINVAL, "negative size");
  if (d->num_nodes >= (int64_t(1) << 31)) return fail(KBISIM_EINVAL, "num_nodes >= 2^31");
  if (d->num_edges >= int64_t(0xffffffffll)) return fail(KBISIM_EINVAL, "num_edges >= 2^32 - 1");
  if (d->num_nodes > 0 && !d->node_label) return fail(KBISIM_EINVAL, "null node_label");
  if (d->num_edges > 0 && (!d->edge_src || !d->edge_label || !d->edge_dst))
    return fail(KBISIM_EINVAL, "null edge array");
  if (d->mem != KBISIM_MEM_HOST && d->mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  return guarded([&]() {
    *req_id = h->s->submit(d->node_label, d->edge_src, d->edge_label, d->edge_dst, d->num_nodes, d->num_edges,
                           d->mem == KBISIM_MEM_DEVICE, k, static_cast<hipStream_t>(d->stream));
    return KBISIM_OK;
  });
}

kbisim_status kbisim_server_wait(kbisim_server* h, uint64_t req_id, int32_t* pid_out, kbisim_mem mem,
                                 int64_t* num_blocks, int32_t* rounds_done, double timeout_s) {
  if (!h || !h->s) return fail(KBISIM_EINVAL, "null handle");
  if (mem != KBISIM_MEM_HOST && mem != KBISIM_MEM_DEVICE) return fail(KBISIM_EINVAL, "bad mem kind");
  return guarded([&]() {
    std::string err;
    const int st = h->s->wait(req_id, pid_out, mem == KBISIM_MEM_DEVICE, num_blocks, rounds_done, timeout_s, &err);
    if (st != KBISIM_OK) {
      g_last_error = err.empty() ? kbisim_status_str(kbisim_status(st)) : err;
      return kbisim_status(st);
    }
    return KBISIM_OK;
  });
}

kbisim_status kbisim_server_cancel(kbisim_server* h, uint64_t req_id) {
  if (!h || !h->s) return fail(KBISIM_EINVAL, "null handle");
  const int st = h->s->cancel(req_id);
  if (st != KBISIM_OK) return fail(kbisim_status(st), st == KBISIM_ESTATE ? "request already finished" : "unknown id");
  return KBISIM_OK;
}

kbisim_status kbisim_server_timing(kbisim_server* h, uint64_t req_id, double* queued_s, double* total_s) {
  if (!h || !h->s) return fail(KBISIM_EINVAL, "null handle");
  if (!h->s->timing(req_id, queued_s, total_s)) return fail(KBISIM_ESTATE, "request not done");
  return KBISIM_OK;
}

kbisim_status kbisim_server_release(kbisim_server* h, uint64_t req_id) {
  if (!h || !h->s) return fail(KBISIM_EINVAL, "null handle");
  h->s->release(req_id);
  return KBISIM_OK;
}

kbisim_status kbisim_server_state(kbisim_server* h, uint64_t req_id, int32_t* state) {
  if (!h || !h->s || !state) return fail(KBISIM_EINVAL, "null argument");
  if (h->s->state(req_id, state) != KBISIM_OK) return fail(KBISIM_EINVAL, "unknown id");
  return KBISIM_OK;
}

kbisim_status kbisim_server_in_use(kbisim_server* h, uint64_t* bytes) {
  if (!h || !h->s || !bytes) return fail(KBISIM_EINVAL, "null argument");
  *bytes = h->s->in_use();
  return KBISIM_OK;
}

void kbisim_server_destroy(kbisim_server* h) {
  if (!h) return;
  delete h->s;
  delete h;
}

void kbisim_destroy(kbisim_graph* g) {
  if (!g) return;
  delete g->eng;
  delete g;
}

const char* kbisim_status_str(kbisim_status s) {
  switch (s) {
    case KBISIM_OK: return "ok";
    case KBISIM_EINVAL: return "invalid argument";
    case KBISIM_ENOMEM: return "out of memory";
    case KBISIM_EDEVICE: return "device error";
    case KBISIM_ESTATE: return "invalid state";
    case KBISIM_EBUSY: return "busy";
    case KBISIM_ECANCELED: return "cancelled";
    case KBISIM_ETIMEDOUT: return "timed out";
  }
  return "unknown status";
}

const char* kbisim_last_error(void) { return g_last_error.c_str(); }

kbisim_status kbisim_release_cached(int64_t* released_bytes) {
  return guarded([&]() {
    const size_t b = kb::Pool::instance().cached_bytes();
    kb::Pool::instance().trim();
    if (released_bytes) *released_bytes = int64_t(b);
    return KBISIM_OK;
  });
}

}  // extern "C"
