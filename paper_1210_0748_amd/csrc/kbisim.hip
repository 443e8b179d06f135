// k-bisimulation on one MI355X: host round driver and the C ABI (kbisim.h).
//
// Per round (Algorithm 1, one iteration j > 0):
//   signature kernels  -- join with pId_{j-1}(dst), per-node sort + unique
//   order_groups       -- order the signatures inside every block of pId_{j-1}
//   assign_ids         -- scan of class starts -> pId_j, block starts, B_j
// The graph (CSR by source, packed label|dst words) stays in device memory.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <string>

#include "build.h"
#include "common.h"
#include "engine.h"
#include "refine.h"
#include "scan_radix.h"
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

Engine::Engine(int64_t n, int64_t m, hipStream_t s, const Options& o) : n_(n), m_(m), st_(s), opt_(o) {}

Engine::~Engine() {
  for (auto& e : ev_pool_) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
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
  }
  ev_used_ = 0;
}

// ---------------------------------------------------------------------------
// Build: validation, pId_0, edge-label ranks, CSR.

template <typename AdjT>
void Engine::build_adj(const int32_t* src, const uint32_t* erank, const int32_t* dst) {
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  DevBuf deg, cursor;
  deg.ensure((N + 1) * sizeof(uint32_t));
  cursor.ensure((N + 1) * sizeof(uint32_t));
  KB_CHECK(hipMemsetAsync(deg.p, 0, (N + 1) * sizeof(uint32_t), st_));
  KB_CHECK(hipMemsetAsync(cursor.p, 0, (N + 1) * sizeof(uint32_t), st_));
  if (E) {
    degree_k<<<grid_stride_blocks(E), kNT, 0, st_>>>(src, E, deg.as<uint32_t>());
    KB_LAUNCH_CHECK();
  }
  rowptr_.ensure((N + 1) * sizeof(uint32_t));
  scan_dev<uint32_t, uint32_t, false>(deg.as<uint32_t>(), rowptr_.as<uint32_t>(), N + 1);
  adj_.ensure(std::max<uint64_t>(E, 1) * sizeof(AdjT));
  if (E) {
    fill_adj_k<AdjT><<<grid_stride_blocks(E), kNT, 0, st_>>>(src, erank, dst, E, rowptr_.as<uint32_t>(),
                                                           cursor.as<uint32_t>(), dst_bits_, adj_.as<AdjT>());
    KB_LAUNCH_CHECK();
  }
  // degree buckets
  if (N) {
    DevBuf fw, fb, fh, hd, ow, ob, oh;
    for (DevBuf* b : {&fw, &fb, &fh, &hd, &ow, &ob, &oh}) b->ensure((N + 1) * sizeof(uint32_t));
    for (DevBuf* b : {&fw, &fb, &fh, &hd})
      KB_CHECK(hipMemsetAsync(b->p, 0, (N + 1) * sizeof(uint32_t), st_));
    bucket_flags_k<<<grid_for(N), kNT, 0, st_>>>(rowptr_.as<uint32_t>(), uint32_t(N), kThreadMaxDeg,
                                                 kWaveMaxDeg, kBlockMaxDeg, fw.as<uint32_t>(),
                                                 fb.as<uint32_t>(), fh.as<uint32_t>(), hd.as<uint32_t>());
    KB_LAUNCH_CHECK();
    scan_dev<uint32_t, uint32_t, false>(fw.as<uint32_t>(), ow.as<uint32_t>(), N + 1);
    scan_dev<uint32_t, uint32_t, false>(fb.as<uint32_t>(), ob.as<uint32_t>(), N + 1);
    scan_dev<uint32_t, uint32_t, false>(fh.as<uint32_t>(), oh.as<uint32_t>(), N + 1);
    hw_.p[1] = hw_.p[2] = hw_.p[3] = 0;  // before the copies are queued
    KB_CHECK(hipMemcpyAsync(&hw_.p[1], ow.as<uint32_t>() + N, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipMemcpyAsync(&hw_.p[2], ob.as<uint32_t>() + N, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipMemcpyAsync(&hw_.p[3], oh.as<uint32_t>() + N, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    nw_ = uint32_t(hw_.p[1]);
    nb_ = uint32_t(hw_.p[2]);
    nh_ = uint32_t(hw_.p[3]);
    wlist_.ensure(std::max<uint32_t>(nw_, 1) * sizeof(uint32_t));
    blist_.ensure(std::max<uint32_t>(nb_, 1) * sizeof(uint32_t));
    hlist_.ensure(std::max<uint32_t>(nh_, 1) * sizeof(uint32_t));
    compact_index_k<<<grid_for(N), kNT, 0, st_>>>(fw.as<uint32_t>(), ow.as<uint32_t>(), uint32_t(N),
                                                  wlist_.as<uint32_t>());
    compact_index_k<<<grid_for(N), kNT, 0, st_>>>(fb.as<uint32_t>(), ob.as<uint32_t>(), uint32_t(N),
                                                  blist_.as<uint32_t>());
    compact_index_k<<<grid_for(N), kNT, 0, st_>>>(fh.as<uint32_t>(), oh.as<uint32_t>(), uint32_t(N),
                                                  hlist_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    hub_off_.ensure((nh_ + 1) * sizeof(uint32_t));
    if (nh_) {
      DevBuf hdl;
      hdl.ensure((nh_ + 1) * sizeof(uint32_t));
      KB_CHECK(hipMemsetAsync(hdl.p, 0, (nh_ + 1) * sizeof(uint32_t), st_));
      gather_u32_k<<<grid_for(nh_), kNT, 0, st_>>>(hd.as<uint32_t>(), hlist_.as<uint32_t>(), nh_,
                                                   hdl.as<uint32_t>());
      KB_LAUNCH_CHECK();
      scan_dev<uint32_t, uint32_t, false>(hdl.as<uint32_t>(), hub_off_.as<uint32_t>(), nh_ + 1);
      const uint64_t tot = read_word(hub_off_.as<uint32_t>() + nh_, 4);
      hub_tmp_.ensure(std::max<uint64_t>(tot, 1) * (key64_ ? 8 : 4));
    }
    KB_CHECK(hipStreamSynchronize(st_));  // temporaries are freed on return
  }
}

void Engine::build(const int32_t* node_label, const int32_t* src, const int32_t* lab, const int32_t* dst) {
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  DevBuf errb;
  errb.ensure(4 * sizeof(uint32_t));
  KB_CHECK(hipMemsetAsync(errb.p, 0, 4 * sizeof(uint32_t), st_));
  uint32_t* err = errb.as<uint32_t>();
  if (N) {
    validate_nodes_k<<<grid_stride_blocks(N), kNT, 0, st_>>>(node_label, N, err, err + 1);
    KB_LAUNCH_CHECK();
  }
  if (E) {
    validate_edges_k<<<grid_stride_blocks(E), kNT, 0, st_>>>(src, lab, dst, E, n_, err, err + 1);
    KB_LAUNCH_CHECK();
  }
  KB_CHECK(hipMemcpyAsync(hw_.p, err, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  uint32_t words[3];
  std::memcpy(words, hw_.p, sizeof(words));
  if (words[0] & 1u) throw InvalidInput("edge endpoint outside [0, num_nodes)");
  if (words[0] & 2u) throw InvalidInput("negative edge label");
  if (words[0] & 4u) throw InvalidInput("negative node label");
  const uint32_t max_nlab = words[1], max_elab = words[2];

  const uint64_t big = std::max<uint64_t>(std::max<uint64_t>(N, E), 1);
  DevBuf ka, kb2, va, vb;
  ka.ensure(big * 4);
  kb2.ensure(big * 4);
  va.ensure(big * 4);
  vb.ensure(big * 4);

  // pId_0: nodes sorted by label; a new id per new label (Section 3.1, k = 0)
  pid_[0].ensure(std::max<uint64_t>(N, 1) * 4);
  pid_[1].ensure(std::max<uint64_t>(N, 1) * 4);
  ord_.ensure(std::max<uint64_t>(N, 1) * 4);
  flag_.ensure(std::max<uint64_t>(N, 1));
  bstart_.ensure((N + 1) * 4);
  cls_.ensure(std::max<uint64_t>(N, 1) * 4);
  cur_ = 0;
  if (N) {
    to_u32_iota_k<<<grid_for(N), kNT, 0, st_>>>(node_label, ka.as<uint32_t>(), va.as<uint32_t>(), uint32_t(N));
    KB_LAUNCH_CHECK();
    const bool f = radix_sort<uint32_t>(ka.as<uint32_t>(), va.as<uint32_t>(), kb2.as<uint32_t>(),
                                        vb.as<uint32_t>(), N, 0, bits_for(max_nlab), radix_scratch(N), st_);
    const uint32_t* keys = f ? kb2.as<uint32_t>() : ka.as<uint32_t>();
    const uint32_t* vals = f ? vb.as<uint32_t>() : va.as<uint32_t>();
    KB_CHECK(hipMemcpyAsync(ord_.p, vals, N * 4, hipMemcpyDeviceToDevice, st_));
    run_start_flags_k<<<grid_for(N), kNT, 0, st_>>>(keys, uint32_t(N), flag_.as<uint8_t>(), nullptr);
    KB_LAUNCH_CHECK();
  }
  assign_ids_into(pid_[0].as<int32_t>());
  counts_.assign(1, B_);
  rounds_ = 0;
  fixed_ = false;

  // edge labels: dense ascending ranks
  DevBuf erank;
  erank.ensure(std::max<uint64_t>(E, 1) * 4);
  n_elab_ = 0;
  if (E) {
    to_u32_iota_k<<<grid_for(E), kNT, 0, st_>>>(lab, ka.as<uint32_t>(), va.as<uint32_t>(), uint32_t(E));
    KB_LAUNCH_CHECK();
    const bool f = radix_sort<uint32_t>(ka.as<uint32_t>(), va.as<uint32_t>(), kb2.as<uint32_t>(),
                                        vb.as<uint32_t>(), E, 0, bits_for(max_elab), radix_scratch(E), st_);
    uint32_t* keys = f ? kb2.as<uint32_t>() : ka.as<uint32_t>();
    uint32_t* vals = f ? vb.as<uint32_t>() : va.as<uint32_t>();
    uint32_t* fl = f ? ka.as<uint32_t>() : kb2.as<uint32_t>();  // the free key buffer
    run_start_flags_k<<<grid_for(E), kNT, 0, st_>>>(keys, uint32_t(E), nullptr, fl);
    KB_LAUNCH_CHECK();
    uint32_t* clsE = f ? va.as<uint32_t>() : vb.as<uint32_t>();  // the free value buffer
    scan_dev<uint32_t, uint32_t, true>(fl, clsE, E);
    rank_scatter_k<<<grid_for(E), kNT, 0, st_>>>(vals, clsE, uint32_t(E), erank.as<uint32_t>());
    KB_LAUNCH_CHECK();
    n_elab_ = uint32_t(read_word(clsE + (E - 1), 4));
  }
  lab_bits_ = n_elab_ > 1 ? bits_for(n_elab_ - 1) : 0;
  dst_bits_ = bits_for(N > 1 ? N - 1 : 1);
  adj64_ = dst_bits_ + lab_bits_ > 32;
  key64_ = lab_bits_ + bits_for(N > 1 ? N - 1 : 1) > 32;
  if (adj64_)
    build_adj<uint64_t>(src, erank.as<uint32_t>(), dst);
  else
    build_adj<uint32_t>(src, erank.as<uint32_t>(), dst);

  // per-round buffers
  ukey_.ensure(std::max<uint64_t>(E, 1) * (key64_ ? 8 : 4));
  ucnt_.ensure(std::max<uint64_t>(N, 1) * 4);
  KB_CHECK(hipStreamSynchronize(st_));
}

// cls = inclusive scan of flag; pid[ord[p]] = cls[p]-1; bstart at class starts.
void Engine::assign_ids_into(int32_t* pid_out) {
  const uint64_t N = uint64_t(n_);
  if (N == 0) {
    set_u32_k<<<1, 1, 0, st_>>>(bstart_.as<uint32_t>(), 0u);
    KB_LAUNCH_CHECK();
    B_ = 0;
    return;
  }
  scan_dev<uint8_t, uint32_t, true>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), N);
  assign_k<<<grid_for(N), kNT, 0, st_>>>(ord_.as<uint32_t>(), flag_.as<uint8_t>(), cls_.as<uint32_t>(),
                                         uint32_t(N), pid_out, bstart_.as<uint32_t>());
  KB_LAUNCH_CHECK();
  const uint64_t b = read_word(cls_.as<uint32_t>() + (N - 1), 4);
  set_u32_k<<<1, 1, 0, st_>>>(bstart_.as<uint32_t>() + b, uint32_t(N));
  KB_LAUNCH_CHECK();
  B_ = int64_t(b);
}

// ---------------------------------------------------------------------------
// Group ordering.

void Engine::make_lists(const uint32_t* seg_start, const uint32_t* seg_size, const uint32_t* seg_depth,
                        const uint8_t* seg_done, uint32_t nseg, SegLists& out) {
  out.ns = out.nm = out.nl = 0;
  if (nseg == 0) return;
  const uint64_t n1 = uint64_t(nseg) + 1;
  for (DevBuf* b : {&cf_small_, &cf_medium_, &cf_large_}) b->ensure(n1 * 4);
  off_.ensure(3 * n1 * 4);
  classify_segments_k<<<grid_for(nseg), kNT, 0, st_>>>(seg_size, seg_done, nseg, opt_.medium_cap,
                                                       cf_small_.as<uint32_t>(),
                                                       cf_medium_.as<uint32_t>(), cf_large_.as<uint32_t>());
  KB_LAUNCH_CHECK();
  // exclusive scans over nseg + 1 entries: entry nseg is the list length
  // (the flag at index nseg is never read into it)
  uint32_t* o = off_.as<uint32_t>();
  scan_dev<uint32_t, uint32_t, false>(cf_small_.as<uint32_t>(), o, n1);
  scan_dev<uint32_t, uint32_t, false>(cf_medium_.as<uint32_t>(), o + n1, n1);
  scan_dev<uint32_t, uint32_t, false>(cf_large_.as<uint32_t>(), o + 2 * n1, n1);
  uint32_t* hw32 = reinterpret_cast<uint32_t*>(hw_.p);
  hw32[0] = hw32[1] = hw32[2] = 0;
  KB_CHECK(hipMemcpyAsync(hw32 + 0, o + nseg, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipMemcpyAsync(hw32 + 1, o + n1 + nseg, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipMemcpyAsync(hw32 + 2, o + 2 * n1 + nseg, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  out.ns = hw32[0];
  out.nm = hw32[1];
  out.nl = hw32[2];
  struct {
    DevBuf *st, *sz, *dp;
    uint32_t cnt;
    const uint32_t* f;
    const uint32_t* off;
  } parts[3] = {{&out.s_start, &out.s_size, &out.s_depth, out.ns, cf_small_.as<uint32_t>(), o},
                {&out.m_start, &out.m_size, &out.m_depth, out.nm, cf_medium_.as<uint32_t>(), o + n1},
                {&out.l_start, &out.l_size, &out.l_depth, out.nl, cf_large_.as<uint32_t>(), o + 2 * n1}};
  for (auto& pp : parts) {
    if (!pp.cnt) continue;
    pp.st->ensure(uint64_t(pp.cnt) * 4);
    pp.sz->ensure(uint64_t(pp.cnt) * 4);
    pp.dp->ensure(uint64_t(pp.cnt) * 4);
    scatter_segments_k<<<grid_for(nseg), kNT, 0, st_>>>(seg_start, seg_size, seg_depth, nseg, pp.f, pp.off,
                                                        pp.st->as<uint32_t>(), pp.sz->as<uint32_t>(),
                                                        pp.dp->as<uint32_t>());
    KB_LAUNCH_CHECK();
  }
}

template <typename KeyT>
void Engine::resolve_lists(SegLists& L, const void* kvp) {
  const KeyView<KeyT>& kv = *static_cast<const KeyView<KeyT>*>(kvp);
  if (L.ns) {
    resolve_k<64, kSmallCap, KeyT><<<L.ns, 64, 0, st_>>>(L.s_start.as<uint32_t>(), L.s_size.as<uint32_t>(),
                                                        L.s_depth.as<uint32_t>(), ord_.as<uint32_t>(),
                                                        flag_.as<uint8_t>(), kv);
    KB_LAUNCH_CHECK();
  }
  if (L.nm) {
    resolve_k<kMediumNT, kMediumCap, KeyT><<<L.nm, kMediumNT, 0, st_>>>(
        L.m_start.as<uint32_t>(), L.m_size.as<uint32_t>(), L.m_depth.as<uint32_t>(), ord_.as<uint32_t>(),
        flag_.as<uint8_t>(), kv);
    KB_LAUNCH_CHECK();
  }
}

template <typename KeyT>
void Engine::order_groups(int key_bits, const void* kvp) {
  const KeyView<KeyT>& kv = *static_cast<const KeyView<KeyT>*>(kvp);
  const uint32_t B = uint32_t(B_);
  seg_start_.ensure(uint64_t(B) * 4 + 4);
  seg_size_.ensure(uint64_t(B) * 4 + 4);
  seg_depth_.ensure(uint64_t(B) * 4 + 4);
  seg_done_.ensure(uint64_t(B) + 1);
  blocks_as_segments_k<<<grid_for(B), kNT, 0, st_>>>(bstart_.as<uint32_t>(), B, seg_start_.as<uint32_t>(),
                                                     seg_size_.as<uint32_t>(), seg_depth_.as<uint32_t>(),
                                                     seg_done_.as<uint8_t>());
  KB_LAUNCH_CHECK();
  make_lists(seg_start_.as<uint32_t>(), seg_size_.as<uint32_t>(), seg_depth_.as<uint32_t>(),
             seg_done_.as<uint8_t>(), B, lists_a_);
  resolve_lists<KeyT>(lists_a_, kvp);

  // Large groups: global passes, each splitting every open group.
  const uint32_t* Ls = lists_a_.l_start.as<uint32_t>();
  const uint32_t* Lz = lists_a_.l_size.as<uint32_t>();
  const uint32_t* Ld = lists_a_.l_depth.as<uint32_t>();
  uint32_t nl = lists_a_.nl;
  int nx = 0;
  const int dbits = key_bits + 1;
  const uint64_t last_mask = dbits >= 64 ? ~0ull : ((1ull << dbits) - 1);
  while (nl > 0) {
    // item offsets of the large groups (sizes with a trailing zero)
    l_ioff_.ensure((uint64_t(nl) + 1) * 4);
    l_open_.ensure((uint64_t(nl) + 1) * 4);
    KB_CHECK(hipMemcpyAsync(l_open_.p, Lz, uint64_t(nl) * 4, hipMemcpyDeviceToDevice, st_));
    KB_CHECK(hipMemsetAsync(l_open_.as<uint32_t>() + nl, 0, 4, st_));
    scan_dev<uint32_t, uint32_t, false>(l_open_.as<uint32_t>(), l_ioff_.as<uint32_t>(), uint64_t(nl) + 1);
    const uint32_t M = uint32_t(read_word(l_ioff_.as<uint32_t>() + nl, 4));
    // split position of every group (kNoDiff: all members identical)
    l_split_.ensure(uint64_t(nl) * 4);
    KB_CHECK(hipMemsetAsync(l_split_.p, 0xff, uint64_t(nl) * 4, st_));
    l_long_.ensure((uint64_t(M) + 1) * 4);
    KB_CHECK(hipMemsetAsync(l_long_.as<uint32_t>() + M, 0, 4, st_));
    large_split_pos_k<KeyT><<<grid_for(M), kNT, 0, st_>>>(Ls, Ld, l_ioff_.as<uint32_t>(), nl, M,
                                                         ord_.as<uint32_t>(), l_split_.as<uint32_t>(),
                                                         l_long_.as<uint32_t>(), l_long_.as<uint32_t>() + M, kv);
    KB_LAUNCH_CHECK();
    large_split_pos_wave_k<KeyT><<<std::min<uint32_t>(grid_for(uint64_t(M) * kWave), 4096), kNT, 0, st_>>>(
        Ls, Ld, l_ioff_.as<uint32_t>(), nl, ord_.as<uint32_t>(), l_split_.as<uint32_t>(), l_long_.as<uint32_t>(),
        l_long_.as<uint32_t>() + M, kv);
    KB_LAUNCH_CHECK();
    l_open_off_.ensure((uint64_t(nl) + 1) * 4);
    open_flags_k<<<grid_for(nl), kNT, 0, st_>>>(l_split_.as<uint32_t>(), nl, l_open_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemsetAsync(l_open_.as<uint32_t>() + nl, 0, 4, st_));
    scan_dev<uint32_t, uint32_t, false>(l_open_.as<uint32_t>(), l_open_off_.as<uint32_t>(), uint64_t(nl) + 1);
    const uint32_t nU = uint32_t(read_word(l_open_off_.as<uint32_t>() + nl, 4));
    if (nU == 0) break;
    u_start_.ensure(uint64_t(nU) * 4);
    u_size_.ensure((uint64_t(nU) + 1) * 4);
    u_pos_.ensure(uint64_t(nU) * 4);
    scatter_segments_k<<<grid_for(nl), kNT, 0, st_>>>(Ls, Lz, l_split_.as<uint32_t>(), nl, l_open_.as<uint32_t>(),
                                                      l_open_off_.as<uint32_t>(), u_start_.as<uint32_t>(),
                                                      u_size_.as<uint32_t>(), u_pos_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemsetAsync(u_size_.as<uint32_t>() + nU, 0, 4, st_));
    u_ioff_.ensure((uint64_t(nU) + 1) * 4);
    scan_dev<uint32_t, uint32_t, false>(u_size_.as<uint32_t>(), u_ioff_.as<uint32_t>(), uint64_t(nU) + 1);
    const uint32_t MU = uint32_t(read_word(u_ioff_.as<uint32_t>() + nU, 4));

    // positions per sort digit and chunks of groups whose index fits beside
    // the packed digits in 64 bits
    const int need_g = nU > 1 ? bits_for(nU - 1) : 0;
    uint32_t width = uint32_t(std::max(1, (64 - need_g) / dbits));
    const int dig_bits = int(width) * dbits;
    const int gb = 64 - dig_bits;
    const uint32_t chunk = gb >= 32 ? nU : std::max<uint32_t>(1, std::min<uint32_t>(nU, 1u << std::max(gb, 0)));
    const int nxt = nx ^ 1;
    for (DevBuf* b : {&next_l_start_[nxt], &next_l_size_[nxt], &next_l_depth_[nxt]})
      b->ensure(uint64_t(MU / (std::max(opt_.medium_cap, kSmallCap) + 1) + 1) * 4);
    uint32_t nnext = 0;
    for (uint32_t c0 = 0; c0 < nU; c0 += chunk) {
      const uint32_t cn = std::min(chunk, nU - c0);
      const uint32_t I0 = (c0 == 0) ? 0u : uint32_t(read_word(u_ioff_.as<uint32_t>() + c0, 4));
      const uint32_t I1 = (c0 + cn == nU) ? MU : uint32_t(read_word(u_ioff_.as<uint32_t>() + c0 + cn, 4));
      const uint32_t cnt = I1 - I0;
      const uint32_t* gst = u_start_.as<uint32_t>() + c0;
      const uint32_t* gps = u_pos_.as<uint32_t>() + c0;
      const uint32_t* gio = u_ioff_.as<uint32_t>() + c0;
      for (DevBuf* b : {&k0_, &k1_}) b->ensure(uint64_t(cnt) * 8);
      for (DevBuf* b : {&v0_, &v1_, &ipos_, &sub_item_}) b->ensure(uint64_t(cnt) * 4);
      for (DevBuf* b : {&sflag_, &soff_}) b->ensure((uint64_t(cnt) + 1) * 4);
      large_gather_k<KeyT><<<grid_for(cnt), kNT, 0, st_>>>(gst, gps, gio, cn, cnt, I0, ord_.as<uint32_t>(), dig_bits,
                                                          width, k0_.as<uint64_t>(), v0_.as<uint32_t>(), kv);
      KB_LAUNCH_CHECK();
      const int g_bits = cn > 1 ? bits_for(cn - 1) : 0;
      const bool f = radix_sort<uint64_t>(k0_.as<uint64_t>(), v0_.as<uint32_t>(), k1_.as<uint64_t>(),
                                          v1_.as<uint32_t>(), cnt, 0, dig_bits + g_bits, radix_scratch(cnt), st_);
      const uint64_t* K = f ? k1_.as<uint64_t>() : k0_.as<uint64_t>();
      const uint32_t* V = f ? v1_.as<uint32_t>() : v0_.as<uint32_t>();
      large_write_k<<<grid_for(cnt), kNT, 0, st_>>>(gst, gio, cnt, I0, K, V, dig_bits, ord_.as<uint32_t>(),
                                                    flag_.as<uint8_t>(), sflag_.as<uint32_t>(), ipos_.as<uint32_t>());
      KB_LAUNCH_CHECK();
      KB_CHECK(hipMemsetAsync(sflag_.as<uint32_t>() + cnt, 0, 4, st_));
      scan_dev<uint32_t, uint32_t, false>(sflag_.as<uint32_t>(), soff_.as<uint32_t>(), uint64_t(cnt) + 1);
      const uint32_t ns = uint32_t(read_word(soff_.as<uint32_t>() + cnt, 4));
      seg_start_.ensure(uint64_t(ns) * 4 + 4);
      seg_size_.ensure(uint64_t(ns) * 4 + 4);
      seg_depth_.ensure(uint64_t(ns) * 4 + 4);
      seg_done_.ensure(uint64_t(ns) + 1);
      large_subgroups_k<<<grid_for(cnt), kNT, 0, st_>>>(sflag_.as<uint32_t>(), soff_.as<uint32_t>(), cnt,
                                                        ipos_.as<uint32_t>(), K, dig_bits, width, last_mask, gps,
                                                        sub_item_.as<uint32_t>(), seg_start_.as<uint32_t>(),
                                                        seg_depth_.as<uint32_t>(), seg_done_.as<uint8_t>());
      subgroup_sizes_k<<<grid_for(ns), kNT, 0, st_>>>(sub_item_.as<uint32_t>(), ns, cnt, seg_size_.as<uint32_t>());
      KB_LAUNCH_CHECK();
      make_lists(seg_start_.as<uint32_t>(), seg_size_.as<uint32_t>(), seg_depth_.as<uint32_t>(),
                 seg_done_.as<uint8_t>(), ns, lists_b_);
      resolve_lists<KeyT>(lists_b_, kvp);
      if (lists_b_.nl) {
        const uint64_t bytes = uint64_t(lists_b_.nl) * 4;
        KB_CHECK(hipMemcpyAsync(next_l_start_[nxt].as<uint32_t>() + nnext, lists_b_.l_start.p, bytes,
                                hipMemcpyDeviceToDevice, st_));
        KB_CHECK(hipMemcpyAsync(next_l_size_[nxt].as<uint32_t>() + nnext, lists_b_.l_size.p, bytes,
                                hipMemcpyDeviceToDevice, st_));
        KB_CHECK(hipMemcpyAsync(next_l_depth_[nxt].as<uint32_t>() + nnext, lists_b_.l_depth.p, bytes,
                                hipMemcpyDeviceToDevice, st_));
        nnext += lists_b_.nl;
      }
    }
    Ls = next_l_start_[nxt].as<uint32_t>();
    Lz = next_l_size_[nxt].as<uint32_t>();
    Ld = next_l_depth_[nxt].as<uint32_t>();
    nl = nnext;
    nx = nxt;
  }
}

template <typename AdjT, typename KeyT>
void Engine::round_impl() {
  const uint32_t N = uint32_t(n_);
  const int pid_bits = bits_for(B_ > 1 ? uint64_t(B_ - 1) : 1);
  const int key_bits = lab_bits_ + pid_bits;
  SigArgs<AdjT, KeyT> a;
  a.rowptr = rowptr_.as<uint32_t>();
  a.adj = adj_.as<AdjT>();
  a.pid = pid_[cur_].as<int32_t>();
  a.bstart = bstart_.as<uint32_t>();
  a.ukey = ukey_.as<KeyT>();
  a.ucnt = ucnt_.as<uint32_t>();
  a.dst_bits = dst_bits_;
  a.pid_bits = pid_bits;
  if (opt_.profile) {
    if (!work_.p) {
      work_.ensure(8 * sizeof(unsigned long long));
      KB_CHECK(hipMemsetAsync(work_.p, 0, 8 * sizeof(unsigned long long), st_));
    }
    work_count_k<<<grid_for(N), kNT, 0, st_>>>(a.rowptr, a.pid, a.bstart, N, work_.as<unsigned long long>());
    KB_LAUNCH_CHECK();
  }

  int ev = ev_begin(0);
  sig_thread_k<AdjT, KeyT><<<grid_for(N), kNT, 0, st_>>>(a, N);
  KB_LAUNCH_CHECK();
  ev_end(ev);
  if (nw_) {
    ev = ev_begin(1);
    sig_wave_k<AdjT, KeyT><<<grid_for(uint64_t(nw_) * kWave), kNT, 0, st_>>>(a, wlist_.as<uint32_t>(), nw_);
    KB_LAUNCH_CHECK();
    ev_end(ev);
  }
  if (nb_) {
    ev = ev_begin(2);
    sig_block_k<AdjT, KeyT><<<nb_, kSigBlockNT, 0, st_>>>(a, blist_.as<uint32_t>(), nb_);
    KB_LAUNCH_CHECK();
    ev_end(ev);
  }
  if (nh_) {
    ev = ev_begin(3);
    sig_hub_k<AdjT, KeyT><<<nh_, kHubNT, 0, st_>>>(a, hlist_.as<uint32_t>(), hub_off_.as<uint32_t>(),
                                                   hub_tmp_.as<KeyT>(), key_bits);
    KB_LAUNCH_CHECK();
    ev_end(ev);
  }

  KeyView<KeyT> kv{rowptr_.as<uint32_t>(), ukey_.as<KeyT>(), ucnt_.as<uint32_t>(), key_bits + 1};
  const int evo = ev_begin(4);
  order_groups<KeyT>(key_bits, &kv);
  ev_end(evo);
}

void Engine::run_round() {
  const int64_t B_old = B_;
  const int evr = ev_begin(6);
  if (n_ > 0) {
    if (adj64_) {
      if (key64_) round_impl<uint64_t, uint64_t>(); else round_impl<uint64_t, uint32_t>();
    } else {
      if (key64_) round_impl<uint32_t, uint64_t>(); else round_impl<uint32_t, uint32_t>();
    }
  }
  const int eva = ev_begin(5);
  assign_ids_into(pid_[cur_ ^ 1].as<int32_t>());
  ev_end(eva);
  ev_end(evr);
  cur_ ^= 1;
  ++rounds_;
  counts_.push_back(B_);
  fixed_ = (B_ == B_old);
  ev_collect();
}

void Engine::work_counts(uint64_t* out8) {
  for (int i = 0; i < 8; ++i) out8[i] = 0;
  if (!work_.p) return;
  KB_CHECK(hipMemcpyAsync(out8, work_.p, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
}

void Engine::reset_work() {
  if (work_.p) KB_CHECK(hipMemsetAsync(work_.p, 0, 8 * sizeof(unsigned long long), st_));
}

void Engine::refine(int32_t k) {
  while (rounds_ < k) {
    if (fixed_ && opt_.early_stop) break;
    run_round();
  }
  KB_CHECK(hipStreamSynchronize(st_));
}

void Engine::result(int32_t* pid_out, bool to_device) const {
  if (n_ == 0) return;
  KB_CHECK(hipMemcpyAsync(pid_out, pid_[cur_].p, uint64_t(n_) * 4,
                          to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
}

}  // namespace kb

// ===========================================================================
// C ABI

struct kbisim_graph {
  kb::Engine* eng = nullptr;
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
  if (opt) {
    o.early_stop = opt->early_stop != 0;
    if (opt->medium_cap < 0 || opt->medium_cap > int32_t(kb::kMediumCap))
      return fail(KBISIM_EINVAL, "medium_cap outside [0, 2048]");
    if (opt->medium_cap > 0) o.medium_cap = uint32_t(opt->medium_cap);
    o.profile = opt->profile != 0;
  }
  return guarded([&]() {
    hipStream_t s = static_cast<hipStream_t>(d->stream);
    auto* eng = new kb::Engine(d->num_nodes, d->num_edges, s, o);
    try {
      const uint64_t N = uint64_t(d->num_nodes), E = uint64_t(d->num_edges);
      if (d->mem == KBISIM_MEM_HOST) {
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

}  // extern "C"
