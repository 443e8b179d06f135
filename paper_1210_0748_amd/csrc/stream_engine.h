// Engine methods of the streamed edge table (included by kbisim.hip inside
// namespace kb, after the Engine's other methods). See stream.h.

// Edges per chunk when the input table is read from host memory.
constexpr uint64_t kStreamChunk = uint64_t(1) << 24;

// The input edge table in host memory, read chunk by chunk into two device
// staging buffers on the engine's stream (a chunk's copy is ordered after the
// last kernel that read its buffer).
struct EdgeChunks {
  const int32_t *src, *lab, *dst;
  uint64_t m, chunk;
  DevBuf s[2], l[2], d[2];
  EdgeChunks(const int32_t* src_, const int32_t* lab_, const int32_t* dst_, uint64_t m_)
      : src(src_), lab(lab_), dst(dst_), m(m_), chunk(std::min<uint64_t>(std::max<uint64_t>(m_, 1), kStreamChunk)) {
    for (int b = 0; b < 2; ++b)
      for (DevBuf* x : {&s[b], &l[b], &d[b]}) x->ensure(chunk * 4);
  }
  // fn(src, lab, dst, count) for every chunk, device pointers
  template <typename F>
  void each(hipStream_t st, F&& fn) {
    uint64_t c = 0;
    for (uint64_t off = 0; off < m; off += chunk, ++c) {
      const uint64_t cnt = std::min(chunk, m - off);
      const int b = int(c & 1);
      KB_CHECK(hipMemcpyAsync(s[b].p, src + off, cnt * 4, hipMemcpyHostToDevice, st));
      KB_CHECK(hipMemcpyAsync(l[b].p, lab + off, cnt * 4, hipMemcpyHostToDevice, st));
      KB_CHECK(hipMemcpyAsync(d[b].p, dst + off, cnt * 4, hipMemcpyHostToDevice, st));
      fn(s[b].as<int32_t>(), l[b].as<int32_t>(), d[b].as<int32_t>(), cnt);
    }
  }
};

inline uint32_t stream_grid(uint64_t n) { return std::max<uint32_t>(1, std::min<uint32_t>(ceil_div(n, 256), 4096)); }

void Engine::build_streamed(const int32_t* node_label, const int32_t* src, const int32_t* lab, const int32_t* dst) {
  StreamScope scope(st_);
  streamed_ = true;
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  constexpr size_t kErrBytes = 16 + 8 * sizeof(uint64_t);
  DevBuf errb, deg;
  errb.ensure(kErrBytes);
  deg.ensure((N + 1) * 4);
  KB_CHECK(hipMemsetAsync(errb.p, 0, kErrBytes, st_));
  KB_CHECK(hipMemsetAsync(deg.p, 0, (N + 1) * 4, st_));
  uint32_t* err = errb.as<uint32_t>();
  unsigned long long* masks = reinterpret_cast<unsigned long long*>(errb.as<uint8_t>() + 16);
  if (N) {
    validate_nodes_k<<<validate_blocks(N), kRadixNT, 0, st_>>>(node_label, N, err, err + 1, masks);
    KB_LAUNCH_CHECK();
  }
  // first read of the table: validation, edge-label maximum and mask, out-degrees
  EdgeChunks in(src, lab, dst, E);
  in.each(st_, [&](const int32_t* s, const int32_t* l, const int32_t* d, uint64_t cnt) {
    stream_scan_k<<<stream_grid(cnt), kRadixNT, 0, st_>>>(s, l, d, cnt, n_, err, err + 2, masks + 4,
                                                           deg.as<uint32_t>());
    KB_LAUNCH_CHECK();
  });
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
  build_nodes(node_label, max_nlab, masks, mask_host);

  // edge labels: dense ascending ranks through a table of every label value
  // (from the mask, or from a second read of the labels)
  DevBuf etable, unused;
  if (E == 0 || max_elab < kMaskLabels) {
    n_elab_ = label_ranks(nullptr, E, max_elab, masks + 4, mask_host + 4, etable, unused, nullptr);
  } else if (max_elab < kRankTableMax) {
    const uint64_t t = uint64_t(max_elab) + 2;
    DevBuf present;
    present.ensure(t * 4);
    etable.ensure(t * 4);
    KB_CHECK(hipMemsetAsync(present.p, 0, t * 4, st_));
    in.each(st_, [&](const int32_t*, const int32_t* l, const int32_t*, uint64_t cnt) {
      stream_mark_k<<<stream_grid(cnt), 256, 0, st_>>>(l, cnt, max_elab + 1, present.as<uint32_t>(), err);
      KB_LAUNCH_CHECK();
    });
    scan_dev<uint32_t, uint32_t, false>(present.as<uint32_t>(), etable.as<uint32_t>(), t);
    n_elab_ = uint32_t(read_word(etable.as<uint32_t>() + (t - 1), 4));
    if (read_word(err, 4)) throw InvalidInput("the edge table changed while it was read");
  } else {
    throw InvalidInput("a streamed edge table needs edge labels below 2^24");
  }
  set_edge_layout();
  rowptr_.ensure((N + 1) * 4);
  scan_dev<uint32_t, uint32_t, false>(deg.as<uint32_t>(), rowptr_.as<uint32_t>(), N + 1);
  const uint32_t rank_size = E ? max_elab + 1 : 0;  // labels 0..max_elab have a rank
  if (adj64_)
    stream_adj<uint64_t>(src, lab, dst, etable.as<uint32_t>(), rank_size);
  else
    stream_adj<uint32_t>(src, lab, dst, etable.as<uint32_t>(), rank_size);
  adj_.ensure(8);  // the table itself is in host memory
  degree_stats();
  finish_build();
}

// Lays the edge table out as CSR edge words in pinned host memory: the
// nodes are cut into partitions of consecutive ids whose rows fit half of the
// window budget, and each partition is filled in a device window by one more
// read of the input table, then copied out.
template <typename AdjT>
void Engine::stream_adj(const int32_t* src, const int32_t* lab, const int32_t* dst, const uint32_t* rank_table,
                        uint32_t rank_size) {
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  std::vector<uint32_t> rp(N + 1);
  KB_CHECK(hipMemcpyAsync(rp.data(), rowptr_.p, (N + 1) * 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  const uint64_t win_edges = opt_.edge_window / 2 / sizeof(AdjT);
  uint64_t longest = 0;
  for (uint64_t u = 0; u < N; ++u) longest = std::max<uint64_t>(longest, rp[u + 1] - rp[u]);
  if (longest > win_edges || win_edges == 0)
    throw InvalidInput("edge_window_bytes is below twice the longest row (" + std::to_string(longest) +
                       " edges of " + std::to_string(sizeof(AdjT)) + " bytes)");
  part_node_.assign(1, 0u);
  part_edge_.assign(1, 0ull);
  for (uint64_t u = 0; u < N;) {
    // the last node v with rp[v] - rp[u] <= win_edges ends the partition
    const uint64_t lim = uint64_t(rp[u]) + win_edges;
    uint64_t v = uint64_t(std::upper_bound(rp.begin() + u + 1, rp.end(), uint32_t(std::min<uint64_t>(lim, 0xffffffffull))) -
                          rp.begin()) - 1;
    v = std::max<uint64_t>(v, u + 1);
    part_node_.push_back(uint32_t(v));
    part_edge_.push_back(rp[v]);
    u = v;
  }
  KB_CHECK(hipHostMalloc(&host_adj_, std::max<uint64_t>(E, 1) * sizeof(AdjT), hipHostMallocMapped));
  uint64_t max_nodes = 1, max_edges = 1;
  for (size_t p = 0; p + 1 < part_node_.size(); ++p) {
    max_nodes = std::max<uint64_t>(max_nodes, part_node_[p + 1] - part_node_[p]);
    max_edges = std::max<uint64_t>(max_edges, part_edge_[p + 1] - part_edge_[p]);
  }
  for (DevBuf& w : win_) w.ensure(max_edges * sizeof(AdjT));
  DevBuf cursor, errw;
  cursor.ensure(max_nodes * 4);
  errw.ensure(4);
  KB_CHECK(hipMemsetAsync(errw.p, 0, 4, st_));
  EdgeChunks in(src, lab, dst, E);
  for (size_t p = 0; p + 1 < part_node_.size(); ++p) {
    const uint32_t lo = part_node_[p], hi = part_node_[p + 1];
    const uint64_t cnt_e = part_edge_[p + 1] - part_edge_[p];
    if (cnt_e == 0) continue;
    stream_cursor_k<<<ceil_div(hi - lo, 256), 256, 0, st_>>>(rowptr_.as<uint32_t>(), lo, hi, cursor.as<uint32_t>());
    KB_LAUNCH_CHECK();
    in.each(st_, [&](const int32_t* s, const int32_t* l, const int32_t* d, uint64_t cnt) {
      stream_fill_k<AdjT><<<stream_grid(cnt), 256, 0, st_>>>(s, l, d, cnt, lo, hi, uint32_t(N),
                                                             rowptr_.as<uint32_t>(), rank_table, rank_size,
                                                             dst_bits_, cursor.as<uint32_t>(), win_[0].as<AdjT>(),
                                                             errw.as<uint32_t>());
      KB_LAUNCH_CHECK();
    });
    KB_CHECK(hipMemcpyAsync(static_cast<AdjT*>(host_adj_) + part_edge_[p], win_[0].p, cnt_e * sizeof(AdjT),
                            hipMemcpyDeviceToHost, st_));
  }
  if (read_word(errw.p, 4)) throw InvalidInput("the edge table changed while it was read");
}

// The signature launch of one round over a streamed edge table. Rounds with
// few active nodes read the rows of those nodes in place (the pinned table
// is mapped into the device's address space); others move every partition
// through the two windows on a copy stream, the copy of one partition
// overlapping the signature launch of the previous one.
template <typename AdjT, typename KeyT>
void Engine::streamed_signature(const void* sig_args, const void* sig_work) {
  SigArgs<AdjT, KeyT> a = *static_cast<const SigArgs<AdjT, KeyT>*>(sig_args);
  SigWork w = *static_cast<const SigWork*>(sig_work);
  const uint64_t table_bytes = uint64_t(m_) * sizeof(AdjT);
  if (uint64_t(M_act_) * 128 < table_bytes) {
    void* mapped = nullptr;
    KB_CHECK(hipHostGetDevicePointer(&mapped, host_adj_, 0));
    a.adj = static_cast<const AdjT*>(mapped);
    signature_k<AdjT, KeyT><<<w.grid(), kSigNT, 0, st_>>>(a, w);
    KB_LAUNCH_CHECK();
    ++direct_rounds_;
    return;
  }
  if (!copy_st_) {
    KB_CHECK(hipStreamCreateWithFlags(&copy_st_, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
      KB_CHECK(hipEventCreateWithFlags(&win_full_[b], hipEventDisableTiming));
      KB_CHECK(hipEventCreateWithFlags(&win_free_[b], hipEventDisableTiming));
      KB_CHECK(hipEventRecord(win_free_[b], st_));  // nothing reads the windows yet
    }
  }
  for (size_t p = 0; p + 1 < part_node_.size(); ++p) {
    const int b = int(p & 1);
    const uint64_t e0 = part_edge_[p], cnt = part_edge_[p + 1] - e0;
    KB_CHECK(hipStreamWaitEvent(copy_st_, win_free_[b], 0));  // the launch that last read window b is done
    if (cnt)
      KB_CHECK(hipMemcpyAsync(win_[b].p, static_cast<const AdjT*>(host_adj_) + e0, cnt * sizeof(AdjT),
                              hipMemcpyHostToDevice, copy_st_));
    KB_CHECK(hipEventRecord(win_full_[b], copy_st_));
    KB_CHECK(hipStreamWaitEvent(st_, win_full_[b], 0));
    // row offsets are global: the window holds edges [e0, e0 + cnt)
    a.adj = reinterpret_cast<const AdjT*>(reinterpret_cast<uintptr_t>(win_[b].p) - e0 * sizeof(AdjT));
    w.node_lo = part_node_[p];
    w.node_hi = part_node_[p + 1];
    signature_k<AdjT, KeyT><<<w.grid(), kSigNT, 0, st_>>>(a, w);
    KB_LAUNCH_CHECK();
    KB_CHECK(hipEventRecord(win_free_[b], st_));
    streamed_bytes_ += cnt * sizeof(AdjT);
  }
}
