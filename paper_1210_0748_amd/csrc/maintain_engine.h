// Host side of the maintenance of a k-bisimulation partition (Section 4):
// the stored history (change of k), and updates of the graph (Add_Nodes,
// Add_Edges, deletions) brought through every stored round level by level.
// Included by kbisim.hip inside namespace kb, after the round driver.

// ---- history -------------------------------------------------------------------

void Engine::save_level(int32_t j) {
  if (int32_t(hist_.size()) <= j) hist_.resize(size_t(j) + 1);
  const uint64_t N = uint64_t(n_);
  Level& L = hist_[size_t(j)];
  L.ord.ensure(std::max<uint64_t>(N, 1) * 4);
  L.pid.ensure(std::max<uint64_t>(N, 1) * 4);
  if (N) {
    KB_CHECK(hipMemcpyAsync(L.ord.p, ord_.p, N * 4, hipMemcpyDeviceToDevice, st_));
    KB_CHECK(hipMemcpyAsync(L.pid.p, pid_.p, N * 4, hipMemcpyDeviceToDevice, st_));
  }
}

void Engine::load_level(int32_t j) {
  const uint64_t N = uint64_t(n_);
  if (!N) return;
  const Level& L = hist_[size_t(j)];
  KB_CHECK(hipMemcpyAsync(ord_.p, L.ord.p, N * 4, hipMemcpyDeviceToDevice, st_));
  KB_CHECK(hipMemcpyAsync(pid_.p, L.pid.p, N * 4, hipMemcpyDeviceToDevice, st_));
  flags_from_level_k<<<grid_for(N), kNT, 0, st_>>>(ord_.as<uint32_t>(), pid_.as<int32_t>(), uint32_t(N),
                                                   flag_.as<uint8_t>());
  KB_LAUNCH_CHECK();
}

// Dense ids of round j (Section 4, "Change k": a smaller k is answered from
// the stored pId_0..pId_k). Rounds after an early stop equal the last one.
void Engine::result_round(int32_t j, int32_t* pid_out, bool to_device, int64_t* blocks) {
  StreamScope scope(st_);
  if (j < 0) throw InvalidInput("round < 0");
  if (j >= rounds_) {
    if (j > rounds_ && !fixed_) throw StateError("round not computed yet (refine to it first)");
    if (blocks) *blocks = B_;
    if (pid_out) result(pid_out, to_device);
    return;
  }
  if (!opt_.history) throw StateError("earlier rounds need the history option");
  if (blocks) *blocks = counts_[size_t(j)];
  const uint64_t N = uint64_t(n_);
  if (!pid_out || !N) return;
  DevBuf fl, cl, out;
  fl.ensure(N);
  cl.ensure(N * 4);
  const Level& L = hist_[size_t(j)];
  flags_from_level_k<<<grid_for(N), kNT, 0, st_>>>(L.ord.as<uint32_t>(), L.pid.as<int32_t>(), uint32_t(N),
                                                   fl.as<uint8_t>());
  KB_LAUNCH_CHECK();
  scan_dev<uint8_t, uint32_t, true>(fl.as<uint8_t>(), cl.as<uint32_t>(), N);
  int32_t* dst = pid_out;
  if (!to_device) {
    out.ensure(N * 4);
    dst = out.as<int32_t>();
  }
  dense_ids_k<<<grid_for(N), kNT, 0, st_>>>(L.pid.as<int32_t>(), cl.as<uint32_t>(), uint32_t(N), dst);
  KB_LAUNCH_CHECK();
  if (!to_device) KB_CHECK(hipMemcpyAsync(pid_out, dst, N * 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
}

// Reverse table E_ts (edges by target) from the forward one.
void Engine::build_reverse() {
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  rrowptr_.ensure((N + 1) * 4);
  const int wb = adj_bytes();
  radj_.ensure(std::max<uint64_t>(E, 1) * uint64_t(wb));
  if (!E) {
    KB_CHECK(hipMemsetAsync(rrowptr_.p, 0, (N + 1) * 4, st_));
    return;
  }
  DevBuf ka, kb2, vb;
  ka.ensure(E * 4);
  kb2.ensure(E * 4);
  vb.ensure(E * uint64_t(wb));
  const uint32_t tiles = ceil_div(E, kMergeTile);
  bool f;
  if (adj64_) {
    reverse_items_k<uint64_t><<<tiles, 256, 0, st_>>>(rowptr_.as<uint32_t>(), uint32_t(N), adj_.as<uint64_t>(), E,
                                                      dst_bits_, ka.as<uint32_t>(), radj_.as<uint64_t>());
    KB_LAUNCH_CHECK();
    f = radix_sort<uint32_t, uint64_t>(ka.as<uint32_t>(), radj_.as<uint64_t>(), kb2.as<uint32_t>(),
                                       vb.as<uint64_t>(), E, 0, bits_for(N > 1 ? N - 1 : 1), radix_scratch(E), st_, ipt());
  } else {
    reverse_items_k<uint32_t><<<tiles, 256, 0, st_>>>(rowptr_.as<uint32_t>(), uint32_t(N), adj_.as<uint32_t>(), E,
                                                      dst_bits_, ka.as<uint32_t>(), radj_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    f = radix_sort<uint32_t, uint32_t>(ka.as<uint32_t>(), radj_.as<uint32_t>(), kb2.as<uint32_t>(),
                                       vb.as<uint32_t>(), E, 0, bits_for(N > 1 ? N - 1 : 1), radix_scratch(E), st_, ipt());
  }
  if (f) radj_.swap(vb);
  const uint32_t* skey = f ? kb2.as<uint32_t>() : ka.as<uint32_t>();
  DevBuf gaps;
  gaps.ensure((3 * (N / kRowGap + 2) + 1) * 4);
  uint32_t* ng = gaps.as<uint32_t>() + 3 * (N / kRowGap + 2);
  KB_CHECK(hipMemsetAsync(ng, 0, 4, st_));
  csr_rowptr_k<<<grid_stride_blocks(E + 1), kNT, 0, st_>>>(skey, E, uint32_t(N), rrowptr_.as<uint32_t>(),
                                                          gaps.as<uint32_t>(), ng);
  KB_LAUNCH_CHECK();
  csr_rowptr_gaps_k<<<256, kNT, 0, st_>>>(gaps.as<uint32_t>(), ng, rrowptr_.as<uint32_t>());
  KB_LAUNCH_CHECK();
  KB_CHECK(hipStreamSynchronize(st_));  // the temporaries are freed here
}

// Hub offsets, largest degree and the per-round buffers sized by the graph.
void Engine::graph_stats() {
  const uint64_t N = uint64_t(n_), E = uint64_t(m_);
  hub_off_.ensure((E / (uint64_t(kBlockMaxDeg) + 1) + 2) * 4);
  ukey_.ensure(std::max<uint64_t>(E, 1) * (key64_ ? 8 : 4));
  if (!N) return;
  DevBuf hd;
  hd.ensure((N + 1) * sizeof(uint32_t));
  hub_toff_.ensure((N + 1) * sizeof(uint32_t));
  KB_CHECK(hipMemsetAsync(hd.as<uint32_t>() + N, 0, 4, st_));
  hub_degree_k<<<grid_for(N), kNT, 0, st_>>>(rowptr_.as<uint32_t>(), uint32_t(N), kBlockMaxDeg, hd.as<uint32_t>());
  KB_LAUNCH_CHECK();
  scan_dev<uint32_t, uint32_t, false>(hd.as<uint32_t>(), hub_toff_.as<uint32_t>(), N + 1);
  KB_CHECK(hipMemsetAsync(hd.p, 0, 4, st_));
  max_degree_k<<<std::min<uint32_t>(grid_for(N), 1024), kNT, 0, st_>>>(rowptr_.as<uint32_t>(), uint32_t(N),
                                                                     hd.as<uint32_t>());
  KB_LAUNCH_CHECK();
  uint32_t* hw32 = reinterpret_cast<uint32_t*>(hw_.p);
  hw32[0] = hw32[1] = 0;
  KB_CHECK(hipMemcpyAsync(hw32, hub_toff_.as<uint32_t>() + N, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipMemcpyAsync(hw32 + 1, hd.p, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  hub_edges_ = hw32[0];
  maxdeg_ = hw32[1];
  hub_toff_valid_ = true;
  maxdeg_pending_ = false;
}

// Per-node buffers for n_new nodes; the partition state arrays keep their
// contents (new entries zero).
static void grow_keep(DevBuf& b, uint64_t old_bytes, uint64_t new_bytes, hipStream_t s) {
  if (!b.p) old_bytes = 0;  // never allocated: all of it starts at zero
  if (b.p && b.bytes >= new_bytes) {
    if (new_bytes > old_bytes) KB_CHECK(hipMemsetAsync(static_cast<char*>(b.p) + old_bytes, 0, new_bytes - old_bytes, s));
    return;
  }
  DevBuf nb;
  nb.ensure(new_bytes);
  if (b.p && old_bytes) KB_CHECK(hipMemcpyAsync(nb.p, b.p, std::min(old_bytes, new_bytes), hipMemcpyDeviceToDevice, s));
  if (new_bytes > old_bytes) KB_CHECK(hipMemsetAsync(static_cast<char*>(nb.p) + old_bytes, 0, new_bytes - old_bytes, s));
  b.swap(nb);
}

void Engine::grow_nodes(uint64_t n_new) {
  const uint64_t n_old = uint64_t(n_);
  const uint64_t N1 = std::max<uint64_t>(n_new, 1);
  for (DevBuf* b : {&pid_, &ord_, &actr_, &rtag_, &ctag_}) grow_keep(*b, n_old * 4, N1 * 4, st_);
  grow_keep(flag_, n_old, N1, st_);
  for (DevBuf* b : {&cls_, &dtag_, &cont_}) grow_keep(*b, n_old * 4, N1 * 4, st_);
  for (DevBuf* b : {&act_.start, &act_.size, &act_.depth, &soff_}) b->ensure((n_new + 1) * 4);
  for (DevBuf* b : {&apos_, &anode_, &blists_, &fl_, &first_, &ucnt_}) b->ensure(N1 * 4);
  head_.ensure(N1 * 8);
  if (bmslot_.p) bmslot_.ensure(N1 * 4);
}

// Active segments of the coming round from the current partition: every
// class with two or more members (except classes of nodes without edges
// after round 0: their signatures stay empty).
void Engine::rebuild_active() {
  const uint64_t N = uint64_t(n_);
  if (!N) return;
  class_scan();
  ufirst_.ensure(N * 4);
  class_starts_k<<<grid_for(N), kNT, 0, st_>>>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), uint32_t(N),
                                               ufirst_.as<uint32_t>());
  KB_LAUNCH_CHECK();
  const uint32_t med = std::min(medium_cap(), kMediumCapSmall), big = medium_cap();
  KB_CHECK(hipMemsetAsync(act_.size.p, 0, (N + 1) * 4, st_));
  uint32_t* info = info_.as<uint32_t>();
  ClassSegOf of{ufirst_.as<uint32_t>(), cls_.as<uint32_t>() + (N - 1), uint32_t(N), ord_.as<uint32_t>(),
                rowptr_.as<uint32_t>(), med, big, rounds_ > 0};
  compact<kSegClasses>(of, ClassSegWrite{of, act_.start.as<uint32_t>(), act_.size.as<uint32_t>(),
                                         act_.depth.as<uint32_t>()},
                       uint32_t(N), cls_.as<uint32_t>() + (N - 1), compact_scratch(compact_part_words<kSegClasses>(N)),
                       info + kInfoSeg, st_);
  large_offsets(act_, info + kInfoSeg, info + kInfoLargeItems, N);
  prepare_active(uint32_t(N), uint32_t(N), tag_ + 1, true);
}

namespace {
// Host-side merge of sorted distinct values with new ones; map[i] = new rank
// of old value i. Returns whether anything was added.
bool merge_values(const std::vector<int32_t>& old_vals, std::vector<int32_t> add, std::vector<int32_t>& merged,
                  std::vector<uint32_t>& map) {
  std::sort(add.begin(), add.end());
  add.erase(std::unique(add.begin(), add.end()), add.end());
  merged.clear();
  std::set_union(old_vals.begin(), old_vals.end(), add.begin(), add.end(), std::back_inserter(merged));
  map.resize(old_vals.size());
  for (size_t i = 0; i < old_vals.size(); ++i)
    map[i] = uint32_t(std::lower_bound(merged.begin(), merged.end(), old_vals[i]) - merged.begin());
  return merged.size() != old_vals.size();
}

void upload_values(DevBuf& d, const std::vector<int32_t>& v, hipStream_t s) {
  d.ensure(std::max<size_t>(v.size(), 1) * 4);
  if (!v.empty()) KB_CHECK(hipMemcpyAsync(d.p, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
}
}  // namespace

// Sorted update items of one table: added (row, word) by row; deleted by
// (row, word).
template <typename W>
struct TableDelta {
  DevBuf a_row, a_word, d_row, d_word;
  uint32_t m_a = 0, m_d = 0;
};

// One CSR table (forward or reverse) with the update applied: touched rows
// rebuilt, the others moved. Returns the new edge count.
template <typename Wo, typename Wn>
static uint64_t merge_table(DevBuf& rowptr, DevBuf& adj, uint32_t n_o, uint32_t n_n, const TableDelta<Wn>& dt,
                            Reencode<Wo, Wn> re, uint64_t e_o, uint32_t* hw, hipStream_t st,
                            DevBuf& scanpart, DevBuf& radix) {
  const uint32_t m_t = dt.m_a + dt.m_d;
  // touched rows: distinct rows of both lists
  DevBuf rows, rows2, fl, ex, R, cnt, cnt_old;
  const uint64_t mt1 = std::max<uint32_t>(m_t, 1);
  for (DevBuf* b : {&rows, &rows2, &fl, &ex, &R}) b->ensure(mt1 * 4);
  cnt.ensure(16);
  KB_CHECK(hipMemsetAsync(cnt.p, 0, 16, st));
  if (dt.m_a) KB_CHECK(hipMemcpyAsync(rows.p, dt.a_row.p, uint64_t(dt.m_a) * 4, hipMemcpyDeviceToDevice, st));
  if (dt.m_d)
    KB_CHECK(hipMemcpyAsync(rows.as<uint32_t>() + dt.m_a, dt.d_row.p, uint64_t(dt.m_d) * 4, hipMemcpyDeviceToDevice, st));
  auto scan_u32 = [&](const uint32_t* in, uint32_t* out, uint64_t n) {
    scanpart.ensure(scan_partials_count(n) * sizeof(uint64_t));
    scan<uint32_t, uint32_t, false>(in, out, n, scanpart.as<uint32_t>(), st);
  };
  uint32_t r = 0, r_old = 0;
  if (m_t) {
    radix.ensure(radix_scratch_words(m_t) * 4);
    const bool f = radix_sort<uint32_t>(rows.as<uint32_t>(), static_cast<uint32_t*>(nullptr), rows2.as<uint32_t>(),
                                        static_cast<uint32_t*>(nullptr), m_t, 0, bits_for(n_n > 1 ? n_n - 1 : 1),
                                        radix.as<uint32_t>(), st);
    const uint32_t* sk = f ? rows2.as<uint32_t>() : rows.as<uint32_t>();
    run_flags_k<<<grid_for(m_t), kNT, 0, st>>>(sk, m_t, fl.as<uint32_t>());
    KB_LAUNCH_CHECK();
    scan_u32(fl.as<uint32_t>(), ex.as<uint32_t>(), m_t);
    run_scatter_k<<<grid_for(m_t), kNT, 0, st>>>(sk, fl.as<uint32_t>(), ex.as<uint32_t>(), m_t, R.as<uint32_t>(),
                                                 cnt.as<uint32_t>());
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemcpyAsync(hw, cnt.p, 4, hipMemcpyDeviceToHost, st));
    KB_CHECK(hipStreamSynchronize(st));
    r = hw[0];
  }
  const uint32_t r1 = std::max<uint32_t>(r, 1);
  DevBuf a_lo, a_hi, d_lo, d_hi, begs, ends, newdeg, delta, cum, deg, rp_n, adj_n;
  for (DevBuf* b : {&a_lo, &a_hi, &d_lo, &d_hi, &begs, &ends, &newdeg}) b->ensure(uint64_t(r1) * 4);
  delta.ensure((uint64_t(r1) + 1) * 8);
  cum.ensure((uint64_t(r1) + 1) * 8);
  MergeRows mr{R.as<uint32_t>(), cnt.as<uint32_t>(), a_lo.as<uint32_t>(), a_hi.as<uint32_t>(),
               d_lo.as<uint32_t>(), d_hi.as<uint32_t>(), begs.as<uint32_t>(), ends.as<uint32_t>()};
  const uint32_t* rp_o = rowptr.as<uint32_t>();
  if (r) {
    merge_rows_k<<<grid_for(r), kNT, 0, st>>>(mr, dt.a_row.template as<uint32_t>(), dt.m_a,
                                              dt.d_row.template as<uint32_t>(), dt.m_d, rp_o, n_o);
    KB_LAUNCH_CHECK();
    merge_count_k<Wo, Wn><<<std::min<uint32_t>(ceil_div(uint64_t(r) * kWave, 256), 4096), 256, 0, st>>>(
        mr, adj.as<Wo>(), dt.d_word.template as<Wn>(), re, newdeg.as<uint32_t>(),
        delta.as<unsigned long long>());
    KB_LAUNCH_CHECK();
  }
  // new row offsets
  deg.ensure((uint64_t(n_n) + 1) * 4);
  rp_n.ensure((uint64_t(n_n) + 1) * 4);
  old_degrees_k<<<grid_for(uint64_t(n_n) + 1), kNT, 0, st>>>(rp_o, n_o, n_n, deg.as<uint32_t>());
  KB_LAUNCH_CHECK();
  if (r) {
    set_degrees_k<<<grid_for(r), kNT, 0, st>>>(mr, newdeg.as<uint32_t>(), deg.as<uint32_t>());
    KB_LAUNCH_CHECK();
  }
  scan_u32(deg.as<uint32_t>(), rp_n.as<uint32_t>(), uint64_t(n_n) + 1);
  // touched rows of old nodes come first (rows are sorted): their count,
  // and the prefix sums of their degree changes
  KB_CHECK(hipMemcpyAsync(hw, rp_n.as<uint32_t>() + n_n, 4, hipMemcpyDeviceToHost, st));
  KB_CHECK(hipStreamSynchronize(st));
  const uint64_t e_n = hw[0];
  if (r) {
    std::vector<uint32_t> Rh(r);
    KB_CHECK(hipMemcpyAsync(Rh.data(), R.p, uint64_t(r) * 4, hipMemcpyDeviceToHost, st));
    KB_CHECK(hipStreamSynchronize(st));
    r_old = uint32_t(std::lower_bound(Rh.begin(), Rh.end(), n_o) - Rh.begin());
  }
  cnt_old.ensure(4);
  hw[0] = r_old;
  KB_CHECK(hipMemcpyAsync(cnt_old.p, hw, 4, hipMemcpyHostToDevice, st));
  KB_CHECK(hipMemsetAsync(delta.as<unsigned long long>() + r_old, 0, 8, st));
  scanpart.ensure(scan_partials_count(uint64_t(r_old) + 1) * sizeof(uint64_t));
  scan<unsigned long long, unsigned long long, false>(delta.as<unsigned long long>(), cum.as<unsigned long long>(),
                                                      uint64_t(r_old) + 1, scanpart.as<unsigned long long>(), st);
  adj_n.ensure(std::max<uint64_t>(e_n, 1) * sizeof(Wn));
  if (e_o) {
    merge_copy_k<Wo, Wn><<<ceil_div(e_o, kMergeTile), 256, 0, st>>>(mr, cnt_old.as<uint32_t>(),
                                                                   cum.as<unsigned long long>(), adj.as<Wo>(), e_o, re,
                                                                   adj_n.as<Wn>());
    KB_LAUNCH_CHECK();
  }
  if (r) {
    merge_rows_copy_k<Wo, Wn><<<std::min<uint32_t>(ceil_div(uint64_t(r) * kWave, 256), 4096), 256, 0, st>>>(
        mr, adj.as<Wo>(), dt.d_word.template as<Wn>(), dt.a_word.template as<Wn>(), re, rp_n.as<uint32_t>(),
        adj_n.as<Wn>());
    KB_LAUNCH_CHECK();
  }
  KB_CHECK(hipStreamSynchronize(st));  // the temporaries (and hw) are released after this
  rowptr.swap(rp_n);
  adj.swap(adj_n);
  return e_n;
}

// Added and deleted items of both tables: validation and packing (words in
// the new encoding), deleted triples whose label does not occur dropped, then
// sorts by row (and word). err gets the validation bits.
template <typename Wn>
static void pack_delta(const int32_t* src, const int32_t* lab, const int32_t* dst, uint32_t m, uint32_t n_n,
                       const int32_t* vals, uint32_t nv, int bits, bool deleting, TableDelta<Wn>& fwd,
                       TableDelta<Wn>& rev, uint32_t* err, uint32_t* hw, hipStream_t st, DevBuf& scanpart,
                       DevBuf& radix, DevBuf& part) {
  const uint64_t m1 = std::max<uint32_t>(m, 1);
  DevBuf fk, rk, fw, rw, keep, meta;
  for (DevBuf* b : {&fk, &rk, &keep}) b->ensure(m1 * 4);
  fw.ensure(m1 * sizeof(Wn));
  rw.ensure(m1 * sizeof(Wn));
  meta.ensure(16);
  pack_update_k<Wn><<<grid_for(m), kNT, 0, st>>>(src, lab, dst, m, n_n, vals, nv, bits, fk.as<uint32_t>(),
                                                 fw.as<Wn>(), rk.as<uint32_t>(), rw.as<Wn>(), keep.as<uint32_t>(),
                                                 err);
  KB_LAUNCH_CHECK();
  // compact the kept items (deleted triples with unknown labels cannot exist)
  struct KeepOf {
    const uint32_t* keep;
    __device__ int operator()(uint32_t i) const { return keep[i] ? 0 : -1; }
  };
  struct KeepWrite {
    const uint32_t *fk, *rk;
    const Wn *fw, *rw;
    uint32_t *ofk, *ork;
    Wn *ofw, *orw;
    __device__ void operator()(uint32_t i, int, uint32_t o) const {
      ofk[o] = fk[i];
      ork[o] = rk[i];
      ofw[o] = fw[i];
      orw[o] = rw[i];
    }
  };
  TableDelta<Wn>* tabs[2] = {&fwd, &rev};
  DevBuf ck[2], cw[2];
  for (int t = 0; t < 2; ++t) {
    ck[t].ensure(m1 * 4);
    cw[t].ensure(m1 * sizeof(Wn));
  }
  part.ensure(compact_part_words<1>(m1) * 4);
  compact<1>(KeepOf{keep.as<uint32_t>()},
             KeepWrite{fk.as<uint32_t>(), rk.as<uint32_t>(), fw.as<Wn>(), rw.as<Wn>(), ck[0].as<uint32_t>(),
                       ck[1].as<uint32_t>(), cw[0].as<Wn>(), cw[1].as<Wn>()},
             m, nullptr, part.as<uint32_t>(), meta.as<uint32_t>(), st);
  KB_CHECK(hipMemcpyAsync(hw, meta.p, 4, hipMemcpyDeviceToHost, st));
  KB_CHECK(hipStreamSynchronize(st));
  const uint32_t mk = hw[0];
  const int row_bits = bits_for(n_n > 1 ? n_n - 1 : 1);
  const int word_bits = int(sizeof(Wn) * 8);
  radix.ensure(radix_scratch_words(std::max<uint32_t>(mk, 1)) * 4);
  for (int t = 0; t < 2; ++t) {
    TableDelta<Wn>& T = *tabs[t];
    DevBuf& rows = deleting ? T.d_row : T.a_row;
    DevBuf& words = deleting ? T.d_word : T.a_word;
    (deleting ? T.m_d : T.m_a) = mk;
    rows.ensure(std::max<uint32_t>(mk, 1) * 4);
    words.ensure(std::max<uint32_t>(mk, 1) * sizeof(Wn));
    if (!mk) continue;
    DevBuf k2, w2;
    k2.ensure(uint64_t(mk) * 4);
    w2.ensure(uint64_t(mk) * sizeof(Wn));
    if (deleting) {
      // by word (carrying the row), then stably by row
      const bool f1 = radix_sort<Wn, uint32_t>(cw[t].as<Wn>(), ck[t].as<uint32_t>(), w2.as<Wn>(), k2.as<uint32_t>(),
                                               mk, 0, word_bits, radix.as<uint32_t>(), st);
      Wn* W1 = f1 ? w2.as<Wn>() : cw[t].as<Wn>();
      uint32_t* K1 = f1 ? k2.as<uint32_t>() : ck[t].as<uint32_t>();
      Wn* W1b = f1 ? cw[t].as<Wn>() : w2.as<Wn>();
      uint32_t* K1b = f1 ? ck[t].as<uint32_t>() : k2.as<uint32_t>();
      const bool f2 = radix_sort<uint32_t, Wn>(K1, W1, K1b, W1b, mk, 0, row_bits, radix.as<uint32_t>(), st);
      KB_CHECK(hipMemcpyAsync(rows.p, f2 ? K1b : K1, uint64_t(mk) * 4, hipMemcpyDeviceToDevice, st));
      KB_CHECK(hipMemcpyAsync(words.p, f2 ? W1b : W1, uint64_t(mk) * sizeof(Wn), hipMemcpyDeviceToDevice, st));
    } else {
      const bool f = radix_sort<uint32_t, Wn>(ck[t].as<uint32_t>(), cw[t].as<Wn>(), k2.as<uint32_t>(), w2.as<Wn>(),
                                              mk, 0, row_bits, radix.as<uint32_t>(), st);
      KB_CHECK(hipMemcpyAsync(rows.p, f ? k2.p : ck[t].p, uint64_t(mk) * 4, hipMemcpyDeviceToDevice, st));
      KB_CHECK(hipMemcpyAsync(words.p, f ? w2.p : cw[t].p, uint64_t(mk) * sizeof(Wn), hipMemcpyDeviceToDevice, st));
    }
  }
  KB_CHECK(hipStreamSynchronize(st));
}

// The graph part of an update: new label values, both tables merged, new
// encoding. src_list receives the sources of kept changed edges.
template <typename Wo, typename Wn>
static void update_tables(Engine& e, DevBuf& rowptr, DevBuf& adj, DevBuf& rrowptr, DevBuf& radj, uint32_t n_o,
                          uint32_t n_n, uint64_t e_o, const TableDelta<Wn>& fwd, const TableDelta<Wn>& rev,
                          const uint32_t* lmap, int bits_o, int bits_n, uint64_t* e_n, uint32_t* hw, hipStream_t st,
                          DevBuf& scanpart, DevBuf& radix) {
  (void)e;
  Reencode<Wo, Wn> re{lmap, bits_o, bits_n};
  *e_n = merge_table<Wo, Wn>(rowptr, adj, n_o, n_n, fwd, re, e_o, hw, st, scanpart, radix);
  const uint64_t e_r = merge_table<Wo, Wn>(rrowptr, radj, n_o, n_n, rev, re, e_o, hw, st, scanpart, radix);
  if (e_r != *e_n) throw DeviceError(hipErrorUnknown, "edge tables out of step after an update");
}

void Engine::update_core(const UpdateArgs& u) {
  StreamScope scope(st_);
  if (!opt_.history) throw StateError("updates need the history option");
  if (u.n_new < 0 || u.m_add < 0 || u.m_del < 0) throw InvalidInput("negative update size");
  const uint64_t n_o = uint64_t(n_), e_o = uint64_t(m_);
  const uint64_t n_n = n_o + uint64_t(u.n_new);
  if (n_n >= (uint64_t(1) << 31)) throw InvalidInput("num_nodes would reach 2^31");
  if (e_o + uint64_t(u.m_add) >= 0xffffffffull) throw InvalidInput("num_edges would reach 2^32 - 1");
  uint32_t* hw = reinterpret_cast<uint32_t*>(hw_.p);
  DevBuf errb;
  errb.ensure(16);
  KB_CHECK(hipMemsetAsync(errb.p, 0, 16, st_));
  uint32_t* err = errb.as<uint32_t>();

  // --- new label values (validated before anything changes)
  std::vector<int32_t> nvals = nlab_vals_, evals = elab_vals_;
  std::vector<uint32_t> nmap, emap;
  bool nchanged = false, echanged = false;
  DevBuf new_rank;
  if (u.n_new) {
    upload_values(d_nvals_, nlab_vals_, st_);
    new_rank.ensure(uint64_t(u.n_new) * 4);
    rank_new_nodes_k<<<grid_for(uint64_t(u.n_new)), kNT, 0, st_>>>(u.new_label, uint32_t(u.n_new),
                                                                  d_nvals_.as<int32_t>(), uint32_t(nlab_vals_.size()),
                                                                  new_rank.as<uint32_t>(), err);
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemcpyAsync(hw, err, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    if (hw[0] & 2u) throw InvalidInput("negative node label");
    if (hw[0] & 4u) {
      std::vector<int32_t> lab(static_cast<size_t>(u.n_new));
      KB_CHECK(hipMemcpyAsync(lab.data(), u.new_label, lab.size() * 4, hipMemcpyDeviceToHost, st_));
      KB_CHECK(hipStreamSynchronize(st_));
      nchanged = merge_values(nlab_vals_, lab, nvals, nmap);
    }
  }
  const int dst_bits_n = bits_for(n_n > 1 ? n_n - 1 : 1);
  auto check_edges = [&](const int32_t* s, const int32_t* l, const int32_t* d, int64_t m, bool adding) {
    if (!m) return;
    DevBuf fk, rk, w, keep;
    for (DevBuf* b : {&fk, &rk, &keep}) b->ensure(uint64_t(m) * 4);
    w.ensure(uint64_t(m) * 16);
    KB_CHECK(hipMemsetAsync(err, 0, 4, st_));
    upload_values(d_evals_, evals, st_);
    pack_update_k<uint64_t><<<grid_for(uint64_t(m)), kNT, 0, st_>>>(
        s, l, d, uint32_t(m), uint32_t(n_n), d_evals_.as<int32_t>(), uint32_t(evals.size()), dst_bits_n,
        fk.as<uint32_t>(), w.as<uint64_t>(), rk.as<uint32_t>(), w.as<uint64_t>() + m, keep.as<uint32_t>(), err);
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemcpyAsync(hw, err, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    if (hw[0] & 1u) throw InvalidInput("edge endpoint outside [0, num_nodes)");
    if (hw[0] & 2u) throw InvalidInput("negative edge label");
    if (adding && (hw[0] & 4u)) {
      std::vector<int32_t> lab(static_cast<size_t>(m));
      KB_CHECK(hipMemcpyAsync(lab.data(), l, lab.size() * 4, hipMemcpyDeviceToHost, st_));
      KB_CHECK(hipStreamSynchronize(st_));
      std::vector<int32_t> merged;
      std::vector<uint32_t> m2;
      if (merge_values(evals, lab, merged, m2)) {
        // compose with a map from an earlier merge (none here: additions are checked first)
        evals = merged;
        emap = m2;
        echanged = true;
      }
    }
  };
  check_edges(u.add_src, u.add_lab, u.add_dst, u.m_add, true);
  check_edges(u.del_src, u.del_lab, u.del_dst, u.m_del, false);
  if (n_n == 0) return;  // no nodes: nothing can change (every edge was rejected above)

  // --- commit: encodings and both tables
  const uint32_t ne_n = uint32_t(evals.size());
  const int lab_bits_n = ne_n > 1 ? bits_for(ne_n - 1) : 0;
  const bool adj64_n = dst_bits_n + lab_bits_n > 32;
  const bool key64_n = lab_bits_n + bits_for(n_n > 1 ? n_n - 1 : 1) > 32;
  upload_values(d_evals_, evals, st_);
  DevBuf lmap;
  if (echanged) {
    lmap.ensure(std::max<size_t>(emap.size(), 1) * 4);
    if (!emap.empty())
      KB_CHECK(hipMemcpyAsync(lmap.p, emap.data(), emap.size() * 4, hipMemcpyHostToDevice, st_));
  }
  const uint32_t* lm = echanged ? lmap.as<uint32_t>() : nullptr;
  ustat_ = UpdateStat{};
  src_list_.ensure((uint64_t(u.m_add) + uint64_t(u.m_del) + uint64_t(u.n_new) + 1) * 4);
  uint64_t e_n = 0;
  auto run = [&](auto wo_tag, auto wn_tag) {
    using Wo = decltype(wo_tag);
    using Wn = decltype(wn_tag);
    TableDelta<Wn> fwd, rev;
    DevBuf part;
    pack_delta<Wn>(u.add_src, u.add_lab, u.add_dst, uint32_t(u.m_add), uint32_t(n_n), d_evals_.as<int32_t>(), ne_n,
                   dst_bits_n, false, fwd, rev, err, hw, st_, scanpart_, radix_, part);
    pack_delta<Wn>(u.del_src, u.del_lab, u.del_dst, uint32_t(u.m_del), uint32_t(n_n), d_evals_.as<int32_t>(), ne_n,
                   dst_bits_n, true, fwd, rev, err, hw, st_, scanpart_, radix_, part);
    // sources of the kept changed edges are checked at every level
    n_src_ = 0;
    if (fwd.m_a)
      KB_CHECK(hipMemcpyAsync(src_list_.p, fwd.a_row.p, uint64_t(fwd.m_a) * 4, hipMemcpyDeviceToDevice, st_));
    if (fwd.m_d)
      KB_CHECK(hipMemcpyAsync(src_list_.as<uint32_t>() + fwd.m_a, fwd.d_row.p, uint64_t(fwd.m_d) * 4,
                              hipMemcpyDeviceToDevice, st_));
    n_src_ = fwd.m_a + fwd.m_d;
    update_tables<Wo, Wn>(*this, rowptr_, adj_, rrowptr_, radj_, uint32_t(n_o), uint32_t(n_n), e_o, fwd, rev, lm,
                          dst_bits_, dst_bits_n, &e_n, hw, st_, scanpart_, radix_);
  };
  if (adj64_) {
    if (adj64_n) run(uint64_t(), uint64_t()); else run(uint64_t(), uint32_t());
  } else {
    if (adj64_n) run(uint32_t(), uint64_t()); else run(uint32_t(), uint32_t());
  }
  if (e_n >= 0xffffffffull) throw DeviceError(hipErrorUnknown, "edge count overflow after an update");
  // new nodes are checked at every level too (they are new at level 0)
  if (u.n_new) {
    std::vector<uint32_t> ids(static_cast<size_t>(u.n_new));
    for (size_t i = 0; i < ids.size(); ++i) ids[i] = uint32_t(n_o + i);
    KB_CHECK(hipMemcpyAsync(src_list_.as<uint32_t>() + n_src_, ids.data(), ids.size() * 4, hipMemcpyHostToDevice,
                            st_));
    KB_CHECK(hipStreamSynchronize(st_));
    n_src_ += uint32_t(u.n_new);
  }
  nlab_vals_ = nvals;
  elab_vals_ = evals;
  n_elab_ = ne_n;
  lab_bits_ = lab_bits_n;
  dst_bits_ = dst_bits_n;
  adj64_ = adj64_n;
  key64_ = key64_n;
  m_ = int64_t(e_n);
  grow_nodes(n_n);
  const uint64_t n_prev = n_o;
  n_ = int64_t(n_n);
  graph_stats();
  dense_round_ = -1;
  cls_round_ = -1;

  // --- level 0: new nodes join the label classes (new labels: new classes)
  DevBuf nm;
  const bool remap0 = nchanged && !nmap.empty();  // old nodes' label ranks move
  if (remap0) {
    nm.ensure(nmap.size() * 4);
    KB_CHECK(hipMemcpyAsync(nm.p, nmap.data(), nmap.size() * 4, hipMemcpyHostToDevice, st_));
  }
  old_prev_pid_.ensure(std::max<uint64_t>(n_prev, 1) * 4);
  if (n_prev) KB_CHECK(hipMemcpyAsync(old_prev_pid_.p, hist_[0].pid.p, n_prev * 4, hipMemcpyDeviceToDevice, st_));
  const uint32_t T0 = ++utag_;
  if (u.n_new) {
    const uint32_t nl = uint32_t(nvals.size());
    const int nb = nl <= 256 ? 1 : nl <= 65536 ? 2 : 4;
    const uint32_t N = uint32_t(n_n);
    DevBuf ka, kb2, va, vb, p0, bstart;
    for (DevBuf* b : {&ka, &kb2, &va, &vb}) b->ensure(uint64_t(N) * 4);
    p0.ensure(uint64_t(N) * uint64_t(nb));
    bstart.ensure((uint64_t(N) + 1) * 4);
    const uint32_t* rm = remap0 ? nm.as<uint32_t>() : nullptr;
    auto ranks = [&](auto told) {
      using To = decltype(told);
      const To* po = pid0_.as<To>();
      if (nb == 1)
        level0_ranks_k<To, uint8_t><<<grid_for(N), kNT, 0, st_>>>(po, uint32_t(n_prev), new_rank.as<uint32_t>(), N, rm,
                                                                 ka.as<uint32_t>(), va.as<uint32_t>(), p0.as<uint8_t>());
      else if (nb == 2)
        level0_ranks_k<To, uint16_t><<<grid_for(N), kNT, 0, st_>>>(po, uint32_t(n_prev), new_rank.as<uint32_t>(), N, rm,
                                                                  ka.as<uint32_t>(), va.as<uint32_t>(), p0.as<uint16_t>());
      else
        level0_ranks_k<To, uint32_t><<<grid_for(N), kNT, 0, st_>>>(po, uint32_t(n_prev), new_rank.as<uint32_t>(), N, rm,
                                                                  ka.as<uint32_t>(), va.as<uint32_t>(), p0.as<uint32_t>());
      KB_LAUNCH_CHECK();
    };
    // ranks of the new nodes' labels among the merged values
    if (nchanged) {
      upload_values(d_nvals_, nvals, st_);
      KB_CHECK(hipMemsetAsync(err, 0, 4, st_));
      rank_new_nodes_k<<<grid_for(uint64_t(u.n_new)), kNT, 0, st_>>>(u.new_label, uint32_t(u.n_new),
                                                                    d_nvals_.as<int32_t>(), nl, new_rank.as<uint32_t>(),
                                                                    err);
      KB_LAUNCH_CHECK();
    }
    if (pid0_bytes_ == 1) ranks(uint8_t()); else if (pid0_bytes_ == 2) ranks(uint16_t()); else ranks(uint32_t());
    pid0_.swap(p0);
    pid0_bytes_ = nb;
    const bool f = radix_sort<uint32_t>(ka.as<uint32_t>(), va.as<uint32_t>(), kb2.as<uint32_t>(), vb.as<uint32_t>(),
                                        N, 0, bits_for(nl > 1 ? nl - 1 : 1), radix_scratch(N), st_, ipt());
    const uint32_t* keys = f ? kb2.as<uint32_t>() : ka.as<uint32_t>();
    const uint32_t* vals = f ? vb.as<uint32_t>() : va.as<uint32_t>();
    KB_CHECK(hipMemcpyAsync(ord_.p, vals, uint64_t(N) * 4, hipMemcpyDeviceToDevice, st_));
    run_start_flags_k<<<grid_for(N), kNT, 0, st_>>>(keys, N, flag_.as<uint8_t>(), nullptr);
    KB_LAUNCH_CHECK();
    scan_dev<uint8_t, uint32_t, true>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), N);
    block_starts_k<<<grid_for(N), kNT, 0, st_>>>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), N, bstart.as<uint32_t>());
    KB_LAUNCH_CHECK();
    set_u32_k<<<1, 1, 0, st_>>>(bstart.as<uint32_t>() + nl, N);
    KB_LAUNCH_CHECK();
    const uint32_t t0 = ++tag_;  // active marks of a first round, in case none is stored
    if (nb == 1)
      node_ids0_k<uint8_t><<<grid_for(N), kNT, 0, st_>>>(pid0_.as<uint8_t>(), bstart.as<uint32_t>(), N,
                                                         pid_.as<int32_t>(), actr_.as<uint32_t>(), t0);
    else if (nb == 2)
      node_ids0_k<uint16_t><<<grid_for(N), kNT, 0, st_>>>(pid0_.as<uint16_t>(), bstart.as<uint32_t>(), N,
                                                          pid_.as<int32_t>(), actr_.as<uint32_t>(), t0);
    else
      node_ids0_k<uint32_t><<<grid_for(N), kNT, 0, st_>>>(pid0_.as<uint32_t>(), bstart.as<uint32_t>(), N,
                                                          pid_.as<int32_t>(), actr_.as<uint32_t>(), t0);
    KB_LAUNCH_CHECK();
    b0_ = nl;
    save_level(0);
    // the new nodes changed at level 0
    clist_.ensure(std::max<uint64_t>(n_n, 1) * 4);
    KB_CHECK(hipMemcpyAsync(clist_.p, src_list_.as<uint32_t>() + (n_src_ - uint32_t(u.n_new)),
                            uint64_t(u.n_new) * 4, hipMemcpyDeviceToDevice, st_));
    KB_CHECK(hipStreamSynchronize(st_));
  } else {
    load_level(0);
  }
  counts_.assign(1, int64_t(nvals.size()));
  const uint32_t n_c0 = uint32_t(u.n_new);  // changed at level 0 (tagged T0 below)
  clist_.ensure(std::max<uint64_t>(n_n, 1) * 4);
  {
    // tag the new nodes as changed at level 0
    DevBuf tmp;
    if (n_c0) {
      std::vector<uint32_t> t(n_c0, T0);
      tmp.ensure(uint64_t(n_c0) * 4);
      KB_CHECK(hipMemcpyAsync(tmp.p, t.data(), uint64_t(n_c0) * 4, hipMemcpyHostToDevice, st_));
      KB_CHECK(hipMemcpyAsync(ctag_.as<uint32_t>() + n_prev, tmp.p, uint64_t(n_c0) * 4, hipMemcpyDeviceToDevice, st_));
      KB_CHECK(hipStreamSynchronize(st_));
    }
  }
  old_n_nodes_ = uint32_t(n_prev);
  if (adj64_) {
    if (key64_) update_levels<uint64_t, uint64_t>(); else update_levels<uint64_t, uint32_t>();
  } else {
    if (key64_) update_levels<uint32_t, uint64_t>(); else update_levels<uint32_t, uint32_t>();
  }
  // the rest of the rounds asked for, when the fixed point moved; the
  // active set of the next round is rebuilt either way (a later
  // kbisim_refine continues from it)
  rebuild_active();
  while (rounds_ < k_target_) {
    if (fixed_ && opt_.early_stop) break;
    run_round();
  }
  KB_CHECK(hipStreamSynchronize(st_));
}

// Levels 1..rounds_ after the graph and level 0 changed (see maintain.h):
// per level, the frontier, the classes of the level below that hold it
// (re-ordered by signature), the other classes (split as stored), change
// detection and the new stored round. The number of changed nodes at level
// 0 is the number of new nodes (listed in clist_, tagged utag_).
// Graphs from this many nodes on may switch to full rounds on measured times.
constexpr uint32_t kTimedSwitchNodes = 1u << 20;

template <typename AdjT, typename KeyT>
void Engine::update_levels() {
  const uint32_t N = uint32_t(n_);
  const int32_t K = rounds_;
  const uint32_t n_o = old_n_nodes_;
  uint32_t* hw = reinterpret_cast<uint32_t*>(hw_.p);
  // [0] frontier, [1] classes, [2] members, [3] items, [4..5] members of a full round (u64)
  DevBuf cnt;
  cnt.ensure(32);
  uint32_t T_prev = utag_;
  // number of changed nodes of the level below, on the device; at level 0
  // these are the new nodes (listed in clist_)
  DevBuf nch;
  nch.ensure(4);
  hw[0] = N - n_o;
  KB_CHECK(hipMemcpyAsync(nch.p, hw, 4, hipMemcpyHostToDevice, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  const uint64_t N1 = std::max<uint32_t>(N, 1), O1 = uint64_t(n_o) + 1;
  for (DevBuf* b : {&rlist_, &dlist_, &ufirst_, &fill_, &dszpos_, &gw_, &inode_}) b->ensure(N1 * 4);
  for (DevBuf* b : {&dsize_, &isize_, &w_, &wscan_, &chunk_}) b->ensure((N1 + 1) * 4);
  iflag_.ensure(N1);
  for (DevBuf* b : {&keep_, &kscan_, &inu_, &kus_, &oflag_, &ocls_, &ofirst_, &xpos_}) b->ensure(O1 * 4);
  xflag_.ensure(O1);
  const uint32_t med = std::min(medium_cap(), kMediumCapSmall), big = medium_cap();
  int32_t stop_at = -1;
  bool switched = false;
  auto level_start = std::chrono::steady_clock::now();
  double last_level_secs = 0.0;  // host time of the previous level, done level by level
  for (int32_t j = 1; j <= K; ++j) {
    if (j > 1) {
      const auto now = std::chrono::steady_clock::now();
      last_level_secs = std::chrono::duration<double>(now - level_start).count();
      level_start = now;
    }
    const uint32_t T = ++utag_;
    KB_CHECK(hipMemsetAsync(cnt.p, 0, 32, st_));
    uint32_t* c = cnt.as<uint32_t>();
    // frontier: chunks of the changed nodes' sources, then one wave per item
    frontier_chunks_k<<<grid_for(uint64_t(N) + 1), kNT, 0, st_>>>(clist_.as<uint32_t>(), nch.as<uint32_t>(),
                                                                  rrowptr_.as<uint32_t>(), chunk_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    scan_dev<uint32_t, uint32_t, false>(chunk_.as<uint32_t>(), chunk_.as<uint32_t>(), uint64_t(N) + 1);
    const uint32_t fgrid = 2048;
    if (adj64_)
      frontier_k<uint64_t><<<fgrid, 256, 0, st_>>>(src_list_.as<uint32_t>(), n_src_, clist_.as<uint32_t>(),
                                                   nch.as<uint32_t>(), chunk_.as<uint32_t>(), rrowptr_.as<uint32_t>(),
                                                   radj_.as<uint64_t>(), dst_bits_, rtag_.as<uint32_t>(), T,
                                                   rlist_.as<uint32_t>(), c);
    else
      frontier_k<uint32_t><<<fgrid, 256, 0, st_>>>(src_list_.as<uint32_t>(), n_src_, clist_.as<uint32_t>(),
                                                   nch.as<uint32_t>(), chunk_.as<uint32_t>(), rrowptr_.as<uint32_t>(),
                                                   radj_.as<uint32_t>(), dst_bits_, rtag_.as<uint32_t>(), T,
                                                   rlist_.as<uint32_t>(), c);
    KB_LAUNCH_CHECK();
    // classes of level j - 1 that hold the frontier
    class_scan();
    class_starts_k<<<grid_for(N), kNT, 0, st_>>>(flag_.as<uint8_t>(), cls_.as<uint32_t>(), N, ufirst_.as<uint32_t>());
    KB_LAUNCH_CHECK();
    dirty_classes_k<<<std::min<uint32_t>(grid_for(N), kListGrid), kNT, 0, st_>>>(rlist_.as<uint32_t>(), c, pid_.as<int32_t>(), dtag_.as<uint32_t>(), T,
                                                 dlist_.as<uint32_t>(), c + 1);
    KB_LAUNCH_CHECK();
    dirty_sizes_k<<<std::min<uint32_t>(grid_for(N), kListGrid), kNT, 0, st_>>>(dlist_.as<uint32_t>(), c + 1, cls_.as<uint32_t>(),
                                               ufirst_.as<uint32_t>(), N, dsize_.as<uint32_t>(),
                                               dszpos_.as<uint32_t>(), fill_.as<uint32_t>(), c + 2);
    KB_LAUNCH_CHECK();
    multi_members_k<<<std::min<uint32_t>(grid_for(N), 2048), kNT, 0, st_>>>(flag_.as<uint8_t>(), N,
                                                 reinterpret_cast<unsigned long long*>(c + 4));
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemcpyAsync(hw, c, 24, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipMemcpyAsync(hw + 6, cls_.as<uint32_t>() + (N - 1), 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipMemcpyAsync(hw + 7, nch.p, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    const uint32_t nr = hw[0], nd = hw[1], members = hw[2], B_prev = hw[6];
    uint64_t full_members = 0;
    std::memcpy(&full_members, hw + 4, 8);
    if (j > 1) ustat_.changed += hw[7];
    if (j - 1 >= 1) counts_.push_back(int64_t(B_prev));
    if (opt_.early_stop && j - 1 >= 1 && counts_[size_t(j - 1)] == counts_[size_t(j - 2)]) {
      stop_at = j - 1;
      break;
    }
    // Switch back to Algorithm 1 (Section 4, "When to switch back"): when
    // the frontier, or below the frontier and the items to re-order, outnumber
    // the nodes a full round would compute, the remaining rounds run in full
    // from this level (checked first on the frontier alone, before the
    // passes over the stored round).
    // Cost model: a level by level round pays about 0.45 node-passes over
    // all N nodes (the stored round's order, its scans and copies) plus about
    // two node-costs per frontier node and per item; a full round pays one
    // per member of a class with two or more members (measured on the
    // 10M-node power-law graph: 1.8 ms of passes per level, 0.4 ns per node of
    // a full round).
    const uint64_t fixed_cost = uint64_t(N) * 9 / 20;
    auto go_full = [&](uint64_t work) {
      if (opt_.update_mode == 1) return false;
      if (opt_.update_mode == 2) return true;
      return fixed_cost + 2 * work > full_members;
    };
    // The estimate's constant depends on the graph (a full round of
    // identical subtrees is cheap to order); once a level has been done level
    // by level, its measured time against the last full computation of round
    // j can also send the rest to full rounds (on graphs large enough for
    // the times to mean something, with a margin for their noise)
    const bool slower_than_full = opt_.update_mode == 0 && j > 1 && N >= kTimedSwitchNodes &&
                                  last_level_secs > 0.0 && size_t(j) < round_secs_.size() &&
                                  round_secs_[size_t(j)] > 0.0 && last_level_secs > 1.2 * round_secs_[size_t(j)];
    if (go_full(nr) || slower_than_full) {
      stop_at = j - 1;
      switched = true;
      ustat_.full_from = j;
      break;
    }
    // the stored round j: frontier membership, kept classes, class starts
    old_ord_.swap(hist_[size_t(j)].ord);
    old_pid_.swap(hist_[size_t(j)].pid);
    if (n_o) {
      old_flags_k<<<grid_for(n_o), kNT, 0, st_>>>(old_ord_.as<uint32_t>(), old_pid_.as<int32_t>(), n_o,
                                                  rtag_.as<uint32_t>(), T, ctag_.as<uint32_t>(), T_prev,
                                                  inu_.as<uint32_t>(), keep_.as<uint32_t>(), oflag_.as<uint32_t>());
      KB_LAUNCH_CHECK();
      KB_CHECK(hipMemsetAsync(inu_.as<uint32_t>() + n_o, 0, 4, st_));
      KB_CHECK(hipMemsetAsync(keep_.as<uint32_t>() + n_o, 0, 4, st_));
      scan_dev<uint32_t, uint32_t, false>(inu_.as<uint32_t>(), kus_.as<uint32_t>(), O1);
      scan_dev<uint32_t, uint32_t, false>(keep_.as<uint32_t>(), kscan_.as<uint32_t>(), O1);
      scan_dev<uint32_t, uint32_t, true>(oflag_.as<uint32_t>(), ocls_.as<uint32_t>(), n_o);
      old_starts_k<<<grid_for(n_o), kNT, 0, st_>>>(oflag_.as<uint32_t>(), ocls_.as<uint32_t>(), n_o,
                                                   ofirst_.as<uint32_t>());
      KB_LAUNCH_CHECK();
    }
    // items of the re-ordered classes (counted only: the partition of level
    // j - 1 stays intact until the choice below)
    auto items = [&](bool place) {
      items_frontier_k<<<std::min<uint32_t>(grid_for(N), kListGrid), kNT, 0, st_>>>(rlist_.as<uint32_t>(), c, pid_.as<int32_t>(),
                                                    dszpos_.as<uint32_t>(), fill_.as<uint32_t>(), place,
                                                    ord_.as<uint32_t>(), gw_.as<uint32_t>());
      KB_LAUNCH_CHECK();
      if (n_o) {
        items_reps_k<<<grid_for(n_o), kNT, 0, st_>>>(old_ord_.as<uint32_t>(), old_pid_.as<int32_t>(), n_o,
                                                     inu_.as<uint32_t>(), kus_.as<uint32_t>(), ocls_.as<uint32_t>(),
                                                     ofirst_.as<uint32_t>(), pid_.as<int32_t>(), dtag_.as<uint32_t>(), T,
                                                     dszpos_.as<uint32_t>(), fill_.as<uint32_t>(), place,
                                                     ord_.as<uint32_t>(), gw_.as<uint32_t>());
        KB_LAUNCH_CHECK();
      }
    };
    items(false);
    item_sizes_k<<<std::min<uint32_t>(grid_for(N), kListGrid), kNT, 0, st_>>>(dlist_.as<uint32_t>(), c + 1, dszpos_.as<uint32_t>(),
                                              fill_.as<uint32_t>(), isize_.as<uint32_t>(), c + 3);
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemcpyAsync(hw, c + 3, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    const uint32_t n_items = hw[0];
    if (go_full(uint64_t(nr) + uint64_t(n_items))) {
      stop_at = j - 1;
      switched = true;
      ustat_.full_from = j;
      break;
    }
    ustat_.rechecked += nr;
    ustat_.recomputed += n_items;
    ustat_.levels = j;
    // re-ordered classes: segments of their items
    KB_CHECK(hipMemsetAsync(act_.size.p, 0, (uint64_t(nd) + 1) * 4, st_));
    uint32_t* info = info_.as<uint32_t>();
    compact<kSegClasses>(DirtySegOf{dlist_.as<uint32_t>(), isize_.as<uint32_t>(), med, big},
                         DirtySegWrite{dlist_.as<uint32_t>(), isize_.as<uint32_t>(), act_.start.as<uint32_t>(),
                                       act_.size.as<uint32_t>(), act_.depth.as<uint32_t>()},
                         nd, nullptr, compact_scratch(compact_part_words<kSegClasses>(std::max<uint32_t>(nd, 1))),
                         info + kInfoSeg, st_);
    large_offsets(act_, info + kInfoSeg, info + kInfoLargeItems, n_items);
    items(true);
    prepare_active(nd, n_items, tag_ + 1, true);
    const uint32_t M_items = M_act_;
    if (M_items > 0) {
      // level 1 keys from the dense label ranks (narrow, as in a first
      // round: they order exactly as the level-0 class positions)
      round_impl<AdjT, KeyT>(j == 1);
      // expand: items to their final positions, groups behind their representatives
      items_read_k<<<grid_for(uint64_t(M_items) + 1), kNT, 0, st_>>>(apos_.as<uint32_t>(), M_items, ord_.as<uint32_t>(),
                                                                     flag_.as<uint8_t>(), gw_.as<uint32_t>(),
                                                                     inode_.as<uint32_t>(), iflag_.as<uint8_t>(),
                                                                     w_.as<uint32_t>());
      KB_LAUNCH_CHECK();
      scan_dev<uint32_t, uint32_t, false>(w_.as<uint32_t>(), wscan_.as<uint32_t>(), uint64_t(M_items) + 1);
      items_place_k<<<grid_for(M_items), kNT, 0, st_>>>(apos_.as<uint32_t>(), M_items, inode_.as<uint32_t>(),
                                                        iflag_.as<uint8_t>(), wscan_.as<uint32_t>(), pid_.as<int32_t>(),
                                                        rtag_.as<uint32_t>(), T, old_pid_.as<int32_t>(),
                                                        ord_.as<uint32_t>(), flag_.as<uint8_t>(), xpos_.as<uint32_t>(),
                                                        xflag_.as<uint8_t>());
      KB_LAUNCH_CHECK();
      if (n_o) {
        groups_place_k<<<grid_for(n_o), kNT, 0, st_>>>(old_ord_.as<uint32_t>(), old_pid_.as<int32_t>(), n_o,
                                                       inu_.as<uint32_t>(), kus_.as<uint32_t>(), pid_.as<int32_t>(),
                                                       dtag_.as<uint32_t>(), T, dszpos_.as<uint32_t>(),
                                                       xpos_.as<uint32_t>(), xflag_.as<uint8_t>(), ord_.as<uint32_t>(),
                                                       flag_.as<uint8_t>());
        KB_LAUNCH_CHECK();
      }
    }
    // the other classes split as stored
    if (n_o) {
      copy_split_k<<<grid_for(n_o), kNT, 0, st_>>>(old_ord_.as<uint32_t>(), n_o, keep_.as<uint32_t>(),
                                                   kscan_.as<uint32_t>(), old_prev_pid_.as<int32_t>(),
                                                   old_pid_.as<int32_t>(), dtag_.as<uint32_t>(), T,
                                                   ord_.as<uint32_t>(), flag_.as<uint8_t>(), pid_.as<int32_t>());
      KB_LAUNCH_CHECK();
    }
    cls_round_ = -1;
    dense_round_ = -1;
    // ids of the re-ordered classes (all their positions) and change detection
    if (members > 0) {
      KB_CHECK(hipMemsetAsync(dsize_.as<uint32_t>() + nd, 0, 4, st_));
      scan_dev<uint32_t, uint32_t, false>(dsize_.as<uint32_t>(), soff_.as<uint32_t>(), uint64_t(nd) + 1);
      expand_k<<<std::max<uint32_t>(1, ceil_div(members, kExpandTile)), 256, 0, st_>>>(
          dlist_.as<uint32_t>(), soff_.as<uint32_t>(), c + 1, members, ord_.as<uint32_t>(), apos_.as<uint32_t>(),
          anode_.as<uint32_t>(), nullptr, 0u, info);
      KB_LAUNCH_CHECK();
      M_act_ = members;
      assign_ids();
      cont_reset_k<<<grid_for(members), kNT, 0, st_>>>(apos_.as<uint32_t>(), members, cont_.as<uint32_t>());
      KB_LAUNCH_CHECK();
      cont_set_k<<<grid_for(members), kNT, 0, st_>>>(apos_.as<uint32_t>(), members, ord_.as<uint32_t>(),
                                                     pid_.as<int32_t>(), rtag_.as<uint32_t>(), T, n_o,
                                                     old_pid_.as<int32_t>(), cont_.as<uint32_t>());
      KB_LAUNCH_CHECK();
    }
    KB_CHECK(hipMemsetAsync(nch.p, 0, 4, st_));
    changed_k<<<std::min<uint32_t>(grid_for(std::max<uint32_t>(nr, 1)), kListGrid), kNT, 0, st_>>>(
        rlist_.as<uint32_t>(), c, actr_.as<uint32_t>(), M_items > 0 ? tag_ : kNoneU32, pid_.as<int32_t>(),
        cont_.as<uint32_t>(), n_o, old_pid_.as<int32_t>(), ctag_.as<uint32_t>(), T, clist_.as<uint32_t>(),
        nch.as<uint32_t>());
    KB_LAUNCH_CHECK();
    save_level(j);
    old_prev_pid_.swap(old_pid_);
    T_prev = T;
  }
  const int32_t last = stop_at >= 0 ? stop_at : K;
  if (stop_at < 0 && K >= 1) {
    // class count of the last level
    class_scan();
    KB_CHECK(hipMemcpyAsync(hw, cls_.as<uint32_t>() + (N - 1), 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipMemcpyAsync(hw + 1, nch.p, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    counts_.push_back(int64_t(hw[0]));
    ustat_.changed += hw[1];
  }
  rounds_ = last;
  hist_.resize(size_t(last) + 1);
  counts_.resize(size_t(last) + 1);
  B_ = counts_.back();
  fixed_ = !switched && last >= 1 && counts_[size_t(last)] == counts_[size_t(last) - 1];
  cls_round_ = -1;
  dense_round_ = -1;
}

// ---- node deletion --------------------------------------------------------------

// An update with deleted nodes: their incoming and outgoing edges are deleted
// (Section 4, "Deletions": a node goes after its edges), added edges are
// mapped to the numbering before the deletion, one level-by-level update
// runs, and the then isolated nodes leave every stored round (a node without
// edges is in no other node's signature, so the others keep their classes;
// positions and node ids close up).
void Engine::update(const UpdateArgs& u) {
  StreamScope scope(st_);
  if (!opt_.history) throw StateError("updates need the history option");
  if (u.n_del < 0 || u.n_new < 0 || u.m_add < 0 || u.m_del < 0) throw InvalidInput("negative update size");
  if (u.n_del == 0) return update_core(u);
  const uint64_t n_all = uint64_t(n_) + uint64_t(u.n_new);
  if (n_all >= (uint64_t(1) << 31)) throw InvalidInput("num_nodes would reach 2^31");
  uint32_t* hw = reinterpret_cast<uint32_t*>(hw_.p);
  // survivors: alive[v] over the nodes after the new ones; newid = exclusive scan
  DevBuf alive, newid, oldid, errb;
  alive.ensure((n_all + 1) * 4);
  newid.ensure((n_all + 1) * 4);
  oldid.ensure(std::max<uint64_t>(n_all, 1) * 4);
  errb.ensure(8);
  KB_CHECK(hipMemsetAsync(errb.p, 0, 8, st_));
  fill_u32_k<<<grid_for(n_all + 1), kNT, 0, st_>>>(alive.as<uint32_t>(), n_all + 1, 1u);
  KB_LAUNCH_CHECK();
  KB_CHECK(hipMemsetAsync(alive.as<uint32_t>() + n_all, 0, 4, st_));
  mark_deleted_k<<<grid_for(uint64_t(u.n_del)), kNT, 0, st_>>>(u.del_nodes, uint32_t(u.n_del), uint32_t(n_all),
                                                              alive.as<uint32_t>(), errb.as<uint32_t>());
  KB_LAUNCH_CHECK();
  scan_dev<uint32_t, uint32_t, false>(alive.as<uint32_t>(), newid.as<uint32_t>(), n_all + 1);
  KB_CHECK(hipMemcpyAsync(hw, errb.p, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipMemcpyAsync(hw + 1, newid.as<uint32_t>() + n_all, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  if (hw[0]) throw InvalidInput("deleted node outside [0, num_nodes + num_new_nodes)");
  const uint32_t n_keep = hw[1];
  survivors_k<<<grid_for(n_all), kNT, 0, st_>>>(newid.as<uint32_t>(), uint32_t(n_all), oldid.as<uint32_t>());
  KB_LAUNCH_CHECK();
  // added edges in the numbering before the deletion
  DevBuf as, ad;
  as.ensure(std::max<int64_t>(u.m_add, 1) * 4);
  ad.ensure(std::max<int64_t>(u.m_add, 1) * 4);
  if (u.m_add) {
    KB_CHECK(hipMemsetAsync(errb.p, 0, 4, st_));
    unmap_edges_k<<<grid_for(uint64_t(u.m_add)), kNT, 0, st_>>>(u.add_src, u.add_dst, uint32_t(u.m_add), n_keep,
                                                                oldid.as<uint32_t>(), as.as<int32_t>(),
                                                                ad.as<int32_t>(), errb.as<uint32_t>());
    KB_LAUNCH_CHECK();
    KB_CHECK(hipMemcpyAsync(hw, errb.p, 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    if (hw[0]) throw InvalidInput("added edge endpoint outside [0, num_nodes) after the deletions");
  }
  // edges of the deleted nodes (old nodes only: new nodes have none yet),
  // as triples with label values, plus the explicit deletions
  const uint32_t n_old = uint32_t(n_);
  DevBuf dn, cntb, off;
  dn.ensure(uint64_t(u.n_del) * 4);
  cntb.ensure((uint64_t(u.n_del) + 1) * 4);
  off.ensure((uint64_t(u.n_del) + 1) * 4);
  incident_counts_k<<<grid_for(uint64_t(u.n_del)), kNT, 0, st_>>>(u.del_nodes, uint32_t(u.n_del), n_old,
                                                                 rowptr_.as<uint32_t>(), rrowptr_.as<uint32_t>(),
                                                                 cntb.as<uint32_t>());
  KB_LAUNCH_CHECK();
  KB_CHECK(hipMemsetAsync(cntb.as<uint32_t>() + u.n_del, 0, 4, st_));
  scan_dev<uint32_t, uint32_t, false>(cntb.as<uint32_t>(), off.as<uint32_t>(), uint64_t(u.n_del) + 1);
  KB_CHECK(hipMemcpyAsync(hw, off.as<uint32_t>() + u.n_del, 4, hipMemcpyDeviceToHost, st_));
  KB_CHECK(hipStreamSynchronize(st_));
  const uint64_t m_inc = hw[0];
  const uint64_t m_d = uint64_t(u.m_del) + m_inc;
  DevBuf ds, dl, dd;
  for (DevBuf* b : {&ds, &dl, &dd}) b->ensure(std::max<uint64_t>(m_d, 1) * 4);
  if (u.m_del) {
    KB_CHECK(hipMemcpyAsync(ds.p, u.del_src, uint64_t(u.m_del) * 4, hipMemcpyDeviceToDevice, st_));
    KB_CHECK(hipMemcpyAsync(dl.p, u.del_lab, uint64_t(u.m_del) * 4, hipMemcpyDeviceToDevice, st_));
    KB_CHECK(hipMemcpyAsync(dd.p, u.del_dst, uint64_t(u.m_del) * 4, hipMemcpyDeviceToDevice, st_));
  }
  if (m_inc) {
    upload_values(d_evals_, elab_vals_, st_);
    const uint32_t waves = uint32_t(u.n_del) * 2;
    if (adj64_)
      incident_edges_k<uint64_t><<<std::min<uint32_t>(ceil_div(uint64_t(waves) * kWave, 256), 4096), 256, 0, st_>>>(
          u.del_nodes, uint32_t(u.n_del), n_old, rowptr_.as<uint32_t>(), adj_.as<uint64_t>(), rrowptr_.as<uint32_t>(),
          radj_.as<uint64_t>(), dst_bits_, d_evals_.as<int32_t>(), off.as<uint32_t>(), ds.as<int32_t>() + u.m_del,
          dl.as<int32_t>() + u.m_del, dd.as<int32_t>() + u.m_del);
    else
      incident_edges_k<uint32_t><<<std::min<uint32_t>(ceil_div(uint64_t(waves) * kWave, 256), 4096), 256, 0, st_>>>(
          u.del_nodes, uint32_t(u.n_del), n_old, rowptr_.as<uint32_t>(), adj_.as<uint32_t>(), rrowptr_.as<uint32_t>(),
          radj_.as<uint32_t>(), dst_bits_, d_evals_.as<int32_t>(), off.as<uint32_t>(), ds.as<int32_t>() + u.m_del,
          dl.as<int32_t>() + u.m_del, dd.as<int32_t>() + u.m_del);
    KB_LAUNCH_CHECK();
  }
  UpdateArgs core = u;
  core.n_del = 0;
  core.del_nodes = nullptr;
  core.m_del = int64_t(m_d);
  core.del_src = ds.as<int32_t>();
  core.del_lab = dl.as<int32_t>();
  core.del_dst = dd.as<int32_t>();
  core.add_src = as.as<int32_t>();
  core.add_dst = ad.as<int32_t>();
  update_core(core);
  remove_nodes(newid.as<uint32_t>(), n_keep);
}

// Removes the nodes with newid[v] == newid[v + 1] (isolated by now) from
// the tables and every stored round, renumbering the others newid[v].
void Engine::remove_nodes(const uint32_t* newid, uint32_t n_keep) {
  const uint32_t n_all = uint32_t(n_);
  const int32_t K = rounds_;
  uint32_t* hw = reinterpret_cast<uint32_t*>(hw_.p);
  if (n_keep == 0) {  // nothing left: the state of an empty graph
    n_ = 0;
    m_ = 0;
    hist_.clear();
    nlab_vals_.clear();
    elab_vals_.clear();
    const int32_t kt = k_target_;
    build(nullptr, nullptr, nullptr, nullptr);
    k_target_ = 0;
    refine(kt);
    return;
  }
  // tables: rows of removed nodes are empty; endpoints renumbered
  const int bits_n = bits_for(n_keep > 1 ? n_keep - 1 : 1);
  auto table = [&](DevBuf& rowptr, DevBuf& adj) {
    DevBuf rp;
    rp.ensure((uint64_t(n_keep) + 1) * 4);
    compact_rowptr_k<<<grid_for(uint64_t(n_all) + 1), kNT, 0, st_>>>(rowptr.as<uint32_t>(), newid, n_all,
                                                                     rp.as<uint32_t>());
    KB_LAUNCH_CHECK();
    rowptr.swap(rp);
    const uint64_t E = uint64_t(m_);
    if (E) {
      if (adj64_)
        renumber_words_k<uint64_t><<<grid_stride_blocks(E), kNT, 0, st_>>>(adj.as<uint64_t>(), E, dst_bits_, bits_n,
                                                                           newid);
      else
        renumber_words_k<uint32_t><<<grid_stride_blocks(E), kNT, 0, st_>>>(adj.as<uint32_t>(), E, dst_bits_, bits_n,
                                                                           newid);
      KB_LAUNCH_CHECK();
    }
  };
  table(rowptr_, adj_);
  table(rrowptr_, radj_);
  dst_bits_ = bits_n;
  // (a narrower endpoint field only shrinks the words: the word and key
  // types stay wide enough)
  // every stored round: positions close up, class starts move to the first
  // surviving member, ids renumbered
  DevBuf alivep, npos, fl8;
  alivep.ensure((uint64_t(n_all) + 1) * 4);
  npos.ensure((uint64_t(n_all) + 1) * 4);
  fl8.ensure(std::max<uint32_t>(n_keep, 1));
  counts_.assign(size_t(K) + 1, 0);
  for (int32_t j = 0; j <= K; ++j) {
    Level& L = hist_[size_t(j)];
    alive_positions_k<<<grid_for(uint64_t(n_all) + 1), kNT, 0, st_>>>(L.ord.as<uint32_t>(), newid, n_all,
                                                                      alivep.as<uint32_t>());
    KB_LAUNCH_CHECK();
    scan_dev<uint32_t, uint32_t, false>(alivep.as<uint32_t>(), npos.as<uint32_t>(), uint64_t(n_all) + 1);
    DevBuf no, np;
    no.ensure(uint64_t(n_keep) * 4);
    np.ensure(uint64_t(n_keep) * 4);
    close_level_k<<<grid_for(n_all), kNT, 0, st_>>>(L.ord.as<uint32_t>(), L.pid.as<int32_t>(), n_all, newid,
                                                    npos.as<uint32_t>(), no.as<uint32_t>(), np.as<int32_t>(),
                                                    fl8.as<uint8_t>());
    KB_LAUNCH_CHECK();
    L.ord.swap(no);
    L.pid.swap(np);
    // classes left: flags of the closed-up round
    scan_dev<uint8_t, uint32_t, true>(fl8.as<uint8_t>(), cls_.as<uint32_t>(), n_keep);
    KB_CHECK(hipMemcpyAsync(hw, cls_.as<uint32_t>() + (n_keep - 1), 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    counts_[size_t(j)] = hw[0];
  }
  // label values still present (one per level-0 class left, read through
  // the old narrow pId_0 of each class's first member) and the new narrow
  // pId_0 (dense level-0 ranks)
  {
    const Level& L0 = hist_[0];
    const uint32_t B0 = uint32_t(counts_[0]);
    DevBuf first, oldid, oldrank, p0;
    first.ensure(std::max<uint32_t>(B0, 1) * 4);
    oldid.ensure(uint64_t(n_keep) * 4);
    oldrank.ensure(std::max<uint32_t>(B0, 1) * 4);
    flags_from_level_k<<<grid_for(n_keep), kNT, 0, st_>>>(L0.ord.as<uint32_t>(), L0.pid.as<int32_t>(), n_keep,
                                                          fl8.as<uint8_t>());
    KB_LAUNCH_CHECK();
    scan_dev<uint8_t, uint32_t, true>(fl8.as<uint8_t>(), cls_.as<uint32_t>(), n_keep);
    class_starts_k<<<grid_for(n_keep), kNT, 0, st_>>>(fl8.as<uint8_t>(), cls_.as<uint32_t>(), n_keep,
                                                      first.as<uint32_t>());
    KB_LAUNCH_CHECK();
    survivors_k<<<grid_for(n_all), kNT, 0, st_>>>(newid, n_all, oldid.as<uint32_t>());
    KB_LAUNCH_CHECK();
    auto ranks = [&](auto told) {
      using To = decltype(told);
      level0_labels_k<To><<<grid_for(B0), kNT, 0, st_>>>(first.as<uint32_t>(), L0.ord.as<uint32_t>(), B0,
                                                         oldid.as<uint32_t>(), pid0_.as<To>(), oldrank.as<uint32_t>());
      KB_LAUNCH_CHECK();
    };
    if (pid0_bytes_ == 1) ranks(uint8_t()); else if (pid0_bytes_ == 2) ranks(uint16_t()); else ranks(uint32_t());
    std::vector<uint32_t> fr(B0);
    if (B0) KB_CHECK(hipMemcpyAsync(fr.data(), oldrank.p, uint64_t(B0) * 4, hipMemcpyDeviceToHost, st_));
    KB_CHECK(hipStreamSynchronize(st_));
    std::vector<int32_t> vals(B0);
    for (uint32_t b = 0; b < B0; ++b) vals[b] = nlab_vals_[fr[b]];
    nlab_vals_ = vals;
    const int nb = B0 <= 256 ? 1 : B0 <= 65536 ? 2 : 4;
    p0.ensure(uint64_t(n_keep) * uint64_t(nb));
    auto narrow = [&](auto tnew) {
      using Tn = decltype(tnew);
      dense_level0_k<Tn><<<grid_for(n_keep), kNT, 0, st_>>>(L0.pid.as<int32_t>(), cls_.as<uint32_t>(), n_keep,
                                                            p0.as<Tn>());
      KB_LAUNCH_CHECK();
    };
    if (nb == 1) narrow(uint8_t()); else if (nb == 2) narrow(uint16_t()); else narrow(uint32_t());
    KB_CHECK(hipStreamSynchronize(st_));
    pid0_.swap(p0);
    pid0_bytes_ = nb;
    b0_ = B0;
  }
  n_ = int64_t(n_keep);
  // the first fixed point of the closed-up counts ends the stored rounds
  int32_t last = K;
  if (opt_.early_stop)
    for (int32_t j = 1; j <= K; ++j)
      if (counts_[size_t(j)] == counts_[size_t(j - 1)]) {
        last = j;
        break;
      }
  rounds_ = last;
  hist_.resize(size_t(last) + 1);
  counts_.resize(size_t(last) + 1);
  B_ = counts_.back();
  fixed_ = last >= 1 && counts_[size_t(last)] == counts_[size_t(last) - 1];
  for (DevBuf* b : {&rtag_, &ctag_, &dtag_}) KB_CHECK(hipMemsetAsync(b->p, 0, b->bytes, st_));
  load_level(rounds_);
  graph_stats();
  dense_round_ = -1;
  cls_round_ = -1;
  if (!(fixed_ && opt_.early_stop) && rounds_ < k_target_) {
    rebuild_active();
    while (rounds_ < k_target_) {
      if (fixed_ && opt_.early_stop) break;
      run_round();
    }
  } else {
    rebuild_active();
  }
  KB_CHECK(hipStreamSynchronize(st_));
}
