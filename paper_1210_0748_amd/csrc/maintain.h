// Kernels of the maintenance of a k-bisimulation partition (Section 4 of the
// paper: change of k, Add_Nodes, Add_Edges and deletions) on a handle that
// keeps the history of every round.
//
// The paper keeps pId_0..pId_k per node (Table 3), the edge table sorted by
// source and by target (E_st, E_ts) and the signature store S, and pushes
// changes level by level through a priority queue (Algorithm 3). Here a
// round's partition is stored as its node order `ord` (classes contiguous,
// in canonical order) and class-start position ids; E_st and E_ts are two
// CSR tables; the queue becomes one device frontier per level: the sources
// of changed edges, the nodes whose class changed at the level below, and
// their sources through the reverse table. Classes of the level below that
// hold no frontier node keep their split of the old history (copied with a
// scan over the old order); the others are re-ordered by signature with the
// round kernels.
#pragma once

#include "common.h"
#include "scan_radix.h"

namespace kb {

constexpr uint32_t kNoneU32 = 0xffffffffu;

// flag[p] = 1 at the first position of every class of a stored round:
// the class-start position id of the node at p is p itself.
__global__ void flags_from_level_k(const uint32_t* __restrict__ ord, const int32_t* __restrict__ pid, uint32_t n,
                                   uint8_t* __restrict__ flag) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) flag[p] = uint32_t(pid[ord[p]]) == p ? 1 : 0;
}

// Rank of value v among the sorted distinct values vals[0..nv), or kNoneU32.
__device__ __forceinline__ uint32_t value_rank(const int32_t* vals, uint32_t nv, int32_t v) {
  uint32_t lo = 0, hi = nv;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (vals[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < nv && vals[lo] == v) ? lo : kNoneU32;
}

// Edges of an update: validation and packing into the words of both tables.
// Forward: key = src, word = (label rank << bits) | dst; reverse: key = dst,
// word = (label rank << bits) | src. err bits: 1 an endpoint outside [0, n),
// 2 a negative label, 4 a label value not among vals. keep[e] = 1 for an
// edge with neither.
template <typename W>
__global__ void pack_update_k(const int32_t* __restrict__ src, const int32_t* __restrict__ lab,
                              const int32_t* __restrict__ dst, uint32_t m, uint32_t n,
                              const int32_t* __restrict__ vals, uint32_t nv, int bits,
                              uint32_t* __restrict__ fkey, W* __restrict__ fword, uint32_t* __restrict__ rkey,
                              W* __restrict__ rword, uint32_t* __restrict__ keep, uint32_t* __restrict__ err) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t s = src[e], l = lab[e], t = dst[e];
  uint32_t bad = 0;
  if (s < 0 || uint32_t(s) >= n || t < 0 || uint32_t(t) >= n) bad |= 1u;
  if (l < 0) bad |= 2u;
  const uint32_t r = bad ? kNoneU32 : value_rank(vals, nv, l);
  if (!bad && r == kNoneU32) bad |= 4u;
  if (bad) atomicOr(err, bad);
  keep[e] = bad ? 0u : 1u;
  fkey[e] = bad ? 0u : uint32_t(s);
  rkey[e] = bad ? 0u : uint32_t(t);
  fword[e] = bad ? W(0) : (W(r) << bits) | W(uint32_t(t));
  rword[e] = bad ? W(0) : (W(r) << bits) | W(uint32_t(s));
}

// Node labels of new nodes: err bit 2 for a negative label, 4 for a value
// not among vals; rank[i] otherwise.
__global__ void rank_new_nodes_k(const int32_t* __restrict__ lab, uint32_t m, const int32_t* __restrict__ vals,
                                 uint32_t nv, uint32_t* __restrict__ rank, uint32_t* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t l = lab[i];
  uint32_t bad = l < 0 ? 2u : 0u;
  const uint32_t r = bad ? kNoneU32 : value_rank(vals, nv, l);
  if (!bad && r == kNoneU32) bad |= 4u;
  if (bad) atomicOr(err, bad);
  rank[i] = r;
}

// Old table words in the new encoding: label rank through lmap (or kept),
// endpoint bits from bits_o to bits_n.
template <typename Wo, typename Wn>
struct Reencode {
  const uint32_t* lmap;  // old rank -> new rank, or null
  int bits_o, bits_n;
  __device__ __forceinline__ Wn operator()(Wo w) const {
    const Wo mask = (Wo(1) << bits_o) - 1;
    const uint32_t end = uint32_t(w & mask);
    uint32_t r = uint32_t(w >> bits_o);
    if (lmap) r = lmap[r];
    return (Wn(r) << bits_n) | Wn(end);
  }
};

// Distinct values of a sorted key array: flags for a scan.
__global__ void run_flags_k(const uint32_t* __restrict__ key, uint32_t m, uint32_t* __restrict__ fl) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) fl[i] = (i == 0 || key[i] != key[i - 1]) ? 1u : 0u;
}
__global__ void run_scatter_k(const uint32_t* __restrict__ key, const uint32_t* __restrict__ fl,
                              const uint32_t* __restrict__ ex, uint32_t m, uint32_t* __restrict__ out,
                              uint32_t* __restrict__ count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  if (fl[i]) out[ex[i]] = key[i];
  if (i == m - 1) *count = ex[i] + fl[i];
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t v) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t v) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
// Whether v occurs in the sorted range a[lo, hi).
template <typename W>
__device__ __forceinline__ bool contains_sorted(const W* a, uint32_t lo, uint32_t hi, W v) {
  uint32_t l = lo, h = hi;
  while (l < h) {
    const uint32_t mid = (l + h) >> 1;
    if (a[mid] < v)
      l = mid + 1;
    else
      h = mid;
  }
  return l < hi && a[l] == v;
}

// Rows touched by an update (sorted distinct row ids R[0..r)): their ranges
// in the sorted added (a_row) and deleted (d_row) lists, old degree, and the
// old row range (begs/ends, E_o for rows of new nodes).
struct MergeRows {
  const uint32_t* R;
  const uint32_t* count;  // r on the device
  uint32_t *a_lo, *a_hi, *d_lo, *d_hi, *begs, *ends;
};
__global__ void merge_rows_k(MergeRows mr, const uint32_t* __restrict__ a_row, uint32_t m_a,
                             const uint32_t* __restrict__ d_row, uint32_t m_d, const uint32_t* __restrict__ rp_o,
                             uint32_t n_o) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *mr.count) return;
  const uint32_t row = mr.R[i];
  mr.a_lo[i] = lower_bound_u32(a_row, 0, m_a, row);
  mr.a_hi[i] = upper_bound_u32(a_row, 0, m_a, row);
  mr.d_lo[i] = lower_bound_u32(d_row, 0, m_d, row);
  mr.d_hi[i] = upper_bound_u32(d_row, 0, m_d, row);
  const uint32_t e_o = rp_o[n_o];
  mr.begs[i] = row < n_o ? rp_o[row] : e_o;
  mr.ends[i] = row < n_o ? rp_o[row + 1] : e_o;
}

// One wave per touched row: old edges that survive the deletions, new
// degree and the change of degree.
template <typename Wo, typename Wn>
__global__ __launch_bounds__(256) void merge_count_k(MergeRows mr, const Wo* __restrict__ adj_o,
                                                     const Wn* __restrict__ d_word, Reencode<Wo, Wn> re,
                                                     uint32_t* __restrict__ newdeg,
                                                     unsigned long long* __restrict__ delta) {
  const uint32_t r = *mr.count;
  const uint32_t lane = __lane_id();
  for (uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < r;
       i += (gridDim.x * blockDim.x) / kWave) {
    const uint32_t b = mr.begs[i], e = mr.ends[i], dl = mr.d_lo[i], dh = mr.d_hi[i];
    uint32_t kept = 0;
    for (uint32_t x = b + lane; x < e; x += kWave) {
      const Wn w = re(adj_o[x]);
      kept += contains_sorted(d_word, dl, dh, w) ? 0u : 1u;
    }
    kept = wave_sum(kept);
    if (lane == 0) {
      const uint32_t nd = kept + (mr.a_hi[i] - mr.a_lo[i]);
      newdeg[i] = nd;
      delta[i] = (unsigned long long)(int64_t(nd) - int64_t(e - b));
    }
  }
}

// Degrees of all rows of the new table (old degree, 0 for new nodes), then
// the touched rows' new degrees.
__global__ void old_degrees_k(const uint32_t* __restrict__ rp_o, uint32_t n_o, uint32_t n_n, uint32_t* __restrict__ deg) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s <= n_n) deg[s] = s < n_o ? rp_o[s + 1] - rp_o[s] : 0u;
}
__global__ void set_degrees_k(MergeRows mr, const uint32_t* __restrict__ newdeg, uint32_t* __restrict__ deg) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < *mr.count) deg[mr.R[i]] = newdeg[i];
}

// Edges of untouched rows move by the change of degree of the touched rows
// before them: with ends[] non-decreasing, the touched rows before edge e
// are those with ends <= e (t of them), and e lies in touched row t when
// begs[t] <= e. One tile of kMergeTile edges per workgroup; the tile's range
// of touched rows is found once.
constexpr uint32_t kMergeTile = 4096;
template <typename Wo, typename Wn>
__global__ __launch_bounds__(256) void merge_copy_k(MergeRows mr, const uint32_t* __restrict__ r_old_dev,
                                                    const unsigned long long* __restrict__ cum,
                                                    const Wo* __restrict__ adj_o, uint64_t e_o,
                                                    Reencode<Wo, Wn> re, Wn* __restrict__ adj_n) {
  __shared__ uint32_t range[2];
  const uint64_t t0 = uint64_t(blockIdx.x) * kMergeTile;
  if (t0 >= e_o) return;
  const uint64_t t1 = t0 + kMergeTile < e_o ? t0 + kMergeTile : e_o;
  const uint32_t ro = *r_old_dev;
  if (threadIdx.x == 0) {
    range[0] = upper_bound_u32(mr.ends, 0, ro, uint32_t(t0));
    range[1] = upper_bound_u32(mr.ends, 0, ro, uint32_t(t1 - 1));
  }
  __syncthreads();
  const uint32_t lo = range[0], hi = range[1];
  for (uint64_t e = t0 + threadIdx.x; e < t1; e += blockDim.x) {
    const uint32_t i = lo == hi ? lo : upper_bound_u32(mr.ends, lo, hi, uint32_t(e));
    if (i < ro && mr.begs[i] <= uint32_t(e)) continue;  // inside a touched row
    adj_n[e + cum[i]] = re(adj_o[e]);
  }
}

// One wave per touched row: surviving old edges in their order, then the
// added ones.
template <typename Wo, typename Wn>
__global__ __launch_bounds__(256) void merge_rows_copy_k(MergeRows mr, const Wo* __restrict__ adj_o,
                                                         const Wn* __restrict__ d_word,
                                                         const Wn* __restrict__ a_word, Reencode<Wo, Wn> re,
                                                         const uint32_t* __restrict__ rp_n, Wn* __restrict__ adj_n) {
  const uint32_t r = *mr.count;
  const uint32_t lane = __lane_id();
  for (uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < r;
       i += (gridDim.x * blockDim.x) / kWave) {
    const uint32_t b = mr.begs[i], e = mr.ends[i], dl = mr.d_lo[i], dh = mr.d_hi[i];
    uint32_t base = rp_n[mr.R[i]];
    for (uint32_t x0 = b; x0 < e; x0 += kWave) {
      const uint32_t x = x0 + lane;
      Wn w = 0;
      bool keep = false;
      if (x < e) {
        w = re(adj_o[x]);
        keep = !contains_sorted(d_word, dl, dh, w);
      }
      const uint64_t bal = __ballot(keep);
      if (keep) adj_n[base + uint32_t(__popcll(bal & lanemask_lt()))] = w;
      base += uint32_t(__popcll(bal));
    }
    const uint32_t al = mr.a_lo[i], ah = mr.a_hi[i];
    for (uint32_t j = al + lane; j < ah; j += kWave) adj_n[base + (j - al)] = a_word[j];
  }
}

// Reverse table items from the forward table: for every edge of row s with
// word (r << bits) | t, key t and word (r << bits) | s. One tile of
// kMergeTile edges per workgroup, rows found by binary search in rowptr.
template <typename W>
__global__ __launch_bounds__(256) void reverse_items_k(const uint32_t* __restrict__ rowptr, uint32_t n,
                                                       const W* __restrict__ adj, uint64_t m, int bits,
                                                       uint32_t* __restrict__ rkey, W* __restrict__ rword) {
  __shared__ uint32_t range[2];
  const uint64_t t0 = uint64_t(blockIdx.x) * kMergeTile;
  if (t0 >= m) return;
  const uint64_t t1 = t0 + kMergeTile < m ? t0 + kMergeTile : m;
  if (threadIdx.x == 0) {  // rows containing the first and last edge
    range[0] = upper_bound_u32(rowptr, 0, n + 1, uint32_t(t0)) - 1;
    range[1] = upper_bound_u32(rowptr, 0, n + 1, uint32_t(t1 - 1)) - 1;
  }
  __syncthreads();
  const uint32_t lo = range[0], hi = range[1];
  const W mask = (W(1) << bits) - 1;
  for (uint64_t e = t0 + threadIdx.x; e < t1; e += blockDim.x) {
    const uint32_t s = lo == hi ? lo : upper_bound_u32(rowptr, lo, hi + 1, uint32_t(e)) - 1;
    const W w = adj[e];
    rkey[e] = uint32_t(w & mask);
    rword[e] = ((w >> bits) << bits) | W(s);
  }
}

// ---- level-wise propagation -------------------------------------------------

// Marks node p for the frontier of this level (once per tag) and appends it.
// Every lane of the wave calls it.
__device__ __forceinline__ void frontier_mark(bool want, uint32_t p, uint32_t* __restrict__ rtag, uint32_t tag,
                                              uint32_t* __restrict__ rlist, uint32_t* __restrict__ rcount) {
  const bool fresh = want && atomicExch(&rtag[p], tag) != tag;
  const uint32_t slot = wave_append(fresh, rcount);
  if (fresh) rlist[slot] = p;
}

// Frontier of level j (Algorithm 3's queue at level j): every node of
// `always` (sources of changed edges and new nodes, checked at every level),
// and every node of `changed` (its class changed at level j - 1, so its own
// head changed) with its sources through the reverse table. Work items are
// one listed node, or one chunk of kFrontierChunk sources of a changed node
// (chunk_off = exclusive scan of the chunks per changed node), one wave each,
// so a node with very many sources is spread over many waves.
constexpr uint32_t kFrontierChunk = 2048;
__global__ void frontier_chunks_k(const uint32_t* __restrict__ changed, const uint32_t* __restrict__ n_changed_dev,
                                  const uint32_t* __restrict__ rrowptr, uint32_t* __restrict__ chunks) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = *n_changed_dev;
  if (i > n) return;
  if (i == n) {
    chunks[i] = 0;
    return;
  }
  const uint32_t u = changed[i];
  chunks[i] = (rrowptr[u + 1] - rrowptr[u] + kFrontierChunk - 1) / kFrontierChunk;
}
template <typename W>
__global__ __launch_bounds__(256) void frontier_k(const uint32_t* __restrict__ always, uint32_t n_always,
                                                  const uint32_t* __restrict__ changed,
                                                  const uint32_t* __restrict__ n_changed_dev,
                                                  const uint32_t* __restrict__ chunk_off,
                                                  const uint32_t* __restrict__ rrowptr, const W* __restrict__ radj,
                                                  int bits, uint32_t* __restrict__ rtag, uint32_t tag,
                                                  uint32_t* __restrict__ rlist, uint32_t* __restrict__ rcount) {
  const uint32_t n_changed = *n_changed_dev;
  const uint32_t n_chunks = chunk_off[n_changed];
  const uint32_t total = n_always + n_changed + n_chunks;
  const uint32_t lane = __lane_id();
  const W mask = (W(1) << bits) - 1;
  for (uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < total;
       i += (gridDim.x * blockDim.x) / kWave) {
    if (i < n_always + n_changed) {  // a listed node itself
      const uint32_t u = i < n_always ? always[i] : changed[i - n_always];
      frontier_mark(lane == 0, u, rtag, tag, rlist, rcount);
      continue;
    }
    // chunk q of the sources of changed node t (chunk_off[t] <= q < chunk_off[t + 1])
    const uint32_t q = i - n_always - n_changed;
    uint32_t lo = 0, hi = n_changed;  // last t with chunk_off[t] <= q
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (chunk_off[mid] <= q)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t u = changed[lo];
    const uint32_t b = rrowptr[u] + (q - chunk_off[lo]) * kFrontierChunk;
    const uint32_t e = min(b + kFrontierChunk, rrowptr[u + 1]);
    // each lane marks its sources of the chunk, keeps the fresh ones, and
    // the wave appends them with one atomic
    constexpr int kPer = int(kFrontierChunk / kWave);
    uint32_t fresh[kPer];
    int nf = 0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const uint32_t x = b + uint32_t(t) * kWave + lane;
      if (x < e) {
        const uint32_t p = uint32_t(radj[x] & mask);
        if (atomicExch(&rtag[p], tag) != tag) fresh[nf++] = p;
      }
    }
    const uint32_t incl = wave_inclusive_scan(uint32_t(nf));
    const uint32_t tot = __shfl(incl, kWave - 1, kWave);
    uint32_t base = 0;
    if (lane == 0 && tot) base = atomicAdd(rcount, tot);
    base = __shfl(base, 0, kWave) + incl - uint32_t(nf);
    for (int t = 0; t < nf; ++t) rlist[base + uint32_t(t)] = fresh[t];
  }
}

// Classes of level j - 1 holding a frontier node (by class-start position).
// Kernels over device-sized lists run a capped grid; every wave steps
// through the list together (wave_append needs all its lanes).
#define KB_LIST_LOOP(i, n)                                                                        \
  for (uint32_t kb_base = blockIdx.x * blockDim.x; kb_base < (n); kb_base += gridDim.x * blockDim.x) \
    if (const uint32_t i = kb_base + threadIdx.x; true)
constexpr uint32_t kListGrid = 1024;

__global__ void dirty_classes_k(const uint32_t* __restrict__ rlist, const uint32_t* __restrict__ rcount,
                                const int32_t* __restrict__ pid, uint32_t* __restrict__ dtag, uint32_t tag,
                                uint32_t* __restrict__ dlist, uint32_t* __restrict__ dcount) {
  const uint32_t n = *rcount;
  KB_LIST_LOOP(i, n) {
    const bool in = i < n;
    const uint32_t c = in ? uint32_t(pid[rlist[i]]) : 0u;
    const bool fresh = in && atomicExch(&dtag[c], tag) != tag;
    const uint32_t slot = wave_append(fresh, dcount);
    if (fresh) dlist[slot] = c;
  }
}

// First position of every class (cls = inclusive scan of the class-start flags).
__global__ void class_starts_k(const uint8_t* __restrict__ flag, const uint32_t* __restrict__ cls, uint32_t n,
                               uint32_t* __restrict__ firstpos) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n && flag[p]) firstpos[cls[p] - 1] = p;
}

// Size of every listed class; members of those with two or more summed.
__global__ void dirty_sizes_k(const uint32_t* __restrict__ dlist, const uint32_t* __restrict__ dcount,
                              const uint32_t* __restrict__ cls, const uint32_t* __restrict__ firstpos, uint32_t n,
                              uint32_t* __restrict__ dsize, uint32_t* __restrict__ dsz_pos, uint32_t* __restrict__ fill,
                              uint32_t* __restrict__ members) {
  const uint32_t nd = *dcount, B = cls[n - 1];
  KB_LIST_LOOP(i, nd) {
    uint32_t z = 0;
    if (i < nd) {
      const uint32_t c = dlist[i];
      const uint32_t ci = cls[c] - 1;
      const uint32_t next = ci + 1 < B ? firstpos[ci + 1] : n;
      z = next - c;
      dsize[i] = z >= 2 ? z : 0u;
      dsz_pos[c] = z;
      fill[c] = 0;
    }
    z = wave_sum(z >= 2 ? z : 0u);
    if (__lane_id() == 0 && z) atomicAdd(members, z);
  }
}

// Members of the classes with two or more members (an upper bound on the
// nodes a full round re-orders), from the class-start flags alone.
__global__ __launch_bounds__(256) void multi_members_k(const uint8_t* __restrict__ flag, uint32_t n,
                                                       unsigned long long* __restrict__ total) {
  __shared__ uint32_t sh[256 / kWave];
  uint32_t z = 0;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
    z += (flag[p] && (p + 1 == n || flag[p + 1])) ? 0u : 1u;
  z = block_sum<256>(z, sh);
  if (threadIdx.x == 0 && z) atomicAdd(total, (unsigned long long)z);
}

// ---- re-ordered classes through representatives ----------------------------
// A class of level j - 1 that holds frontier nodes (R) also holds nodes
// outside the frontier (U); U nodes keep their level-j signature, so the U
// nodes of one stored class X of round j stay together (one new class, the
// continuation of X). Only one representative per such group (the first U
// member of X in the stored order) and the R nodes are ordered by signature;
// the groups are expanded to their members afterwards.

// Slot of this lane among the lanes of its wave that add to the same
// counter (one atomic per distinct counter in the wave, not per lane: the
// items of one big class arrive together). Every lane of the wave calls it.
__device__ __forceinline__ uint32_t wave_group_add(bool want, uint32_t key, uint32_t* __restrict__ counters) {
  uint64_t pending = __ballot(want);
  uint32_t slot = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t k = __shfl(key, leader, kWave);
    const uint64_t same = __ballot(want && key == k);
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(&counters[k], uint32_t(__popcll(same)));
    base = __shfl(base, leader, kWave);
    if (want && key == k) slot = base + uint32_t(__popcll(same & lanemask_lt()));
    pending &= ~same;
  }
  return slot;
}

// Per old position p of the stored round j: inU[p] = the node is outside
// the frontier; keep[p] = the node kept its class at level j - 1; oflag[p] =
// p starts a stored class.
__global__ void old_flags_k(const uint32_t* __restrict__ old_ord, const int32_t* __restrict__ old_pid, uint32_t n_o,
                            const uint32_t* __restrict__ rtag, uint32_t tag, const uint32_t* __restrict__ ctag,
                            uint32_t tag_prev, uint32_t* __restrict__ inU, uint32_t* __restrict__ keep,
                            uint32_t* __restrict__ oflag) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_o) return;
  const uint32_t u = old_ord[p];
  inU[p] = rtag[u] != tag ? 1u : 0u;
  keep[p] = ctag[u] != tag_prev ? 1u : 0u;
  oflag[p] = uint32_t(old_pid[u]) == p ? 1u : 0u;
}

// Items of the re-ordered classes (dsz[class start] >= 2): the frontier
// nodes and the representatives. With place = false only counted (per class
// start, in fill), with place = true also written to ord from the class
// start on (fill counted from zero again). gw[u] = the item's weight: the
// size of its group for a representative, 1 for a frontier node.
__global__ void items_frontier_k(const uint32_t* __restrict__ rlist, const uint32_t* __restrict__ rcount,
                                 const int32_t* __restrict__ pid, const uint32_t* __restrict__ dsz,
                                 uint32_t* __restrict__ fill, bool place, uint32_t* __restrict__ ord,
                                 uint32_t* __restrict__ gw) {
  const uint32_t n = *rcount;
  KB_LIST_LOOP(i, n) {
    bool want = false;
    uint32_t u = 0, c = 0;
    if (i < n) {
      u = rlist[i];
      c = uint32_t(pid[u]);
      want = dsz[c] >= 2;
    }
    const uint32_t slot = wave_group_add(want, c, fill);
    if (want && place) {
      ord[c + slot] = u;
      gw[u] = 1u;
    }
  }
}
__global__ void items_reps_k(const uint32_t* __restrict__ old_ord, const int32_t* __restrict__ old_pid, uint32_t n_o,
                             const uint32_t* __restrict__ inU, const uint32_t* __restrict__ kus,
                             const uint32_t* __restrict__ ocls, const uint32_t* __restrict__ ofirst,
                             const int32_t* __restrict__ pid, const uint32_t* __restrict__ dtag, uint32_t tag,
                             const uint32_t* __restrict__ dsz, uint32_t* __restrict__ fill, bool place,
                             uint32_t* __restrict__ ord, uint32_t* __restrict__ gw) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  bool want = false;
  uint32_t u = 0, c = 0, xs = 0;
  if (p < n_o && inU[p]) {
    u = old_ord[p];
    c = uint32_t(pid[u]);
    if (dtag[c] == tag && dsz[c] >= 2) {
      xs = uint32_t(old_pid[u]);
      want = kus[p] == kus[xs];  // the first U member of its stored class
    }
  }
  const uint32_t slot = wave_group_add(want, c, fill);
  if (!want || !place) return;
  const uint32_t ci = ocls[xs] - 1, B = ocls[n_o - 1];
  const uint32_t xe = ci + 1 < B ? ofirst[ci + 1] : n_o;
  ord[c + slot] = u;
  gw[u] = kus[xe] - kus[xs];
}

// Per re-ordered class: its item count becomes the segment size; fill is
// cleared for the placing pass; the items are summed.
__global__ void item_sizes_k(const uint32_t* __restrict__ dlist, const uint32_t* __restrict__ dcount,
                             const uint32_t* __restrict__ dsz, uint32_t* __restrict__ fill,
                             uint32_t* __restrict__ isize, uint32_t* __restrict__ total) {
  const uint32_t nd = *dcount;
  KB_LIST_LOOP(i, nd) {
    uint32_t z = 0;
    if (i < nd) {
      const uint32_t c = dlist[i];
      z = dsz[c] >= 2 ? fill[c] : 0u;
      isize[i] = z;
      fill[c] = 0;
    }
    z = wave_sum(z);
    if (__lane_id() == 0 && z) atomicAdd(total, z);
  }
}

// First position of every stored class (u32 flags, ocls inclusive scan).
__global__ void old_starts_k(const uint32_t* __restrict__ oflag, const uint32_t* __restrict__ ocls, uint32_t n,
                             uint32_t* __restrict__ ofirst) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n && oflag[p]) ofirst[ocls[p] - 1] = p;
}

// After the ordering: the items in their order, and their weights.
__global__ void items_read_k(const uint32_t* __restrict__ apos, uint32_t m, const uint32_t* __restrict__ ord,
                             const uint8_t* __restrict__ flag, const uint32_t* __restrict__ gw,
                             uint32_t* __restrict__ inode, uint8_t* __restrict__ iflag, uint32_t* __restrict__ w) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > m) return;
  if (j == m) {
    w[j] = 0;
    return;
  }
  const uint32_t u = ord[apos[j]];
  inode[j] = u;
  iflag[j] = flag[apos[j]];
  w[j] = gw[u];
}
// Final position of item j: its class start plus the weights of the items
// before it in the class (W = exclusive scan of the weights; the first item
// of j's class is j - (apos[j] - class start)). A frontier node goes there;
// a representative leaves the position and its flag for its group.
__global__ void items_place_k(const uint32_t* __restrict__ apos, uint32_t m, const uint32_t* __restrict__ inode,
                              const uint8_t* __restrict__ iflag, const uint32_t* __restrict__ W,
                              const int32_t* __restrict__ pid, const uint32_t* __restrict__ rtag, uint32_t tag,
                              const int32_t* __restrict__ old_pid, uint32_t* __restrict__ ord,
                              uint8_t* __restrict__ flag, uint32_t* __restrict__ xpos, uint8_t* __restrict__ xflag) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const uint32_t u = inode[j];
  const uint32_t c = uint32_t(pid[u]);
  const uint32_t j0 = j - (apos[j] - c);
  const uint32_t fp = c + (W[j] - W[j0]);
  if (rtag[u] == tag) {
    ord[fp] = u;
    flag[fp] = iflag[j];
  } else {
    xpos[uint32_t(old_pid[u])] = fp;
    xflag[uint32_t(old_pid[u])] = iflag[j];
  }
}
// The groups: every U member of a re-ordered class at its representative's
// position plus its rank in the group (stored order).
__global__ void groups_place_k(const uint32_t* __restrict__ old_ord, const int32_t* __restrict__ old_pid, uint32_t n_o,
                               const uint32_t* __restrict__ inU, const uint32_t* __restrict__ kus,
                               const int32_t* __restrict__ pid, const uint32_t* __restrict__ dtag, uint32_t tag,
                               const uint32_t* __restrict__ dsz, const uint32_t* __restrict__ xpos,
                               const uint8_t* __restrict__ xflag, uint32_t* __restrict__ ord,
                               uint8_t* __restrict__ flag) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_o || !inU[p]) return;
  const uint32_t u = old_ord[p];
  const uint32_t c = uint32_t(pid[u]);
  if (dtag[c] != tag || dsz[c] < 2) return;
  const uint32_t xs = uint32_t(old_pid[u]);
  const uint32_t t = kus[p] - kus[xs];
  const uint32_t dest = xpos[xs] + t;
  ord[dest] = u;
  flag[dest] = t == 0 ? xflag[xs] : 0;
}

// Old positions p of the stored round j whose node kept its class at level
// j - 1 (not changed there): keep[p] = 1.
__global__ void keep_flags_k(const uint32_t* __restrict__ old_ord, uint32_t n_o, const uint32_t* __restrict__ ctag,
                             uint32_t tag_prev, uint32_t* __restrict__ keep) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_o) keep[p] = ctag[old_ord[p]] != tag_prev ? 1u : 0u;
}

// Classes of level j - 1 without frontier nodes split as in the stored
// round j: their members (exactly the kept members of one old class of
// level j - 1, which starts at old_prev_pid[u] in the old order) keep their
// old order, and the first kept member of each old class of level j starts
// a class. ks = exclusive scan of keep over old positions.
__global__ void copy_split_k(const uint32_t* __restrict__ old_ord, uint32_t n_o, const uint32_t* __restrict__ keep,
                             const uint32_t* __restrict__ ks, const int32_t* __restrict__ old_prev_pid,
                             const int32_t* __restrict__ old_pid, const uint32_t* __restrict__ dtag, uint32_t tag,
                             uint32_t* __restrict__ ord, uint8_t* __restrict__ flag, int32_t* __restrict__ pid) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_o || !keep[p]) return;
  const uint32_t u = old_ord[p];
  const uint32_t c = uint32_t(pid[u]);
  if (dtag[c] == tag) return;  // re-ordered by signature instead
  const uint32_t base = ks[uint32_t(old_prev_pid[u])];
  const uint32_t first = ks[uint32_t(old_pid[u])];
  const uint32_t dest = c + (ks[p] - base);
  ord[dest] = u;
  flag[dest] = ks[p] == first ? 1 : 0;
  pid[u] = int32_t(c + (first - base));
}

// Change detection in the re-ordered classes. A new class that holds a node
// outside the frontier continues that node's old class (every such node of
// one old class lands in one new class, and no two old classes share one);
// cont[class start] = the old class (its old start position).
__global__ void cont_reset_k(const uint32_t* __restrict__ apos, uint32_t m, uint32_t* __restrict__ cont) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) cont[apos[i]] = kNoneU32;
}
__global__ void cont_set_k(const uint32_t* __restrict__ apos, uint32_t m, const uint32_t* __restrict__ ord,
                           const int32_t* __restrict__ pid, const uint32_t* __restrict__ rtag, uint32_t tag,
                           uint32_t n_o, const int32_t* __restrict__ old_pid, uint32_t* __restrict__ cont) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t u = ord[apos[i]];
  if (rtag[u] == tag || u >= n_o) return;
  cont[uint32_t(pid[u])] = uint32_t(old_pid[u]);
}
// A frontier node changed at level j unless it joined the continuation of
// its own old class. Nodes of classes that were not re-ordered (alone at
// level j - 1) and new nodes count as changed. Changed nodes are listed and
// tagged for the next level.
__global__ void changed_k(const uint32_t* __restrict__ rlist, const uint32_t* __restrict__ rcount,
                          const uint32_t* __restrict__ actr, uint32_t act_tag, const int32_t* __restrict__ pid,
                          const uint32_t* __restrict__ cont, uint32_t n_o, const int32_t* __restrict__ old_pid,
                          uint32_t* __restrict__ ctag, uint32_t tag, uint32_t* __restrict__ clist,
                          uint32_t* __restrict__ ccount) {
  const uint32_t n = *rcount;
  KB_LIST_LOOP(i, n) {
    bool ch = false;
    uint32_t u = 0;
    if (i < n) {
      u = rlist[i];
      ch = u >= n_o || actr[u] != act_tag || cont[uint32_t(pid[u])] != uint32_t(old_pid[u]);
      if (ch) ctag[u] = tag;
    }
    const uint32_t slot = wave_append(ch, ccount);
    if (ch) clist[slot] = u;
  }
}

// Classes with two or more members whose members have out-edges (the
// active segments of the coming round, from a full class scan).
struct ClassSegOf {
  const uint32_t* firstpos;
  const uint32_t* nclass;
  uint32_t n;
  const uint32_t* ord;
  const uint32_t* rowptr;
  uint32_t medium_cap, big_cap;
  bool skip_edgeless;  // members of a class of round >= 1 share their signature: all or none have edges
  __device__ __forceinline__ uint32_t size(uint32_t c) const {
    return (c + 1 < *nclass ? firstpos[c + 1] : n) - firstpos[c];
  }
  __device__ __forceinline__ int operator()(uint32_t c) const {
    const uint32_t z = size(c);
    if (z < 2) return -1;
    const uint32_t u = ord[firstpos[c]];
    if (skip_edgeless && rowptr[u + 1] == rowptr[u]) return -1;
    return seg_class(z, medium_cap, big_cap);
  }
};
struct ClassSegWrite {
  ClassSegOf of;
  uint32_t *o_start, *o_size, *o_depth;
  __device__ __forceinline__ void operator()(uint32_t c, int, uint32_t o) const {
    o_start[o] = of.firstpos[c];
    o_size[o] = of.size(c);
    o_depth[o] = 0;
  }
};

// Re-ordered classes of level j - 1 (size >= 2) as segments.
struct DirtySegOf {
  const uint32_t* dlist;
  const uint32_t* dsize;  // 0 or 1: no segment
  uint32_t medium_cap, big_cap;
  __device__ __forceinline__ int operator()(uint32_t i) const {
    const uint32_t z = dsize[i];
    return z >= 2 ? seg_class(z, medium_cap, big_cap) : -1;
  }
};
struct DirtySegWrite {
  const uint32_t* dlist;
  const uint32_t* dsize;
  uint32_t *o_start, *o_size, *o_depth;
  __device__ __forceinline__ void operator()(uint32_t i, int, uint32_t o) const {
    o_start[o] = dlist[i];
    o_size[o] = dsize[i];
    o_depth[o] = 0;
  }
};

// Distinct values of a sorted array (run starts fl, cl = inclusive scan of fl).
__global__ void distinct_values_k(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ fl,
                                  const uint32_t* __restrict__ cl, uint32_t n, int32_t* __restrict__ vals) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && fl[i]) vals[cl[i] - 1] = int32_t(keys[i]);
}

// Level 0 after new nodes: every node's label rank (old nodes through the
// map of old ranks to new ones), as sort items and in the narrow id type.
template <typename Told, typename Tnew>
__global__ void level0_ranks_k(const Told* __restrict__ old_rank, uint32_t n_o, const uint32_t* __restrict__ new_rank,
                               uint32_t n_n, const uint32_t* __restrict__ rmap, uint32_t* __restrict__ key,
                               uint32_t* __restrict__ idx, Tnew* __restrict__ narrow) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_n) return;
  uint32_t r = u < n_o ? uint32_t(old_rank[u]) : new_rank[u - n_o];
  if (u < n_o && rmap) r = rmap[r];
  key[u] = r;
  idx[u] = u;
  narrow[u] = Tnew(r);
}

// ---- node deletion --------------------------------------------------------------

__global__ void fill_u32_k(uint32_t* __restrict__ a, uint64_t n, uint32_t v) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// alive[v] = 0 for every listed node; err = 1 for an id outside [0, n).
__global__ void mark_deleted_k(const int32_t* __restrict__ del, uint32_t m, uint32_t n, uint32_t* __restrict__ alive,
                               uint32_t* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t v = del[i];
  if (v < 0 || uint32_t(v) >= n) {
    atomicOr(err, 1u);
    return;
  }
  alive[v] = 0;
}

// oldid[newid[v]] = v for the surviving nodes (newid[v + 1] > newid[v]).
__global__ void survivors_k(const uint32_t* __restrict__ newid, uint32_t n, uint32_t* __restrict__ oldid) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && newid[v + 1] != newid[v]) oldid[newid[v]] = v;
}

// Added edges from the numbering after the deletion to the one before.
__global__ void unmap_edges_k(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, uint32_t m,
                              uint32_t n_keep, const uint32_t* __restrict__ oldid, int32_t* __restrict__ osrc,
                              int32_t* __restrict__ odst, uint32_t* __restrict__ err) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t s = src[e], t = dst[e];
  if (s < 0 || uint32_t(s) >= n_keep || t < 0 || uint32_t(t) >= n_keep) {
    atomicOr(err, 1u);
    osrc[e] = odst[e] = 0;
    return;
  }
  osrc[e] = int32_t(oldid[s]);
  odst[e] = int32_t(oldid[t]);
}

// Out- and in-degree of every deleted node (nodes added in this update have none).
__global__ void incident_counts_k(const int32_t* __restrict__ del, uint32_t m, uint32_t n_old,
                                  const uint32_t* __restrict__ rowptr, const uint32_t* __restrict__ rrowptr,
                                  uint32_t* __restrict__ cnt) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t x = uint32_t(del[i]);
  cnt[i] = x < n_old ? (rowptr[x + 1] - rowptr[x]) + (rrowptr[x + 1] - rrowptr[x]) : 0u;
}

// The edges of the deleted nodes as (src, label value, dst) triples: one
// wave per deleted node and table.
template <typename W>
__global__ __launch_bounds__(256) void incident_edges_k(const int32_t* __restrict__ del, uint32_t m, uint32_t n_old,
                                                        const uint32_t* __restrict__ rowptr, const W* __restrict__ adj,
                                                        const uint32_t* __restrict__ rrowptr,
                                                        const W* __restrict__ radj, int bits,
                                                        const int32_t* __restrict__ vals,
                                                        const uint32_t* __restrict__ off, int32_t* __restrict__ s,
                                                        int32_t* __restrict__ l, int32_t* __restrict__ d) {
  const uint32_t lane = __lane_id();
  const W mask = (W(1) << bits) - 1;
  for (uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; w < 2 * m;
       w += (gridDim.x * blockDim.x) / kWave) {
    const uint32_t i = w >> 1;
    const uint32_t x = uint32_t(del[i]);
    if (x >= n_old) continue;
    const bool reverse = w & 1u;
    const uint32_t fdeg = rowptr[x + 1] - rowptr[x];
    const uint32_t b = reverse ? rrowptr[x] : rowptr[x];
    const uint32_t e = reverse ? rrowptr[x + 1] : rowptr[x + 1];
    const uint32_t o = off[i] + (reverse ? fdeg : 0u);
    const W* a = reverse ? radj : adj;
    for (uint32_t q = b + lane; q < e; q += kWave) {
      const W word = a[q];
      const uint32_t other = uint32_t(word & mask);
      const uint32_t out = o + (q - b);
      s[out] = int32_t(reverse ? other : x);
      d[out] = int32_t(reverse ? x : other);
      l[out] = vals[uint32_t(word >> bits)];
    }
  }
}

// Row offsets of the surviving rows (removed rows are empty).
__global__ void compact_rowptr_k(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ newid, uint32_t n,
                                 uint32_t* __restrict__ rp_n) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  if (v == n) {
    rp_n[newid[n]] = rp[n];
    return;
  }
  if (newid[v + 1] != newid[v]) rp_n[newid[v]] = rp[v];
}

// Endpoint ids of every word renumbered (and moved to a narrower field).
template <typename W>
__global__ void renumber_words_k(W* __restrict__ adj, uint64_t m, int bits_o, int bits_n,
                                 const uint32_t* __restrict__ newid) {
  const W mask = (W(1) << bits_o) - 1;
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += uint64_t(gridDim.x) * blockDim.x) {
    const W w = adj[e];
    adj[e] = ((w >> bits_o) << bits_n) | W(newid[uint32_t(w & mask)]);
  }
}

// Per position of a stored round: does its node survive.
__global__ void alive_positions_k(const uint32_t* __restrict__ ord, const uint32_t* __restrict__ newid, uint32_t n,
                                  uint32_t* __restrict__ alivep) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > n) return;
  if (p == n) {
    alivep[p] = 0;
    return;
  }
  const uint32_t u = ord[p];
  alivep[p] = newid[u + 1] != newid[u] ? 1u : 0u;
}

// A stored round closed up: surviving positions move to npos[p] (exclusive
// scan of the survivors), a class starts at its first surviving member
// (npos of its old start), ids renumbered; flags of the closed-up round.
__global__ void close_level_k(const uint32_t* __restrict__ ord, const int32_t* __restrict__ pid, uint32_t n,
                              const uint32_t* __restrict__ newid, const uint32_t* __restrict__ npos,
                              uint32_t* __restrict__ ord_n, int32_t* __restrict__ pid_n, uint8_t* __restrict__ flag_n) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t u = ord[p];
  if (newid[u + 1] == newid[u]) return;
  const uint32_t q = npos[p];
  const uint32_t start = npos[uint32_t(pid[u])];
  ord_n[q] = newid[u];
  pid_n[newid[u]] = int32_t(start);
  flag_n[q] = q == start ? 1 : 0;
}

// Old narrow pId_0 (label rank) of the first member of every level-0 class.
template <typename T>
__global__ void level0_labels_k(const uint32_t* __restrict__ first, const uint32_t* __restrict__ ord, uint32_t B,
                                const uint32_t* __restrict__ oldid, const T* __restrict__ old_rank,
                                uint32_t* __restrict__ out) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) out[b] = uint32_t(old_rank[oldid[ord[first[b]]]]);
}

// Dense level-0 ids in the narrow type: cls[pid[v]] - 1.
template <typename T>
__global__ void dense_level0_k(const int32_t* __restrict__ pid, const uint32_t* __restrict__ cls, uint32_t n,
                               T* __restrict__ out) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = T(cls[uint32_t(pid[v])] - 1);
}

}  // namespace kb
