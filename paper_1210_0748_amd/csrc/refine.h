// Id assignment for one refinement round: the signature store S.insert of
// Algorithm 1 realised as an ordering of the signatures (Section 3.2, "Data
// structures for S": sort all signatures, then hand out ids while scanning).
//
// Canonical ids are lexicographic ranks of the signatures
// [pid_prev(u), k1, k2, ...] (k = unique keys in ascending order, a proper
// prefix is smaller). Because pid_prev(u) leads the signature, the new order
// refines the old one block by block: the array `ord` holds the nodes sorted by
// pid_prev (blocks contiguous, block b starting at bstart[b]), and only blocks
// with two or more members need their members ordered by the key sequence.
//
// Ordering a group is a most-significant-digit refinement with common-prefix
// skipping. Every open subgroup S has a depth t(S): all members agree on the
// keys before t(S). Each member finds the first position >= t(S) where its
// sequence differs from that of the subgroup's first member (the leader); the
// minimum d over the members is where S splits. If no member differs, S is a
// set of identical signatures and closes. Otherwise the members are sorted by
// digit(d) = key[d] + 1 (0 once the sequence has ended), split where the digit
// changes, and every new subgroup gets depth d + 1. A subgroup whose sequences
// ended at d, or that has one member, closes. When keys are narrow, several
// consecutive digits are packed into one 64-bit sort digit (most significant
// first), which consumes that many positions per iteration. Each iteration splits every
// open subgroup, so the number of iterations does not depend on how long the
// shared prefixes are. All comparisons are exact.
//
// flag[p] = 1 marks the first position of every class (distinct signature) in
// `ord`; an inclusive scan of flag then yields the new dense ids.
#pragma once

#include "common.h"
#include "scan_radix.h"

namespace kb {

constexpr uint32_t kSmallCap = 64;     // groups handled by one wave
constexpr uint32_t kMediumCap = 1024;  // largest group one workgroup can order in LDS
constexpr uint32_t kMediumCapSmall = 512;  // LDS size class for medium_cap <= 512
constexpr int kMediumNT = 256;
constexpr uint32_t kNoDiff = 0xffffffffu;
constexpr uint32_t kUndecided = 0xfffffffeu;
constexpr uint32_t kThreadWindow = 32;  // keys one thread compares before asking its wave

template <typename KeyT>
struct KeyView {
  const uint32_t* rowptr;
  const KeyT* ukey;
  const uint32_t* ucnt;
  int dbits;  // bits of one digit: key bits + 1

  __device__ __forceinline__ uint64_t digit(uint32_t node, uint32_t t) const {
    return t < ucnt[node] ? uint64_t(ukey[rowptr[node] + t]) + 1ull : 0ull;
  }
  // Digits of positions t .. t+w-1 packed most significant first (w * dbits
  // <= 64), so comparing packed values compares the w positions in order.
  __device__ __forceinline__ uint64_t digits(uint32_t node, uint32_t t, uint32_t w) const {
    if (w == 1) return digit(node, t);
    const uint32_t c = ucnt[node];
    const KeyT* k = ukey + rowptr[node];
    uint64_t v = 0;
    for (uint32_t j = 0; j < w; ++j) {
      const uint64_t d = (t + j < c) ? uint64_t(k[t + j]) + 1ull : 0ull;
      v = (v << dbits) | d;
    }
    return v;
  }
  // Mask of the last packed digit: zero there means the sequence ended.
  __device__ __forceinline__ uint64_t last_digit_mask() const {
    return dbits >= 64 ? ~0ull : ((1ull << dbits) - 1);
  }
  // First position >= t where the key sequences of a and b differ (one of
  // them ending counts as a difference), or kNoDiff if they are equal.
  __device__ __forceinline__ uint32_t first_diff(uint32_t a, uint32_t b, uint32_t t) const {
    const uint32_t ca = ucnt[a], cb = ucnt[b];
    const uint32_t n = ca < cb ? ca : cb;
    const KeyT* ka = ukey + rowptr[a];
    const KeyT* kb_ = ukey + rowptr[b];
    uint32_t j = t;
    for (; j + 4 <= n; j += 4) {
      const KeyT a0 = ka[j], a1 = ka[j + 1], a2 = ka[j + 2], a3 = ka[j + 3];
      const KeyT b0 = kb_[j], b1 = kb_[j + 1], b2 = kb_[j + 2], b3 = kb_[j + 3];
      if (a0 != b0) return j;
      if (a1 != b1) return j + 1;
      if (a2 != b2) return j + 2;
      if (a3 != b3) return j + 3;
    }
    for (; j < n; ++j)
      if (ka[j] != kb_[j]) return j;
    if (ca == cb) return kNoDiff;
    return n > t ? n : t;
  }
  // As first_diff, but looks at most at `window` positions from t; returns
  // kUndecided when the sequences agree on the whole window and continue.
  __device__ __forceinline__ uint32_t first_diff_window(uint32_t a, uint32_t b, uint32_t t,
                                                        uint32_t window) const {
    const uint32_t ca = ucnt[a], cb = ucnt[b];
    const uint32_t n = ca < cb ? ca : cb;
    const uint32_t stop = n > t ? ((n - t > window) ? t + window : n) : t;
    const KeyT* ka = ukey + rowptr[a];
    const KeyT* kb_ = ukey + rowptr[b];
    uint32_t j = t;
    for (; j + 4 <= stop; j += 4) {
      const KeyT a0 = ka[j], a1 = ka[j + 1], a2 = ka[j + 2], a3 = ka[j + 3];
      const KeyT b0 = kb_[j], b1 = kb_[j + 1], b2 = kb_[j + 2], b3 = kb_[j + 3];
      if (a0 != b0) return j;
      if (a1 != b1) return j + 1;
      if (a2 != b2) return j + 2;
      if (a3 != b3) return j + 3;
    }
    for (; j < stop; ++j)
      if (ka[j] != kb_[j]) return j;
    if (stop < n) return kUndecided;
    if (ca == cb) return kNoDiff;
    return n > t ? n : t;
  }
  // first_diff computed by a whole wave, 64 positions per step; every lane
  // of the wave must call it with the same arguments.
  __device__ __forceinline__ uint32_t wave_first_diff(uint32_t a, uint32_t b, uint32_t t) const {
    const uint32_t ca = ucnt[a], cb = ucnt[b];
    const uint32_t n = ca < cb ? ca : cb;
    const KeyT* ka = ukey + rowptr[a];
    const KeyT* kb_ = ukey + rowptr[b];
    const uint32_t lane = __lane_id();
    for (uint32_t base = t; base < n; base += kWave) {
      const uint32_t j = base + lane;
      const bool ne = j < n && ka[j] != kb_[j];
      const uint64_t bal = __ballot(ne);
      if (bal) return base + uint32_t(__ffsll((unsigned long long)bal) - 1);
    }
    if (ca == cb) return kNoDiff;
    return n > t ? n : t;
  }
};

// Block-wide inclusive max-scan of one uint32 per thread; *total = block max.
template <int NT>
__device__ __forceinline__ uint32_t block_inclusive_max(uint32_t v, uint32_t* sh, uint32_t* total) {
  constexpr int NW = NT / kWave;
  const int lane = __lane_id();
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t u = __shfl_up(v, o, kWave);
    if (lane >= o) v = u > v ? u : v;
  }
  if (NW == 1) {
    *total = __shfl(v, kWave - 1, kWave);
    return v;
  }
  if (lane == kWave - 1) sh[w] = v;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint32_t s = sh[i];
    if (i < w) before = s > before ? s : before;
    tot = s > tot ? s : tot;
  }
  __syncthreads();
  *total = tot;
  return v > before ? v : before;
}

// Side of a member relative to the subgroup's leader, from the first
// position d where they differ: below (0) when the member's digit there is
// smaller, above (2) when larger; identical members are "equal" (1).
// Ordering members by (side, d ascending for below / descending for above,
// digits from d on) is their lexicographic order, except among members
// with equal (side, d, digits), which agree on all positions before
// d + width and form the next subgroups.
__device__ __forceinline__ uint64_t side_key(uint32_t side, uint32_t rel) {
  // below: rel ascending; equal; above: rel descending
  return side == 0 ? uint64_t(rel) : side == 1 ? (1ull << 32) : ((2ull << 32) | uint64_t(0xffffffffu - rel));
}

// Orders the members of one group (positions [s, s+m) of ord, m <= CAP,
// all agreeing on keys before gdepth) lexicographically and sets flag[] at
// the first position of every class inside the group (the group's own first
// position is already flagged). Each iteration splits every open subgroup
// around its first member as a pivot (see side_key).
template <int NT, int CAP, typename KeyT>
__global__ __launch_bounds__(NT) void resolve_k(const uint32_t* __restrict__ gstart,
                                                const uint32_t* __restrict__ gsize,
                                                const uint32_t* __restrict__ gdepth,
                                                uint32_t* __restrict__ ord, uint8_t* __restrict__ flag,
                                                KeyView<KeyT> kv) {
  __shared__ uint32_t node[CAP];
  __shared__ uint32_t sub[CAP];    // index of the subgroup's first member (the pivot)
  __shared__ uint32_t dep[CAP];    // depth of the member's subgroup
  __shared__ uint64_t hk[CAP];     // first difference with the pivot, then side_key
  __shared__ uint64_t dig[CAP];    // packed digits from the first difference on
  __shared__ uint8_t res[CAP];     // member's subgroup is closed
  __shared__ uint8_t mark[CAP];
  __shared__ uint32_t queue[CAP];  // members whose comparison needs a whole wave
  __shared__ uint32_t qn;
  __shared__ uint32_t shm[NT / kWave > 0 ? NT / kWave : 1];

  const uint32_t s = gstart[blockIdx.x];
  const uint32_t m = gsize[blockIdx.x];
  const uint32_t d0 = gdepth[blockIdx.x];
  const uint32_t width = kv.dbits >= 64 ? 1u : uint32_t(64 / kv.dbits);  // positions per digit
  uint32_t P = 2;
  while (P < m) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += NT) {
    const bool in = i < m;
    node[i] = in ? ord[s + i] : 0xffffffffu;
    sub[i] = in ? 0u : 0xffffffffu;
    dep[i] = d0;
    res[i] = in ? 0 : 1;
    hk[i] = in ? 0ull : ~0ull;
    dig[i] = in ? 0ull : ~0ull;
  }
  __syncthreads();

  for (;;) {
    // (a) first difference of every open member with its pivot: a short
    // window per thread, then whole waves (64 positions per step)
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += NT) {
      uint32_t d = kNoDiff;
      const uint32_t L = sub[i];
      if (!res[i] && i != L) {
        d = kv.first_diff_window(node[i], node[L], dep[i], kThreadWindow);
        if (d == kUndecided) queue[atomicAdd(&qn, 1u)] = i;
      }
      hk[i] = d;
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x / kWave; q < qn; q += NT / kWave) {
      const uint32_t i = queue[q];
      const uint32_t d = kv.wave_first_diff(node[i], node[sub[i]], dep[i] + kThreadWindow);
      if (__lane_id() == 0) hk[i] = d;
    }
    __syncthreads();

    // (b) sort keys: (side, distance of the first difference, digits there)
    bool open = false;
    for (uint32_t i = threadIdx.x; i < m; i += NT) {
      if (res[i]) {
        hk[i] = 0;
        dig[i] = 0;
        continue;
      }
      const uint32_t d = uint32_t(hk[i]);
      if (d == kNoDiff) {
        hk[i] = side_key(1, 0);
        dig[i] = 0;
      } else {
        const uint32_t L = sub[i];
        const uint64_t da = kv.digit(node[i], d), dl = kv.digit(node[L], d);
        hk[i] = side_key(da < dl ? 0u : 2u, d - dep[i]);
        dig[i] = kv.digits(node[i], d, width);
        dep[i] = d + width;
        open = true;
      }
    }
    if (!__syncthreads_or(open)) {
      // every open subgroup consists of copies of its pivot: one class each
      for (uint32_t i = threadIdx.x; i < m; i += NT) res[i] = 1;
      __syncthreads();
      break;
    }

    // (c) sort by (subgroup, side key, digits); subgroups keep their ranges
    for (uint32_t size = 2; size <= P; size <<= 1) {
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
        for (uint32_t i = threadIdx.x; i < P / 2; i += NT) {
          const uint32_t lo = 2 * i - (i & (stride - 1));
          const uint32_t hi = lo + stride;
          const bool up = (lo & size) == 0;
          const bool gt = sub[lo] != sub[hi] ? sub[lo] > sub[hi]
                          : hk[lo] != hk[hi] ? hk[lo] > hk[hi]
                                             : dig[lo] > dig[hi];
          if (gt == up) {
            uint32_t tu = sub[lo]; sub[lo] = sub[hi]; sub[hi] = tu;
            tu = node[lo]; node[lo] = node[hi]; node[hi] = tu;
            tu = dep[lo]; dep[lo] = dep[hi]; dep[hi] = tu;
            uint64_t td = hk[lo]; hk[lo] = hk[hi]; hk[hi] = td;
            td = dig[lo]; dig[lo] = dig[hi]; dig[hi] = td;
            const uint8_t tr = res[lo]; res[lo] = res[hi]; res[hi] = tr;
          }
        }
        __syncthreads();
      }
    }

    // (d) split where the key changes; close copies of the pivot, ended
    // sequences and single members
    for (uint32_t i = threadIdx.x; i < m; i += NT)
      mark[i] = (i == 0 || sub[i] != sub[i - 1] || hk[i] != hk[i - 1] || dig[i] != dig[i - 1]) ? 1 : 0;
    __syncthreads();
    uint32_t carry = 0;
    for (uint32_t base = 0; base < m; base += NT) {
      const uint32_t i = base + threadIdx.x;
      const uint32_t v = (i < m && mark[i]) ? i : 0u;
      uint32_t tot;
      uint32_t r = block_inclusive_max<NT>(v, shm, &tot);
      r = r > carry ? r : carry;
      if (i < m) sub[i] = r;
      carry = tot > carry ? tot : carry;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += NT) {
      if (mark[i] && i > 0) flag[s + i] = 1;
      if (!res[i]) {
        const bool single = mark[i] && (i + 1 == m || mark[i + 1]);
        const bool copies = (hk[i] >> 32) == 1;
        if (copies || (dig[i] & kv.last_digit_mask()) == 0 || single) res[i] = 1;
      }
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < m; i += NT) ord[s + i] = node[i];
}

// ---------------------------------------------------------------------------
// Segments (blocks of the previous round, or subgroups after a global split)
// and their classification into work lists by size.

// Segment j of the previous partition: block j with start bstart[j], depth 0.
__global__ void blocks_as_segments_k(const uint32_t* __restrict__ bstart, uint32_t nblocks,
                                     uint32_t* __restrict__ seg_start, uint32_t* __restrict__ seg_size,
                                     uint32_t* __restrict__ seg_depth, uint8_t* __restrict__ seg_done) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nblocks) return;
  const uint32_t a = bstart[j], b = bstart[j + 1];
  seg_start[j] = a;
  seg_size[j] = b - a;
  seg_depth[j] = 0;
  seg_done[j] = (b - a) <= 1;
}

// Open segments of up to kSmallCap members go to the wave resolver, up to
// medium_cap (<= kMediumCap) to the workgroup resolver, the rest to the
// global pass.
// nseg is an upper bound; when nseg_dev is given, segments at or past
// *nseg_dev get no class.
__global__ void classify_segments_k(const uint32_t* __restrict__ seg_size,
                                    const uint8_t* __restrict__ seg_done, uint32_t nseg,
                                    const uint32_t* __restrict__ nseg_dev, uint32_t medium_cap,
                                    uint32_t* __restrict__ c_small, uint32_t* __restrict__ c_medium,
                                    uint32_t* __restrict__ c_large) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  if (nseg_dev && j >= *nseg_dev) {
    c_small[j] = c_medium[j] = c_large[j] = 0;
    return;
  }
  const uint32_t z = seg_size[j];
  const bool done = seg_done[j] || z <= 1;
  c_small[j] = !done && z <= kSmallCap;
  c_medium[j] = !done && z > kSmallCap && z <= medium_cap;
  c_large[j] = !done && z > kSmallCap && z > medium_cap;
}

// Scatters segment j to list position off[j] when its class flag is set
// (off = exclusive scan of the flags).
__global__ void scatter_segments_k(const uint32_t* __restrict__ seg_start,
                                   const uint32_t* __restrict__ seg_size,
                                   const uint32_t* __restrict__ seg_depth, uint32_t nseg,
                                   const uint32_t* __restrict__ cflag, const uint32_t* __restrict__ off,
                                   uint32_t* __restrict__ out_start, uint32_t* __restrict__ out_size,
                                   uint32_t* __restrict__ out_depth) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  if (cflag[j]) {
    const uint32_t o = off[j];
    out_start[o] = seg_start[j];
    out_size[o] = seg_size[j];
    out_depth[o] = seg_depth[j];
  }
}

// ---------------------------------------------------------------------------
// Global pass for groups too large for the resolvers. Items are the members of
// the large groups laid out group after group; ioff[g] is the absolute index
// of the first item of group g.

__device__ __forceinline__ uint32_t group_of_item(const uint32_t* ioff, uint32_t ng, uint32_t i) {
  uint32_t lo = 0, hi = ng;  // last g with ioff[g] <= i
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ioff[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// fdv[i] = first difference of item i's sequence with its group leader's
// (kNoDiff for the leader and its copies). Each thread compares one item
// over a short window; items that still agree are appended to `longq` for
// large_fd_wave_k.
template <typename KeyT>
__global__ __launch_bounds__(256) void large_fd_k(
    const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ gdepth, const uint32_t* __restrict__ ioff,
    uint32_t ng, uint32_t nitems, const uint32_t* __restrict__ ord, uint32_t* __restrict__ fdv,
    uint32_t* __restrict__ longq, uint32_t* __restrict__ nlong, KeyView<KeyT> kv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint32_t g = group_of_item(ioff, ng, i);
  const uint32_t a = ord[gstart[g] + (i - ioff[g])];
  const uint32_t b = ord[gstart[g]];
  uint32_t d = kNoDiff;
  if (a != b) {
    d = kv.first_diff_window(a, b, gdepth[g], kThreadWindow);
    if (d == kUndecided) longq[atomicAdd(nlong, 1u)] = i;
  }
  fdv[i] = d;
}

// One wave per queued item, grid-stride over the queue length in *nlong.
template <typename KeyT>
__global__ void large_fd_wave_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ gdepth,
                                const uint32_t* __restrict__ ioff, uint32_t ng, const uint32_t* __restrict__ ord,
                                uint32_t* __restrict__ fdv, const uint32_t* __restrict__ longq,
                                const uint32_t* __restrict__ nlong, KeyView<KeyT> kv) {
  const uint32_t nq = *nlong;
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  for (uint32_t q = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < nq; q += waves) {
    const uint32_t i = longq[q];
    const uint32_t g = group_of_item(ioff, ng, i);
    const uint32_t a = ord[gstart[g] + (i - ioff[g])];
    const uint32_t b = ord[gstart[g]];
    const uint32_t d = kv.wave_first_diff(a, b, gdepth[g] + kThreadWindow);
    if (__lane_id() == 0) fdv[i] = d;
  }
}

// Layout of the global sort key of an item of group g (see side_key):
//   hi = g << (2 + fd_bits) | side << fd_bits | fdkey
//   lo = `width` packed digits from the first difference on
// fdkey = distance of the first difference from the group depth (below),
// or its complement in fd_bits (above). Packed into one word as
// hi << dig_bits | lo when it fits, else kept as two words.
struct LargeKey {
  int fd_bits;
  int dig_bits;   // width * dbits
  uint32_t width;
  bool packed;
  __device__ __forceinline__ uint64_t hi_of(const uint64_t* ka, const uint64_t* kb, uint32_t i) const {
    return packed ? (dig_bits >= 64 ? 0ull : ka[i] >> dig_bits) : ka[i];
  }
  __device__ __forceinline__ uint64_t lo_of(const uint64_t* ka, const uint64_t* kb, uint32_t i) const {
    return packed ? (dig_bits >= 64 ? ka[i] : (ka[i] & ((1ull << dig_bits) - 1))) : kb[i];
  }
};

template <typename KeyT>
__global__ void large_gather_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ gdepth,
                               const uint32_t* __restrict__ ioff, uint32_t ng, uint32_t nitems,
                               const uint32_t* __restrict__ ord, const uint32_t* __restrict__ fdv, LargeKey lk,
                               uint64_t* __restrict__ ka, uint64_t* __restrict__ kb, uint32_t* __restrict__ val,
                               KeyView<KeyT> kv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint32_t g = group_of_item(ioff, ng, i);
  const uint32_t node = ord[gstart[g] + (i - ioff[g])];
  const uint32_t d = fdv[i];
  uint64_t side = 1, fdkey = 0, lo = 0;
  if (d != kNoDiff) {
    const uint32_t leader = ord[gstart[g]];
    const uint64_t fdmask = (1ull << lk.fd_bits) - 1;
    const uint64_t rel = d - gdepth[g];
    side = kv.digit(node, d) < kv.digit(leader, d) ? 0 : 2;
    fdkey = side == 0 ? rel : (fdmask - rel);
    lo = kv.digits(node, d, lk.width);
  }
  const uint64_t hi = (uint64_t(g) << (2 + lk.fd_bits)) | (side << lk.fd_bits) | fdkey;
  if (lk.packed) {
    ka[i] = (lk.dig_bits >= 64 ? 0ull : (hi << lk.dig_bits)) | lo;
  } else {
    ka[i] = hi;
    kb[i] = lo;
  }
  val[i] = node;
}

// After the sort: write members back to ord, flag class starts, and mark the
// first item of every subgroup.
__global__ void large_write_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ ioff,
                              uint32_t nitems, const uint64_t* __restrict__ ka, const uint64_t* __restrict__ kb,
                              const uint32_t* __restrict__ val, LargeKey lk, uint32_t* __restrict__ ord,
                              uint8_t* __restrict__ flag, uint32_t* __restrict__ start_flag,
                              uint32_t* __restrict__ item_pos) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint64_t hi = lk.hi_of(ka, kb, i), lo = lk.lo_of(ka, kb, i);
  const uint32_t g = uint32_t(hi >> (2 + lk.fd_bits));
  const uint32_t p = gstart[g] + (i - ioff[g]);
  ord[p] = val[i];
  item_pos[i] = p;
  const bool st = (i == ioff[g]) || hi != lk.hi_of(ka, kb, i - 1) || lo != lk.lo_of(ka, kb, i - 1);
  start_flag[i] = st;
  if (st && i != ioff[g]) flag[p] = 1;
}

// Subgroup j starts at item S[j] (S = compacted start flags). Its depth is
// `width` past its first difference with the pivot; it is closed when it
// holds copies of the pivot or its sequences ended inside the digits.
__global__ void large_subgroups_k(const uint32_t* __restrict__ start_flag,
                                  const uint32_t* __restrict__ start_off, uint32_t nitems,
                                  const uint32_t* __restrict__ item_pos, const uint64_t* __restrict__ ka,
                                  const uint64_t* __restrict__ kb, LargeKey lk, uint64_t last_mask,
                                  const uint32_t* __restrict__ gdepth, uint32_t* __restrict__ sub_item,
                                  uint32_t* __restrict__ seg_start, uint32_t* __restrict__ seg_depth,
                                  uint8_t* __restrict__ seg_done) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  if (start_flag[i]) {
    const uint32_t j = start_off[i];
    const uint64_t hi = lk.hi_of(ka, kb, i), lo = lk.lo_of(ka, kb, i);
    const uint64_t fdmask = (1ull << lk.fd_bits) - 1;
    const uint32_t g = uint32_t(hi >> (2 + lk.fd_bits));
    const uint32_t side = uint32_t(hi >> lk.fd_bits) & 3u;
    const uint64_t fdkey = hi & fdmask;
    const uint64_t rel = side == 0 ? fdkey : (fdmask - fdkey);
    sub_item[j] = i;
    seg_start[j] = item_pos[i];
    seg_depth[j] = side == 1 ? 0u : uint32_t(gdepth[g] + rel + lk.width);
    seg_done[j] = side == 1 || (lo & last_mask) == 0;
  }
}

// ns_dev: number of subgroups (device); at most nitems.
__global__ void subgroup_sizes_k(const uint32_t* __restrict__ sub_item, const uint32_t* __restrict__ ns_dev,
                                 uint32_t nitems, uint32_t* __restrict__ seg_size) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t ns = *ns_dev;
  if (j >= ns) return;
  const uint32_t end = (j + 1 < ns) ? sub_item[j + 1] : nitems;
  seg_size[j] = end - sub_item[j];
}

// Two-word sort support: out[i] = in[idx[i]].
__global__ void gather_u64_k(const uint64_t* __restrict__ in, const uint32_t* __restrict__ idx, uint32_t n,
                             uint64_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[idx[i]];
}

// Final two-word order: lo_out[i] = lo[perm[i]], val_out[i] = val[idx1[perm[i]]].
__global__ void two_word_finish_k(const uint64_t* __restrict__ lo, const uint32_t* __restrict__ idx1,
                                  const uint32_t* __restrict__ perm, const uint32_t* __restrict__ val, uint32_t n,
                                  uint64_t* __restrict__ lo_out, uint32_t* __restrict__ val_out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t p = perm[i];
  lo_out[i] = lo[p];
  val_out[i] = val[idx1[p]];
}

// ---------------------------------------------------------------------------
// New ids: cls = inclusive scan of flag; pid_next[ord[p]] = cls[p] - 1 and
// bstart[cls[p] - 1] = p at class starts.
__global__ void assign_k(const uint32_t* __restrict__ ord, const uint8_t* __restrict__ flag,
                         const uint32_t* __restrict__ cls, uint32_t n, int32_t* __restrict__ pid_next,
                         uint32_t* __restrict__ bstart) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t c = cls[p];
  pid_next[ord[p]] = int32_t(c - 1);
  if (flag[p]) bstart[c - 1] = p;
}

__global__ void set_u32_k(uint32_t* __restrict__ dst, uint32_t v) { *dst = v; }

}  // namespace kb
