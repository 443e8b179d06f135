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
// Ordering a group of positions is a most-significant-digit refinement over
// key positions t = 0, 1, ...: at depth t the members of every still-open
// subgroup are sorted by digit(t) = key[t] + 1, or 0 once the sequence has
// ended, and split where the digit changes. A subgroup whose members end
// together is a set of identical signatures. A subgroup whose members all
// carry the same 64-bit hash and length is checked element by element and,
// when identical, closed early; on any mismatch refinement simply continues,
// so the hash can only save work and never changes an id.
//
// flag[p] = 1 marks the first position of every class (distinct signature) in
// `ord`; an inclusive scan of flag then yields the new dense ids.
#pragma once

#include "common.h"
#include "scan_radix.h"

namespace kb {

constexpr uint32_t kSmallCap = 64;     // groups handled by one wave
constexpr uint32_t kMediumCap = 2048;  // groups handled by one workgroup in LDS
constexpr int kMediumNT = 256;

template <typename KeyT>
struct KeyView {
  const uint32_t* rowptr;
  const KeyT* ukey;
  const uint32_t* ucnt;
  const uint64_t* hsh;

  __device__ __forceinline__ uint64_t digit(uint32_t node, uint32_t t) const {
    return t < ucnt[node] ? uint64_t(ukey[rowptr[node] + t]) + 1ull : 0ull;
  }
  // True when the key sequences of a and b agree from position t on (their
  // earlier keys agree by construction) and their lengths agree.
  __device__ __forceinline__ bool same_tail(uint32_t a, uint32_t b, uint32_t t) const {
    const uint32_t ca = ucnt[a];
    if (ca != ucnt[b]) return false;
    const KeyT* ka = ukey + rowptr[a];
    const KeyT* kb_ = ukey + rowptr[b];
    for (uint32_t j = t; j < ca; ++j)
      if (ka[j] != kb_[j]) return false;
    return true;
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

// Orders the members of one group (positions [s, s+m) of ord, m <= CAP)
// lexicographically by their key sequences from depth d0 on, and sets flag[]
// at the first position of every class inside the group (the group's own
// first position is already flagged).
template <int NT, int CAP, typename KeyT>
__global__ __launch_bounds__(NT) void resolve_k(const uint32_t* __restrict__ gstart,
                                                const uint32_t* __restrict__ gsize, uint32_t d0,
                                                uint32_t* __restrict__ ord, uint8_t* __restrict__ flag,
                                                KeyView<KeyT> kv) {
  __shared__ uint32_t node[CAP];
  __shared__ uint32_t sub[CAP];
  __shared__ uint64_t dig[CAP];
  __shared__ uint8_t res[CAP];
  __shared__ uint8_t mark[CAP];
  __shared__ uint32_t shm[NT / kWave > 0 ? NT / kWave : 1];

  const uint32_t s = gstart[blockIdx.x];
  const uint32_t m = gsize[blockIdx.x];
  uint32_t P = 2;
  while (P < m) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += NT) {
    if (i < m) {
      node[i] = ord[s + i];
      sub[i] = 0;
      res[i] = 0;
      dig[i] = 0;
    } else {
      node[i] = 0xffffffffu;
      sub[i] = 0xffffffffu;
      res[i] = 1;
      dig[i] = ~0ull;
    }
  }
  __syncthreads();

  for (uint32_t t = d0;; ++t) {
    // (a) close subgroups whose members carry identical signatures
    for (uint32_t i = threadIdx.x; i < m; i += NT) mark[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += NT) {
      const uint32_t L = sub[i];
      if (!res[i] && i != L) {
        const uint32_t a = node[i], b = node[L];
        if (kv.hsh[a] != kv.hsh[b] || kv.ucnt[a] != kv.ucnt[b]) mark[L] = 1;
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += NT) {
      const uint32_t L = sub[i];
      if (!res[i] && i != L && !mark[L] && !kv.same_tail(node[i], node[L], t)) mark[L] = 1;
    }
    __syncthreads();
    bool open = false;
    for (uint32_t i = threadIdx.x; i < m; i += NT) {
      if (!res[i]) {
        if (!mark[sub[i]])
          res[i] = 1;
        else
          open = true;
      }
    }
    if (!__syncthreads_or(open)) break;

    // (b) digit at depth t of every open member
    for (uint32_t i = threadIdx.x; i < m; i += NT) dig[i] = res[i] ? 0ull : kv.digit(node[i], t);
    __syncthreads();

    // (c) sort by (subgroup, digit); subgroups keep their position ranges
    for (uint32_t size = 2; size <= P; size <<= 1) {
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
        for (uint32_t i = threadIdx.x; i < P / 2; i += NT) {
          const uint32_t lo = 2 * i - (i & (stride - 1));
          const uint32_t hi = lo + stride;
          const bool up = (lo & size) == 0;
          const bool gt = sub[lo] != sub[hi] ? sub[lo] > sub[hi] : dig[lo] > dig[hi];
          if (gt == up) {
            uint32_t tu = sub[lo]; sub[lo] = sub[hi]; sub[hi] = tu;
            uint64_t td = dig[lo]; dig[lo] = dig[hi]; dig[hi] = td;
            tu = node[lo]; node[lo] = node[hi]; node[hi] = tu;
            uint8_t tr = res[lo]; res[lo] = res[hi]; res[hi] = tr;
          }
        }
        __syncthreads();
      }
    }

    // (d) split where the digit changes; close ended and single subgroups
    for (uint32_t i = threadIdx.x; i < m; i += NT)
      mark[i] = (i == 0 || sub[i] != sub[i - 1] || dig[i] != dig[i - 1]) ? 1 : 0;
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
        const uint32_t L = sub[i];
        const bool single = mark[i] && (i + 1 == m || mark[i + 1]);
        if (dig[i] == 0 || single) res[i] = 1;
        (void)L;
      }
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < m; i += NT) ord[s + i] = node[i];
}

// ---------------------------------------------------------------------------
// Segments (blocks of the previous round, or subgroups after a global split)
// and their classification into work lists by size.

// Segment j of the previous partition: block j with start bstart[j].
__global__ void blocks_as_segments_k(const uint32_t* __restrict__ bstart, uint32_t nblocks,
                                     uint32_t* __restrict__ seg_start, uint32_t* __restrict__ seg_size,
                                     uint8_t* __restrict__ seg_done) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nblocks) return;
  const uint32_t a = bstart[j], b = bstart[j + 1];
  seg_start[j] = a;
  seg_size[j] = b - a;
  seg_done[j] = (b - a) <= 1;
}

// cls[j] bits: 1 small, 2 medium, 4 large (exactly one bit, or none if done).
__global__ void classify_segments_k(const uint32_t* __restrict__ seg_size,
                                    const uint8_t* __restrict__ seg_done, uint32_t nseg,
                                    uint32_t* __restrict__ c_small, uint32_t* __restrict__ c_medium,
                                    uint32_t* __restrict__ c_large) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  const uint32_t z = seg_size[j];
  const bool done = seg_done[j] || z <= 1;
  c_small[j] = !done && z <= kSmallCap;
  c_medium[j] = !done && z > kSmallCap && z <= kMediumCap;
  c_large[j] = !done && z > kMediumCap;
}

// Scatters segment j to list position off[j] when its class flag is set
// (off = exclusive scan of the flags).
__global__ void scatter_segments_k(const uint32_t* __restrict__ seg_start,
                                   const uint32_t* __restrict__ seg_size, uint32_t nseg,
                                   const uint32_t* __restrict__ cflag, const uint32_t* __restrict__ off,
                                   uint32_t* __restrict__ out_start, uint32_t* __restrict__ out_size) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  if (cflag[j]) {
    out_start[off[j]] = seg_start[j];
    out_size[off[j]] = seg_size[j];
  }
}

// ---------------------------------------------------------------------------
// Global most-significant-digit pass for groups larger than kMediumCap.
// Items are the members of the large groups laid out group after group;
// ioff[g] is the first item of group g (exclusive scan of the sizes).

__device__ __forceinline__ uint32_t group_of_item(const uint32_t* ioff, uint32_t ng, uint32_t i) {
  uint32_t lo = 0, hi = ng;  // find last g with ioff[g] <= i
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ioff[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// mixed[g] = 1 unless every member of g has the leader's hash and length.
template <typename KeyT>
__global__ void large_mixed_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ ioff,
                              uint32_t ng, uint32_t nitems, const uint32_t* __restrict__ ord,
                              uint8_t* __restrict__ mixed, KeyView<KeyT> kv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint32_t g = group_of_item(ioff, ng, i);
  const uint32_t a = ord[gstart[g] + (i - ioff[g])];
  const uint32_t b = ord[gstart[g]];
  if (kv.hsh[a] != kv.hsh[b] || kv.ucnt[a] != kv.ucnt[b]) mixed[g] = 1;
}

template <typename KeyT>
__global__ void large_verify_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ ioff,
                               uint32_t ng, uint32_t nitems, const uint32_t* __restrict__ ord,
                               uint8_t* __restrict__ mixed, uint32_t t, KeyView<KeyT> kv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint32_t g = group_of_item(ioff, ng, i);
  if (mixed[g]) return;
  const uint32_t a = ord[gstart[g] + (i - ioff[g])];
  const uint32_t b = ord[gstart[g]];
  if (a != b && !kv.same_tail(a, b, t)) mixed[g] = 1;
}

__global__ void u8_to_u32_k(const uint8_t* __restrict__ in, uint32_t* __restrict__ out, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

// Sort keys of the open large groups: (group << dig_bits) | digit(t). Items
// are numbered from item_base (ioff holds absolute item offsets).
template <typename KeyT>
__global__ void large_gather_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ ioff,
                               uint32_t ng, uint32_t nitems, uint32_t item_base,
                               const uint32_t* __restrict__ ord, uint32_t t, int dig_bits,
                               uint64_t* __restrict__ key, uint32_t* __restrict__ val, KeyView<KeyT> kv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint32_t ia = item_base + i;
  const uint32_t g = group_of_item(ioff, ng, ia);
  const uint32_t node = ord[gstart[g] + (ia - ioff[g])];
  const uint64_t hi = dig_bits >= 64 ? 0ull : (uint64_t(g) << dig_bits);
  key[i] = hi | kv.digit(node, t);
  val[i] = node;
}

// After the sort: write members back to ord, flag class starts, and emit the
// subgroups (start position, size, ended) via start flags.
__global__ void large_split_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ ioff,
                              uint32_t ng, uint32_t nitems, uint32_t item_base,
                              const uint64_t* __restrict__ key, const uint32_t* __restrict__ val,
                              int dig_bits, uint32_t* __restrict__ ord, uint8_t* __restrict__ flag,
                              uint32_t* __restrict__ start_flag, uint32_t* __restrict__ item_pos) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint32_t ia = item_base + i;
  const uint32_t g = dig_bits >= 64 ? 0u : uint32_t(key[i] >> dig_bits);
  const uint32_t p = gstart[g] + (ia - ioff[g]);
  ord[p] = val[i];
  item_pos[i] = p;
  const bool st = (ia == ioff[g]) || key[i] != key[i - 1];
  start_flag[i] = st;
  if (st && ia != ioff[g]) flag[p] = 1;
  (void)ng;
}

// Subgroup j starts at item S[j] (S = compacted start flags, S[ns] = nitems).
__global__ void large_subgroups_k(const uint32_t* __restrict__ start_flag,
                                  const uint32_t* __restrict__ start_off, uint32_t nitems,
                                  const uint32_t* __restrict__ item_pos, const uint64_t* __restrict__ key,
                                  uint64_t dig_mask, uint32_t* __restrict__ sub_item,
                                  uint32_t* __restrict__ seg_start, uint8_t* __restrict__ seg_done) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  if (start_flag[i]) {
    const uint32_t j = start_off[i];
    sub_item[j] = i;
    seg_start[j] = item_pos[i];
    seg_done[j] = (key[i] & dig_mask) == 0;  // sequences ended: identical signatures
  }
}

__global__ void subgroup_sizes_k(const uint32_t* __restrict__ sub_item, uint32_t ns, uint32_t nitems,
                                 uint32_t* __restrict__ seg_size) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ns) return;
  const uint32_t end = (j + 1 < ns) ? sub_item[j + 1] : nitems;
  seg_size[j] = end - sub_item[j];
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
