// The active set of a refinement round and the id assignment that ends it.
//
// Refinement never merges classes (Proposition 1), so a class with a single
// member stays alone and keeps its place in `ord`. A round therefore only
// works on the active segments: the classes of the previous round with two
// or more members. Ids are kept as class-start positions: the id of node u
// is the position in `ord` of the first member of u's class. These ids order
// the classes exactly as the dense ids do (both increase along `ord`), so
// they serve as pId_{i-1} inside signatures, and a node of an untouched class
// keeps its id from round to round. Dense 0-based ids are a scan of the
// class-start flags, computed only when ids are read out.
#pragma once

#include "common.h"
#include "compact.h"
#include "refine.h"
#include "signature.h"

namespace kb {

// Words of the per-round summary the host reads back in one copy.
constexpr int kInfoSeg = 0;                          // next segments: counts, list starts, total
constexpr int kInfoBucket = 2 * kSegClasses + 1;     // degree buckets: counts, list starts, total
constexpr int kNumBuckets = 4;                       // wave, mid, block, hub lists
constexpr int kBucketWave = 0, kBucketMid = 1, kBucketBlock = 2, kBucketHub = 3;
constexpr int kInfoClasses = kInfoBucket + 2 * kNumBuckets + 1;  // classes among the active positions
constexpr int kInfoItems = kInfoClasses + 1;         // positions of the next active segments
constexpr int kInfoHubEdges = kInfoItems + 1;        // edges of the hubs in the hub list
constexpr int kInfoLargeItems = kInfoHubEdges + 1;   // items in the large segments
constexpr int kInfoMaxDeg = kInfoLargeItems + 1;      // largest out-degree (after a build)
constexpr int kInfoWords = kInfoMaxDeg + 1;

// apos[j] = position of active item j, anode[j] = ord[apos[j]]; segment t of
// the list covers positions [seg_s[t], seg_s[t] + size), soff is the
// exclusive scan of the sizes (soff[S] = number of items), S = *s_dev.
// Thread 0 of workgroup 0 also records the number of items in info.
// actr[anode[j]] = tag marks the active nodes of the round (unless actr is
// null: marked by the caller). One tile of kExpandTile items per workgroup:
// the segments of the tile's first and last items are found once, items in
// between search only that range.
constexpr uint32_t kExpandTile = 2048;
__device__ __forceinline__ uint32_t seg_of(const uint32_t* soff, uint32_t lo, uint32_t hi, uint32_t j) {
  while (hi - lo > 1) {  // last t in [lo, hi) with soff[t] <= j
    const uint32_t mid = (lo + hi) >> 1;
    if (soff[mid] <= j)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}
__global__ __launch_bounds__(256) void expand_k(const uint32_t* __restrict__ seg_s, const uint32_t* __restrict__ soff,
                                                const uint32_t* __restrict__ s_dev, uint32_t m_cap,
                                                const uint32_t* __restrict__ ord, uint32_t* __restrict__ apos,
                                                uint32_t* __restrict__ anode, uint32_t* __restrict__ actr,
                                                uint32_t tag, uint32_t* __restrict__ info) {
  __shared__ uint32_t range[2];
  const uint32_t S = *s_dev;
  const uint32_t M = soff[S] < m_cap ? soff[S] : m_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) info[kInfoItems] = soff[S];
  const uint32_t t0 = blockIdx.x * kExpandTile;
  if (t0 >= M) return;  // uniform over the workgroup
  const uint32_t t1 = t0 + kExpandTile < M ? t0 + kExpandTile : M;
  if (threadIdx.x == 0) {
    range[0] = seg_of(soff, 0, S, t0);
    range[1] = seg_of(soff, 0, S, t1 - 1);
  }
  __syncthreads();
  const uint32_t lo = range[0], hi = range[1];
  for (uint32_t j = t0 + threadIdx.x; j < t1; j += blockDim.x) {
    const uint32_t t = lo == hi ? lo : seg_of(soff, lo, hi + 1, j);
    const uint32_t p = seg_s[t] + (j - soff[t]);
    const uint32_t u = ord[p];
    apos[j] = p;
    anode[j] = u;
    if (actr) actr[u] = tag;
  }
}

// Out-degree bucket of an active node for the signature kernel: wave (17..64
// edges), mid (65..512), block (513..4096) or hub; nodes with at most 16
// edges need no list.
__device__ __forceinline__ int degree_bucket(uint32_t d) {
  return d <= kThreadMaxDeg ? -1
         : d <= kWaveMaxDeg ? kBucketWave
         : d <= kMidMaxDeg  ? kBucketMid
         : d <= kBlockMaxDeg ? kBucketBlock
                             : kBucketHub;
}
struct NodeBucketOf {
  const uint32_t* anode;
  const uint32_t* rowptr;
  __device__ __forceinline__ int operator()(uint32_t j) const {
    const uint32_t n = anode[j];
    return degree_bucket(rowptr[n + 1] - rowptr[n]);
  }
};
struct NodeWrite {
  const uint32_t* anode;
  uint32_t* list;
  __device__ __forceinline__ void operator()(uint32_t j, int, uint32_t o) const { list[o] = anode[j]; }
};
// The same over all nodes in id order (lists in node order: neighbouring
// nodes have neighbouring rows), for rounds where most nodes are active.
struct NodeBucketDenseOf {
  const uint32_t* actr;
  uint32_t tag;
  const uint32_t* rowptr;
  __device__ __forceinline__ int operator()(uint32_t n) const {
    if (actr[n] != tag) return -1;
    return degree_bucket(rowptr[n + 1] - rowptr[n]);
  }
};
struct NodeWriteDense {
  uint32_t* list;
  __device__ __forceinline__ void operator()(uint32_t n, int, uint32_t o) const { list[o] = n; }
};

// hoff[h] = exclusive scan of the out-degrees of the hub list (*nh_dev
// entries from lists + *start_dev), hoff[nh] = *total = their sum. One
// workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void hub_offsets_k(const uint32_t* __restrict__ rowptr,
                                                      const uint32_t* __restrict__ lists,
                                                      const uint32_t* __restrict__ nh_dev,
                                                      const uint32_t* __restrict__ start_dev,
                                                      uint32_t* __restrict__ hoff, uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[1024 / kWave];
  const uint32_t nh = *nh_dev;
  const uint32_t* hl = lists + *start_dev;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nh; base += 1024) {
    const uint32_t h = base + threadIdx.x;
    uint32_t d = 0;
    if (h < nh) {
      const uint32_t n = hl[h];
      d = rowptr[n + 1] - rowptr[n];
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024>(d, sh, &tot);
    if (h < nh) hoff[h] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    hoff[nh] = carry;
    *total = carry;
  }
}

// Initial segments: the blocks of pId_0 (block b spans [bstart[b], bstart[b+1])).
struct BlockSegOf {
  const uint32_t* bstart;
  uint32_t medium_cap, big_cap;
  __device__ __forceinline__ int operator()(uint32_t b) const {
    const uint32_t z = bstart[b + 1] - bstart[b];
    return z >= 2 ? seg_class(z, medium_cap, big_cap) : -1;
  }
};
struct BlockSegWrite {
  const uint32_t* bstart;
  uint32_t *o_start, *o_size, *o_depth;
  __device__ __forceinline__ void operator()(uint32_t b, int, uint32_t o) const {
    o_start[o] = bstart[b];
    o_size[o] = bstart[b + 1] - bstart[b];
    o_depth[o] = 0;
  }
};

// ---- assignment over the active positions -----------------------------------

__global__ void act_flags_k(const uint32_t* __restrict__ apos, const uint8_t* __restrict__ flag, uint32_t m,
                            uint32_t* __restrict__ fl) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) fl[j] = flag[apos[j]];
}

// cls = inclusive scan of fl: class c (0-based, in position order) of the
// active positions starts at item first[c]. info[kInfoClasses] = classes.
__global__ void class_first_k(const uint32_t* __restrict__ fl, const uint32_t* __restrict__ cls, uint32_t m,
                              uint32_t* __restrict__ first, uint32_t* __restrict__ info) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  if (fl[j]) first[cls[j] - 1] = j;
  if (j == m - 1) info[kInfoClasses] = cls[j];
}

// pid[u] = position of the first member of u's class, for every active u.
__global__ void assign_pos_k(const uint32_t* __restrict__ apos, const uint32_t* __restrict__ cls,
                             const uint32_t* __restrict__ first, const uint32_t* __restrict__ ord, uint32_t m,
                             int32_t* __restrict__ pid) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  pid[ord[apos[j]]] = int32_t(apos[first[cls[j] - 1]]);
}

// Classes of the active positions with two or more members become the next
// round's segments (class c spans items first[c] .. first[c+1]), except
// classes of nodes without out-edges: all members of a class share this
// round's signature, so when the first member's is empty they all have no
// edges, their signatures stay empty in every later round, and the class
// never splits.
struct NextSegOf {
  const uint32_t* first;
  const uint32_t* nclass;  // device count of classes
  uint32_t m;
  uint32_t medium_cap, big_cap;
  const uint32_t* apos;
  const uint32_t* ord;
  const uint32_t* ucnt;
  __device__ __forceinline__ uint32_t size(uint32_t c) const {
    const uint32_t C = *nclass;
    return (c + 1 < C ? first[c + 1] : m) - first[c];
  }
  __device__ __forceinline__ int operator()(uint32_t c) const {
    const uint32_t z = size(c);
    if (z < 2 || ucnt[ord[apos[first[c]]]] == 0) return -1;
    return seg_class(z, medium_cap, big_cap);
  }
};
struct NextSegWrite {
  NextSegOf of;
  const uint32_t* apos;
  uint32_t *o_start, *o_size, *o_depth;
  __device__ __forceinline__ void operator()(uint32_t c, int, uint32_t o) const {
    o_start[o] = apos[of.first[c]];
    o_size[o] = of.size(c);
    o_depth[o] = 0;
  }
};

// ---- ids ---------------------------------------------------------------------

// Dense ids in node order: pid[v] is the position of the first member of
// v's class and cls (inclusive scan of the class-start flags) numbers the
// classes along ord, so v's dense id is cls[pid[v]] - 1.
__global__ void dense_ids_k(const int32_t* __restrict__ pid, const uint32_t* __restrict__ cls, uint32_t n,
                            int32_t* __restrict__ dense) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) dense[v] = int32_t(cls[uint32_t(pid[v])] - 1);
}

// Start position of every block of pId_0: bstart[cls[p] - 1] = p at the
// first position p of each block (cls = inclusive scan of the flags).
__global__ void block_starts_k(const uint8_t* __restrict__ flag, const uint32_t* __restrict__ cls, uint32_t n,
                               uint32_t* __restrict__ bstart) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n && flag[p]) bstart[cls[p] - 1] = p;
}

// In node order: the class-start position id of node v (the start of its
// block of pId_0, rank0[v] = its block) and its active mark (tag when the
// block has two or more members, else 0).
template <typename T>
__global__ void node_ids0_k(const T* __restrict__ rank0, const uint32_t* __restrict__ bstart, uint32_t n,
                            int32_t* __restrict__ pid, uint32_t* __restrict__ actr, uint32_t tag) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t r = uint32_t(rank0[v]);
  const uint32_t s = bstart[r];
  pid[v] = int32_t(s);
  actr[v] = bstart[r + 1] - s >= 2 ? tag : 0u;
}

// Narrow copy of ids below 2^16 (the first round's keys gather pId_0 for
// every edge; a smaller table keeps more of it in cache).
template <typename T>
__global__ void narrow_ids_k(const uint32_t* __restrict__ in, uint32_t n, T* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = T(in[i]);
}

}  // namespace kb
