// Id assignment for one refinement round: the signature store S.insert of
// Algorithm 1 realised as an ordering of the signatures (Section 3.2, "Data
// structures for S": sort all signatures, then hand out ids while scanning).
//
// Canonical ids are lexicographic ranks of the signatures
// [pid_prev(u), k1, k2, ...] (k = unique keys in ascending order, a proper
// prefix is smaller). Because pid_prev(u) leads the signature, the new order
// refines the old one class by class: the array `ord` holds the nodes sorted
// by class (classes contiguous), and only classes with two or more members
// need their members ordered by the key sequence.
//
// A group (a class, or a part of one whose members agree on all keys before
// the group's depth t) is ordered by most-significant-digit refinement, with
// digit(t) = key[t] + 1 (0 once the sequence has ended, so a proper prefix
// sorts first). A group splits around its first member (the pivot): each
// member finds the first position d where it differs from the pivot, and
// members are ordered by (below/equal/above the pivot at d, d, digits from d
// on); members that tie agree on everything before d + width and form the
// next subgroups. Groups of up to a few thousand members do this in registers
// or LDS (resolve_lanes_k, resolve_k); larger ones in global passes
// (large_*_k) that sort the members of all large groups with one device-wide
// radix sort. The first global pass of a round works on whole classes at
// depth 0 and sorts by the leading digits only (no pivot), which every node's
// signature kernel wrote out.
// When keys are narrow, several consecutive digits are packed into one
// 64-bit sort digit (most significant first), which consumes that many
// positions per step. A subgroup whose sequences ended inside the packed
// digits, or that holds copies of one sequence, or a single member, closes.
// All comparisons are exact.
//
// flag[p] = 1 marks the first position of every class (distinct signature) in
// `ord`.
#pragma once

#include "common.h"
#include "compact.h"
#include "scan_radix.h"

namespace kb {

constexpr uint32_t kSmallCap = 64;     // groups handled by one wave
constexpr uint32_t kMediumCapSmall = 512;  // groups one 256-thread workgroup orders in LDS
constexpr uint32_t kBigCap = 4096;         // groups one 1024-thread workgroup orders in LDS
constexpr int kMediumNT = 256;
constexpr int kBigNT = 1024;
constexpr uint32_t kNoDiff = 0xffffffffu;
constexpr uint32_t kUndecided = 0xfffffffeu;
constexpr uint32_t kThreadWindow = 32;  // keys one thread compares before asking its wave

template <typename KeyT>
struct KeyView {
  const uint32_t* rowptr;
  const KeyT* ukey;
  const uint32_t* ucnt;
  int dbits;  // bits of one digit: key bits + 1
  // Optional key-set bitmaps (bm_words64 > 0) of every node with more than
  // bm_min_deg edges: bitmap of node u at bm + bmslot[u] * bm_words64.
  const uint64_t* bm = nullptr;
  const uint32_t* bmslot = nullptr;
  uint32_t bm_words64 = 0;
  uint32_t bm_min_deg = 0;

  __device__ __forceinline__ bool has_bm(uint32_t node) const {
    return bm_words64 && rowptr[node + 1] - rowptr[node] > bm_min_deg;
  }
  // First difference of two key sets given as bitmaps: the smallest key x in
  // exactly one of them; both sequences hold the same keys below x, so they
  // first differ at the position equal to the number of those keys.
  __device__ __forceinline__ uint32_t first_diff_bm(uint32_t a, uint32_t b) const {
    const uint64_t* A = bm + size_t(bmslot[a]) * bm_words64;
    const uint64_t* B = bm + size_t(bmslot[b]) * bm_words64;
    uint32_t below = 0;
    // eight words of each bitmap in flight per step
    uint32_t w = 0;
    for (; w + 8 <= bm_words64; w += 8) {
      uint64_t va[8], vb[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        va[q] = A[w + q];
        vb[q] = B[w + q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint64_t x = va[q] ^ vb[q];
        if (x) return below + uint32_t(__popcll(va[q] & ((x & (~x + 1)) - 1)));
        below += uint32_t(__popcll(va[q]));
      }
    }
    for (; w < bm_words64; ++w) {
      const uint64_t x = A[w] ^ B[w];
      if (x) return below + uint32_t(__popcll(A[w] & ((x & (~x + 1)) - 1)));
      below += uint32_t(__popcll(A[w]));
    }
    return kNoDiff;
  }
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
  // them ending counts as a difference; kNoDiff if they are equal), looking
  // at most at `window` positions from t: kUndecided when the sequences agree
  // on the whole window and continue.
  __device__ __forceinline__ uint32_t first_diff_window(uint32_t a, uint32_t b, uint32_t t,
                                                        uint32_t window) const {
    if (has_bm(a) && has_bm(b)) return first_diff_bm(a, b);
    const uint32_t ca = ucnt[a], cb = ucnt[b];
    const uint32_t n = ca < cb ? ca : cb;
    const uint32_t stop = n > t ? ((n - t > window) ? t + window : n) : t;
    const KeyT* ka = ukey + rowptr[a];
    const KeyT* kb_ = ukey + rowptr[b];
    uint32_t j = t;
    for (; j + 8 <= stop; j += 8) {
      KeyT va[8], vb[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        va[q] = ka[j + q];
        vb[q] = kb_[j + q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (va[q] != vb[q]) return j + q;
    }
    for (; j < stop; ++j)
      if (ka[j] != kb_[j]) return j;
    if (stop < n) return kUndecided;
    if (ca == cb) return kNoDiff;
    return n > t ? n : t;
  }
  // Member a against pivot b from position t, with the rows and counts of
  // both loaded once: the first difference d (kUndecided when a window of
  // `window` keys agrees and both continue, kNoDiff when equal) and, when d
  // is decided, the digits of both at d (da, dl: side) and a's packed digits
  // from d on (width positions). Saves reloading the rows for the keys.
  struct Cmp {
    uint32_t d;
    uint64_t da, dl, dig;
  };
  __device__ __forceinline__ Cmp compare(uint32_t a, uint32_t b, uint32_t t, uint32_t window,
                                         uint32_t width) const {
    const uint32_t ra = rowptr[a], rb = rowptr[b];
    const uint32_t ea = rowptr[a + 1], eb = rowptr[b + 1];
    const uint32_t ca = ucnt[a], cb = ucnt[b];
    const KeyT* ka = ukey + ra;
    const KeyT* kb_ = ukey + rb;
    Cmp c{kNoDiff, 0, 0, 0};
    if (bm_words64 && ea - ra > bm_min_deg && eb - rb > bm_min_deg) {
      c.d = first_diff_bm(a, b);
    } else {
      const uint32_t n = ca < cb ? ca : cb;
      const uint32_t stop = n > t ? ((n - t > window) ? t + window : n) : t;
      uint32_t j = t, d = kNoDiff;
      for (; j + 8 <= stop && d == kNoDiff; j += 8) {
        KeyT va[8], vb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          va[q] = ka[j + q];
          vb[q] = kb_[j + q];
        }
#pragma unroll
        for (int q = 7; q >= 0; --q)
          if (va[q] != vb[q]) d = j + uint32_t(q);
      }
      for (; j < stop && d == kNoDiff; ++j)
        if (ka[j] != kb_[j]) d = j;
      if (d == kNoDiff) {
        if (stop < n) d = kUndecided;
        else if (ca != cb) d = n > t ? n : t;
      }
      c.d = d;
    }
    if (c.d == kNoDiff || c.d == kUndecided) return c;
    const uint32_t d = c.d;
    c.da = d < ca ? uint64_t(ka[d]) + 1ull : 0ull;
    c.dl = d < cb ? uint64_t(kb_[d]) + 1ull : 0ull;
    if (width == 1 || dbits >= 64) {
      c.dig = c.da;
    } else {
      uint64_t v = 0;
      for (uint32_t q = 0; q < width; ++q) v = (v << dbits) | (d + q < ca ? uint64_t(ka[d + q]) + 1ull : 0ull);
      c.dig = v;
    }
    return c;
  }
  // The first difference computed by a whole wave, 64 positions per step; every lane
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
// around its first member as a pivot (see side_key). Only members of open
// subgroups take part in an iteration: their positions are listed in order
// (an open subgroup is a contiguous range), the list is sorted by (subgroup,
// side key, digits) through a permutation of positions, and the members are
// then moved once to their new places.
template <int NT, int CAP, typename KeyT>
__global__ __launch_bounds__(NT) void resolve_k(const uint32_t* __restrict__ gstart,
                                                const uint32_t* __restrict__ gsize,
                                                const uint32_t* __restrict__ gdepth,
                                                uint32_t* __restrict__ ord, uint8_t* __restrict__ flag,
                                                KeyView<KeyT> kv) {
  static_assert(CAP < 65535 && CAP % NT == 0, "positions are 16-bit");
  constexpr int kPer = CAP / NT;
  __shared__ uint32_t node[CAP];
  __shared__ uint32_t dep[CAP];
  __shared__ uint32_t sub[CAP];    // position of the member's subgroup pivot
  __shared__ uint64_t hk[CAP];     // first difference with the pivot, then side_key
  __shared__ uint64_t dig[CAP];    // packed digits from the first difference on
  __shared__ uint16_t opos[CAP];   // positions of the open members, ascending
  __shared__ uint16_t perm[CAP];   // sorted order of the open members (positions)
  __shared__ uint16_t queue[CAP];  // members whose comparison needs a whole wave
  __shared__ uint8_t res[CAP];     // member's subgroup is closed
  __shared__ uint8_t mark[CAP];    // open-list entry starts a new subgroup
  __shared__ uint32_t qn;
  __shared__ uint32_t shm[NT / kWave > 0 ? NT / kWave : 1];

  const uint32_t s = gstart[blockIdx.x];
  const uint32_t m = gsize[blockIdx.x];
  const uint32_t d0 = gdepth[blockIdx.x];
  const uint32_t width = kv.dbits >= 64 ? 1u : uint32_t(64 / kv.dbits);  // positions per digit
  const uint64_t last_mask = kv.last_digit_mask();
  for (uint32_t i = threadIdx.x; i < m; i += NT) {
    node[i] = ord[s + i];
    sub[i] = 0;
    dep[i] = d0;
    res[i] = 0;
  }
  __syncthreads();

  for (;;) {
    // (a) list the open members
    uint32_t n = 0;
    for (uint32_t base = 0; base < m; base += NT) {
      const uint32_t i = base + threadIdx.x;
      const bool f = i < m && !res[i];
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan<NT>(uint32_t(f), shm, &tot);
      if (f) opos[n + ex] = uint16_t(i);
      n += tot;
    }
    if (n == 0) break;
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();

    // (b) first difference with the pivot and the sort key there: (side,
    // distance of the first difference, digits from it on). A short window
    // per thread; members whose window agreed go to whole waves (64
    // positions per step) and get their key after.
    bool open = false;
    for (uint32_t k = threadIdx.x; k < n; k += NT) {
      const uint32_t i = opos[k];
      const uint32_t L = sub[i];
      if (i == L) {
        hk[i] = side_key(1, 0);
        dig[i] = 0;
        continue;
      }
      const typename KeyView<KeyT>::Cmp c = kv.compare(node[i], node[L], dep[i], kThreadWindow, width);
      if (c.d == kUndecided) {
        queue[atomicAdd(&qn, 1u)] = uint16_t(i);
      } else if (c.d == kNoDiff) {
        hk[i] = side_key(1, 0);
        dig[i] = 0;
      } else {
        hk[i] = side_key(c.da < c.dl ? 0u : 2u, c.d - dep[i]);
        dig[i] = c.dig;
        dep[i] = c.d + width;
        open = true;
      }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x / kWave; q < qn; q += NT / kWave) {
      const uint32_t i = queue[q];
      const uint32_t L = sub[i];
      const uint32_t d = kv.wave_first_diff(node[i], node[L], dep[i] + kThreadWindow);
      if (__lane_id() == 0) {
        if (d == kNoDiff) {
          hk[i] = side_key(1, 0);
          dig[i] = 0;
        } else {
          const uint64_t da = kv.digit(node[i], d), dl = kv.digit(node[L], d);
          hk[i] = side_key(da < dl ? 0u : 2u, d - dep[i]);
          dig[i] = kv.digits(node[i], d, width);
          dep[i] = d + width;
          open = true;
        }
      }
    }
    for (uint32_t k = threadIdx.x; k < n; k += NT) perm[k] = opos[k];
    if (!__syncthreads_or(open)) break;  // what is still open consists of copies of its pivot

    // (d) stable merge sort of the open list by (subgroup, side key,
    // digits): runs of width w = 1, 2, 4, ... merged pairwise, one
    // workgroup barrier per level. Each thread writes a fixed range of
    // outputs: it finds where its first output splits the pair's two runs
    // (merge path: the number of entries of the first run among the first
    // outputs, by binary search) and merges sequentially from there.
    // Ping-pongs between perm and queue (free after the comparisons).
    auto before = [&](uint32_t a, uint32_t b) {
      return sub[a] != sub[b] ? sub[a] < sub[b] : hk[a] != hk[b] ? hk[a] < hk[b] : dig[a] < dig[b];
    };
    uint16_t* src = perm;
    uint16_t* dst = queue;
    const uint32_t per = (n + NT - 1) / NT;  // outputs per thread
    for (uint32_t w = 1; w < n; w <<= 1) {
      uint32_t o = threadIdx.x * per;
      const uint32_t o_end = min(o + per, n);
      while (o < o_end) {
        const uint32_t base = o - o % (2 * w);  // the pair's first run starts here
        const uint32_t a_len = min(w, n - base);
        const uint32_t b_beg = base + a_len;
        const uint32_t b_len = b_beg < n ? min(w, n - b_beg) : 0u;
        const uint32_t diag = o - base;
        uint32_t lo = diag > b_len ? diag - b_len : 0u, hi = min(diag, a_len);
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (!before(src[b_beg + diag - 1 - mid], src[base + mid]))
            lo = mid + 1;
          else
            hi = mid;
        }
        uint32_t i = lo, j = diag - lo;
        const uint32_t stop = min(o_end, b_beg + b_len);
        for (; o < stop; ++o) {
          const bool take_a = i < a_len && (j >= b_len || !before(src[b_beg + j], src[base + i]));
          dst[o] = take_a ? src[base + i++] : src[b_beg + j++];
        }
      }
      __syncthreads();
      uint16_t* t = src;
      src = dst;
      dst = t;
    }
    const uint16_t* sorted = src;

    // (e) move: the k-th open position receives the k-th member in order
    uint32_t tn[kPer], td[kPer];
    uint64_t th[kPer], tg[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t k = uint32_t(j) * NT + threadIdx.x;
      if (k < n) {
        const uint32_t from = sorted[k];
        tn[j] = node[from];
        td[j] = dep[from];
        th[j] = hk[from];
        tg[j] = dig[from];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t k = uint32_t(j) * NT + threadIdx.x;
      if (k < n) {
        const uint32_t dst = opos[k];
        node[dst] = tn[j];
        dep[dst] = td[j];
        hk[dst] = th[j];
        dig[dst] = tg[j];
      }
    }
    __syncthreads();

    // (f) split where the key changes; close copies of the pivot, ended
    // sequences and single members
    for (uint32_t k = threadIdx.x; k < n; k += NT) {
      const uint32_t i = opos[k];
      bool mk = k == 0;
      if (!mk) {
        const uint32_t p = opos[k - 1];
        mk = sub[i] != sub[p] || hk[i] != hk[p] || dig[i] != dig[p];
      }
      mark[k] = mk ? 1 : 0;
    }
    __syncthreads();
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n; base += NT) {
      const uint32_t k = base + threadIdx.x;
      const uint32_t i = k < n ? opos[k] : 0u;
      const uint32_t v = (k < n && mark[k]) ? i : 0u;
      uint32_t tot;
      uint32_t r = block_inclusive_max<NT>(v, shm, &tot);
      r = r > carry ? r : carry;
      if (k < n) {
        if (mark[k] && i > 0) flag[s + i] = 1;
        const bool single = mark[k] && (k + 1 == n || mark[k + 1]);
        const bool copies = (hk[i] >> 32) == 1;
        if (copies || (dig[i] & last_mask) == 0 || single) res[i] = 1;
        sub[i] = r;
      }
      carry = tot > carry ? tot : carry;
    }
    __syncthreads();
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < m; i += NT) ord[s + i] = node[i];
}

// Orders groups of at most W members (W a power of two <= 64), W lanes per
// group and 256 / W groups per workgroup, with the same pivot splitting as
// resolve_k: the members live in registers and are sorted by a bitonic
// network over the group's lanes. Lanes past a group's size, and whole groups
// past `ngroups`, are padding that sorts last and writes nothing.
template <int W, typename KeyT>
__global__ __launch_bounds__(256) void resolve_lanes_k(const uint32_t* __restrict__ gstart,
                                                       const uint32_t* __restrict__ gsize,
                                                       const uint32_t* __restrict__ gdepth, uint32_t ngroups,
                                                       uint32_t* __restrict__ ord, uint8_t* __restrict__ flag,
                                                       KeyView<KeyT> kv) {
  static_assert(W >= 2 && W <= kWave && (W & (W - 1)) == 0, "W must be a power of two <= 64");
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  const uint32_t gi = t / W;
  const uint32_t l = t % W;
  uint32_t s = 0, m = 0, d0 = 0;
  if (gi < ngroups) {
    s = gstart[gi];
    m = gsize[gi];
    d0 = gdepth[gi];
  }
  const bool in = l < m;
  const uint32_t width = kv.dbits >= 64 ? 1u : uint32_t(64 / kv.dbits);
  const uint64_t last_mask = kv.last_digit_mask();
  uint32_t node = in ? ord[s + l] : 0xffffffffu;
  uint32_t sub = in ? 0u : 0xffffffffu;  // lane of the subgroup's pivot
  uint32_t dep = d0;
  bool res = !in;
  uint64_t hk = in ? 0ull : ~0ull, dig = in ? 0ull : ~0ull;

  for (;;) {
    // (a) first difference with the pivot: a short window per lane, then
    // the whole wave for every lane whose window agreed
    const uint32_t lead = __shfl(node, in ? sub : l, W);
    typename KeyView<KeyT>::Cmp c{kNoDiff, 0, 0, 0};
    if (!res && l != sub) c = kv.compare(node, lead, dep, kThreadWindow, width);
    bool late = false;  // decided by the whole wave: keys still to fetch
    for (uint64_t pend = __ballot(c.d == kUndecided); pend; pend &= pend - 1) {
      const int q = __ffsll((unsigned long long)pend) - 1;
      const uint32_t qa = __shfl(node, q, kWave), qb = __shfl(lead, q, kWave), qt = __shfl(dep, q, kWave);
      const uint32_t r = kv.wave_first_diff(qa, qb, qt + kThreadWindow);
      if (__lane_id() == q) {
        c.d = r;
        late = true;
      }
    }
    const uint32_t d = c.d;
    // (b) sort keys
    bool open = false;
    if (res) {
      hk = in ? 0ull : ~0ull;
      dig = in ? 0ull : ~0ull;
    } else if (d == kNoDiff) {
      hk = side_key(1, 0);
      dig = 0;
    } else {
      const uint64_t da = late ? kv.digit(node, d) : c.da, dl = late ? kv.digit(lead, d) : c.dl;
      hk = side_key(da < dl ? 0u : 2u, d - dep);
      dig = late ? kv.digits(node, d, width) : c.dig;
      dep = d + width;
      open = true;
    }
    if (!__any(open)) break;  // what is still open consists of copies of its pivot
    // (c) bitonic sort over the group's lanes by (sub, hk, dig)
#pragma unroll
    for (int size = 2; size <= W; size <<= 1) {
#pragma unroll
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const uint32_t o_sub = __shfl_xor(sub, stride, W);
        const uint64_t o_hk = __shfl_xor(hk, stride, W);
        const uint64_t o_dig = __shfl_xor(dig, stride, W);
        const uint32_t o_node = __shfl_xor(node, stride, W);
        const uint32_t o_dep = __shfl_xor(dep, stride, W);
        const int o_res = __shfl_xor(int(res), stride, W);
        const bool o_less = o_sub != sub ? o_sub < sub : o_hk != hk ? o_hk < hk : o_dig < dig;
        const bool o_more = o_sub != sub ? o_sub > sub : o_hk != hk ? o_hk > hk : o_dig > dig;
        const bool keep_min = ((l & size) == 0) == ((l & stride) == 0);
        if (keep_min ? o_less : o_more) {
          sub = o_sub;
          hk = o_hk;
          dig = o_dig;
          node = o_node;
          dep = o_dep;
          res = o_res != 0;
        }
      }
    }
    // (d) split where the key changes; close copies of the pivot, ended
    // sequences and single members
    const uint32_t p_sub = __shfl_up(sub, 1, W);
    const uint64_t p_hk = __shfl_up(hk, 1, W);
    const uint64_t p_dig = __shfl_up(dig, 1, W);
    const bool mark = in && (l == 0 || p_sub != sub || p_hk != hk || p_dig != dig);
    uint32_t v = mark ? l : 0u;
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
      const uint32_t u = __shfl_up(v, o, W);
      if (l >= uint32_t(o)) v = u > v ? u : v;
    }
    const bool next_mark = __shfl_down(int(mark), 1, W) != 0;
    if (in) {
      if (mark && l > 0) flag[s + l] = 1;
      if (!res) {
        const bool single = mark && (l + 1 == m || next_mark);
        const bool copies = (hk >> 32) == 1;
        if (copies || (dig & last_mask) == 0 || single) res = true;
      }
      sub = v;
    }
  }
  if (in) ord[s + l] = node;
}

// ---------------------------------------------------------------------------
// Segments (open groups) and their classification into work lists by size.
//
// Classes 0-3 hold groups of at most 8, 16, 32, 64 members (resolve_lanes_k
// with that many lanes per group); kMediumClass groups of up to medium_cap
// (<= kMediumCapSmall) members (resolve_k, 256 threads); kBigClass groups of
// up to big_cap (<= kBigCap) members (resolve_k, 1024 threads); kLargeClass
// the rest (global passes). The lists share one set of arrays: list c
// occupies [off[c], off[c] + cnt[c]). Every group is ordered on its own.

constexpr int kLaneClasses = 4;
constexpr int kMediumClass = kLaneClasses;
constexpr int kBigClass = kLaneClasses + 1;
constexpr int kLargeClass = kLaneClasses + 2;
constexpr int kSegClasses = kLaneClasses + 3;

// medium_cap <= kMediumCapSmall <= big_cap; a group above big_cap is large.
__device__ __forceinline__ int seg_class(uint32_t z, uint32_t medium_cap, uint32_t big_cap) {
  return z <= 8 ? 0 : z <= 16 ? 1 : z <= 32 ? 2 : z <= kSmallCap ? 3 : z <= medium_cap ? kMediumClass
         : z <= big_cap ? kBigClass : kLargeClass;
}

// Open segment j (two or more members, not done) -> its size class, for the
// tile compaction (compact.h) that builds the work lists.
struct SegClassOf {
  const uint32_t* size;
  const uint8_t* done;  // optional
  uint32_t medium_cap, big_cap;
  __device__ __forceinline__ int operator()(uint32_t j) const {
    const uint32_t z = size[j];
    if (z <= 1 || (done && done[j])) return -1;
    return seg_class(z, medium_cap, big_cap);
  }
};
struct SegCopy {
  const uint32_t* start;
  const uint32_t* size;
  const uint32_t* depth;  // optional: depth 0
  uint32_t* o_start;
  uint32_t* o_size;
  uint32_t* o_depth;
  __device__ __forceinline__ void operator()(uint32_t j, int, uint32_t o) const {
    o_start[o] = start[j];
    o_size[o] = size[j];
    o_depth[o] = depth ? depth[j] : 0u;
  }
};

// ---------------------------------------------------------------------------
// Global pass for groups too large for the resolvers. Items are the members of
// the large groups laid out group after group; ioff[g] is the absolute index
// of the first item of group g.

// Item offsets of the large groups of a classified list: ioff[g] =
// exclusive scan of the sizes of the meta[kLargeClass] groups listed from
// meta[kSegClasses + kLargeClass], ioff[ng] = *total = their items. One
// workgroup of 1024 threads (computed with the lists, so the host learns the
// total with the list counts).
__global__ __launch_bounds__(1024) void large_offsets_k(const uint32_t* __restrict__ size,
                                                        const uint32_t* __restrict__ meta,
                                                        uint32_t* __restrict__ ioff, uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[1024 / kWave];
  const uint32_t ng = meta[kLargeClass];
  const uint32_t* z = size + meta[kSegClasses + kLargeClass];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < ng; base += 1024) {
    const uint32_t g = base + threadIdx.x;
    const uint32_t v = g < ng ? z[g] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024>(v, sh, &tot);
    if (g < ng) ioff[g] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    ioff[ng] = carry;
    *total = carry;
  }
}

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

// fdv[i] = first difference of item i's sequence with its group's first
// member, the pivot (kNoDiff for the pivot and its copies). Each thread
// compares one item over a short window; items that still agree are appended
// to `longq` for large_fd_wave_k.
template <typename KeyT>
__global__ __launch_bounds__(256) void large_fd_k(const uint32_t* __restrict__ gstart,
                                                  const uint32_t* __restrict__ gdepth,
                                                  const uint32_t* __restrict__ ioff, uint32_t ng, uint32_t nitems,
                                                  const uint32_t* __restrict__ ord, uint32_t* __restrict__ fdv,
                                                  uint32_t* __restrict__ longq, uint32_t* __restrict__ nlong,
                                                  KeyView<KeyT> kv) {
  // no early exit: wave_append needs every lane
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t d = kNoDiff;
  if (i < nitems) {
    const uint32_t g = group_of_item(ioff, ng, i);
    const uint32_t a = ord[gstart[g] + (i - ioff[g])];
    const uint32_t b = ord[gstart[g]];
    if (a != b) d = kv.first_diff_window(a, b, gdepth[g], kThreadWindow);
    fdv[i] = d;
  }
  const uint32_t slot = wave_append(d == kUndecided, nlong);
  if (d == kUndecided) longq[slot] = i;
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

// Global sort key of an item of group g, hi above lo:
//  * head pass (groups are whole classes at depth 0): hi = g, lo = the first
//    `width` digits of the sequence;
//  * pivot pass: hi = g << (2 + fd_bits) | side << fd_bits | fdkey, lo =
//    `width` digits from the item's first difference d with the pivot on,
//    where side says whether the item is below, equal to or above the pivot
//    at d, and fdkey = d - depth (below) or its complement in fd_bits
//    (above), as in side_key.
// Packed into one word as hi << dig_bits | lo when that fits, else two words.
struct LargeKey {
  int fd_bits;   // 0 in the head pass
  int dig_bits;  // width * dbits
  uint32_t width;
  bool packed;
  __device__ __forceinline__ uint64_t hi_of(const uint64_t* ka, uint32_t i) const {
    return packed ? (dig_bits >= 64 ? 0ull : ka[i] >> dig_bits) : ka[i];
  }
  __device__ __forceinline__ uint64_t lo_of(const uint64_t* ka, const uint64_t* kb, uint32_t i) const {
    return packed ? (dig_bits >= 64 ? ka[i] : (ka[i] & ((1ull << dig_bits) - 1))) : kb[i];
  }
  __device__ __forceinline__ uint32_t group_of(uint64_t hi) const {
    return uint32_t(fd_bits ? hi >> (2 + fd_bits) : hi);
  }
};

// head (head pass only): the first head_w digits of every node, packed as by
// KeyView::digits; fdv (pivot pass only): first differences with the pivots.
template <typename KeyT>
__global__ void large_gather_k(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ gdepth,
                               const uint32_t* __restrict__ ioff, uint32_t ng, uint32_t nitems,
                               const uint32_t* __restrict__ ord, const uint32_t* __restrict__ fdv, LargeKey lk,
                               uint64_t* __restrict__ ka, uint64_t* __restrict__ kb, uint32_t* __restrict__ val,
                               KeyView<KeyT> kv, const uint64_t* __restrict__ head, uint32_t head_w) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const uint32_t g = group_of_item(ioff, ng, i);
  const uint32_t node = ord[gstart[g] + (i - ioff[g])];
  uint64_t hi, lo;
  if (!lk.fd_bits) {
    const uint32_t drop = (head_w - lk.width) * uint32_t(kv.dbits);
    lo = drop >= 64 ? 0ull : head[node] >> drop;
    hi = g;
  } else {
    const uint32_t d = fdv[i];
    uint64_t side = 1, fdkey = 0;
    lo = 0;
    if (d != kNoDiff) {
      const uint32_t leader = ord[gstart[g]];
      const uint64_t fdmask = (1ull << lk.fd_bits) - 1;
      const uint64_t rel = d - gdepth[g];
      side = kv.digit(node, d) < kv.digit(leader, d) ? 0 : 2;
      fdkey = side == 0 ? rel : (fdmask - rel);
      lo = kv.digits(node, d, lk.width);
    }
    hi = (uint64_t(g) << (2 + lk.fd_bits)) | (side << lk.fd_bits) | fdkey;
  }
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
  const uint64_t hi = lk.hi_of(ka, i), lo = lk.lo_of(ka, kb, i);
  const uint32_t g = lk.group_of(hi);
  const uint32_t p = gstart[g] + (i - ioff[g]);
  ord[p] = val[i];
  item_pos[i] = p;
  const bool st = (i == ioff[g]) || hi != lk.hi_of(ka, i - 1) || lo != lk.lo_of(ka, kb, i - 1);
  start_flag[i] = st;
  if (st && i != ioff[g]) flag[p] = 1;
}

// Subgroup j starts at item S[j] (S = compacted start flags). Head pass: its
// depth is `width`; pivot pass: `width` past its first difference with the
// pivot. It is closed when it holds copies of the pivot or its sequences
// ended inside the digits.
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
    const uint64_t hi = lk.hi_of(ka, i), lo = lk.lo_of(ka, kb, i);
    const uint32_t g = lk.group_of(hi);
    bool copies = false;
    uint32_t depth = lk.width;
    if (lk.fd_bits) {
      const uint64_t fdmask = (1ull << lk.fd_bits) - 1;
      const uint32_t side = uint32_t(hi >> lk.fd_bits) & 3u;
      const uint64_t fdkey = hi & fdmask;
      const uint64_t rel = side == 0 ? fdkey : (fdmask - fdkey);
      copies = side == 1;
      depth = copies ? 0u : uint32_t(gdepth[g] + rel + lk.width);
    }
    sub_item[j] = i;
    seg_start[j] = item_pos[i];
    seg_depth[j] = depth;
    seg_done[j] = copies || (lo & last_mask) == 0;
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

__global__ void set_u32_k(uint32_t* __restrict__ dst, uint32_t v) { *dst = v; }

}  // namespace kb
