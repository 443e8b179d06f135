// Signature construction for one refinement round (Definition 3; Algorithm 1,
// the join that fills pId_old(tId), the projection/sort/de-duplication that
// builds F, and the per-node signature string).
//
// For every active node u (a member of a class with two or more members) the
// kernel gathers key(e) = (edge label rank << pid_bits) | pid_prev[dst(e)]
// over u's out-edges, sorts the keys of u ascending, drops duplicates and
// writes the unique keys to ukey[rowptr[u] ...] and their number to ucnt[u].
// The key order equals the order of the pairs (label, pid) because the label
// occupies the high bits.
//
// Nodes alone in their class are skipped: a refinement never merges classes
// (Proposition 1), so such a node stays alone whatever its signature.
//
// One launch covers all active nodes. Work is split by out-degree: one thread
// (<= 16 keys, register sorting network; the wave's rows staged in LDS so
// that loads and stores are contiguous), one wave (two nodes per wave when
// both have <= 32 keys) (<= 64 keys, shuffle
// bitonic; <= 512 keys, 2, 4 or 8 keys per lane in registers), one workgroup
// (<= 4096 keys, LDS bitonic); hubs (more keys) are sorted by (hub, key)
// together with the device-wide radix sort before the launch, or, when that
// key does not fit 64 bits, by one workgroup each with a global-memory radix
// sort. When every key is below 2^kBmKeyBits the nodes above 64 keys
// de-duplicate through a bitmap instead (one wave per node, hubs in chunks of
// one workgroup), and keep the bitmap for the ordering's first-difference
// searches. Workgroups are laid out hubs first, so the longest ones start
// first.
#pragma once

#include "common.h"
#include "scan_radix.h"

namespace kb {

constexpr uint32_t kThreadMaxDeg = 16;
constexpr uint32_t kWaveMaxDeg = 64;
constexpr uint32_t kMidMaxDeg = 512;
constexpr uint32_t kBlockMaxDeg = 4096;
constexpr int kSigNT = 256;
constexpr int kBmKeyBits = 12;
constexpr uint32_t kHubChunk = 8192;  // edges per hub unit in bitmap rounds (at least)
constexpr uint32_t kHubUnits = 16;    // units per hub (at most)
constexpr uint32_t kBmMaxWords = (1u << kBmKeyBits) / 32;

template <typename AdjT, typename KeyT>
struct SigArgs {
  const uint32_t* rowptr;  // [N+1]
  const AdjT* adj;         // [E] (label rank << dst_bits) | dst, CSR order
  const void* pid;         // [N] previous-round ids, pid_bytes (1, 2 or 4) each
  int pid_bytes;
  KeyT* ukey;              // [E] unique keys per node at rowptr offsets
  uint32_t* ucnt;          // [N]
  uint64_t* head;          // [N] first hw digits (key + 1, 0 past the end), most significant first
  int dst_bits;
  int pid_bits;
  int hdbits;              // bits of one digit: key bits + 1
  uint32_t hw;             // digits per head word: 64 / hdbits

  __device__ __forceinline__ KeyT key_of(AdjT a) const {
    const uint32_t dst = uint32_t(a & ((AdjT(1) << dst_bits) - 1));
    const uint64_t lab = uint64_t(a >> dst_bits);
    const uint32_t p = pid_bytes == 4   ? static_cast<const uint32_t*>(pid)[dst]
                       : pid_bytes == 2 ? uint32_t(static_cast<const uint16_t*>(pid)[dst])
                                        : uint32_t(static_cast<const uint8_t*>(pid)[dst]);
    return KeyT((lab << pid_bits) | uint64_t(p));
  }
  __device__ __forceinline__ uint64_t head_of(const KeyT* k, uint32_t c) const {
    if (hdbits >= 64) return c ? uint64_t(k[0]) + 1ull : 0ull;
    uint64_t v = 0;
    for (uint32_t j = 0; j < hw; ++j) v = (v << hdbits) | (j < c ? uint64_t(k[j]) + 1ull : 0ull);
    return v;
  }
};

// Work of one launch. Lists hold node ids by out-degree: wave (17..64), mid
// (65..512), block (513..4096) and hub lists. With bitmaps (bm != nullptr)
// mid and block nodes take one wave each (slot i for entry i of the mid list
// followed by the block list) and hub h takes slot hub_slot0() + h; without,
// a mid node takes one wave and a block node one workgroup.
struct SigWork {
  const uint32_t* anode;  // all active nodes (the thread part skips those above kThreadMaxDeg)
  const uint32_t* actr;   // dense thread part: node n is active when actr[n] == tag
  uint32_t tag, n_nodes;
  bool dense;             // thread part over all node ids (in order) instead of anode
  const uint32_t* wl;     // wave list
  const uint32_t* ml;     // mid list
  const uint32_t* bl;     // block list
  const uint32_t* hl;     // hub list
  uint32_t nact, nw, nm, nb, nh;
  uint32_t* bm;           // bitmaps, `words` 32-bit words each, or nullptr
  uint32_t* bmslot;       // [N]
  uint32_t words;
  void* hub_tmp;          // radix ping-pong space of the hubs (KeyT)
  const uint32_t* hub_toff;  // [N] offset of a hub's space in hub_tmp
  uint32_t hub_units;     // workgroups per hub (bitmap rounds; else 1)
  uint32_t hub_chunk;     // edges per unit
  int key_bits;
  // nodes outside [node_lo, node_hi) are skipped: a launch over one
  // partition of a streamed edge table, whose rows alone are in the window
  uint32_t node_lo = 0, node_hi = 0xffffffffu;

  __host__ __device__ bool in(uint32_t n) const { return n >= node_lo && n < node_hi; }
  static constexpr uint32_t kWavesPerUnit = kSigNT / kWave;
  __host__ __device__ uint32_t hub_slot0() const { return nm + nb; }
  // two wave-list entries per wave (sig_wave_pair)
  __host__ __device__ uint32_t wave_units() const { return ((nw + 1) / 2 + kWavesPerUnit - 1) / kWavesPerUnit; }
  __host__ __device__ uint32_t thread_units() const { return ((dense ? n_nodes : nact) + kSigNT - 1) / kSigNT; }
  // bitmap rounds: one wave per mid or block node; else one workgroup per
  // block node and one wave per mid node
  __host__ __device__ uint32_t block_units() const {
    return bm ? (nm + nb + kWavesPerUnit - 1) / kWavesPerUnit : nb;
  }
  __host__ __device__ uint32_t mid_units() const { return bm ? 0u : (nm + kWavesPerUnit - 1) / kWavesPerUnit; }
  __host__ __device__ uint32_t grid() const {
    return nh * hub_units + block_units() + mid_units() + wave_units() + thread_units();
  }
};

template <typename KeyT>
__device__ __forceinline__ void cas_up(KeyT& a, KeyT& b, bool up) {
  const KeyT lo = a < b ? a : b;
  const KeyT hi = a < b ? b : a;
  a = up ? lo : hi;
  b = up ? hi : lo;
}

// ---- one thread per node, out-degree <= 16 ------------------------------------
// Each lane sorts its node's keys with a 16-key sorting network in registers
// and de-duplicates them. The rows pass through LDS: the wave lists the edges
// of its 64 nodes one node after another, loads them (consecutive lanes read
// consecutive edges of a row; a lane reading its own row would put the
// wave's accesses 64 rows apart) and turns them into keys; each lane takes
// its keys from the list and puts its unique keys back in place, and the
// wave writes those out the same way. `n` is kNone for lanes without a node
// (or whose node has more than kThreadMaxDeg edges). Every thread of the
// workgroup calls it (three workgroup barriers).
template <typename KeyT>
struct ThreadLds {
  static constexpr uint32_t kCap = kWave * kThreadMaxDeg;
  KeyT key[kSigNT / kWave][kCap];
  uint8_t own[kSigNT / kWave][kCap];      // lane of the node the listed edge belongs to
  uint32_t delta[kSigNT / kWave][kWave];  // per lane: row start in adj minus list start
  uint32_t lim[kSigNT / kWave][kWave];    // per lane: end of its unique keys in the list
};
constexpr uint32_t kNone = 0xffffffffu;

template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_thread_wave(const SigArgs<AdjT, KeyT>& a, uint32_t n, ThreadLds<KeyT>& t) {
  constexpr int M = kThreadMaxDeg;
  const int wv = threadIdx.x / kWave;
  const int lane = __lane_id();
  uint32_t beg = 0, deg = 0;
  if (n != kNone) {
    beg = a.rowptr[n];
    deg = a.rowptr[n + 1] - beg;
    if (deg > kThreadMaxDeg) n = kNone, deg = 0;
  }
  const uint32_t incl = wave_inclusive_scan(deg);
  const uint32_t o = incl - deg;  // this lane's first list position
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  t.delta[wv][lane] = beg - o;
  for (uint32_t q = 0; q < deg; ++q) t.own[wv][o + q] = uint8_t(lane);
  __syncthreads();
  for (uint32_t i = lane; i < total; i += kWave) t.key[wv][i] = a.key_of(a.adj[t.delta[wv][t.own[wv][i]] + i]);
  __syncthreads();
  KeyT k[M];
#pragma unroll
  for (int j = 0; j < M; ++j) k[j] = (uint32_t(j) < deg) ? t.key[wv][o + j] : ~KeyT(0);
#pragma unroll
  for (int size = 2; size <= M; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const int j = i ^ stride;
        if (j > i) cas_up(k[i], k[j], (i & size) == 0);
      }
    }
  }
  uint32_t c = 0;
  uint64_t hv = 0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    if (uint32_t(j) < deg && (j == 0 || k[j] != k[j - 1])) {
      t.key[wv][o + c] = k[j];
      if (c < a.hw) hv = a.hdbits >= 64 ? uint64_t(k[j]) + 1ull : (hv << a.hdbits) | (uint64_t(k[j]) + 1ull);
      ++c;
    }
  }
  if (a.hdbits < 64 && c < a.hw) hv <<= (a.hw - c) * a.hdbits;
  t.lim[wv][lane] = o + c;
  if (n != kNone) {
    a.ucnt[n] = c;
    a.head[n] = hv;
  }
  __syncthreads();
  for (uint32_t i = lane; i < total; i += kWave) {
    const uint32_t ow = t.own[wv][i];
    if (i < t.lim[wv][ow]) a.ukey[t.delta[wv][ow] + i] = t.key[wv][i];
  }
}

// ---- one wave per node, 16 < out-degree <= 64 ---------------------------------
template <typename KeyT>
__device__ __forceinline__ KeyT wave_bitonic64(KeyT k) {
  const int lane = __lane_id();
#pragma unroll
  for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const KeyT o = __shfl_xor(k, stride, kWave);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const KeyT mn = k < o ? k : o;
      const KeyT mx = k < o ? o : k;
      k = (lower == up) ? mn : mx;
    }
  }
  return k;
}

// Every lane of the wave calls it with the same n.
template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_wave_node(const SigArgs<AdjT, KeyT>& a, uint32_t n) {
  const int lane = __lane_id();
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  KeyT k = uint32_t(lane) < deg ? a.key_of(a.adj[beg + lane]) : ~KeyT(0);
  k = wave_bitonic64(k);
  const KeyT prev = __shfl_up(k, 1, kWave);
  const bool f = uint32_t(lane) < deg && (lane == 0 || k != prev);
  const uint64_t b = __ballot(f);
  const uint32_t r = uint32_t(__popcll(b & lanemask_lt()));
  if (f) a.ukey[beg + r] = k;
  // head word: the first hw unique keys, OR-reduced over the wave
  uint64_t hv = 0;
  if (f && r < a.hw) hv = a.hdbits >= 64 ? uint64_t(k) + 1ull : (uint64_t(k) + 1ull) << ((a.hw - 1 - r) * a.hdbits);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) hv |= __shfl_xor(hv, o, kWave);
  if (lane == 0) {
    a.ucnt[n] = __popcll(b);
    a.head[n] = hv;
  }
}

// Two wave-list nodes per wave. When both have at most 32 edges (or the
// second is kNone) each takes a half-wave: a 32-lane bitonic sort (15
// stages instead of the full wave's 21, with a 32-wide shuffle network that
// stays inside the half) and the same de-duplication over the half's lanes;
// else the wave runs sig_wave_node for one node after the other. With one
// node per wave, a node of 17..32 edges left half of the lanes idle.
template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_wave_pair(const SigArgs<AdjT, KeyT>& a, uint32_t n0, uint32_t n1) {
  const uint32_t b0 = a.rowptr[n0];
  const uint32_t d0 = a.rowptr[n0 + 1] - b0;
  uint32_t b1 = 0, d1 = 0;
  if (n1 != kNone) {
    b1 = a.rowptr[n1];
    d1 = a.rowptr[n1 + 1] - b1;
  }
  if (d0 > kWave / 2 || d1 > kWave / 2) {
    sig_wave_node(a, n0);
    if (n1 != kNone) sig_wave_node(a, n1);
    return;
  }
  const int lane = __lane_id();
  const int half = lane >> 5;
  const uint32_t l = uint32_t(lane & 31);
  const uint32_t n = half ? n1 : n0;
  const uint32_t beg = half ? b1 : b0;
  const uint32_t deg = half ? d1 : d0;
  KeyT k = l < deg ? a.key_of(a.adj[beg + l]) : ~KeyT(0);
#pragma unroll
  for (uint32_t size = 2; size <= 32; size <<= 1) {
#pragma unroll
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      const KeyT o = __shfl_xor(k, int(stride), kWave);
      const bool up = (l & size) == 0;  // size 32: both halves ascending
      const bool lower = (l & stride) == 0;
      const KeyT mn = k < o ? k : o;
      const KeyT mx = k < o ? o : k;
      k = (lower == up) ? mn : mx;
    }
  }
  const KeyT prev = __shfl_up(k, 1, kWave);
  const bool f = l < deg && (l == 0 || k != prev);
  const uint32_t bh = uint32_t(__ballot(f) >> (32 * half));
  const uint32_t r = uint32_t(__popc(bh & ((1u << l) - 1u)));
  if (f) a.ukey[beg + r] = k;
  uint64_t hv = 0;
  if (f && r < a.hw) hv = a.hdbits >= 64 ? uint64_t(k) + 1ull : (uint64_t(k) + 1ull) << ((a.hw - 1 - r) * a.hdbits);
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) hv |= __shfl_xor(hv, o, kWave);
  if (l == 0 && n != kNone) {
    a.ucnt[n] = uint32_t(__popc(bh));
    a.head[n] = hv;
  }
}

// ---- one wave per node, K keys per lane, out-degree <= 64 K ----------------------
// Bitonic sort of 64 K keys held in registers, element i = lane * K + q in
// lane `lane`, register q: partners closer than K are in the same lane, the
// others K-aligned in lane ^ (stride / K).
template <int K, typename KeyT>
__device__ __forceinline__ void wave_bitonic_k(KeyT (&k)[K]) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (uint32_t size = 2; size <= kWave * K; size <<= 1) {
#pragma unroll
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride < K) {
#pragma unroll
        for (uint32_t q = 0; q < K; ++q) {
          const uint32_t p = q ^ stride;
          if (p > q) cas_up(k[q], k[p], ((lane * K + q) & size) == 0);
        }
      } else {
#pragma unroll
        for (uint32_t q = 0; q < K; ++q) {
          const uint32_t i = lane * K + q;
          const KeyT o = __shfl_xor(k[q], int(stride / K), kWave);
          const bool up = (i & size) == 0;
          const bool lower = (i & stride) == 0;
          const KeyT mn = k[q] < o ? k[q] : o;
          const KeyT mx = k[q] < o ? o : k[q];
          k[q] = (lower == up) ? mn : mx;
        }
      }
    }
  }
}

// Every lane of the wave calls it with the same n (out-degree <= 64 K).
template <int K, typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_wave_multi_node(const SigArgs<AdjT, KeyT>& a, uint32_t n, uint32_t beg,
                                                    uint32_t deg) {
  const uint32_t lane = __lane_id();
  KeyT k[K];
#pragma unroll
  for (uint32_t q = 0; q < K; ++q) {  // coalesced loads; the sort places them
    const uint32_t j = q * kWave + lane;
    k[q] = j < deg ? a.key_of(a.adj[beg + j]) : ~KeyT(0);
  }
  wave_bitonic_k<K>(k);
  // first of each run of equal keys, in sorted order
  const KeyT before = __shfl_up(k[K - 1], 1, kWave);
  uint32_t first = 0;
#pragma unroll
  for (uint32_t q = 0; q < K; ++q) {
    const uint32_t i = lane * K + q;
    const KeyT pv = q == 0 ? before : k[q > 0 ? q - 1 : 0];
    if (i < deg && (i == 0 || k[q] != pv)) first |= 1u << q;
  }
  const uint32_t c = uint32_t(__popc(first));
  const uint32_t incl = wave_inclusive_scan(c);
  uint32_t r = incl - c;
  uint64_t hv = 0;
#pragma unroll
  for (uint32_t q = 0; q < K; ++q) {
    if ((first >> q) & 1u) {
      a.ukey[beg + r] = k[q];
      if (r < a.hw)
        hv |= a.hdbits >= 64 ? uint64_t(k[q]) + 1ull : (uint64_t(k[q]) + 1ull) << ((a.hw - 1 - r) * a.hdbits);
      ++r;
    }
  }
  hv = wave_or(hv);
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  if (lane == 0) {
    a.ucnt[n] = total;
    a.head[n] = hv;
  }
}

template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_mid_node(const SigArgs<AdjT, KeyT>& a, uint32_t n) {
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  if (deg <= 2 * kWave)
    sig_wave_multi_node<2>(a, n, beg, deg);
  else if (deg <= 4 * kWave)
    sig_wave_multi_node<4>(a, n, beg, deg);
  else
    sig_wave_multi_node<8>(a, n, beg, deg);
}

// ---- one workgroup per node, 64 < out-degree <= 4096 ----------------------------
template <typename KeyT>
__device__ __forceinline__ void block_bitonic(KeyT* s, uint32_t P) {
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < P / 2; i += kSigNT) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool up = (lo & size) == 0;
        const KeyT x = s[lo], y = s[hi];
        if ((x > y) == up) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_block_node(const SigArgs<AdjT, KeyT>& a, uint32_t n, KeyT* s, uint32_t* shc) {
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  uint32_t P = 128;
  while (P < deg) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += kSigNT) s[i] = i < deg ? a.key_of(a.adj[beg + i]) : ~KeyT(0);
  __syncthreads();
  block_bitonic(s, P);
  KeyT* out = a.ukey + beg;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < deg; base += kSigNT) {
    const uint32_t i = base + threadIdx.x;
    const bool f = i < deg && (i == 0 || s[i] != s[i - 1]);
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kSigNT>(uint32_t(f), shc, &tot);
    if (f) out[carry + ex] = s[i];
    carry += tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ucnt[n] = carry;
    a.head[n] = a.head_of(out, carry);
  }
}

// ---- small key universes: bitmap de-duplication ---------------------------------
// The workgroup ORs the node's keys into an LDS bitmap of `words` 32-bit
// words, then lists the set bits in ascending order (a block scan of the word
// popcounts gives each word's first output slot). The bitmap itself is kept
// in bm[slot * words ...] for first-difference searches, and bmslot[n] = slot.
// Head word (first hw keys) of a key set held as a bitmap in LDS.
template <typename AdjT, typename KeyT>
__device__ __forceinline__ uint64_t head_of_bits(const SigArgs<AdjT, KeyT>& a, const uint32_t* bits, uint32_t nw) {
  uint64_t v = 0;
  uint32_t c = 0;
  for (uint32_t j = 0; j < nw && c < a.hw; ++j) {
    uint32_t x = bits[j];
    while (x && c < a.hw) {
      const uint32_t key = j * 32u + uint32_t(__ffs(x) - 1);
      v = a.hdbits >= 64 ? uint64_t(key) + 1ull : (v << a.hdbits) | (uint64_t(key) + 1ull);
      ++c;
      x &= x - 1;
    }
  }
  if (a.hdbits < 64 && c < a.hw) v <<= (a.hw - c) * a.hdbits;
  return v;
}

// The same for one wave per node (out-degree <= 4096), each wave with its
// own LDS bitmap: all 64 lanes call it with the same n; LDS operations of
// one wave are performed in order, so no barrier is needed between its steps.
template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_bitmap_wave_node(const SigArgs<AdjT, KeyT>& a, uint32_t n, const SigWork& w,
                                                     uint32_t slot, uint32_t* bits) {
  const uint32_t lane = __lane_id();
  const uint32_t nw = w.words;
  for (uint32_t i = lane; i < nw; i += kWave) bits[i] = 0;
  __builtin_amdgcn_wave_barrier();
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  uint32_t i = lane;
  for (; i + 3 * kWave < deg; i += 4 * kWave) {
    const AdjT e0 = a.adj[beg + i], e1 = a.adj[beg + i + kWave];
    const AdjT e2 = a.adj[beg + i + 2 * kWave], e3 = a.adj[beg + i + 3 * kWave];
    const uint32_t k0 = uint32_t(a.key_of(e0)), k1 = uint32_t(a.key_of(e1));
    const uint32_t k2 = uint32_t(a.key_of(e2)), k3 = uint32_t(a.key_of(e3));
    atomicOr(&bits[k0 >> 5], 1u << (k0 & 31));
    atomicOr(&bits[k1 >> 5], 1u << (k1 & 31));
    atomicOr(&bits[k2 >> 5], 1u << (k2 & 31));
    atomicOr(&bits[k3 >> 5], 1u << (k3 & 31));
  }
  for (; i < deg; i += kWave) {
    const uint32_t k = uint32_t(a.key_of(a.adj[beg + i]));
    atomicOr(&bits[k >> 5], 1u << (k & 31));
  }
  __builtin_amdgcn_wave_barrier();
  uint32_t* out = w.bm + size_t(slot) * nw;
  KeyT* uk = a.ukey + beg;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nw; base += kWave) {
    const uint32_t j = base + lane;
    uint32_t v = j < nw ? bits[j] : 0u;
    if (j < nw) out[j] = v;
    const uint32_t pc = uint32_t(__popc(v));
    const uint32_t incl = wave_inclusive_scan(pc);
    uint32_t r = carry + incl - pc;
    while (v) {
      uk[r++] = KeyT(j * 32u + uint32_t(__ffs(v) - 1));
      v &= v - 1;
    }
    carry += __shfl(incl, kWave - 1, kWave);
  }
  if (lane == 0) {
    a.ucnt[n] = carry;
    a.head[n] = head_of_bits(a, bits, nw);
    w.bmslot[n] = slot;
  }
}

// Lists the set bits of a bitmap in LDS in ascending order as the node's
// unique keys (a block scan of the word popcounts gives each word's first
// output slot) and writes its count and head word.
template <typename AdjT, typename KeyT>
__device__ __forceinline__ void list_bits(const SigArgs<AdjT, KeyT>& a, uint32_t n, const uint32_t* bits,
                                          uint32_t nw, uint32_t* shs) {
  KeyT* uk = a.ukey + a.rowptr[n];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nw; base += kSigNT) {
    const uint32_t j = base + threadIdx.x;
    uint32_t v = j < nw ? bits[j] : 0u;
    uint32_t tot;
    uint32_t r = carry + block_exclusive_scan<kSigNT>(uint32_t(__popc(v)), shs, &tot);
    while (v) {
      uk[r++] = KeyT(j * 32u + uint32_t(__ffs(v) - 1));
      v &= v - 1;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    a.ucnt[n] = carry;
    a.head[n] = head_of_bits(a, bits, nw);
  }
}

// Workgroup bitmap node. Hubs in bitmap rounds are split into `units` chunks
// of hub_chunk edges, one workgroup each, which OR their LDS bitmaps into the
// hub's bitmap in global memory (zeroed before the launch); sig_hub_list_k
// lists the keys after the launch. With one unit the workgroup lists them.
template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_bitmap_node(const SigArgs<AdjT, KeyT>& a, uint32_t n, const SigWork& w,
                                                uint32_t slot, uint32_t unit, uint32_t units, uint32_t* bits,
                                                uint32_t* shs) {
  const uint32_t nw = w.words;
  for (uint32_t i = threadIdx.x; i < nw; i += kSigNT) bits[i] = 0;
  __syncthreads();
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  const uint32_t lo = units == 1 ? 0u : min(deg, unit * w.hub_chunk);
  const uint32_t hi = units == 1 ? deg : min(deg, lo + w.hub_chunk);
  if (lo >= hi) return;  // nothing of this hub in this unit (uniform over the workgroup)
  // four edges in flight per thread
  uint32_t i = lo + threadIdx.x;
  for (; i + 3 * kSigNT < hi; i += 4 * kSigNT) {
    const AdjT e0 = a.adj[beg + i], e1 = a.adj[beg + i + kSigNT];
    const AdjT e2 = a.adj[beg + i + 2 * kSigNT], e3 = a.adj[beg + i + 3 * kSigNT];
    const uint32_t k0 = uint32_t(a.key_of(e0)), k1 = uint32_t(a.key_of(e1));
    const uint32_t k2 = uint32_t(a.key_of(e2)), k3 = uint32_t(a.key_of(e3));
    atomicOr(&bits[k0 >> 5], 1u << (k0 & 31));
    atomicOr(&bits[k1 >> 5], 1u << (k1 & 31));
    atomicOr(&bits[k2 >> 5], 1u << (k2 & 31));
    atomicOr(&bits[k3 >> 5], 1u << (k3 & 31));
  }
  for (; i < hi; i += kSigNT) {
    const uint32_t k = uint32_t(a.key_of(a.adj[beg + i]));
    atomicOr(&bits[k >> 5], 1u << (k & 31));
  }
  __syncthreads();
  uint32_t* out = w.bm + size_t(slot) * nw;
  if (units > 1) {
    for (uint32_t j = threadIdx.x; j < nw; j += kSigNT)
      if (bits[j]) atomicOr(&out[j], bits[j]);
    return;
  }
  for (uint32_t j = threadIdx.x; j < nw; j += kSigNT) out[j] = bits[j];
  list_bits(a, n, bits, nw, shs);
  if (threadIdx.x == 0) w.bmslot[n] = slot;
}

// After a launch with chunked hubs: one workgroup per hub lists the keys of
// its merged bitmap.
template <typename AdjT, typename KeyT>
__global__ __launch_bounds__(kSigNT) void sig_hub_list_k(SigArgs<AdjT, KeyT> a, SigWork w) {
  __shared__ uint32_t bits[kBmMaxWords];
  __shared__ uint32_t shs[kSigNT / kWave];
  const uint32_t h = blockIdx.x;
  const uint32_t n = w.hl[h];
  const uint32_t slot = w.hub_slot0() + h;
  const uint32_t* src = w.bm + size_t(slot) * w.words;
  for (uint32_t j = threadIdx.x; j < w.words; j += kSigNT) bits[j] = src[j];
  __syncthreads();
  list_bits(a, n, bits, w.words, shs);
  if (threadIdx.x == 0) w.bmslot[n] = slot;
}

// ---- hubs, out-degree > 4096 -------------------------------------------------------
// One workgroup sorts the node's keys with an LSD radix sort (8-bit digits)
// that ping-pongs between ukey[beg..] and tmp[0..deg), then writes the unique
// keys to ukey[beg..].
struct HubLds {
  uint32_t cnt[256];
  uint32_t base_d[256];
  uint32_t wcnt[kSigNT / kWave][256];
  uint32_t shs[kSigNT / kWave];
};

template <typename AdjT, typename KeyT>
__device__ __forceinline__ void sig_hub_node(const SigArgs<AdjT, KeyT>& a, uint32_t n, KeyT* tmp, int key_bits,
                                             HubLds& L) {
  constexpr int NW = kSigNT / kWave;
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  KeyT* A = a.ukey + beg;
  KeyT* B = tmp;
  for (uint32_t i = threadIdx.x; i < deg; i += kSigNT) A[i] = a.key_of(a.adj[beg + i]);
  __syncthreads();
  const int w = threadIdx.x / kWave;
  KeyT* src = A;
  KeyT* dst = B;
  for (int shift = 0; shift < key_bits; shift += 8) {
    for (int d = threadIdx.x; d < 256; d += kSigNT) L.cnt[d] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < deg; i += kSigNT) atomicAdd(&L.cnt[uint32_t(src[i] >> shift) & 255u], 1u);
    __syncthreads();
    {
      uint32_t tot;
      const uint32_t v = threadIdx.x < 256 ? L.cnt[threadIdx.x] : 0u;
      const uint32_t ex = block_exclusive_scan<kSigNT>(v, L.shs, &tot);
      if (threadIdx.x < 256) L.base_d[threadIdx.x] = ex;
    }
    __syncthreads();
    for (uint32_t row = 0; row < deg; row += kSigNT) {
      for (int j = threadIdx.x; j < NW * 256; j += kSigNT) (&L.wcnt[0][0])[j] = 0;
      __syncthreads();
      const uint32_t i = row + threadIdx.x;
      const bool valid = i < deg;
      const KeyT key = valid ? src[i] : KeyT(0);
      const uint32_t d = valid ? (uint32_t(key >> shift) & 255u) : 0u;
      const uint64_t m = match_digit8(d, __ballot(valid));
      const uint32_t rank = __popcll(m & lanemask_lt());
      if (valid && rank == 0) L.wcnt[w][d] = __popcll(m);
      __syncthreads();
      if (valid) {
        uint32_t off = L.base_d[d] + rank;
        for (int q = 0; q < w; ++q) off += L.wcnt[q][d];
        dst[off] = key;
      }
      __syncthreads();
      for (int dd = threadIdx.x; dd < 256; dd += kSigNT) {
        uint32_t s2 = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) s2 += L.wcnt[q][dd];
        L.base_d[dd] += s2;
      }
      __syncthreads();
    }
    KeyT* t = src;
    src = dst;
    dst = t;
  }
  // unique pass: read src (sorted), write A; in place when src == A, so each
  // chunk is read completely before any of it is written.
  uint32_t carry = 0;
  for (uint32_t base = 0; base < deg; base += kSigNT) {
    const uint32_t i = base + threadIdx.x;
    KeyT cur = 0;
    bool f = false;
    if (i < deg) {
      cur = src[i];
      f = (i == 0) || cur != src[i - 1];
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kSigNT>(uint32_t(f), L.shs, &tot);  // has barriers
    if (f) A[carry + ex] = cur;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.ucnt[n] = carry;
    a.head[n] = a.head_of(A, carry);
  }
}

// ---- the launch ----------------------------------------------------------------------
template <typename KeyT>
union SigLds {
  KeyT block[kBlockMaxDeg];
  ThreadLds<KeyT> th;
  HubLds hub;
  struct {
    uint32_t bits[kSigNT / kWave][kBmMaxWords];  // one per wave (the workgroup path uses the first)
    uint32_t shs[kSigNT / kWave];
  } bm;
};

template <typename AdjT, typename KeyT>
__global__ __launch_bounds__(kSigNT) void signature_k(SigArgs<AdjT, KeyT> a, SigWork w) {
  __shared__ SigLds<KeyT> lds;
  __shared__ uint32_t shc[kSigNT / kWave];
  uint32_t b = blockIdx.x;
  if (b < w.nh * w.hub_units) {
    const uint32_t h = b / w.hub_units;
    const uint32_t n = w.hl[h];
    if (!w.in(n)) return;
    if (w.bm)
      sig_bitmap_node(a, n, w, w.hub_slot0() + h, b % w.hub_units, w.hub_units, lds.bm.bits[0], lds.bm.shs);
    else
      sig_hub_node(a, n, static_cast<KeyT*>(w.hub_tmp) + w.hub_toff[n], w.key_bits, lds.hub);
    return;
  }
  b -= w.nh * w.hub_units;
  if (b < w.block_units()) {
    if (w.bm) {
      const uint32_t bi = b * (kSigNT / kWave) + threadIdx.x / kWave;
      if (bi < w.nm + w.nb) {
        const uint32_t n = bi < w.nm ? w.ml[bi] : w.bl[bi - w.nm];
        if (w.in(n)) sig_bitmap_wave_node(a, n, w, bi, lds.bm.bits[threadIdx.x / kWave]);
      }
    } else if (w.in(w.bl[b])) {
      sig_block_node(a, w.bl[b], lds.block, shc);
    }
    return;
  }
  b -= w.block_units();
  if (b < w.mid_units()) {
    const uint32_t mi = b * (kSigNT / kWave) + threadIdx.x / kWave;
    if (mi < w.nm && w.in(w.ml[mi])) sig_mid_node(a, w.ml[mi]);
    return;
  }
  b -= w.mid_units();
  if (b < w.wave_units()) {
    const uint32_t wi = 2 * (b * (kSigNT / kWave) + threadIdx.x / kWave);
    if (wi < w.nw) {
      uint32_t n0 = w.wl[wi], n1 = wi + 1 < w.nw ? w.wl[wi + 1] : kNone;
      if (n1 != kNone && !w.in(n1)) n1 = kNone;
      if (!w.in(n0)) {
        n0 = n1;
        n1 = kNone;
      }
      if (n0 != kNone) sig_wave_pair(a, n0, n1);
    }
    return;
  }
  b -= w.wave_units();
  const uint32_t j = b * kSigNT + threadIdx.x;
  uint32_t n = kNone;
  if (w.dense) {
    if (j < w.n_nodes && w.in(j) && w.actr[j] == w.tag) n = j;
  } else if (j < w.nact) {
    n = w.anode[j];
    if (!w.in(n)) n = kNone;
  }
  sig_thread_wave(a, n, lds.th);
}

// ---- hubs in rounds with wide keys: one device-wide sort ----------------------
// A hub sorted by one workgroup gathers its keys one workgroup's worth at a
// time, which for hubs of 10^5 edges and more takes milliseconds. Instead the
// edges of all hubs of the round are sorted together by (hub, key) with the
// device-wide radix sort: hub h of the hub list owns items [hoff[h],
// hoff[h+1]) (exclusive scan of the hub out-degrees).

// comp[i] = (h << key_bits) | key of item i. One tile of kHubKeyTile items
// per workgroup: the hubs of its first and last items are found once.
constexpr uint32_t kHubKeyTile = 2048;
__device__ __forceinline__ uint32_t hub_of(const uint32_t* hoff, uint32_t lo, uint32_t hi, uint32_t i) {
  while (hi - lo > 1) {  // last h in [lo, hi) with hoff[h] <= i
    const uint32_t mid = (lo + hi) >> 1;
    if (hoff[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}
template <typename AdjT, typename KeyT, typename CompT>
__global__ __launch_bounds__(256) void hub_keys_k(SigArgs<AdjT, KeyT> a, const uint32_t* __restrict__ hl,
                                                  const uint32_t* __restrict__ hoff, uint32_t nh, uint32_t n_items,
                                                  int key_bits, CompT* __restrict__ comp) {
  __shared__ uint32_t range[2];
  const uint32_t t0 = blockIdx.x * kHubKeyTile;
  const uint32_t t1 = t0 + kHubKeyTile < n_items ? t0 + kHubKeyTile : n_items;
  if (threadIdx.x == 0) {
    range[0] = hub_of(hoff, 0, nh, t0);
    range[1] = hub_of(hoff, 0, nh, t1 - 1);
  }
  __syncthreads();
  const uint32_t lo = range[0], hi = range[1];
  for (uint32_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
    const uint32_t h = lo == hi ? lo : hub_of(hoff, lo, hi + 1, i);
    const uint32_t e = a.rowptr[hl[h]] + (i - hoff[h]);
    comp[i] = (CompT(h) << key_bits) | CompT(a.key_of(a.adj[e]));
  }
}

// fl[i] = 1 where a run of equal (hub, key) starts; fl[n] = 0.
template <typename CompT>
__global__ void hub_flags_k(const CompT* __restrict__ comp, uint32_t n, uint32_t* __restrict__ fl) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) fl[i] = (i == 0 || comp[i] != comp[i - 1]) ? 1u : 0u;
  if (i == n) fl[n] = 0u;
}

// rank = exclusive scan of the run flags: the unique key starting a run at
// item i is key number rank[i] - rank[hoff[h]] of hub h.
template <typename AdjT, typename KeyT, typename CompT>
__global__ void hub_write_k(SigArgs<AdjT, KeyT> a, const uint32_t* __restrict__ hl, const uint32_t* __restrict__ hoff,
                            const CompT* __restrict__ comp, const uint32_t* __restrict__ rank, uint32_t n,
                            int key_bits) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CompT c = comp[i];
  if (i > 0 && comp[i - 1] == c) return;
  const uint32_t h = uint32_t(c >> key_bits);
  a.ukey[a.rowptr[hl[h]] + (rank[i] - rank[hoff[h]])] = KeyT(c & ((CompT(1) << key_bits) - 1));
}

// Per hub: number of unique keys and the head word.
template <typename AdjT, typename KeyT>
__global__ void hub_finish_k(SigArgs<AdjT, KeyT> a, const uint32_t* __restrict__ hl,
                             const uint32_t* __restrict__ hoff, const uint32_t* __restrict__ rank, uint32_t nh) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  const uint32_t n = hl[h];
  const uint32_t c = rank[hoff[h + 1]] - rank[hoff[h]];
  a.ucnt[n] = c;
  a.head[n] = a.head_of(a.ukey + a.rowptr[n], c);
}

// Profiling reductions over the active list: grid-stride over at most
// kProfGrid workgroups, one global atomic per workgroup and counter (one per
// wave serialises on the counters: milliseconds at 10^7 nodes).
constexpr uint32_t kProfGrid = 512;

// Largest number of unique keys among the active nodes.
__global__ __launch_bounds__(kSigNT) void max_ucnt_k(const uint32_t* __restrict__ anode,
                                                    const uint32_t* __restrict__ ucnt, uint32_t m,
                                                    unsigned long long* __restrict__ mx) {
  __shared__ uint32_t sh[kSigNT / kWave];
  uint32_t c = 0;
  for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < m; j += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t u = ucnt[anode[j]];
    c = u > c ? u : c;
  }
  c = wave_max(c);
  if (__lane_id() == 0) sh[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kSigNT / kWave; ++q) c = sh[q] > c ? sh[q] : c;
    if (c > 0) atomicMax(mx, (unsigned long long)c);
  }
}

// Work of the signature launch: per bucket (thread, wave, block, hub) the
// active nodes and their edges.
__global__ __launch_bounds__(kSigNT) void work_count_k(const uint32_t* __restrict__ anode,
                                                      const uint32_t* __restrict__ rowptr, uint32_t m,
                                                      unsigned long long* __restrict__ acc) {
  __shared__ unsigned long long red[8];
  if (threadIdx.x < 8) red[threadIdx.x] = 0;
  __syncthreads();
  uint64_t ne[4] = {0, 0, 0, 0};
  uint64_t nn[4] = {0, 0, 0, 0};
  for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < m; j += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t n = anode[j];
    const uint32_t d = rowptr[n + 1] - rowptr[n];
    const int c = d <= kThreadMaxDeg ? 0 : d <= kWaveMaxDeg ? 1 : d <= kBlockMaxDeg ? 2 : 3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      nn[q] += q == c ? 1u : 0u;
      ne[q] += q == c ? d : 0u;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint64_t sn = wave_sum(nn[c]), se = wave_sum(ne[c]);
    if (__lane_id() == 0 && (sn || se)) {
      atomicAdd(&red[2 * c], (unsigned long long)sn);
      atomicAdd(&red[2 * c + 1], (unsigned long long)se);
    }
  }
  __syncthreads();
  if (threadIdx.x < 8 && red[threadIdx.x]) atomicAdd(&acc[threadIdx.x], red[threadIdx.x]);
}

}  // namespace kb
