// Signature construction for one refinement round (Definition 3; Algorithm 1,
// the join that fills pId_old(tId), the projection/sort/de-duplication that
// builds F, and the per-node signature string).
//
// For every node u whose current block has at least two members, the kernels
// gather key(e) = (edge label rank << pid_bits) | pid_prev[dst(e)] over u's
// out-edges, sort the keys of u ascending, drop duplicates and write the
// unique keys to ukey[rowptr[u] ...] and their number to ucnt[u]. The key
// order equals the order of the pairs (label, pid) because the label occupies
// the high bits.
//
// Nodes alone in their block are skipped: a refinement never merges blocks
// (Proposition 1), so such a node stays alone and its signature cannot
// change its rank inside the block.
//
// Work is bucketed by out-degree: one thread (<= 16 keys, register sorting
// network), one wave (<= 64 keys, shuffle bitonic), one workgroup (<= 4096
// keys, LDS bitonic) or one workgroup with a global-memory radix sort (hubs).
#pragma once

#include "common.h"
#include "scan_radix.h"

namespace kb {

constexpr uint32_t kThreadMaxDeg = 16;
constexpr uint32_t kWaveMaxDeg = 64;
constexpr uint32_t kBlockMaxDeg = 4096;
constexpr int kSigBlockNT = 256;
constexpr int kHubNT = 256;

template <typename AdjT, typename KeyT>
struct SigArgs {
  const uint32_t* rowptr;  // [N+1]
  const AdjT* adj;         // [E] (label rank << dst_bits) | dst, CSR order
  const int32_t* pid;      // [N] previous-round ids
  const uint32_t* bstart;  // [B+1] block start positions (block sizes)
  KeyT* ukey;              // [E] unique keys per node at rowptr offsets
  uint32_t* ucnt;          // [N]
  uint64_t* head;          // [N] first hw digits (key + 1, 0 past the end), most significant first
  int dst_bits;
  int pid_bits;
  int hdbits;              // bits of one digit: key bits + 1
  uint32_t hw;             // digits per head word: 64 / hdbits

  __device__ __forceinline__ uint64_t head_of(const KeyT* k, uint32_t c) const {
    if (hdbits >= 64) return c ? uint64_t(k[0]) + 1ull : 0ull;
    uint64_t v = 0;
    for (uint32_t j = 0; j < hw; ++j) v = (v << hdbits) | (j < c ? uint64_t(k[j]) + 1ull : 0ull);
    return v;
  }

  __device__ __forceinline__ KeyT key_of(AdjT a) const {
    const uint32_t dst = uint32_t(a & ((AdjT(1) << dst_bits) - 1));
    const uint64_t lab = uint64_t(a >> dst_bits);
    return KeyT((lab << pid_bits) | uint64_t(uint32_t(pid[dst])));
  }
  __device__ __forceinline__ bool active(uint32_t n) const {
    const int32_t p = pid[n];
    return bstart[p + 1] - bstart[p] > 1;
  }
};

template <typename KeyT>
__device__ __forceinline__ void cas_up(KeyT& a, KeyT& b, bool up) {
  const KeyT lo = a < b ? a : b;
  const KeyT hi = a < b ? b : a;
  a = up ? lo : hi;
  b = up ? hi : lo;
}

// ---- bucket 1: one thread per node, out-degree <= 16 ------------------------
template <typename AdjT, typename KeyT>
__global__ __launch_bounds__(256) void sig_thread_k(SigArgs<AdjT, KeyT> a, uint32_t n_nodes) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t beg = 0, deg = 0;
  bool act = false;
  if (n < n_nodes) {
    beg = a.rowptr[n];
    deg = a.rowptr[n + 1] - beg;
    act = deg <= kThreadMaxDeg && a.active(n);
  }
  if (act) {
    constexpr int M = kThreadMaxDeg;
    KeyT k[M];
#pragma unroll
    for (int j = 0; j < M; ++j) k[j] = (uint32_t(j) < deg) ? a.key_of(a.adj[beg + j]) : ~KeyT(0);
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
#pragma unroll
    for (int j = 0; j < M; ++j) {
      if (uint32_t(j) < deg && (j == 0 || k[j] != k[j - 1])) {
        a.ukey[beg + c] = k[j];
        ++c;
      }
    }
    a.ucnt[n] = c;
    a.head[n] = a.head_of(a.ukey + beg, c);
  }
}

// ---- bucket 2: one wave per node, 16 < out-degree <= 64 ----------------------
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

template <typename AdjT, typename KeyT>
__global__ __launch_bounds__(256) void sig_wave_k(SigArgs<AdjT, KeyT> a, const uint32_t* __restrict__ list,
                                                  uint32_t count) {
  const uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (w >= count) return;
  const uint32_t n = list[w];
  if (!a.active(n)) return;
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

// ---- bucket 3: one workgroup per node, 64 < out-degree <= 4096 --------------
template <typename KeyT>
__device__ __forceinline__ void block_bitonic(KeyT* s, uint32_t P) {
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < P / 2; i += blockDim.x) {
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

// Writes the unique keys of the sorted array s[0..deg) to out[0..) and
// returns their number to every thread.
template <int NT, typename KeyT>
__device__ __forceinline__ uint32_t block_unique_write(const KeyT* s, uint32_t deg, KeyT* out) {
  __shared__ uint32_t shc[NT / kWave];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < deg; base += NT) {
    const uint32_t i = base + threadIdx.x;
    const bool f = i < deg && (i == 0 || s[i] != s[i - 1]);
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<NT>(uint32_t(f), shc, &tot);
    if (f) out[carry + ex] = s[i];
    carry += tot;
  }
  return carry;
}

template <typename AdjT, typename KeyT>
__global__ __launch_bounds__(kSigBlockNT) void sig_block_k(SigArgs<AdjT, KeyT> a,
                                                           const uint32_t* __restrict__ list,
                                                           uint32_t count) {
  __shared__ KeyT s[kBlockMaxDeg];
  const uint32_t n = list[blockIdx.x];
  if (!a.active(n)) return;
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  uint32_t P = 128;
  while (P < deg) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += kSigBlockNT)
    s[i] = i < deg ? a.key_of(a.adj[beg + i]) : ~KeyT(0);
  __syncthreads();
  block_bitonic(s, P);
  const uint32_t c = block_unique_write<kSigBlockNT>(s, deg, a.ukey + beg);
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ucnt[n] = c;
    a.head[n] = a.head_of(a.ukey + beg, c);
  }
}

// ---- bucket 4: hubs, out-degree > 4096 -----------------------------------------
// One workgroup sorts the node's keys with an LSD radix sort (8-bit digits)
// that ping-pongs between ukey[beg..] and tmp[hoff..], then writes the
// unique keys to ukey[beg..].
template <typename AdjT, typename KeyT>
__global__ __launch_bounds__(kHubNT) void sig_hub_k(SigArgs<AdjT, KeyT> a, const uint32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ hub_off, KeyT* __restrict__ tmp,
                                                    int key_bits) {
  constexpr int NW = kHubNT / kWave;
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t base_d[256];
  __shared__ uint32_t wcnt[NW][256];
  __shared__ uint32_t shs[NW];
  const uint32_t n = list[blockIdx.x];
  if (!a.active(n)) return;
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  KeyT* A = a.ukey + beg;
  KeyT* B = tmp + hub_off[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < deg; i += kHubNT) A[i] = a.key_of(a.adj[beg + i]);
  __syncthreads();
  const int w = threadIdx.x / kWave;
  KeyT* src = A;
  KeyT* dst = B;
  for (int shift = 0; shift < key_bits; shift += 8) {
    for (int d = threadIdx.x; d < 256; d += kHubNT) cnt[d] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < deg; i += kHubNT)
      atomicAdd(&cnt[uint32_t(src[i] >> shift) & 255u], 1u);
    __syncthreads();
    {
      uint32_t tot;
      const uint32_t v = threadIdx.x < 256 ? cnt[threadIdx.x] : 0u;
      const uint32_t ex = block_exclusive_scan<kHubNT>(v, shs, &tot);
      if (threadIdx.x < 256) base_d[threadIdx.x] = ex;
    }
    __syncthreads();
    for (uint32_t row = 0; row < deg; row += kHubNT) {
      for (int j = threadIdx.x; j < NW * 256; j += kHubNT) (&wcnt[0][0])[j] = 0;
      __syncthreads();
      const uint32_t i = row + threadIdx.x;
      const bool valid = i < deg;
      const KeyT key = valid ? src[i] : KeyT(0);
      const uint32_t d = valid ? (uint32_t(key >> shift) & 255u) : 0u;
      const uint64_t m = match_digit8(d, __ballot(valid));
      const uint32_t rank = __popcll(m & lanemask_lt());
      if (valid && rank == 0) wcnt[w][d] = __popcll(m);
      __syncthreads();
      if (valid) {
        uint32_t off = base_d[d] + rank;
        for (int q = 0; q < w; ++q) off += wcnt[q][d];
        dst[off] = key;
      }
      __syncthreads();
      for (int dd = threadIdx.x; dd < 256; dd += kHubNT) {
        uint32_t s2 = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) s2 += wcnt[q][dd];
        base_d[dd] += s2;
      }
      __syncthreads();
    }
    KeyT* t = src;
    src = dst;
    dst = t;
  }
  // unique pass: read src (sorted), write A; in place when src == A, so each
  // chunk is read completely before any of it is written.
  __shared__ uint32_t shc[NW];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < deg; base += kHubNT) {
    const uint32_t i = base + threadIdx.x;
    KeyT cur = 0;
    bool f = false;
    if (i < deg) {
      cur = src[i];
      f = (i == 0) || cur != src[i - 1];
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kHubNT>(uint32_t(f), shc, &tot);  // has barriers
    if (f) A[carry + ex] = cur;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.ucnt[n] = carry;
    a.head[n] = a.head_of(A, carry);
  }
}

// ---- small key universes: bitmap de-duplication -----------------------------
// When every key is below 2^kBmKeyBits, a node's unique keys are the set bits
// of a bitmap of `words` 32-bit words: the workgroup ORs the node's keys into
// LDS, then lists the set bits in ascending order (a block scan of the word
// popcounts gives each word's first output slot). The bitmap itself is kept
// in bm[slot * words ...] for later first-difference searches, and
// bmslot[n] = slot. Used for nodes with more than kWaveMaxDeg edges: list
// entry i gets slot slot0 + i.
constexpr int kBmKeyBits = 12;
constexpr uint32_t kBmMaxWords = (1u << kBmKeyBits) / 32;

struct BmOut {
  uint32_t* bm;      // [slots * words]
  uint32_t* bmslot;  // [N]
  uint32_t words;    // 32-bit words per bitmap (>= 2)
  uint32_t slot0;
};

template <typename AdjT, typename KeyT, int NT>
__global__ __launch_bounds__(NT) void sig_bitmap_k(SigArgs<AdjT, KeyT> a, const uint32_t* __restrict__ list,
                                                   BmOut o) {
  __shared__ uint32_t w[kBmMaxWords];
  __shared__ uint32_t shs[NT / kWave];
  const uint32_t n = list[blockIdx.x];
  if (!a.active(n)) return;
  const uint32_t nw = o.words;
  for (uint32_t i = threadIdx.x; i < nw; i += NT) w[i] = 0;
  __syncthreads();
  const uint32_t beg = a.rowptr[n];
  const uint32_t deg = a.rowptr[n + 1] - beg;
  // four edges in flight per thread
  uint32_t i = threadIdx.x;
  for (; i + 3 * NT < deg; i += 4 * NT) {
    const AdjT e0 = a.adj[beg + i], e1 = a.adj[beg + i + NT];
    const AdjT e2 = a.adj[beg + i + 2 * NT], e3 = a.adj[beg + i + 3 * NT];
    const uint32_t k0 = uint32_t(a.key_of(e0)), k1 = uint32_t(a.key_of(e1));
    const uint32_t k2 = uint32_t(a.key_of(e2)), k3 = uint32_t(a.key_of(e3));
    atomicOr(&w[k0 >> 5], 1u << (k0 & 31));
    atomicOr(&w[k1 >> 5], 1u << (k1 & 31));
    atomicOr(&w[k2 >> 5], 1u << (k2 & 31));
    atomicOr(&w[k3 >> 5], 1u << (k3 & 31));
  }
  for (; i < deg; i += NT) {
    const uint32_t k = uint32_t(a.key_of(a.adj[beg + i]));
    atomicOr(&w[k >> 5], 1u << (k & 31));
  }
  __syncthreads();
  const uint32_t slot = o.slot0 + blockIdx.x;
  uint32_t* out = o.bm + size_t(slot) * nw;
  KeyT* uk = a.ukey + beg;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nw; base += NT) {
    const uint32_t j = base + threadIdx.x;
    uint32_t v = j < nw ? w[j] : 0u;
    if (j < nw) out[j] = v;
    uint32_t tot;
    uint32_t r = carry + block_exclusive_scan<NT>(uint32_t(__popc(v)), shs, &tot);
    while (v) {
      const uint32_t b = uint32_t(__ffs(v) - 1);
      uk[r++] = KeyT(j * 32u + b);
      v &= v - 1;
    }
    carry += tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ucnt[n] = carry;
    a.head[n] = a.head_of(uk, carry);
    o.bmslot[n] = slot;
  }
}

// Work of the signature kernels (profiling only, launched separately so the
// timed kernels carry no counters): per bucket, active nodes and their edges.
__global__ __launch_bounds__(256) void work_count_k(const uint32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ pid,
                                                    const uint32_t* __restrict__ bstart, uint32_t n,
                                                    unsigned long long* __restrict__ work) {
  __shared__ unsigned long long acc[8];
  if (threadIdx.x < 8) acc[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    const int32_t p = pid[v];
    if (bstart[p + 1] - bstart[p] > 1) {
      const uint32_t d = rowptr[v + 1] - rowptr[v];
      const int b = d <= kThreadMaxDeg ? 0 : d <= kWaveMaxDeg ? 1 : d <= kBlockMaxDeg ? 2 : 3;
      atomicAdd(&acc[2 * b], 1ull);
      atomicAdd(&acc[2 * b + 1], (unsigned long long)d);
    }
  }
  __syncthreads();
  if (threadIdx.x < 8 && acc[threadIdx.x]) atomicAdd(&work[threadIdx.x], acc[threadIdx.x]);
}

}  // namespace kb
