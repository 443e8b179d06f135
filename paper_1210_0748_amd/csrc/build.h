// Once-per-graph steps: input validation, the k = 0 partition (Algorithm 1,
// iteration 0: nodes sorted by label, one id per distinct label), dense
// ranks of the edge labels, and the edge table grouped by source node (the
// sort of the edge table that iteration 1 performs, kept as CSR).
#pragma once

#include "common.h"
#include "scan_radix.h"

namespace kb {

// Streaming kernels keep this many elements per thread in flight.
constexpr int kStreamUnroll = 4;

// Presence of the label values below kMaskLabels, as four 64-bit words held
// in registers (never indexed dynamically, so they stay out of scratch).
constexpr uint32_t kMaskLabels = 256;
struct LabelMask {
  uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  __device__ __forceinline__ void add(uint32_t v) {
    const uint64_t bit = 1ull << (v & 63u);
    const uint32_t q = v >> 6;
    w0 |= q == 0 ? bit : 0ull;
    w1 |= q == 1 ? bit : 0ull;
    w2 |= q == 2 ? bit : 0ull;
    w3 |= q == 3 ? bit : 0ull;
  }
};

// Errors, label maximum and label mask of one workgroup (every thread calls
// it), reduced over the workgroup and reported by thread 0 with one atomic
// each at most (skipped when nothing new is to be reported).
template <int NT>
__device__ __forceinline__ void report(uint32_t e_bits, uint32_t mx, const LabelMask& mk, uint32_t* err,
                                       uint32_t* maxv, unsigned long long* lmask) {
  constexpr int NW = NT / kWave;
  __shared__ uint64_t red[NW][6];
  const int w = threadIdx.x / kWave;
  const uint64_t v[6] = {wave_or(uint64_t(e_bits)), wave_max(uint64_t(mx)), wave_or(mk.w0),
                         wave_or(mk.w1),            wave_or(mk.w2),          wave_or(mk.w3)};
  if (__lane_id() == 0)
    for (int q = 0; q < 6; ++q) red[w][q] = v[q];
  __syncthreads();
  if (threadIdx.x != 0) return;
  uint64_t r[6] = {0, 0, 0, 0, 0, 0};
  for (int i = 0; i < NW; ++i) {
    r[0] |= red[i][0];
    r[1] = red[i][1] > r[1] ? red[i][1] : r[1];
    for (int q = 2; q < 6; ++q) r[q] |= red[i][q];
  }
  if (r[0]) atomicOr(err, uint32_t(r[0]));
  if (uint32_t(r[1]) > __hip_atomic_load(maxv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(maxv, uint32_t(r[1]));
  for (int q = 0; q < 4; ++q) {
    const uint64_t cur = __hip_atomic_load(&lmask[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (r[q + 2] & ~cur) atomicOr(&lmask[q], (unsigned long long)r[q + 2]);
  }
}

// One pass over the edge table (src, lab, dst), grid-stride over the radix
// tiles of the edges in input order:
//   err bit 1: src/dst outside [0, N); bit 2: negative edge label;
//   *maxv = largest edge label; lmask = presence of edge labels < 256;
//   hist[d * nb + t] = edges of tile t (kRadixNT * IPT edges) whose source
//   has lowest byte d (the first pass of the sort by source).
template <int IPT = kRadixIPT>
__global__ __launch_bounds__(kRadixNT) void edge_scan_k(const int32_t* __restrict__ src,
                                                        const int32_t* __restrict__ lab,
                                                        const int32_t* __restrict__ dst, uint64_t m, int64_t n,
                                                        uint32_t* __restrict__ err, uint32_t* __restrict__ maxv,
                                                        unsigned long long* __restrict__ lmask,
                                                        uint32_t* __restrict__ hist, uint32_t nb) {
  constexpr int kTile = kRadixNT * IPT;
  __shared__ uint32_t cnt[kRadixNW][256];
  const int w = threadIdx.x / kWave;
  uint32_t e_bits = 0, mx = 0;
  LabelMask mk;
  const bool vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(lab) |
                     reinterpret_cast<uintptr_t>(dst)) & 15u) == 0;
  auto check = [&](int32_t s, int32_t l, int32_t d) {
    if (s < 0 || s >= n || d < 0 || d >= n) e_bits |= 1u;
    if (l < 0) {
      e_bits |= 2u;
    } else {
      mx = uint32_t(l) > mx ? uint32_t(l) : mx;
      if (uint32_t(l) < kMaskLabels) mk.add(uint32_t(l));
    }
    atomicAdd(&cnt[w][uint32_t(s) & 255u], 1u);
  };
  for (uint32_t t = blockIdx.x; t < nb; t += gridDim.x) {
    for (int j = threadIdx.x; j < kRadixNW * 256; j += kRadixNT) (&cnt[0][0])[j] = 0;
    __syncthreads();
    const uint64_t base = uint64_t(t) * kTile;
    if (vec && base + kTile <= m) {
      constexpr int kVecs = IPT / 4;
      const uint4* vs = reinterpret_cast<const uint4*>(src + base);
      const uint4* vl = reinterpret_cast<const uint4*>(lab + base);
      const uint4* vd = reinterpret_cast<const uint4*>(dst + base);
      uint4 rs[kVecs], rl[kVecs], rd[kVecs];
#pragma unroll
      for (int i = 0; i < kVecs; ++i) {
        rs[i] = vs[i * kRadixNT + threadIdx.x];
        rl[i] = vl[i * kRadixNT + threadIdx.x];
        rd[i] = vd[i * kRadixNT + threadIdx.x];
      }
#pragma unroll
      for (int i = 0; i < kVecs; ++i) {
        check(int32_t(rs[i].x), int32_t(rl[i].x), int32_t(rd[i].x));
        check(int32_t(rs[i].y), int32_t(rl[i].y), int32_t(rd[i].y));
        check(int32_t(rs[i].z), int32_t(rl[i].z), int32_t(rd[i].z));
        check(int32_t(rs[i].w), int32_t(rl[i].w), int32_t(rd[i].w));
      }
    } else {
      for (int i = 0; i < IPT; ++i) {
        const uint64_t e = base + uint64_t(i) * kRadixNT + threadIdx.x;
        if (e < m) check(src[e], lab[e], dst[e]);
      }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kRadixNT) {
      uint32_t c = 0;
#pragma unroll
      for (int q = 0; q < kRadixNW; ++q) c += cnt[q][d];
      hist[uint64_t(d) * nb + t] = c;
    }
    __syncthreads();
  }
  report<kRadixNT>(e_bits, mx, mk, err, maxv, lmask);
}

// err bit 4: negative node label; *maxv = largest node label; lmask =
// presence of node labels < 256.
__global__ __launch_bounds__(kRadixNT) void validate_nodes_k(const int32_t* __restrict__ label, uint64_t n,
                                                       uint32_t* __restrict__ err,
                                 uint32_t* __restrict__ maxv, unsigned long long* __restrict__ lmask) {
  uint32_t bad = 0, mx = 0;
  LabelMask mk;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t b = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < n; b += kStreamUnroll * stride) {
    int32_t l[kStreamUnroll];
#pragma unroll
    for (int q = 0; q < kStreamUnroll; ++q) l[q] = b + q * stride < n ? label[b + q * stride] : 0;
#pragma unroll
    for (int q = 0; q < kStreamUnroll; ++q) {
      if (b + q * stride >= n) continue;
      if (l[q] < 0) {
        bad = 4u;
      } else {
        mx = uint32_t(l[q]) > mx ? uint32_t(l[q]) : mx;
        if (uint32_t(l[q]) < kMaskLabels) mk.add(uint32_t(l[q]));
      }
    }
  }
  report<kRadixNT>(bad, mx, mk, err, maxv, lmask);
}

// Rank table of label values below kMaskLabels from their presence mask:
// table[v] = number of present values below v, for v < t (t = max + 2, so
// table[t - 1] is the number of distinct values).
__global__ void mask_ranks_k(const unsigned long long* __restrict__ lmask, uint32_t t, uint32_t* __restrict__ table) {
  for (uint32_t v = threadIdx.x; v < t; v += blockDim.x) {
    uint32_t c = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t lo = q * 64u;
      if (v >= lo + 64u)
        c += uint32_t(__popcll(lmask[q]));
      else if (v > lo)
        c += uint32_t(__popcll(lmask[q] & ((1ull << (v - lo)) - 1ull)));
    }
    table[v] = c;
  }
}

// Grid for the validation kernels: a few workgroups per CU (each wave
// reports once).
inline uint32_t validate_blocks(uint64_t n) {
  return std::max<uint32_t>(1, std::min<uint32_t>(ceil_div(n, 256), 2048));
}

__global__ void to_u32_iota_k(const int32_t* __restrict__ in, uint32_t* __restrict__ key,
                              uint32_t* __restrict__ val, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = uint32_t(in[i]);
  val[i] = i;
}

__global__ void iota_k(uint32_t* __restrict__ out, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = i;
}

// flag[p] = 1 where the sorted key changes (first position of each run).
__global__ void run_start_flags_k(const uint32_t* __restrict__ key, uint32_t n,
                                  uint8_t* __restrict__ flag8, uint32_t* __restrict__ flag32) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint8_t f = (p == 0 || key[p] != key[p - 1]) ? 1 : 0;
  if (flag8) flag8[p] = f;
  if (flag32) flag32[p] = f;
}

// rank[val[p]] = cls[p] - 1 (cls = inclusive scan of the run-start flags).
__global__ void rank_scatter_k(const uint32_t* __restrict__ val, const uint32_t* __restrict__ cls,
                               uint32_t n, uint32_t* __restrict__ rank) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) rank[val[p]] = cls[p] - 1;
}

// hub_deg[v] = out-degree of v when above b_max (a hub), else 0; an
// exclusive scan of it places every hub's radix-sort space.
__global__ void hub_degree_k(const uint32_t* __restrict__ rowptr, uint32_t n, uint32_t b_max,
                             uint32_t* __restrict__ hub_deg) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t d = rowptr[v + 1] - rowptr[v];
  hub_deg[v] = d > b_max ? d : 0u;
}

// *mx = largest out-degree (grid-stride; one atomic per wave at most).
__global__ void max_degree_k(const uint32_t* __restrict__ rowptr, uint32_t n, uint32_t* __restrict__ mx) {
  uint32_t m = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const uint32_t d = rowptr[v + 1] - rowptr[v];
    m = d > m ? d : m;
  }
  m = wave_max(m);
  if (__lane_id() == 0 && m > __hip_atomic_load(mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(mx, m);
}

// Label values below this bound are ranked through a presence table; larger
// values through a sort.
constexpr uint32_t kRankTableMax = 1u << 24;

// present[v] = 1 for every value v in val[0..n). Values below 64 are
// collected in a register mask per thread and stored once per wave; larger
// ones are stored only when not yet marked (few distinct values would
// otherwise take one store per element on the same few addresses).
__global__ void mark_present_k(const int32_t* __restrict__ val, uint64_t n, uint32_t* __restrict__ present) {
  uint64_t low = 0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t b = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < n; b += kStreamUnroll * stride) {
    uint32_t v[kStreamUnroll];
#pragma unroll
    for (int q = 0; q < kStreamUnroll; ++q) v[q] = b + q * stride < n ? uint32_t(val[b + q * stride]) : 0u;
#pragma unroll
    for (int q = 0; q < kStreamUnroll; ++q) {
      if (v[q] < 64) {
        low |= 1ull << v[q];
      } else {
        uint32_t* p = &present[v[q]];
        if (*p == 0u) *p = 1u;  // a stale 0 only costs a repeated store
      }
    }
  }
  low = wave_or(low);
  if (__lane_id() == 0) {
    while (low) {
      const uint32_t b = uint32_t(__ffsll((unsigned long long)low) - 1);
      if (present[b] == 0u) present[b] = 1u;
      low &= low - 1;
    }
  }
}

// Label rank of every node: the sort input (key = rank, value = node) and
// the rank itself in the narrow id type.
template <typename T>
__global__ void lookup_rank_k(const int32_t* __restrict__ val, const uint32_t* __restrict__ rank, uint32_t n,
                              uint32_t* __restrict__ out_key, uint32_t* __restrict__ out_idx, T* __restrict__ narrow) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t r = rank[uint32_t(val[i])];
  out_key[i] = r;
  out_idx[i] = i;
  narrow[i] = T(r);
}

// Items of the first pass of the sort by source, read from the edge table
// itself: key = source node, value = packed (label rank << dst_bits) | dst.
// `erank` (per edge) or `rank_table` (per label value) gives the label rank.
template <typename AdjT>
struct EdgePackLoad {
  const int32_t* __restrict__ src;
  const int32_t* __restrict__ lab;
  const int32_t* __restrict__ dst;
  const uint32_t* __restrict__ erank;
  const uint32_t* __restrict__ rank_table;
  int dst_bits;
  __device__ __forceinline__ void operator()(uint64_t e, uint32_t& key, AdjT& val) const {
    const uint32_t r = erank ? erank[e] : rank_table[uint32_t(lab[e])];
    key = uint32_t(src[e]);
    val = (AdjT(r) << dst_bits) | AdjT(uint32_t(dst[e]));
  }
};

// First pass of the sort by source straight from the edge table (the
// per-tile counts come from edge_scan_k).
template <typename AdjT, bool kFused, int IPT = kRadixIPT>
__global__ __launch_bounds__(kRadixNT) void pack_scatter_k(EdgePackLoad<AdjT> load, uint32_t* __restrict__ kout,
                                                           AdjT* __restrict__ vout, uint64_t m,
                                                           const uint32_t* __restrict__ hist, uint32_t nb) {
  radix_scatter_tile<uint32_t, AdjT, true, kFused, EdgePackLoad<AdjT>, IPT>(load, kout, vout, m, 0, hist, nb);
}

// Row offsets of the CSR from the edges sorted by source: rowptr[v] = first
// position whose source is >= v (v <= n). The thread at a position where the
// source changes from u to v writes rowptr[u+1 .. v] (nodes without edges in
// between share the offset); position 0 and the end cover the two borders,
// so every entry is written exactly once. Ranges longer than kRowGap are
// queued for csr_rowptr_gaps_k instead (gaps[3i..3i+2] = first, last, value).
constexpr uint32_t kRowGap = 64;
__global__ void csr_rowptr_k(const uint32_t* __restrict__ skey, uint64_t m, uint32_t n,
                             uint32_t* __restrict__ rowptr, uint32_t* __restrict__ gaps,
                             uint32_t* __restrict__ ngaps) {
  // four consecutive positions per thread (one 16-byte load where they are
  // all inside the array) plus the one before them
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x * 4;
  for (uint64_t b = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4; b <= m; b += stride) {
    uint32_t cur[4];
    if (b + 4 <= m) {
      const uint4 v = *reinterpret_cast<const uint4*>(skey + b);
      cur[0] = v.x;
      cur[1] = v.y;
      cur[2] = v.z;
      cur[3] = v.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) cur[q] = b + q < m ? skey[b + q] : n;  // past the end: source n
    }
    uint32_t prev = b > 0 ? skey[b - 1] : 0u;  // before the start: no source
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t p = b + q;
      const uint32_t c = cur[q], pr = prev;
      prev = c;
      if (p > m || (p > 0 && c == pr)) continue;
      const uint32_t from = p == 0 ? 0u : pr + 1, to = c;
      if (to - from < kRowGap) {
        for (uint32_t w = from; w <= to; ++w) rowptr[w] = uint32_t(p);
      } else {
        const uint32_t slot = atomicAdd(ngaps, 1u);
        gaps[3 * slot] = from;
        gaps[3 * slot + 1] = to;
        gaps[3 * slot + 2] = uint32_t(p);
      }
    }
  }
}

// The long ranges: one workgroup per queued range (grid-stride).
__global__ void csr_rowptr_gaps_k(const uint32_t* __restrict__ gaps, const uint32_t* __restrict__ ngaps,
                                  uint32_t* __restrict__ rowptr) {
  const uint32_t ng = *ngaps;
  for (uint32_t i = blockIdx.x; i < ng; i += gridDim.x) {
    const uint32_t from = gaps[3 * i], to = gaps[3 * i + 1], v = gaps[3 * i + 2];
    for (uint32_t w = from + threadIdx.x; w <= to; w += blockDim.x) rowptr[w] = v;
  }
}

}  // namespace kb
