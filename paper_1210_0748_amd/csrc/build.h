// Once-per-graph steps: input validation, the k = 0 partition (Algorithm 1,
// iteration 0: nodes sorted by label, one id per distinct label), dense
// ranks of the edge labels, and the edge table grouped by source node (the
// sort of the edge table that iteration 1 performs, kept as CSR).
#pragma once

#include "common.h"

namespace kb {

// err bit 1: src/dst outside [0, N); bit 2: negative edge label;
// bit 4: negative node label. maxv[0] = max node label, maxv[1] = max edge label.
__global__ void validate_edges_k(const int32_t* __restrict__ src, const int32_t* __restrict__ lab,
                                 const int32_t* __restrict__ dst, uint64_t m, int64_t n,
                                 uint32_t* __restrict__ err, uint32_t* __restrict__ maxv) {
  uint32_t e_bits = 0, mx = 0;
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += uint64_t(gridDim.x) * blockDim.x) {
    const int32_t s = src[e], d = dst[e], l = lab[e];
    if (s < 0 || s >= n || d < 0 || d >= n) e_bits |= 1u;
    if (l < 0)
      e_bits |= 2u;
    else
      mx = uint32_t(l) > mx ? uint32_t(l) : mx;
  }
  // one atomic per wave at most: skipped when nothing new is to be reported
  e_bits = wave_or(e_bits);
  mx = wave_max(mx);
  if (__lane_id() == 0) {
    if (e_bits) atomicOr(err, e_bits);
    if (mx > __hip_atomic_load(&maxv[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&maxv[1], mx);
  }
}

__global__ void validate_nodes_k(const int32_t* __restrict__ label, uint64_t n,
                                 uint32_t* __restrict__ err, uint32_t* __restrict__ maxv) {
  uint32_t bad = 0, mx = 0;
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += uint64_t(gridDim.x) * blockDim.x) {
    const int32_t l = label[v];
    if (l < 0)
      bad = 4u;
    else
      mx = uint32_t(l) > mx ? uint32_t(l) : mx;
  }
  bad = wave_or(bad);
  mx = wave_max(mx);
  if (__lane_id() == 0) {
    if (bad) atomicOr(err, bad);
    if (mx > __hip_atomic_load(&maxv[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&maxv[0], mx);
  }
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

// present[v] = 1 for every value v in val[0..n); a value already marked is
// not stored again (few distinct values would otherwise take one store per
// element on the same few addresses).
__global__ void mark_present_k(const int32_t* __restrict__ val, uint64_t n, uint32_t* __restrict__ present) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * blockDim.x) {
    uint32_t* p = &present[uint32_t(val[i])];
    if (*p == 0u) *p = 1u;  // a stale 0 only costs a repeated store
  }
}

__global__ void lookup_rank_k(const int32_t* __restrict__ val, const uint32_t* __restrict__ rank,
                              uint32_t n, uint32_t* __restrict__ out_key, uint32_t* __restrict__ out_idx) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out_key[i] = rank[uint32_t(val[i])];
  if (out_idx) out_idx[i] = i;
}

// Sort input for the CSR build: key = source node, value = packed
// (label rank << dst_bits) | dst. `erank` (per edge) or `rank_table` (per
// label value) gives the label rank.
template <typename AdjT>
__global__ void pack_edges_k(const int32_t* __restrict__ src, const int32_t* __restrict__ lab,
                             const int32_t* __restrict__ dst, uint64_t m, const uint32_t* __restrict__ erank,
                             const uint32_t* __restrict__ rank_table, int dst_bits, uint32_t* __restrict__ key,
                             AdjT* __restrict__ val) {
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t r = erank ? erank[e] : rank_table[uint32_t(lab[e])];
    key[e] = uint32_t(src[e]);
    val[e] = (AdjT(r) << dst_bits) | AdjT(uint32_t(dst[e]));
  }
}

// Degrees from edges sorted by source: the first and one-past-last position
// of every run of equal sources (end stays 0 for nodes without edges).
__global__ void run_bounds_k(const uint32_t* __restrict__ skey, uint64_t m, uint32_t* __restrict__ run_start,
                             uint32_t* __restrict__ run_end) {
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < m;
       p += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t k = skey[p];
    if (p == 0 || skey[p - 1] != k) run_start[k] = uint32_t(p);
    if (p + 1 == m || skey[p + 1] != k) run_end[k] = uint32_t(p + 1);
  }
}

__global__ void degree_from_runs_k(const uint32_t* __restrict__ run_start, const uint32_t* __restrict__ run_end,
                                   uint32_t n, uint32_t* __restrict__ deg) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) deg[v] = run_end[v] ? run_end[v] - run_start[v] : 0u;
}

}  // namespace kb
