// Batched form: many independent graphs refined together.
//
// The graphs become one disjoint union whose node labels are made
// graph-major: a node's union label orders the pairs (graph, label)
// lexicographically ((graph << b) | label, or their rank when that does not
// fit 31 bits). Every
// signature then starts with an id that orders graphs first, so each round
// of the union keeps the graphs' blocks apart and, inside graph g, orders
// signatures exactly as a run on g alone would (all of g's ids are shifted
// by the same offset, which preserves lexicographic order). Consequently
// the nodes of graph g occupy positions [node_off[g], node_off[g+1]) of the
// sorted order, g's local id of a node is its union id minus the union id at
// position node_off[g], and g's block count is the id range at its ends.
// One launch of every kernel serves all graphs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.h"
#include "build.h"
#include "engine.h"

namespace kb {

__device__ __forceinline__ uint32_t bucket_of(const int64_t* off, uint32_t G, uint64_t i) {
  uint32_t lo = 0, hi = G;  // last g with off[g] <= i
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (uint64_t(off[mid]) <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Items per workgroup of the union kernels: graphs are much larger than a
// tile, so a tile mostly lies inside one graph, found once per tile.
constexpr uint32_t kUnionTile = 4096;

// Graphs owning the first and last items [t0, t1) of a tile, by binary
// search in `off` (thread 0), shared with the workgroup.
__device__ __forceinline__ void tile_graphs(const int64_t* off, uint32_t G, uint64_t t0, uint64_t t1, uint32_t* sh) {
  if (threadIdx.x == 0) {
    sh[0] = bucket_of(off, G, t0);
    sh[1] = bucket_of(off, G, t1 - 1);
  }
  __syncthreads();
}

// Graph of item i of a tile whose items belong to graphs glo..ghi.
__device__ __forceinline__ uint32_t graph_in(const int64_t* off, uint32_t glo, uint32_t ghi, uint64_t i) {
  uint32_t lo = glo, hi = ghi + 1;  // last g in [glo, ghi] with off[g] <= i
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (uint64_t(off[mid]) <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Union edge endpoints: local ids of graph g offset by node_off[g]. One tile
// of kUnionTile edges per workgroup. err bit 1: a local id outside [0, N_g).
__global__ __launch_bounds__(256) void union_edges_k(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                                     uint64_t m, const int64_t* __restrict__ node_off,
                                                     const int64_t* __restrict__ edge_off, uint32_t G,
                                                     int32_t* __restrict__ usrc, int32_t* __restrict__ udst,
                                                     uint32_t* __restrict__ err) {
  __shared__ uint32_t gr[2];
  const uint64_t t0 = uint64_t(blockIdx.x) * kUnionTile;
  const uint64_t t1 = t0 + kUnionTile < m ? t0 + kUnionTile : m;
  tile_graphs(edge_off, G, t0, t1, gr);
  const uint32_t glo = gr[0], ghi = gr[1];
  uint32_t bad = 0;
  for (uint64_t e = t0 + threadIdx.x; e < t1; e += blockDim.x) {
    const uint32_t g = glo == ghi ? glo : graph_in(edge_off, glo, ghi, e);
    const int64_t base = node_off[g], n = node_off[g + 1] - base;
    const int32_t s = src[e], d = dst[e];
    if (s < 0 || s >= n || d < 0 || d >= n) {
      bad = 1u;
      usrc[e] = 0;
      udst[e] = 0;
    } else {
      usrc[e] = int32_t(base + s);
      udst[e] = int32_t(base + d);
    }
  }
  bad = wave_or(bad);
  if (__lane_id() == 0 && bad) atomicOr(err, 1u);
}

// Union label of every node: (graph << lbits) | label (labels already
// validated, below 2^lbits). One tile of kUnionTile nodes per workgroup.
__global__ __launch_bounds__(256) void union_labels_k(const int32_t* __restrict__ label, uint64_t n,
                                                      const int64_t* __restrict__ node_off, uint32_t G, int lbits,
                                                      int32_t* __restrict__ out) {
  __shared__ uint32_t gr[2];
  const uint64_t t0 = uint64_t(blockIdx.x) * kUnionTile;
  const uint64_t t1 = t0 + kUnionTile < n ? t0 + kUnionTile : n;
  tile_graphs(node_off, G, t0, t1, gr);
  const uint32_t glo = gr[0], ghi = gr[1];
  for (uint64_t v = t0 + threadIdx.x; v < t1; v += blockDim.x) {
    const uint32_t g = glo == ghi ? glo : graph_in(node_off, glo, ghi, v);
    out[v] = int32_t((g << lbits) | uint32_t(label[v]));
  }
}

// Sort key (graph, label) of every union node (labels already validated).
__global__ void union_node_keys_k(const int32_t* __restrict__ label, uint64_t n, const int64_t* __restrict__ node_off,
                                  uint32_t G, uint64_t* __restrict__ key, uint32_t* __restrict__ idx) {
  const uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  key[v] = (uint64_t(bucket_of(node_off, G, v)) << 31) | uint64_t(uint32_t(label[v]));
  idx[v] = uint32_t(v);
}

__global__ void u64_run_flags_k(const uint64_t* __restrict__ key, uint32_t n, uint32_t* __restrict__ flag) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) flag[p] = (p == 0 || key[p] != key[p - 1]) ? 1u : 0u;
}

__global__ void scatter_rank_k(const uint32_t* __restrict__ idx, const uint32_t* __restrict__ cls, uint32_t n,
                               int32_t* __restrict__ out) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[idx[p]] = int32_t(cls[p] - 1);
}

// Per graph: dense union id of its first sorted position and its number of
// classes, from the inclusive scan of the class-start flags (graph g holds
// positions [node_off[g], node_off[g+1]), and a graph's first position
// starts a class).
__global__ void graph_id_range_k(const uint32_t* __restrict__ cls, const int64_t* __restrict__ node_off, uint32_t G,
                                 int32_t* __restrict__ base, int32_t* __restrict__ count) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int64_t a = node_off[g], b = node_off[g + 1];
  if (a == b) {
    base[g] = 0;
    count[g] = 0;
    return;
  }
  base[g] = int32_t(cls[a] - 1);
  count[g] = int32_t(cls[b - 1] - cls[a] + 1);
}

// Local ids of the graphs marked in `take`. One tile of kUnionTile nodes per
// workgroup.
__global__ __launch_bounds__(256) void snapshot_k(const int32_t* __restrict__ pid, uint64_t n,
                                                  const int64_t* __restrict__ node_off, uint32_t G,
                                                  const int32_t* __restrict__ base, const uint8_t* __restrict__ take,
                                                  int32_t* __restrict__ out) {
  __shared__ uint32_t gr[2];
  const uint64_t t0 = uint64_t(blockIdx.x) * kUnionTile;
  const uint64_t t1 = t0 + kUnionTile < n ? t0 + kUnionTile : n;
  tile_graphs(node_off, G, t0, t1, gr);
  const uint32_t glo = gr[0], ghi = gr[1];
  for (uint64_t v = t0 + threadIdx.x; v < t1; v += blockDim.x) {
    const uint32_t g = glo == ghi ? glo : graph_in(node_off, glo, ghi, v);
    if (take[g]) out[v] = pid[v] - base[g];
  }
}

class Batch {
 public:
  Batch(int32_t G, const int64_t* node_off, const int64_t* edge_off, const int32_t* label, const int32_t* src,
        const int32_t* lab, const int32_t* dst, bool host_mem, hipStream_t s, const Options& o);
  ~Batch();
  // k_g < 0 is invalid; rounds_done[g] (may be null) receives each graph's rounds.
  void refine(const std::vector<int32_t>& k);
  void result(int32_t* pid_out, bool to_device, int64_t* blocks, int32_t* rounds) const;
  int32_t num_graphs() const { return G_; }
  int64_t total_nodes() const { return ntot_; }
  Engine* engine() { return eng_; }

 private:
  void read_counts(std::vector<int32_t>& cnt);
  void take_snapshot(const std::vector<uint8_t>& take);

  int32_t G_;
  int64_t ntot_, etot_;
  hipStream_t st_;
  Options opt_;
  std::vector<int64_t> node_off_, edge_off_;
  DevBuf d_node_off_, d_edge_off_, out_, base_, cnt_, take_;
  Engine* eng_ = nullptr;
  std::vector<int32_t> k_, rounds_, blocks_, prev_;
  std::vector<uint8_t> done_;
  bool refined_ = false;
};

}  // namespace kb
