// Kernels of the streamed edge table: graphs whose edge table is kept out of
// device memory (the paper's setting, Section 2.2: the graph does not fit in
// the fast memory, so every iteration reads the edge table from the slow one
// in large sequential pieces). The table arrives in host memory, is read in
// chunks to count out-degrees and validate, and is laid out once as CSR edge
// words in pinned host memory, one partition of consecutive source nodes at a
// time; every round then moves the partitions through a device window (or,
// in rounds with few active nodes, reads their rows in place).
#pragma once

#include "build.h"

namespace kb {

// One chunk of the edge table: err bit 1 (endpoint outside [0, n)), bit 2
// (negative label), the largest label and the presence mask of labels below
// kMaskLabels, and out-degree counts deg[src] (valid edges only).
__global__ __launch_bounds__(kRadixNT) void stream_scan_k(const int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ lab,
                                                          const int32_t* __restrict__ dst, uint64_t m, int64_t n,
                                                          uint32_t* __restrict__ err, uint32_t* __restrict__ maxv,
                                                          unsigned long long* __restrict__ lmask,
                                                          uint32_t* __restrict__ deg) {
  uint32_t e_bits = 0, mx = 0;
  LabelMask mk;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += stride) {
    const int32_t s = src[e], l = lab[e], d = dst[e];
    if (s < 0 || s >= n || d < 0 || d >= n) {
      e_bits |= 1u;
    } else {
      atomicAdd(&deg[s], 1u);
    }
    if (l < 0) {
      e_bits |= 2u;
    } else {
      mx = uint32_t(l) > mx ? uint32_t(l) : mx;
      if (uint32_t(l) < kMaskLabels) mk.add(uint32_t(l));
    }
  }
  report<kRadixNT>(e_bits, mx, mk, err, maxv, lmask);
}

// cursor[u - lo] = rowptr[u] - rowptr[lo] for the nodes u of one partition.
__global__ void stream_cursor_k(const uint32_t* __restrict__ rowptr, uint32_t lo, uint32_t hi,
                                uint32_t* __restrict__ cursor) {
  const uint32_t u = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (u < hi) cursor[u - lo] = rowptr[u] - rowptr[lo];
}

// The edges of one chunk whose source lies in [lo, hi), as CSR edge words
// (label rank << dst_bits) | dst, in the partition's window at its rows'
// positions (within a row in arrival order). An edge that no longer passes
// the first read's checks (the table changed since: a row would overflow, a
// label beyond the rank table of `tsize` values, a target outside [0, n))
// sets *err and is not written.
template <typename AdjT>
__global__ void stream_fill_k(const int32_t* __restrict__ src, const int32_t* __restrict__ lab,
                              const int32_t* __restrict__ dst, uint64_t m, uint32_t lo, uint32_t hi, uint32_t n,
                              const uint32_t* __restrict__ rowptr, const uint32_t* __restrict__ rank_table,
                              uint32_t tsize, int dst_bits, uint32_t* __restrict__ cursor, AdjT* __restrict__ win,
                              uint32_t* __restrict__ err) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint32_t base = rowptr[lo];
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += stride) {
    const uint32_t s = uint32_t(src[e]);
    if (s < lo || s >= hi) continue;
    const uint32_t l = uint32_t(lab[e]), d = uint32_t(dst[e]);
    if (l >= tsize || d >= n) {
      atomicOr(err, 1u);
      continue;
    }
    const uint32_t pos = atomicAdd(&cursor[s - lo], 1u);
    if (pos >= rowptr[s + 1] - base) {
      atomicOr(err, 1u);
      continue;
    }
    win[pos] = (AdjT(rank_table[l]) << dst_bits) | AdjT(d);
  }
}

// present[v] = 1 for the label values v < t of one chunk (a value beyond
// the first read's maximum, the table having changed since, sets *err).
__global__ void stream_mark_k(const int32_t* __restrict__ lab, uint64_t m, uint32_t t, uint32_t* __restrict__ present,
                              uint32_t* __restrict__ err) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += stride) {
    const uint32_t v = uint32_t(lab[e]);
    if (v >= t) {
      atomicOr(err, 1u);
      continue;
    }
    uint32_t* p = &present[v];
    if (*p == 0u) *p = 1u;
  }
}

}  // namespace kb
