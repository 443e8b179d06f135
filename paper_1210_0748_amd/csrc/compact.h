// Multi-class compaction by tiles, without atomics: every item j < n gets a
// class c in [0, NC) from a functor (or -1: dropped), and the items of class
// c are written, in a fixed order, to the output range starting at
// meta[NC + c] (the lists of all classes are concatenated, class 0 first).
// Three kernels: per-tile class counts, an exclusive scan of those counts per
// class by one workgroup (meta[c] = count of class c, meta[NC + c] = start of
// its list, meta[2 NC] = total), and the scatter, which ranks every item
// inside its tile with a block scan of packed per-class counters.
#pragma once

#include "common.h"

namespace kb {

constexpr int kTileIPT = 8;
constexpr int kTileItems = 256 * kTileIPT;

// Per-thread class counts packed 16 bits per class (a tile has 2048 items):
// classes 0-3 in lo, 4-7 in hi.
struct PackedCounts {
  uint64_t lo = 0, hi = 0;
  __device__ __forceinline__ void add(int c) {
    if (c < 0) return;
    if (c < 4)
      lo += 1ull << (16 * c);
    else
      hi += 1ull << (16 * (c - 4));
  }
  __device__ __forceinline__ uint32_t get(int c) const {
    return uint32_t(((c < 4 ? lo : hi) >> (16 * (c & 3))) & 0xffffu);
  }
};

__device__ __forceinline__ uint32_t item_count(uint32_t n, const uint32_t* n_dev) {
  return n_dev ? min(n, *n_dev) : n;
}

// part[c * gridDim.x + tile] = number of items of class c in the tile.
template <int NC, typename F>
__global__ __launch_bounds__(256) void tile_count_k(F f, uint32_t n, const uint32_t* __restrict__ n_dev,
                                                    uint32_t* __restrict__ part) {
  static_assert(NC >= 1 && NC <= 8, "at most 8 classes");
  __shared__ uint64_t sh[256 / kWave];
  const uint32_t cnt = item_count(n, n_dev);
  const uint32_t base = blockIdx.x * uint32_t(kTileItems);
  PackedCounts pc;
#pragma unroll
  for (int q = 0; q < kTileIPT; ++q) {
    const uint32_t j = base + q * 256u + threadIdx.x;
    if (j < cnt) pc.add(f(j));
  }
  PackedCounts tot;
  block_exclusive_scan<256>(pc.lo, sh, &tot.lo);
  block_exclusive_scan<256>(pc.hi, sh, &tot.hi);
  if (threadIdx.x < NC) part[threadIdx.x * gridDim.x + blockIdx.x] = tot.get(threadIdx.x);
}

// One workgroup: per class, the exclusive scan of the per-tile counts (in
// place) and the class totals. Every thread takes kOffPer consecutive tiles
// of a chunk (all their counts, of every class, loaded at once), so up to
// 1024 * kOffPer tiles cost one round of loads and one pair of barriers.
constexpr int kOffPer = 8;
template <int NC>
__global__ __launch_bounds__(1024) void tile_offsets_k(uint32_t* __restrict__ part, uint32_t ntiles,
                                                       uint32_t* __restrict__ meta) {
  constexpr int NW = 1024 / kWave;
  __shared__ uint32_t sh[NW][NC];
  const int lane = __lane_id();
  const int w = threadIdx.x / kWave;
  uint32_t carry[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) carry[c] = 0;
  for (uint32_t b = 0; b < ntiles; b += 1024u * kOffPer) {
    const uint32_t i0 = b + threadIdx.x * kOffPer;
    uint32_t v[NC][kOffPer], sum[NC], inc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < kOffPer; ++q) v[c][q] = i0 + q < ntiles ? part[size_t(c) * ntiles + i0 + q] : 0u;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      sum[c] = 0;
#pragma unroll
      for (int q = 0; q < kOffPer; ++q) sum[c] += v[c][q];
      inc[c] = wave_inclusive_scan(sum[c]);
      if (lane == kWave - 1) sh[w][c] = inc[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uint32_t before = 0, tot = 0;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        const uint32_t x = sh[q][c];
        before += q < w ? x : 0u;
        tot += x;
      }
      uint32_t run = carry[c] + before + inc[c] - sum[c];
#pragma unroll
      for (int q = 0; q < kOffPer; ++q) {
        if (i0 + q < ntiles) part[size_t(c) * ntiles + i0 + q] = run;
        run += v[c][q];
      }
      carry[c] += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    uint32_t off = 0;
    for (int c = 0; c < NC; ++c) {
      meta[c] = carry[c];
      meta[NC + c] = off;
      off += carry[c];
    }
    meta[2 * NC] = off;
  }
}

// w(j, c, slot) writes item j of class c to output slot `slot`.
template <int NC, typename F, typename W>
__global__ __launch_bounds__(256) void tile_scatter_k(F f, W w, uint32_t n, const uint32_t* __restrict__ n_dev,
                                                      const uint32_t* __restrict__ part,
                                                      const uint32_t* __restrict__ meta) {
  __shared__ uint64_t sh[256 / kWave];
  const uint32_t cnt = item_count(n, n_dev);
  const uint32_t base = blockIdx.x * uint32_t(kTileItems);
  int cls[kTileIPT];
  PackedCounts pc;
#pragma unroll
  for (int q = 0; q < kTileIPT; ++q) {
    const uint32_t j = base + q * 256u + threadIdx.x;
    cls[q] = j < cnt ? f(j) : -1;
    pc.add(cls[q]);
  }
  PackedCounts tot, ex;
  ex.lo = block_exclusive_scan<256>(pc.lo, sh, &tot.lo);
  ex.hi = block_exclusive_scan<256>(pc.hi, sh, &tot.hi);
#pragma unroll
  for (int q = 0; q < kTileIPT; ++q) {
    const int c = cls[q];
    if (c < 0) continue;
    const uint32_t j = base + q * 256u + threadIdx.x;
    w(j, c, meta[NC + c] + part[c * gridDim.x + blockIdx.x] + ex.get(c));
    ex.add(c);
  }
}

// Scratch words for a compaction of up to n items into NC classes.
template <int NC>
inline size_t compact_part_words(uint64_t n) {
  return size_t(NC) * ceil_div(n > 0 ? n : 1, kTileItems);
}

// Enqueues the three kernels; meta needs 2 NC + 1 words.
template <int NC, typename F, typename W>
void compact(F f, W w, uint32_t n, const uint32_t* n_dev, uint32_t* part, uint32_t* meta, hipStream_t s) {
  const uint32_t ntiles = ceil_div(n > 0 ? n : 1, kTileItems);
  tile_count_k<NC><<<ntiles, 256, 0, s>>>(f, n, n_dev, part);
  KB_LAUNCH_CHECK();
  tile_offsets_k<NC><<<1, 1024, 0, s>>>(part, ntiles, meta);
  KB_LAUNCH_CHECK();
  tile_scatter_k<NC><<<ntiles, 256, 0, s>>>(f, w, n, n_dev, part, meta);
  KB_LAUNCH_CHECK();
}

}  // namespace kb
