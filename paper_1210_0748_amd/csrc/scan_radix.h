// Device-wide exclusive/inclusive scan and stable LSD radix sort (8-bit
// digits), hand-written for gfx950. Both are three-kernel designs with no
// inter-block waiting: reduce -> scan of partials -> apply.
#pragma once

#include "common.h"

namespace kb {

constexpr int kScanNT = 256;
constexpr int kScanIPT = 8;
constexpr int kScanTile = kScanNT * kScanIPT;

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanNT) void scan_reduce_k(const Tin* __restrict__ in, uint64_t n,
                                                         Tout* __restrict__ partial) {
  __shared__ Tout sh[kScanNT / kWave];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const uint64_t idx = base + uint64_t(i) * kScanNT + threadIdx.x;
    if (idx < n) s += Tout(in[idx]);
  }
  Tout tot = block_sum<kScanNT>(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of partial[0..nb) in place by one block; partial[nb] = total.
template <typename Tout>
__global__ __launch_bounds__(1024) void scan_partials_k(Tout* __restrict__ partial, uint32_t nb) {
  __shared__ Tout sh[1024 / kWave];
  Tout carry = 0;
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    Tout v = i < nb ? partial[i] : Tout(0);
    Tout tot;
    Tout ex = block_exclusive_scan<1024>(v, sh, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) partial[nb] = carry;
}

template <typename Tin, typename Tout, bool kInclusive>
__global__ __launch_bounds__(kScanNT) void scan_apply_k(const Tin* __restrict__ in,
                                                        Tout* __restrict__ out, uint64_t n,
                                                        const Tout* __restrict__ partial) {
  __shared__ Tout buf[kScanTile];
  __shared__ Tout sh[kScanNT / kWave];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const uint64_t idx = base + uint64_t(i) * kScanNT + threadIdx.x;
    buf[i * kScanNT + threadIdx.x] = idx < n ? Tout(in[idx]) : Tout(0);
  }
  __syncthreads();
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) s += buf[threadIdx.x * kScanIPT + i];
  Tout tot;
  Tout run = block_exclusive_scan<kScanNT>(s, sh, &tot) + partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const Tout v = buf[threadIdx.x * kScanIPT + i];
    buf[threadIdx.x * kScanIPT + i] = kInclusive ? run + v : run;
    run += v;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const uint64_t idx = base + uint64_t(i) * kScanNT + threadIdx.x;
    if (idx < n) out[idx] = buf[i * kScanNT + threadIdx.x];
  }
}

// Scratch words needed by scan(): one partial per tile plus the total.
inline size_t scan_partials_count(uint64_t n) { return size_t(ceil_div(n, kScanTile)) + 1; }

// out[i] = sum(in[0..i)) (or ..i] when inclusive). partial must hold
// scan_partials_count(n) entries; partial[#tiles] receives the total.
// `out` may alias `in`.
template <typename Tin, typename Tout, bool kInclusive = false>
void scan(const Tin* in, Tout* out, uint64_t n, Tout* partial, hipStream_t s) {
  const uint32_t nb = ceil_div(n, kScanTile);
  if (nb > 0) {
    scan_reduce_k<Tin, Tout><<<nb, kScanNT, 0, s>>>(in, n, partial);
    KB_LAUNCH_CHECK();
  }
  scan_partials_k<Tout><<<1, 1024, 0, s>>>(partial, nb);
  KB_LAUNCH_CHECK();
  if (nb > 0) {
    scan_apply_k<Tin, Tout, kInclusive><<<nb, kScanNT, 0, s>>>(in, out, n, partial);
    KB_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8 bits per pass.

constexpr int kRadixNT = 256;
constexpr int kRadixIPT = 16;
constexpr int kRadixTile = kRadixNT * kRadixIPT;
constexpr int kRadixNW = kRadixNT / kWave;

template <typename K>
__global__ __launch_bounds__(kRadixNT) void radix_hist_k(const K* __restrict__ keys, uint64_t n,
                                                         int shift, uint32_t* __restrict__ hist,
                                                         uint32_t nblocks) {
  __shared__ uint32_t cnt[kRadixNW][256];
  for (int j = threadIdx.x; j < kRadixNW * 256; j += kRadixNT) (&cnt[0][0])[j] = 0;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const uint64_t base = uint64_t(blockIdx.x) * kRadixTile;
#pragma unroll 4
  for (int i = 0; i < kRadixIPT; ++i) {
    const uint64_t idx = base + uint64_t(i) * kRadixNT + threadIdx.x;
    if (idx < n) atomicAdd(&cnt[w][uint32_t(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += kRadixNT) {
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kRadixNW; ++q) s += cnt[q][d];
    hist[uint64_t(d) * nblocks + blockIdx.x] = s;
  }
}

// Lanes of the calling wave whose 8-bit digit equals this lane's digit.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t valid_mask) {
  uint64_t m = valid_mask;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

template <typename K, bool kHasVal>
__global__ __launch_bounds__(kRadixNT) void radix_scatter_k(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, uint64_t n, int shift, const uint32_t* __restrict__ hist_scan,
    uint32_t nblocks) {
  __shared__ uint32_t base_d[256];
  __shared__ uint32_t wcnt[kRadixNW][256];
  for (int d = threadIdx.x; d < 256; d += kRadixNT) base_d[d] = hist_scan[uint64_t(d) * nblocks + blockIdx.x];
  const int w = threadIdx.x / kWave;
  const uint64_t tile = uint64_t(blockIdx.x) * kRadixTile;
  for (int r = 0; r < kRadixIPT; ++r) {
    for (int j = threadIdx.x; j < kRadixNW * 256; j += kRadixNT) (&wcnt[0][0])[j] = 0;
    __syncthreads();
    const uint64_t idx = tile + uint64_t(r) * kRadixNT + threadIdx.x;
    const bool valid = idx < n;
    const K key = valid ? kin[idx] : K(0);
    const uint32_t d = valid ? (uint32_t(key >> shift) & 255u) : 0u;
    const uint64_t m = match_digit8(d, __ballot(valid));
    const uint32_t rank = __popcll(m & lanemask_lt());
    if (valid && rank == 0) wcnt[w][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t off = base_d[d] + rank;
      for (int q = 0; q < w; ++q) off += wcnt[q][d];
      kout[off] = key;
      if (kHasVal) vout[off] = vin[idx];
    }
    __syncthreads();
    for (int dd = threadIdx.x; dd < 256; dd += kRadixNT) {
      uint32_t s = 0;
#pragma unroll
      for (int q = 0; q < kRadixNW; ++q) s += wcnt[q][dd];
      base_d[dd] += s;
    }
    __syncthreads();
  }
}

inline uint32_t radix_blocks(uint64_t n) { return ceil_div(n, kRadixTile); }
// Scratch (uint32 words) radix_sort needs for the histograms and their scan.
inline size_t radix_scratch_words(uint64_t n) {
  const size_t h = size_t(radix_blocks(n)) * 256;
  return h + scan_partials_count(h);
}

// Sorts (keys, vals) of length n by bits [begin_bit, end_bit) of the key,
// stably. Ping-pongs between (k0,v0) and (k1,v1); returns true when the
// result ends in (k1,v1). vals may be null (keys only).
template <typename K>
bool radix_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, uint64_t n, int begin_bit, int end_bit,
                uint32_t* scratch, hipStream_t s) {
  if (n <= 1 || end_bit <= begin_bit) return false;
  const uint32_t nb = radix_blocks(n);
  uint32_t* hist = scratch;
  uint32_t* part = scratch + size_t(nb) * 256;
  bool flip = false;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    const K* ki = flip ? k1 : k0;
    K* ko = flip ? k0 : k1;
    const uint32_t* vi = flip ? v1 : v0;
    uint32_t* vo = flip ? v0 : v1;
    radix_hist_k<K><<<nb, kRadixNT, 0, s>>>(ki, n, shift, hist, nb);
    KB_LAUNCH_CHECK();
    scan<uint32_t, uint32_t, false>(hist, hist, uint64_t(nb) * 256, part, s);
    if (v0 != nullptr)
      radix_scatter_k<K, true><<<nb, kRadixNT, 0, s>>>(ki, vi, ko, vo, n, shift, hist, nb);
    else
      radix_scatter_k<K, false><<<nb, kRadixNT, 0, s>>>(ki, nullptr, ko, nullptr, n, shift, hist, nb);
    KB_LAUNCH_CHECK();
    flip = !flip;
  }
  return flip;
}

}  // namespace kb
