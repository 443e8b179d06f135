// Device-wide exclusive/inclusive scan and stable LSD radix sort (8-bit
// digits), hand-written for gfx950. Both are three-kernel designs with no
// inter-block waiting: reduce -> scan of partials -> apply.
#pragma once

#include <type_traits>

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

// Exclusive scan of partial[0..nb) in place by one block; partial[nb] =
// total. Every thread takes kPartPer consecutive partials of a chunk (loaded
// at once), so up to 1024 * kPartPer partials cost one round of loads.
constexpr int kPartPer = 8;
template <typename Tout>
__global__ __launch_bounds__(1024) void scan_partials_k(Tout* __restrict__ partial, uint32_t nb) {
  __shared__ Tout sh[1024 / kWave];
  Tout carry = 0;
  for (uint32_t base = 0; base < nb; base += 1024u * kPartPer) {
    const uint32_t i0 = base + threadIdx.x * kPartPer;
    Tout v[kPartPer], sum = 0;
#pragma unroll
    for (int q = 0; q < kPartPer; ++q) {
      v[q] = i0 + q < nb ? partial[i0 + q] : Tout(0);
      sum += v[q];
    }
    Tout tot;
    Tout run = carry + block_exclusive_scan<1024>(sum, sh, &tot);
#pragma unroll
    for (int q = 0; q < kPartPer; ++q) {
      if (i0 + q < nb) partial[i0 + q] = run;
      run += v[q];
    }
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

// Scan of up to kScanSmall elements by one workgroup, 1024 elements per step
// with a running carry. partial[0] receives the total.
constexpr uint32_t kScanSmall = 8192;
template <typename Tin, typename Tout, bool kInclusive>
__global__ __launch_bounds__(1024) void scan_small_k(const Tin* __restrict__ in, Tout* __restrict__ out,
                                                     uint32_t n, Tout* __restrict__ partial) {
  // every thread takes kPartPer consecutive elements (loaded at once), so
  // kScanSmall elements are one step
  __shared__ Tout sh[1024 / kWave];
  Tout carry = 0;
  for (uint32_t base = 0; base < n; base += 1024u * kPartPer) {
    const uint32_t i0 = base + threadIdx.x * kPartPer;
    Tout v[kPartPer], sum = 0;
#pragma unroll
    for (int q = 0; q < kPartPer; ++q) {
      v[q] = i0 + q < n ? Tout(in[i0 + q]) : Tout(0);
      sum += v[q];
    }
    Tout tot;
    Tout run = carry + block_exclusive_scan<1024>(sum, sh, &tot);  // reads all of the step before writes
#pragma unroll
    for (int q = 0; q < kPartPer; ++q) {
      if (i0 + q < n) out[i0 + q] = kInclusive ? run + v[q] : run;
      run += v[q];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) partial[0] = carry;
}

// Scratch words needed by scan(): one partial per tile plus the total.
inline size_t scan_partials_count(uint64_t n) { return size_t(ceil_div(n, kScanTile)) + 1; }

// out[i] = sum(in[0..i)) (or ..i] when inclusive). partial must hold
// scan_partials_count(n) entries of scratch. `out` may alias `in`. Up to
// kScanSmall elements one workgroup does it all; beyond, three kernels.
template <typename Tin, typename Tout, bool kInclusive = false>
void scan(const Tin* in, Tout* out, uint64_t n, Tout* partial, hipStream_t s) {
  if (n <= kScanSmall) {
    scan_small_k<Tin, Tout, kInclusive><<<1, 1024, 0, s>>>(in, out, uint32_t(n), partial);
    KB_LAUNCH_CHECK();
    return;
  }
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

// Tiles of kRadixNT threads x IPT items. The default, 3072-item tiles: on
// 10M-item passes with 64-bit keys 4096-item tiles ran about 6% slower and
// 8192-item tiles (one workgroup per CU) far slower; 2048-item tiles slowed
// the 100M-edge passes of the build by about 7%. 2048 and 4096 items are
// compiled too (a tuning option: the best size depends on the item counts).
constexpr int kRadixNT = 256;
constexpr int kRadixIPT = 12;  // a multiple of 4: full tiles are read with 16-byte loads
constexpr int kRadixIPTMin = 8;  // smallest tile compiled: sizes the scratch of every choice
constexpr int kRadixNW = kRadixNT / kWave;

// Items per thread of a tile size in items (2048, 3072 or 4096); 0 = the default.
inline int radix_ipt_of(uint32_t tile_items) {
  return tile_items == 0 ? kRadixIPT : int(tile_items / kRadixNT);
}
inline bool radix_tile_valid(uint32_t tile_items) {
  return tile_items == 0 || tile_items == 2048 || tile_items == 3072 || tile_items == 4096;
}

// Per-tile digit counts, digit-major: hist[d * nblocks + tile]. A full
// tile whose start is 16-byte aligned is read with 16-byte loads (more
// bytes in flight per thread); others element by element.
template <typename K, int IPT = kRadixIPT>
__global__ __launch_bounds__(kRadixNT) void radix_hist_k(const K* __restrict__ keys, uint64_t n,
                                                         int shift, uint32_t* __restrict__ hist,
                                                         uint32_t nblocks) {
  constexpr int kTile = kRadixNT * IPT;
  __shared__ uint32_t cnt[kRadixNW][256];
  for (int j = threadIdx.x; j < kRadixNW * 256; j += kRadixNT) (&cnt[0][0])[j] = 0;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const uint64_t base = uint64_t(blockIdx.x) * kTile;
  constexpr int kPerVec = 16 / sizeof(K);
  constexpr int kVecs = IPT / kPerVec;
  if (base + kTile <= n && (reinterpret_cast<uintptr_t>(keys) & 15u) == 0) {
    const uint4* v = reinterpret_cast<const uint4*>(keys + base);
    uint4 r[kVecs];
#pragma unroll
    for (int i = 0; i < kVecs; ++i) r[i] = v[i * kRadixNT + threadIdx.x];
#pragma unroll
    for (int i = 0; i < kVecs; ++i) {
      const K* e = reinterpret_cast<const K*>(&r[i]);
#pragma unroll
      for (int q = 0; q < kPerVec; ++q) {
        // a digit shared by the whole wave is added once
        const uint32_t d = uint32_t(e[q] >> shift) & 255u;
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        if (__ballot(d != d0) == 0) {
          if (__lane_id() == 0) atomicAdd(&cnt[w][d0], uint32_t(kWave));
        } else {
          atomicAdd(&cnt[w][d], 1u);
        }
      }
    }
  } else {
#pragma unroll 4
    for (int i = 0; i < IPT; ++i) {
      const uint64_t idx = base + uint64_t(i) * kRadixNT + threadIdx.x;
      if (idx < n) atomicAdd(&cnt[w][uint32_t(keys[idx] >> shift) & 255u], 1u);
    }
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

// Key and value of item i of a radix pass, read from two arrays.
template <typename K, typename V, bool kHasVal>
struct KVLoad {
  const K* __restrict__ k;
  const V* __restrict__ v;
  __device__ __forceinline__ void operator()(uint64_t i, K& key, V& val) const {
    key = k[i];
    if (kHasVal) val = v[i];
  }
};

// Scatter of one tile of kRadixNT * IPT items (blockIdx.x). Wave w owns the
// contiguous sub-tile [w*IPT*64, (w+1)*IPT*64) and keeps its IPT rows of 64
// items in registers. The tile is first sorted by digit into LDS (per-wave digit
// counts give every wave its local offsets; each wave places its rows in
// order with wave-local counters, one LDS read and one write per row, which
// a wave completes in order). Then consecutive threads copy consecutive LDS
// items to their global positions, so each digit's run is written
// contiguously. Stable: tile order = wave order, row order, lane order.
// kFused: `hist` holds the raw per-tile counts (digit-major) and every
// workgroup derives its own global offsets from them (for few tiles); else
// it holds their exclusive scan. `load(i, key, val)` reads item i < n.
template <typename K, typename V, bool kHasVal, bool kFused, typename Load, int IPT = kRadixIPT>
__device__ __forceinline__ void radix_scatter_tile(const Load& load, K* __restrict__ kout, V* __restrict__ vout,
                                                   uint64_t n, int shift, const uint32_t* __restrict__ hist_scan,
                                                   uint32_t nblocks) {
  constexpr int kRows = IPT;
  constexpr int kTile = kRadixNT * IPT;
  __shared__ uint32_t wh[kRadixNW][256];   // per-wave counts, then running local offsets
  __shared__ uint32_t gdelta[256];         // global position - local position, per digit
  __shared__ K sk[kTile];
  __shared__ V sv[kHasVal ? kTile : 1];
  for (int j = threadIdx.x; j < kRadixNW * 256; j += kRadixNT) (&wh[0][0])[j] = 0;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const int lane = __lane_id();
  const uint64_t tile = uint64_t(blockIdx.x) * kTile;
  const uint64_t sub = tile + uint64_t(w) * (kRows * kWave);
  const uint32_t tile_n = uint32_t(n - tile < uint64_t(kTile) ? n - tile : uint64_t(kTile));
  K key[kRows];
  V val[kRows];
  uint32_t dg[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const uint64_t idx = sub + uint64_t(r) * kWave + lane;
    const bool valid = idx < n;
    key[r] = K(0);
    val[r] = V(0);
    if (valid) load(idx, key[r], val[r]);
    dg[r] = valid ? (uint32_t(key[r] >> shift) & 255u) : 256u;
  }
  // lanes of the wave sharing each row's digit: one LDS add per distinct
  // digit (equal digits in a row, common in the high digits, would
  // otherwise serialise on one counter), reused for the ranks below
  uint64_t peers[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const bool valid = dg[r] < 256u;
    const uint32_t d = valid ? dg[r] : 0u;
    peers[r] = match_digit8(d, __ballot(valid));
    if (valid && (peers[r] & lanemask_lt()) == 0) atomicAdd(&wh[w][d], uint32_t(__popcll(peers[r])));
  }
  __syncthreads();
  {
    // local exclusive prefix over (digit, wave), and the global shift per digit
    const int d = threadIdx.x;  // kRadixNT == 256: one digit per thread
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < kRadixNW; ++q) tot += wh[q][d];
    __shared__ uint32_t shs[kRadixNW];
    uint32_t all;
    uint32_t local = block_exclusive_scan<kRadixNT>(tot, shs, &all);
    uint32_t gpos;
    if (kFused) {
      // items of digit d in earlier tiles, and in all tiles (eight counts
      // in flight at a time: one load per step would wait out the L2
      // latency nblocks times)
      const uint32_t* h = hist_scan + uint64_t(d) * nblocks;
      uint32_t before = 0, total = 0;
      uint32_t t = 0;
      for (; t + 8 <= nblocks; t += 8) {
        uint32_t c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = h[t + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          before += t + q < blockIdx.x ? c[q] : 0u;
          total += c[q];
        }
      }
      for (; t < nblocks; ++t) {
        const uint32_t c = h[t];
        before += t < blockIdx.x ? c : 0u;
        total += c;
      }
      uint32_t alld;
      gpos = block_exclusive_scan<kRadixNT>(total, shs, &alld) + before;
    } else {
      gpos = hist_scan[uint64_t(d) * nblocks + blockIdx.x];
    }
    gdelta[d] = gpos - local;
#pragma unroll
    for (int q = 0; q < kRadixNW; ++q) {
      const uint32_t c = wh[q][d];
      wh[q][d] = local;
      local += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const bool valid = dg[r] < 256u;
    const uint32_t d = valid ? dg[r] : 0u;
    const uint64_t m = peers[r];
    const uint32_t rank = __popcll(m & lanemask_lt());
    const uint32_t pos = wh[w][d] + rank;
    if (valid) {
      sk[pos] = key[r];
      if (kHasVal) sv[pos] = val[r];
    }
    if (valid && rank == 0) wh[w][d] = pos + __popcll(m);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < tile_n; i += kRadixNT) {
    const K k = sk[i];
    const uint32_t pos = gdelta[uint32_t(k >> shift) & 255u] + i;
    kout[pos] = k;
    if (kHasVal) vout[pos] = sv[i];
  }
}

template <typename K, typename V, bool kHasVal, bool kFused, int IPT = kRadixIPT>
__global__ __launch_bounds__(kRadixNT) void radix_scatter_k(
    const K* __restrict__ kin, const V* __restrict__ vin, K* __restrict__ kout,
    V* __restrict__ vout, uint64_t n, int shift, const uint32_t* __restrict__ hist_scan,
    uint32_t nblocks) {
  radix_scatter_tile<K, V, kHasVal, kFused, KVLoad<K, V, kHasVal>, IPT>(KVLoad<K, V, kHasVal>{kin, vin}, kout, vout,
                                                                        n, shift, hist_scan, nblocks);
}

inline uint32_t radix_blocks(uint64_t n, int ipt = kRadixIPT) { return ceil_div(n, uint64_t(kRadixNT) * ipt); }
// Up to this many tiles the scatter derives its offsets from the raw
// histogram itself, which saves the scan's three launches per digit. On the
// 10M/100M job (ordering passes of 10^5..10^6 items in rounds 1 and 2) 128
// tiles gave 9.38 ms per job against 9.58 with 64, 9.47 with 256 and 9.45
// with 512: each workgroup then reads 256 x nb counts.
constexpr uint32_t kRadixFusedTiles = 128;
// Scratch (uint32 words) radix_sort needs for the histograms and their scan,
// for any of the compiled tile sizes.
inline size_t radix_scratch_words(uint64_t n) {
  const size_t h = size_t(radix_blocks(n, kRadixIPTMin)) * 256;
  return h + scan_partials_count(h);
}

// Sorts (keys, vals) of length n by bits [begin_bit, end_bit) of the key,
// stably. Ping-pongs between (k0,v0) and (k1,v1); returns true when the
// result ends in (k1,v1). vals may be null (keys only).
template <typename K, typename V, int IPT>
bool radix_sort_t(K* k0, V* v0, K* k1, V* v1, uint64_t n, int begin_bit, int end_bit,
                  uint32_t* scratch, hipStream_t s) {
  if (n <= 1 || end_bit <= begin_bit) return false;
  const uint32_t nb = radix_blocks(n, IPT);
  uint32_t* hist = scratch;
  uint32_t* part = scratch + size_t(nb) * 256;
  bool flip = false;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    const K* ki = flip ? k1 : k0;
    K* ko = flip ? k0 : k1;
    const V* vi = flip ? v1 : v0;
    V* vo = flip ? v0 : v1;
    radix_hist_k<K, IPT><<<nb, kRadixNT, 0, s>>>(ki, n, shift, hist, nb);
    KB_LAUNCH_CHECK();
    if (nb <= kRadixFusedTiles) {
      if (v0 != nullptr)
        radix_scatter_k<K, V, true, true, IPT><<<nb, kRadixNT, 0, s>>>(ki, vi, ko, vo, n, shift, hist, nb);
      else
        radix_scatter_k<K, V, false, true, IPT><<<nb, kRadixNT, 0, s>>>(ki, nullptr, ko, nullptr, n, shift, hist, nb);
    } else {
      scan<uint32_t, uint32_t, false>(hist, hist, uint64_t(nb) * 256, part, s);
      if (v0 != nullptr)
        radix_scatter_k<K, V, true, false, IPT><<<nb, kRadixNT, 0, s>>>(ki, vi, ko, vo, n, shift, hist, nb);
      else
        radix_scatter_k<K, V, false, false, IPT><<<nb, kRadixNT, 0, s>>>(ki, nullptr, ko, nullptr, n, shift, hist, nb);
    }
    KB_LAUNCH_CHECK();
    flip = !flip;
  }
  return flip;
}

// Calls f(std::integral_constant<int, IPT>{}) for the compiled tile size
// with `ipt` items per thread (8, 12 or 16; anything else: the default).
template <typename F>
inline void with_radix_ipt(int ipt, F&& f) {
  switch (ipt) {
    case 8:
      f(std::integral_constant<int, 8>{});
      break;
    case 16:
      f(std::integral_constant<int, 16>{});
      break;
    default:
      f(std::integral_constant<int, kRadixIPT>{});
  }
}

// radix_sort_t with the tile size chosen at run time: ipt = items per
// thread (8, 12 or 16; radix_ipt_of), 0 = the default.
template <typename K, typename V = uint32_t>
bool radix_sort(K* k0, V* v0, K* k1, V* v1, uint64_t n, int begin_bit, int end_bit,
                uint32_t* scratch, hipStream_t s, int ipt = kRadixIPT) {
  switch (ipt) {
    case 8:
      return radix_sort_t<K, V, 8>(k0, v0, k1, v1, n, begin_bit, end_bit, scratch, s);
    case 16:
      return radix_sort_t<K, V, 16>(k0, v0, k1, v1, n, begin_bit, end_bit, scratch, s);
    default:
      return radix_sort_t<K, V, kRadixIPT>(k0, v0, k1, v1, n, begin_bit, end_bit, scratch, s);
  }
}

}  // namespace kb
