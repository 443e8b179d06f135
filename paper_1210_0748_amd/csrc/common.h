// Shared device helpers for the k-bisimulation kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace kb {

constexpr int kWave = 64;

struct DeviceError : std::runtime_error {
  hipError_t code;
  DeviceError(hipError_t c, const std::string& what) : std::runtime_error(what), code(c) {}
};

struct InvalidInput : std::runtime_error {
  using std::runtime_error::runtime_error;
};

struct OutOfMemory : std::runtime_error {
  using std::runtime_error::runtime_error;
};

struct StateError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define KB_CHECK(expr)                                                                      \
  do {                                                                                      \
    hipError_t kb_err_ = (expr);                                                            \
    if (kb_err_ != hipSuccess)                                                              \
      throw ::kb::DeviceError(kb_err_, std::string(#expr) + ": " + hipGetErrorString(kb_err_) + \
                                           " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define KB_LAUNCH_CHECK() KB_CHECK(hipGetLastError())

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return uint32_t((a + b - 1) / b); }

// Number of bits needed to represent values 0..v (at least 1).
inline int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Wave-aggregated append: each active lane with `want` receives a distinct
// slot counted from *counter (one atomic per wave). Every active lane of the
// wave must call it; the return value is meaningful only where `want` holds.
__device__ __forceinline__ uint32_t wave_append(bool want, uint32_t* counter) {
  const uint64_t b = __ballot(want);
  if (!b) return 0;
  const int leader = __ffsll((unsigned long long)b) - 1;
  uint32_t base = 0;
  if (__lane_id() == leader) base = atomicAdd(counter, uint32_t(__popcll(b)));
  base = __shfl(base, leader, kWave);
  return base + uint32_t(__popcll(b & lanemask_lt()));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_or(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w < v ? w : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

// Inclusive prefix sum over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T w = __shfl_up(v, o, kWave);
    if (lane >= o) v += w;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total. `sh` needs NT/64 entries.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T* total) {
  constexpr int NW = NT / kWave;
  const int lane = __lane_id();
  const int w = threadIdx.x / kWave;
  T inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) sh[w] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    T s = sh[i];
    if (i < w) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  T tot;
  block_exclusive_scan<NT>(v, sh, &tot);
  return tot;
}

}  // namespace kb
