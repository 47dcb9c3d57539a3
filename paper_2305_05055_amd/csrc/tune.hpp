// Kernels of the autotuner's trial workload: a density-preserving sample of the
// input (the keys below a threshold) and uniform keys / ranges drawn with the
// counter-based splitmix64 generator (Steele, Lea, Flood, OOPSLA 2014).
#pragma once
#include "common.hpp"

namespace cpma_dev {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Appends every key below T (any order: the build sorts); *cnt counts all of
// them, writes stop at cap.
__global__ void k_sample_below(const uint64_t* __restrict__ keys, uint64_t n, uint64_t T,
                               uint64_t* __restrict__ out, uint64_t cap, unsigned long long* cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = keys[i];
    if (x < T) {
      const uint64_t p = atomicAdd(cnt, 1ull);
      if (p < cap) out[p] = x;
    }
  }
}

// out[i] = a uniform key in [0, T) (T > 0).
__global__ void k_gen_uniform(uint64_t* __restrict__ out, uint64_t n, uint64_t T, uint64_t seed) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = splitmix64_at(seed, i) % T;
}

// Ranges [lo, lo + width) with lo uniform in [0, T).
__global__ void k_gen_ranges(uint64_t* __restrict__ lo, uint64_t* __restrict__ hi, uint64_t n, uint64_t T,
                             uint64_t width, uint64_t seed) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t l = splitmix64_at(seed, i) % T;
    lo[i] = l;
    hi[i] = l + width;
  }
}

}  // namespace cpma_dev
