// Device-wide exclusive prefix sums (reduce -> scan of block totals -> apply).
// Inputs come from a functor so producers (flags, costs, counts) fuse into the scan.
#pragma once
#include "common.hpp"

namespace cpma_dev {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr uint64_t kScanTile = (uint64_t)kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* wtot /*LDS [4]*/, T* total) {
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  T incl = wave_incl_scan(v);
  if (lane == kWave - 1) wtot[wid] = incl;
  __syncthreads();
  T wofs = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; w++) {
    T x = wtot[w];
    if (w < wid) wofs += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return wofs + incl - v;
}

template <typename T, typename F>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(F in, uint64_t n, T* partial) {
  __shared__ T wtot[kScanThreads / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++)
    if (base + j < n) s += in(base + j);
  T tot;
  block_excl_scan<T>(s, wtot, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename T, typename F>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(F in, uint64_t n, T* out,
                                                             const T* partial_scan) {
  __shared__ T wtot[kScanThreads / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    v[j] = (base + j < n) ? in(base + j) : (T)0;
    s += v[j];
  }
  T tot;
  T ofs = block_excl_scan<T>(s, wtot, &tot) + (partial_scan ? partial_scan[blockIdx.x] : (T)0);
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    if (base + j < n) out[base + j] = ofs;
    ofs += v[j];
  }
  // The last block also writes the grand total at position n.
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
    T grand = (partial_scan ? partial_scan[blockIdx.x] : (T)0) + tot;
    out[n] = grand;
  }
}

template <typename T>
struct LoadFn {
  const T* p;
  __device__ T operator()(uint64_t i) const { return p[i]; }
};

// Scratch needed by scan_exclusive for n elements (in units of T).
inline uint64_t scan_scratch_elems(uint64_t n) {
  uint64_t total = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    total += 2 * (n + 1);
  }
  return total + 16;
}

// out[0..n] <- exclusive prefix sums of in(0..n-1); out[n] = total.
// tmp must hold scan_scratch_elems(n) elements.
template <typename T, typename F>
hipError_t scan_exclusive(F in, uint64_t n, T* out, T* tmp, hipStream_t s) {
  if (n == 0) {
    hipLaunchKernelGGL((k_fill<T>), dim3(1), dim3(kWave), 0, s, out, (uint64_t)1, (T)0);
    return hipGetLastError();
  }
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL((k_scan_apply<T, F>), dim3(1), dim3(kScanThreads), 0, s, in, n, out,
                       (const T*)nullptr);
    return hipGetLastError();
  }
  T* partial = tmp;
  T* partial_scan = tmp + nb + 1;
  hipLaunchKernelGGL((k_scan_reduce<T, F>), dim3((uint32_t)nb), dim3(kScanThreads), 0, s, in, n,
                     partial);
  hipError_t e = scan_exclusive<T>(LoadFn<T>{partial}, nb, partial_scan,
                                   partial_scan + nb + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_scan_apply<T, F>), dim3((uint32_t)nb), dim3(kScanThreads), 0, s, in, n, out,
                     (const T*)partial_scan);
  return hipGetLastError();
}

}  // namespace cpma_dev
