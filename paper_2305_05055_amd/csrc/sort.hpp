// Batch prep: stable LSD radix sort of 64-bit keys (8-bit digits, only as many
// passes as the OR of the keys needs) followed by removal of repeated keys.
// The paper sorts an unsorted batch in O(k log k) before merging it (Section
// "Parallel Batch Updates in a PMA"); on the GPU a radix sort does it in O(k)
// passes over HBM.
#pragma once
#include "scan.hpp"

namespace cpma_dev {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;  // keys per block

// Validation pass over a batch: OR of all keys (radix pass count), whether a
// reserved key occurs, and whether the batch is already non-decreasing.
struct BatchInfo {
  unsigned long long or_all;
  unsigned int has_reserved;
  unsigned int unsorted;
  unsigned int max_bucket;  // largest MSD bucket of a split (large batches)
  unsigned int ready;       // set last when a kernel publishes the struct to host memory
};

__global__ void __launch_bounds__(256) k_validate(const uint64_t* __restrict__ keys, uint64_t k,
                                                  BatchInfo* info) {
  __shared__ uint64_t red[4];
  uint64_t orv = 0;
  uint32_t res = 0, uns = 0;
  // four independent loads per thread in flight; the right neighbour of a
  // key comes from the next lane (lane 63 loads it)
  constexpr int kU = 4;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const bool last_lane = lane_id() == kWave - 1;
  // wave-uniform trip count, so every lane takes part in the neighbour shifts
  for (uint64_t w0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(uint32_t)(kWave - 1)); w0 < k;
       w0 += kU * stride) {
    const uint64_t i0 = w0 + (uint64_t)lane_id();
    uint64_t x[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint64_t i = i0 + u * stride;
      x[u] = i < k ? keys[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint64_t i = i0 + u * stride;
      uint64_t nx = dpp_next64(x[u]);
      if (last_lane && i + 1 < k) nx = keys[i + 1];
      if (i < k) {
        orv |= x[u];
        res |= (x[u] == kNoKey);
        if (i + 1 < k && nx < x[u]) uns = 1;
      }
    }
  }
  orv = wave_or(orv);
  const uint64_t flags = wave_or((uint64_t)(res | (uns << 1)));
  const int wid = threadIdx.x / kWave;
  if (lane_id() == 0) red[wid] = orv;
  __shared__ uint32_t fl[4];
  if (lane_id() == 0) fl[wid] = (uint32_t)flags;
  __syncthreads();
  if (threadIdx.x == 0) {
    // one atomic per block and field, and only while it still adds bits (a
    // stale read only costs a redundant atomic)
    const uint64_t o = red[0] | red[1] | red[2] | red[3];
    const uint32_t f = fl[0] | fl[1] | fl[2] | fl[3];
    if (o & ~__hip_atomic_load(&info->or_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->or_all, (unsigned long long)o);
    if ((f & 1) && !__hip_atomic_load(&info->has_reserved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->has_reserved, 1u);
    if ((f & 2) && !__hip_atomic_load(&info->unsorted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->unsorted, 1u);
  }
}

// Validation and the first radix pass's histogram in one read: one block per
// sort tile (item i = base + 256 r + tid), the tile's digit-0 counts written as
// k_radix_hist writes them, the batch flags as k_validate sets them.
__global__ void __launch_bounds__(kSortThreads) k_validate_hist(const uint64_t* __restrict__ keys, uint32_t k,
                                                                BatchInfo* info, uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[256];
  __shared__ uint64_t red[kSortThreads / kWave];
  __shared__ uint32_t fl[kSortThreads / kWave];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
  const bool last_lane = lane_id() == kWave - 1;
  uint64_t orv = 0;
  uint32_t res = 0, uns = 0;
  uint64_t x[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; r++) {
    const uint32_t i = base + r * kSortThreads + threadIdx.x;
    x[r] = i < k ? keys[i] : 0;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; r++) {
    const uint32_t i = base + r * kSortThreads + threadIdx.x;
    uint64_t nx = dpp_next64(x[r]);
    if (last_lane && i + 1 < k) nx = keys[i + 1];
    if (i < k) {
      orv |= x[r];
      res |= (x[r] == kNoKey);
      if (i + 1 < k && nx < x[r]) uns = 1;
      atomicAdd(&h[x[r] & 255u], 1u);
    }
  }
  orv = wave_or(orv);
  const uint64_t flags = wave_or((uint64_t)(res | (uns << 1)));
  const int wid = threadIdx.x / kWave;
  if (lane_id() == 0) {
    red[wid] = orv;
    fl[wid] = (uint32_t)flags;
  }
  __syncthreads();
  ghist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
  if (threadIdx.x == 0) {
    uint64_t o = 0;
    uint32_t f = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; w++) {
      o |= red[w];
      f |= fl[w];
    }
    if (o & ~__hip_atomic_load(&info->or_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->or_all, (unsigned long long)o);
    if ((f & 1) && !__hip_atomic_load(&info->has_reserved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->has_reserved, 1u);
    if ((f & 2) && !__hip_atomic_load(&info->unsorted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->unsorted, 1u);
  }
}

__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint64_t* __restrict__ in,
                                                             uint32_t n, int shift,
                                                             uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortItems; r++) {
    uint32_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(in[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  ghist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one tile (kSortTile keys) with stable ranks, written out in digit
// order.  Wave w ranks its own contiguous quarter of the tile (round r, lane l
// holds key w * 1024 + 64 r + l): a lane's rank among equal digits in a round
// comes from eight ballots, and wave-private digit counters in LDS carry it
// across rounds, so no barrier is needed while ranking.  The tile is then
// placed in LDS in digit order and written with consecutive threads on
// consecutive output positions inside each digit's run.
//
// With kKV every key carries a 32-bit value that moves with it (the values
// take a second LDS tile).  A pass without input values (vin null) makes them:
// value i is i | vgen[i] << 31.
constexpr int kScatterWaves = kSortThreads / kWave;
static_assert(kSortItems * kScatterWaves == kWave, "one wave scans the (round, wave) counts of a tile");

template <bool kKV>
__device__ __forceinline__ void radix_scatter_tile(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                   uint32_t n, int shift, const uint32_t* __restrict__ goff,
                                                   const uint32_t* __restrict__ vin, const uint8_t* __restrict__ vgen,
                                                   uint32_t* __restrict__ vout, uint64_t* tile, uint32_t* vtile,
                                                   uint32_t (*cnt)[256], uint32_t* toff, uint32_t* gbase,
                                                   uint32_t* wsum) {
  constexpr int kW = kScatterWaves;
  constexpr int kRounds = kSortTile / kSortThreads;  // rounds per wave (16)
  const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
#pragma unroll
  for (int w = 0; w < kW; w++) cnt[w][tid] = 0;
  gbase[tid] = goff[(uint64_t)tid * gridDim.x + blockIdx.x];
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
  const uint32_t wbase = base + (uint32_t)wid * (kRounds * kWave);
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint64_t x[kRounds];
  uint32_t v[kKV ? kRounds : 1];
#pragma unroll
  for (int r = 0; r < kRounds; r++) {
    const uint32_t i = wbase + (uint32_t)r * kWave + lane;
    x[r] = i < n ? in[i] : 0;
    if constexpr (kKV) v[r] = i < n ? (vin ? vin[i] : (i | ((uint32_t)vgen[i] << 31))) : 0u;
  }
  uint32_t rk[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; r++) {
    const bool valid = wbase + (uint32_t)r * kWave + lane < n;
    const uint32_t d = (uint32_t)(x[r] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    uint32_t pre = 0;
    if (valid) pre = cnt[wid][d];
    rk[r] = pre + below;
    if (valid && below == 0) cnt[wid][d] = pre + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // tile offsets of every digit (exclusive scan over 256 digits) and of every
  // wave's share of it
  uint32_t tot = 0;
#pragma unroll
  for (int w = 0; w < kW; w++) tot += cnt[w][tid];
  const uint32_t incl = wave_incl_scan(tot);
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t wofs = 0;
#pragma unroll
  for (int w = 0; w < kW; w++)
    if (w < wid) wofs += wsum[w];
  const uint32_t ex = wofs + incl - tot;
  toff[tid] = ex;
  uint32_t run = ex;
#pragma unroll
  for (int w = 0; w < kW; w++) {
    const uint32_t c = cnt[w][tid];
    cnt[w][tid] = run;  // becomes the wave's first slot for digit tid
    run += c;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; r++) {
    if (wbase + (uint32_t)r * kWave + lane < n) {
      const uint32_t d = (uint32_t)(x[r] >> shift) & 255u;
      tile[cnt[wid][d] + rk[r]] = x[r];
      if constexpr (kKV) vtile[cnt[wid][d] + rk[r]] = v[r];
    }
  }
  __syncthreads();
  const uint32_t m = min(kSortTile, n - base);
  for (uint32_t i = tid; i < m; i += kSortThreads) {
    const uint64_t y = tile[i];
    const uint32_t d = (uint32_t)(y >> shift) & 255u;
    out[gbase[d] + (i - toff[d])] = y;
    if constexpr (kKV) vout[gbase[d] + (i - toff[d])] = vtile[i];
  }
}

__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint64_t* __restrict__ in,
                                                                uint64_t* __restrict__ out,
                                                                uint32_t n, int shift,
                                                                const uint32_t* __restrict__ goff) {
  __shared__ uint64_t tile[kSortTile];
  __shared__ uint32_t cnt[kScatterWaves][256];
  __shared__ uint32_t toff[256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t wsum[kScatterWaves];
  radix_scatter_tile<false>(in, out, n, shift, goff, nullptr, nullptr, nullptr, tile, nullptr, cnt, toff, gbase,
                            wsum);
}

// Key-value scatter (stable, so equal keys keep the order of their values'
// positions through every pass).
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter_kv(const uint64_t* __restrict__ in,
                                                                   uint64_t* __restrict__ out, uint32_t n, int shift,
                                                                   const uint32_t* __restrict__ goff,
                                                                   const uint32_t* __restrict__ vin,
                                                                   const uint8_t* __restrict__ vgen,
                                                                   uint32_t* __restrict__ vout) {
  __shared__ uint64_t tile[kSortTile];
  __shared__ uint32_t vtile[kSortTile];
  __shared__ uint32_t cnt[kScatterWaves][256];
  __shared__ uint32_t toff[256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t wsum[kScatterWaves];
  radix_scatter_tile<true>(in, out, n, shift, goff, vin, vgen, vout, tile, vtile, cnt, toff, gbase, wsum);
}

// Large batches: one MSD split, then every bucket sorted inside LDS.
//
// The top b bits of a key (b = 8..11, chosen by the host so that an average
// bucket holds about 0.8 kBktCap keys) pick its bucket; the low r = bits - b
// bits (r <= 32) are sorted inside the bucket.  k_msd_hist counts the buckets
// per tile ([bucket][tile], scanned into output offsets as for the LSD
// passes); k_msd_scatter moves every tile's keys to their buckets through an
// LDS copy of the tile in bucket order, so each bucket's run of a tile is
// written contiguously; k_bucket_sort then loads one bucket per block, sorts
// the 32-bit low parts with stable 8-bit LSD passes inside LDS and writes the
// bucket's first occurrences back in order; k_bucket_compact closes the gaps
// the removed repeats leave.  Three passes over HBM replace the five of a
// 40-bit LSD sort and the two of removing repeats.  Order inside a bucket before its sort does not matter, so the
// split ranks keys with LDS atomics.
constexpr int kMsdThreads = 1024;
constexpr int kMsdItems = 16;
constexpr uint32_t kMsdTile = kMsdThreads * kMsdItems;  // keys per split block
constexpr int kMsdMaxBits = 11;                          // at most 2048 buckets
constexpr uint32_t kMsdMaxBuckets = 1u << kMsdMaxBits;
constexpr int kBktThreads = 1024;
constexpr int kBktWaves = kBktThreads / kWave;
constexpr int kBktRounds = 12;                           // rounds of 64 keys per wave
constexpr uint32_t kBktCap = kBktThreads * kBktRounds;   // keys per bucket (12288)
constexpr uint64_t kBktTarget = kBktCap * 4 / 5;          // average bucket the host aims for
constexpr int kMsdMinBits = 8;
constexpr uint64_t kMsdMinKeys = 1ull << 19;              // smaller batches take the LSD passes
constexpr uint64_t kMsdMaxKeys = kBktTarget << kMsdMaxBits;

__device__ __forceinline__ uint32_t msd_bucket(uint64_t x, int r, uint32_t nd) {
  // clamped so that a key outside the announced bit length cannot index past
  // the counters (the host derives r from the OR of the same keys)
  return (uint32_t)min<uint64_t>(x >> r, (uint64_t)(nd - 1));
}

__global__ void __launch_bounds__(kMsdThreads) k_msd_hist(const uint64_t* __restrict__ in, uint32_t n, int r,
                                                          uint32_t nd, uint32_t* __restrict__ counts) {
  __shared__ uint32_t h[kMsdMaxBuckets];
  for (uint32_t d = threadIdx.x; d < kMsdMaxBuckets; d += kMsdThreads) h[d] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kMsdTile;
  uint64_t x[kMsdItems];
#pragma unroll
  for (int j = 0; j < kMsdItems; j++) {
    const uint32_t i = base + j * kMsdThreads + threadIdx.x;
    x[j] = i < n ? in[i] : 0;
  }
#pragma unroll
  for (int j = 0; j < kMsdItems; j++)
    if (base + j * kMsdThreads + threadIdx.x < n) atomicAdd(&h[msd_bucket(x[j], r, nd)], 1u);
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < nd; d += kMsdThreads) counts[(uint64_t)d * gridDim.x + blockIdx.x] = h[d];
}

// Validation and k_msd_hist's counts in one read, for a bucket shift taken
// from an earlier batch (the host discards the counts if this batch has more
// bits).  One block per split tile, item i = base + 1024 j + tid.  A key's
// right neighbour is the next lane's (DPP); lane 63's is lane 0 of the next
// wave (or of wave 0 in the next round), so lane 63 parks its keys in LDS and
// compares them after the barrier, when the keys' registers are free; only
// the tile's last item reads the next tile's first key.
__global__ void __launch_bounds__(kMsdThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_validate_msd(const uint64_t* __restrict__ keys, uint32_t n, int r, uint32_t nd, BatchInfo* __restrict__ info,
               uint32_t* __restrict__ counts) {
  constexpr int kW = kMsdThreads / kWave;
  __shared__ uint32_t h[kMsdMaxBuckets];
  __shared__ uint64_t first[kMsdItems][kW];
  __shared__ uint64_t last[kMsdItems][kW];
  __shared__ uint64_t red[kW];
  __shared__ uint32_t fl[kW];
  const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
  for (uint32_t d = tid; d < kMsdMaxBuckets; d += kMsdThreads) h[d] = 0;
  const uint32_t base = blockIdx.x * kMsdTile;
  __syncthreads();  // counters cleared
  uint64_t orv = 0;
  uint32_t res = 0, uns = 0;
  // two halves of kMsdItems / 2 loads in flight, so two blocks fit a CU
  constexpr int kHalf = kMsdItems / 2;
#pragma unroll
  for (int hf = 0; hf < 2; hf++) {
    uint64_t x[kHalf];
#pragma unroll
    for (int q = 0; q < kHalf; q++) {
      const uint32_t i = base + (hf * kHalf + q) * kMsdThreads + tid;
      x[q] = i < n ? keys[i] : 0;
    }
#pragma unroll
    for (int q = 0; q < kHalf; q++) {
      const int j = hf * kHalf + q;
      const uint32_t i = base + j * kMsdThreads + tid;
      const uint64_t nx = dpp_next64(x[q]);
      if (lane == 0) first[j][wid] = x[q];
      if (lane == kWave - 1) last[j][wid] = x[q];
      if (i < n) {
        orv |= x[q];
        res |= (x[q] == kNoKey);
        if (lane != kWave - 1 && i + 1 < n && nx < x[q]) uns = 1;
        atomicAdd(&h[msd_bucket(x[q], r, nd)], 1u);
      }
    }
  }
  __syncthreads();
  if (lane == kWave - 1) {
    const uint64_t after = base + kMsdTile < n ? keys[base + kMsdTile] : 0;  // the next tile's first key
#pragma unroll
    for (int j = 0; j < kMsdItems; j++) {
      const uint32_t i = base + j * kMsdThreads + tid;
      const uint64_t nx = wid + 1 < kW ? first[j][wid + 1] : (j + 1 < kMsdItems ? first[j + 1][0] : after);
      if (i + 1 < n && nx < last[j][wid]) uns = 1;
    }
  }
  orv = wave_or(orv);
  const uint64_t flags = wave_or((uint64_t)(res | (uns << 1)));
  if (lane == 0) {
    red[wid] = orv;
    fl[wid] = (uint32_t)flags;
  }
  __syncthreads();
  for (uint32_t d = tid; d < nd; d += kMsdThreads) counts[(uint64_t)d * gridDim.x + blockIdx.x] = h[d];
  if (tid == 0) {
    uint64_t o = 0;
    uint32_t f = 0;
#pragma unroll
    for (int w = 0; w < kW; w++) {
      o |= red[w];
      f |= fl[w];
    }
    if (o & ~__hip_atomic_load(&info->or_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->or_all, (unsigned long long)o);
    if ((f & 1) && !__hip_atomic_load(&info->has_reserved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->has_reserved, 1u);
    if ((f & 2) && !__hip_atomic_load(&info->unsorted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicOr(&info->unsorted, 1u);
  }
}

// Largest bucket after the scan of k_msd_hist's counts (koff[d * ntiles] is
// where bucket d starts, koff[nd * ntiles] the total).  One block.  With hout
// (host memory) it also publishes the whole BatchInfo there, the validation's
// fields included, and then sets hout->ready, so the host can poll instead of
// copying and synchronising.
__global__ void __launch_bounds__(kMsdThreads) k_msd_max(const uint32_t* __restrict__ koff, uint32_t ntiles,
                                                         uint32_t nd, BatchInfo* __restrict__ info,
                                                         BatchInfo* hout) {
  __shared__ uint32_t wm[kMsdThreads / kWave];
  uint32_t m = 0;
  for (uint32_t d = threadIdx.x; d < nd; d += kMsdThreads)
    m = max(m, koff[(uint64_t)(d + 1) * ntiles] - koff[(uint64_t)d * ntiles]);
  m = __shfl(dpp_incl_max(m), kWave - 1);
  if (lane_id() == 0) wm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kMsdThreads / kWave; w++) m = max(m, wm[w]);
    m = max(m, atomicMax(&info->max_bucket, m));
    if (hout) {
      hout->or_all = __hip_atomic_load(&info->or_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      hout->has_reserved = __hip_atomic_load(&info->has_reserved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      hout->unsorted = __hip_atomic_load(&info->unsorted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      hout->max_bucket = m;
      __threadfence_system();
      __hip_atomic_store(&hout->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// The bucket's low parts only go out: a key is its bucket number above its
// low r bits, and the bucket sort restores it.
__global__ void __launch_bounds__(kMsdThreads) k_msd_scatter(const uint64_t* __restrict__ in,
                                                             uint32_t* __restrict__ out, uint32_t n, int r,
                                                             uint32_t nd, const uint32_t* __restrict__ koff) {
  __shared__ uint64_t tile[kMsdTile];
  __shared__ uint32_t h[kMsdMaxBuckets];   // counts, then the tile's bucket offsets
  __shared__ uint32_t gb[kMsdMaxBuckets];  // the tile's output position per bucket
  __shared__ uint32_t wsum[kMsdThreads / kWave];
  const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
  for (uint32_t d = tid; d < kMsdMaxBuckets; d += kMsdThreads) h[d] = 0;
  for (uint32_t d = tid; d < nd; d += kMsdThreads) gb[d] = koff[(uint64_t)d * gridDim.x + blockIdx.x];
  __syncthreads();
  const uint32_t base = blockIdx.x * kMsdTile;
  uint64_t x[kMsdItems];
  uint32_t rk[kMsdItems];
#pragma unroll
  for (int j = 0; j < kMsdItems; j++) {
    const uint32_t i = base + j * kMsdThreads + tid;
    x[j] = i < n ? in[i] : 0;
  }
#pragma unroll
  for (int j = 0; j < kMsdItems; j++)
    if (base + j * kMsdThreads + tid < n) rk[j] = atomicAdd(&h[msd_bucket(x[j], r, nd)], 1u);
  __syncthreads();
  // exclusive scan of the 2048 counters, kPer consecutive ones per thread
  constexpr int kPer = kMsdMaxBuckets / kMsdThreads;
  static_assert(kPer * kMsdThreads == kMsdMaxBuckets, "counters split evenly over the threads");
  uint32_t c[kPer], sum = 0;
#pragma unroll
  for (int q = 0; q < kPer; q++) {
    c[q] = h[kPer * tid + q];
    sum += c[q];
  }
  const uint32_t incl = wave_incl_scan(sum);
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
#pragma unroll
  for (int w = 0; w < kMsdThreads / kWave; w++)
    if (w < wid) run += wsum[w];
#pragma unroll
  for (int q = 0; q < kPer; q++) {
    h[kPer * tid + q] = run;
    run += c[q];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kMsdItems; j++)
    if (base + j * kMsdThreads + tid < n) tile[h[msd_bucket(x[j], r, nd)] + rk[j]] = x[j];
  __syncthreads();
  const uint32_t m = min(kMsdTile, n - base);
  const uint32_t lowmask = r >= 32 ? 0xffffffffu : ((1u << r) - 1u);
  for (uint32_t i = tid; i < m; i += kMsdThreads) {
    const uint64_t y = tile[i];
    const uint32_t d = msd_bucket(y, r, nd);
    out[gb[d] + (i - h[d])] = (uint32_t)y & lowmask;
  }
}

// Lanes of the wave whose bit B of y matches this lane's, as two 32-bit
// halves: the sign-extended bit is 0 or all ones, so ~(ballot ^ bit) keeps the
// lanes that agree.
template <int B>
__device__ __forceinline__ void match_bit(uint32_t y, uint32_t& p0, uint32_t& p1) {
  uint32_t sb;
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(sb) : "v"(y), "i"(B));
  const uint64_t m = __ballot(sb != 0);
  p0 &= ~((uint32_t)m ^ sb);
  p1 &= ~((uint32_t)(m >> 32) ^ sb);
}

// One block per bucket (nd blocks).  Wave w holds items w * 768 + 64 j + l of
// the current order (round j, lane l) in registers; each pass sorts them by
// one 8-bit digit of the low part, least significant first, through LDS.
// The first pass may reorder equal digits (the order it starts from is
// arbitrary), so it ranks with LDS atomics.  The later passes are stable: a
// lane's rank among equal digits of its round comes from eight ballots, and
// wave-private counters in LDS carry the count across rounds (every lane
// reads its digit's counter, then the group's lowest lane adds the group;
// LDS executes one wave's operations in order, so no wait is needed between
// rounds).  The host launches this only when every bucket holds at most
// kBktCap keys; a larger one is left unsorted and raises *err (the update's
// device-error counter, which the host checks before it reports success).
__global__ void __launch_bounds__(kBktThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_bucket_sort(const uint32_t* __restrict__ in,
                                                             uint64_t* __restrict__ out,
                                                             const uint32_t* __restrict__ koff, uint32_t ntiles,
                                                             int r, uint32_t* __restrict__ ucnt,
                                                             unsigned int* __restrict__ err) {
  __shared__ uint32_t buf[kBktCap];
  __shared__ uint32_t cnt[kBktWaves][256];  // the first pass uses row 0 for the whole block
  __shared__ uint32_t wsum[256 / kWave];
  __shared__ uint32_t wtot[kBktWaves];
  const uint32_t bkt = blockIdx.x;
  const uint32_t beg = koff[(uint64_t)bkt * ntiles];
  const uint32_t n = koff[(uint64_t)(bkt + 1) * ntiles] - beg;
  if (n > kBktCap) {
    if (threadIdx.x == 0) {
      ucnt[bkt] = 0u;
      atomicOr(err, 1u);
    }
    return;
  }
  const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
  const uint32_t wb = (uint32_t)wid * (kBktRounds * kWave);
  uint32_t x[kBktRounds];
#pragma unroll
  for (int j = 0; j < kBktRounds; j++) {
    const uint32_t i = wb + (uint32_t)j * kWave + lane;
    x[j] = i < n ? in[beg + i] : 0u;
  }
  for (int sh = 0; sh < r; sh += 8) {
    const bool first = sh == 0;
#pragma unroll
    for (int q = 0; q < kBktWaves * 256 / kBktThreads; q++) (&cnt[0][0])[q * kBktThreads + tid] = 0;
    __syncthreads();
    uint32_t rk[kBktRounds];
    if (wb < n) {  // waves past the bucket's end rank nothing
      if (first) {
#pragma unroll
        for (int j = 0; j < kBktRounds; j++)
          if (wb + (uint32_t)j * kWave + lane < n) rk[j] = atomicAdd(&cnt[0][x[j] & 255u], 1u);
      } else {
#pragma unroll
        for (int j = 0; j < kBktRounds; j++) {
          const bool valid = wb + (uint32_t)j * kWave + lane < n;
          const uint32_t y = x[j] >> sh;
          const uint64_t vm = __ballot(valid);
          uint32_t p0 = (uint32_t)vm, p1 = (uint32_t)(vm >> 32);
          match_bit<0>(y, p0, p1);
          match_bit<1>(y, p0, p1);
          match_bit<2>(y, p0, p1);
          match_bit<3>(y, p0, p1);
          match_bit<4>(y, p0, p1);
          match_bit<5>(y, p0, p1);
          match_bit<6>(y, p0, p1);
          match_bit<7>(y, p0, p1);
          const uint32_t below = __builtin_amdgcn_mbcnt_hi(p1, __builtin_amdgcn_mbcnt_lo(p0, 0u));
          uint32_t* c = &cnt[wid][y & 255u];
          rk[j] = below + (valid ? *c : 0u);
          if (valid && below == 0) atomicAdd(c, (uint32_t)(__popc(p0) + __popc(p1)));
        }
      }
    }
    __syncthreads();
    // digit offsets: threads 0..255 own one digit each
    uint32_t tot = 0, incl = 0;
    if (tid < 256) {
      if (first) {
        tot = cnt[0][tid];
      } else {
#pragma unroll
        for (int w = 0; w < kBktWaves; w++) tot += cnt[w][tid];
      }
      incl = wave_incl_scan(tot);
      if (lane == kWave - 1) wsum[wid] = incl;
    }
    __syncthreads();
    if (tid < 256) {
      uint32_t run = incl - tot;
#pragma unroll
      for (int w = 0; w < 256 / kWave; w++)
        if (w < wid) run += wsum[w];
      if (first) {
        cnt[0][tid] = run;
      } else {
#pragma unroll
        for (int w = 0; w < kBktWaves; w++) {
          const uint32_t c = cnt[w][tid];
          cnt[w][tid] = run;  // wave w's first slot for digit tid
          run += c;
        }
      }
    }
    __syncthreads();
    if (wb < n) {
      const int row = first ? 0 : wid;
#pragma unroll
      for (int j = 0; j < kBktRounds; j++)
        if (wb + (uint32_t)j * kWave + lane < n) buf[cnt[row][(x[j] >> sh) & 255u] + rk[j]] = x[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBktRounds; j++) {
      const uint32_t i = wb + (uint32_t)j * kWave + lane;
      if (i < n) x[j] = buf[i];
    }
    __syncthreads();  // the next pass clears the counters the scatter read
  }
  // Repeats removed on the way out: the first occurrences of the sorted
  // bucket go to out[beg ..], in order (item order is wave, round, lane), and
  // their number to ucnt[bkt].  Without a low part every key of the bucket is
  // the same.
  const uint64_t hi = (uint64_t)bkt << r;
  if (r == 0) {
    if (tid == 0) {
      if (n) out[beg] = hi;
      ucnt[bkt] = n ? 1u : 0u;
    }
    return;
  }
  auto first_occ = [&](int j) {
    const uint32_t i = wb + (uint32_t)j * kWave + lane;
    return i < n && (i == 0 || buf[i - 1] != x[j]);
  };
  uint32_t tw = 0;
#pragma unroll
  for (int j = 0; j < kBktRounds; j++) tw += (uint32_t)__popcll(__ballot(first_occ(j)));
  if (lane == 0) wtot[wid] = tw;
  __syncthreads();
  uint32_t woff = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kBktWaves; w++) {
    const uint32_t t = wtot[w];
    if (w < wid) woff += t;
    total += t;
  }
  uint32_t pos = beg + woff;
#pragma unroll
  for (int j = 0; j < kBktRounds; j++) {
    const bool f = first_occ(j);
    const uint64_t fm = __ballot(f);
    if (f) out[pos + __builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0u))] =
        hi | x[j];
    pos += (uint32_t)__popcll(fm);
  }
  if (tid == 0) ucnt[bkt] = total;
}

// Moves every bucket's first occurrences (ucnt of them at the bucket's start
// in `in`) to their place in the repeat-free batch (uoff: exclusive scan of
// ucnt, uoff[nd] the total, which block 0 also stores in *n_out).
__global__ void __launch_bounds__(256) k_bucket_compact(const uint64_t* __restrict__ in,
                                                        const uint32_t* __restrict__ koff, uint32_t ntiles,
                                                        const uint32_t* __restrict__ uoff, uint32_t nd,
                                                        uint64_t* __restrict__ out,
                                                        unsigned long long* __restrict__ n_out) {
  const uint32_t b = blockIdx.x;
  const uint64_t* src = in + koff[(uint64_t)b * ntiles];
  const uint32_t d0 = uoff[b], m = uoff[b + 1] - d0;
  constexpr int kU = 4;
  for (uint32_t i0 = threadIdx.x; i0 < m; i0 += kU * 256) {
    uint64_t v[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) v[u] = i0 + u * 256 < m ? src[i0 + u * 256] : 0;
#pragma unroll
    for (int u = 0; u < kU; u++)
      if (i0 + u * 256 < m) out[d0 + i0 + u * 256] = v[u];
  }
  if (b == 0 && threadIdx.x == 0) *n_out = uoff[nd];
}

// Flags of first occurrences in a sorted array.
struct FirstFlag {
  const uint64_t* a;
  __device__ uint32_t operator()(uint64_t i) const { return (i == 0 || a[i] != a[i - 1]) ? 1u : 0u; }
};

__global__ void k_compact_unique(const uint64_t* __restrict__ a, uint64_t n,
                                 const uint32_t* __restrict__ pos, uint64_t* __restrict__ out,
                                 unsigned long long* __restrict__ n_out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (i == 0 || a[i] != a[i - 1]) out[pos[i]] = a[i];
    if (i == 0) *n_out = pos[n];
  }
}

// Removal of repeats from a sorted batch in two passes over it: per tile of
// kSortTile keys the number of first occurrences, an exclusive scan of those
// (one small launch), then every tile writes its first occurrences to its
// offset.  Inside a tile, item i = base + 256 r + 64 w + l (round r, wave w,
// lane l), so the tile's order is (r, w, l): a ballot per round gives the lane
// offsets, and one wave scan over the 16 x 4 (round, wave) counts the rest.
__device__ __forceinline__ bool first_occurrence(const uint64_t* __restrict__ a, uint64_t i, uint64_t x,
                                                 uint64_t prev_lane) {
  if (i == 0) return true;
  const uint64_t prev = lane_id() == 0 ? a[i - 1] : prev_lane;
  return prev != x;
}

__global__ void __launch_bounds__(kSortThreads) k_unique_count(const uint64_t* __restrict__ a, uint64_t n,
                                                               uint32_t* __restrict__ tcnt) {
  __shared__ uint32_t red[kSortThreads / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  const int wid = threadIdx.x / kWave;
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < kSortItems; r++) {
    const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
    const uint64_t x = i < n ? a[i] : 0;
    const uint64_t pl = dpp_prev64(x);
    if (i < n && first_occurrence(a, i, x, pl)) c++;
  }
  c = wave_sum(c);
  if (lane_id() == 0) red[wid] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; w++) t += red[w];
    tcnt[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kSortThreads) k_unique_write(const uint64_t* __restrict__ a, uint64_t n,
                                                               const uint32_t* __restrict__ toff, uint32_t ntiles,
                                                               uint64_t* __restrict__ out,
                                                               unsigned long long* __restrict__ n_out) {
  constexpr int kW = kSortThreads / kWave;
  __shared__ uint32_t rc[kSortItems * kW];  // (round, wave) counts, then their exclusive offsets
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint64_t x[kSortItems];
  uint64_t fm[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; r++) {
    const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
    x[r] = i < n ? a[i] : 0;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; r++) {
    const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
    const uint64_t pl = dpp_prev64(x[r]);
    fm[r] = __ballot(i < n && first_occurrence(a, i, x[r], pl));
    if (lane == 0) rc[r * kW + wid] = (uint32_t)__popcll(fm[r]);
  }
  __syncthreads();
  if (wid == 0) {
    const uint32_t v = rc[lane];  // kSortItems * kW == 64 entries
    rc[lane] = wave_incl_scan(v) - v;
  }
  __syncthreads();
  const uint64_t tb = toff[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kSortItems; r++) {
    if ((fm[r] >> lane) & 1ull) out[tb + rc[r * kW + wid] + (uint32_t)__popcll(fm[r] & lt_mask)] = x[r];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = toff[ntiles];
}

}  // namespace cpma_dev
