// Query kernels: batched range_map (sum, count over [lo, hi)) and contains.
//
// range_map(start, end, f) is a search for the first element followed by a scan
// (Section "Packed Memory Array", "Design and operations"); in the CPMA the search
// runs on the uncompressed leaf heads and the scan decodes every leaf it passes
// (Section "Compressed Packed Memory Array", "Point queries").  A batch of
// queries becomes a flat list of leaf visits (query q visits leaves
// leaf(lo_q) .. leaf(hi_q - 1)); persistent waves take fixed-size chunks of
// visits, so long and short ranges balance across the GPU.
#pragma once
#include "update.hpp"

namespace cpma_dev {

struct QueryArgs {
  const uint64_t* lo;
  const uint64_t* hi;
  uint64_t q;
  const uint64_t* head;
  const uint8_t* bytes;
  const uint32_t* used;
  uint64_t L;
  uint32_t S;
};

// First leaf of every query and its number of leaf visits; zeroes the outputs.
__global__ void k_rm_locate(QueryArgs a, uint64_t* __restrict__ first_leaf, uint64_t* __restrict__ nvis,
                            unsigned long long* __restrict__ sum, unsigned long long* __restrict__ count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.q;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = a.lo[i], hi = a.hi[i];
    uint64_t f = 0, n = 0;
    if (lo < hi) {
      f = locate_leaf(a.head, a.L, lo);
      n = locate_leaf(a.head, a.L, hi - 1) - f + 1;
    }
    first_leaf[i] = f;
    nvis[i] = n;
    sum[i] = 0;
    count[i] = 0;
  }
}

// Persistent scan: each wave owns chunks of `chunk` consecutive visits.  Per-lane
// partial sums stay in registers while the query is unchanged and are flushed
// with one wave reduction and two 64-bit atomics (exact: integer adds commute).
__global__ void __launch_bounds__(256) k_rm_scan(QueryArgs a, const uint64_t* __restrict__ voff,
                                                 const uint64_t* __restrict__ first_leaf, uint32_t chunk,
                                                 unsigned long long* __restrict__ sum,
                                                 unsigned long long* __restrict__ count,
                                                 unsigned long long* __restrict__ alg) {
  const int lane = lane_id();
  uint64_t visited = 0;  // used bytes decoded by this wave (statistics)
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  const uint64_t wid = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint64_t V = voff[a.q];
  const uint64_t nchunks = (V + chunk - 1) / chunk;
  for (uint64_t c = wid; c < nchunks; c += waves) {
    const uint64_t v0 = c * chunk;
    const uint64_t v1 = min(v0 + chunk, V);
    uint64_t qi = upper_bound_u64(voff, a.q + 1, v0) - 1;
    uint64_t acc_s = 0, acc_c = 0;
    uint64_t qend = voff[qi + 1];
    uint64_t qlo = a.lo[qi], qhi = a.hi[qi];
    for (uint64_t v = v0; v < v1; v++) {
      if (v >= qend) {
        const uint64_t s = wave_sum(acc_s), n = wave_sum(acc_c);
        if (lane == 0 && n) {
          atomicAdd(&sum[qi], (unsigned long long)s);
          atomicAdd(&count[qi], (unsigned long long)n);
        }
        acc_s = acc_c = 0;
        do {
          qi++;
          qend = voff[qi + 1];
        } while (v >= qend);
        qlo = a.lo[qi];
        qhi = a.hi[qi];
      }
      const uint64_t leaf = first_leaf[qi] + (v - voff[qi]);
      const uint32_t u = a.used[leaf];
      visited += u;
      wave_decode_leaf(a.bytes + leaf * (uint64_t)a.S, u, [&](uint32_t, uint64_t x) {
        const bool in = (x >= qlo) & (x < qhi);
        acc_s += in ? x : 0ull;
        acc_c += in ? 1u : 0u;
      });
    }
    const uint64_t s = wave_sum(acc_s), n = wave_sum(acc_c);
    if (lane == 0 && n) {
      atomicAdd(&sum[qi], (unsigned long long)s);
      atomicAdd(&count[qi], (unsigned long long)n);
    }
  }
  if (alg && lane == 0 && visited) atomicAdd(alg, (unsigned long long)visited);
}

// Membership: one wave per key -- locate the leaf, decode it, compare.
__global__ void __launch_bounds__(256) k_contains(QueryArgs a, const uint64_t* __restrict__ keys,
                                                  uint8_t* __restrict__ out) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  const uint64_t wid = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  for (uint64_t i = wid; i < a.q; i += waves) {
    const uint64_t x = keys[i];
    const uint64_t leaf = locate_leaf(a.head, a.L, x);
    uint32_t found = 0;
    wave_decode_leaf(a.bytes + leaf * (uint64_t)a.S, a.used[leaf],
                     [&](uint32_t, uint64_t y) { found |= (y == x); });
    const uint64_t any = __ballot(found != 0);
    if (lane_id() == 0) out[i] = any ? 1 : 0;
  }
}

}  // namespace cpma_dev
