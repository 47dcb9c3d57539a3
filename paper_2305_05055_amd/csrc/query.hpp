// Query kernels: batched range_map (sum, count over [lo, hi)) and contains.
//
// range_map(start, end, f) is a search for the first element followed by a scan
// (Section "Packed Memory Array", "Design and operations"); in the CPMA the search
// runs on the uncompressed leaf heads and the scan decodes every leaf it passes
// (Section "Compressed Packed Memory Array", "Point queries").  A batch of
// queries becomes a flat list of leaf visits (query q visits leaves
// leaf(lo_q) .. leaf(hi_q - 1)).  The two end leaves of each query are scanned
// with comparisons by one lane per query; the interior leaves are flattened over
// all queries and split into fixed-size chunks, so long and short ranges balance
// across the GPU in one launch.
#pragma once
#include "scan_lane.hpp"
#include "update.hpp"
#include "kv.hpp"

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
  uint32_t raw;  // uncompressed leaves (raw 8-byte keys)
  // key-value leaves: `used` above is each leaf's code bytes, `fill` its filled
  // bytes (codes and values); vals: sum values instead of keys
  const uint32_t* fill;
  uint32_t vals;
  uint32_t zero_fill;  // bytes past `used` are zero in place (every set without values)
};

// The values of a key-value leaf (m = (fill - codes) / 8 words at its end).
__device__ __forceinline__ const uint64_t* leaf_vals(const QueryArgs& a, uint64_t leaf, uint32_t codes) {
  const uint32_t m = (a.fill[leaf] - codes) / 8;
  return reinterpret_cast<const uint64_t*>(a.bytes + leaf * (uint64_t)a.S + a.S - 8u * m);
}

// Keys of [lo, hi) in one leaf, one lane, for either leaf format.
__device__ __forceinline__ LeafSum leaf_range_any(const QueryArgs& a, uint64_t leaf, uint32_t used, uint64_t lo,
                                                  uint64_t hi) {
  const uint8_t* p = a.bytes + leaf * (uint64_t)a.S;
  if (a.vals) return kv_leaf_values(p, used, leaf_vals(a, leaf, used), lo, hi);
  return a.raw ? raw_sum_range(p, used, lo, hi) : leaf_sum_range(p, used, lo, hi);
}

// End leaves of every query (the leaf of lo and the leaf of hi - 1), scanned with
// comparisons by one lane per query; the result initialises sum / count.  The
// leaves strictly between them are the query's interior visits.
__global__ void __launch_bounds__(256) k_rm_ends(QueryArgs a, uint64_t* __restrict__ first_int,
                                                 uint64_t* __restrict__ nint,
                                                 unsigned long long* __restrict__ sum,
                                                 unsigned long long* __restrict__ count,
                                                 unsigned long long* __restrict__ alg) {
  uint64_t visited = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.q;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = a.lo[i], hi = a.hi[i];
    uint64_t f = 0, n = 0;
    LeafSum r{0, 0};
    if (lo < hi) {
      f = locate_leaf(a.head, a.L, lo);
      const uint64_t l = locate_leaf(a.head, a.L, hi - 1);
      const uint32_t uf = a.used[f];
      r = leaf_range_any(a, f, uf, lo, hi);
      visited += uf;
      if (l != f) {
        const uint32_t ul = a.used[l];
        const LeafSum r2 = leaf_range_any(a, l, ul, lo, hi);
        r.sum += r2.sum;
        r.count += r2.count;
        visited += ul;
      }
      n = (l > f + 1) ? l - f - 1 : 0;
    }
    first_int[i] = f + 1;
    nint[i] = n;
    sum[i] = r.sum;
    count[i] = r.count;
  }
  if (alg) {  // statistics: one slot per wave (no shared counter), summed by k_fold_sum
    const uint64_t t = wave_sum(visited);
    if (lane_id() == 0) alg[((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave] = t;
  }
}

// Few queries: one wave per query.  The leaf of a key comes from a 64-ary
// search of the heads (64 pivots compared per step, so a few steps for millions
// of leaves), and the two end leaves are decoded by the whole wave.
__device__ __forceinline__ uint64_t wave_locate_leaf(const uint64_t* __restrict__ head, uint64_t L, uint64_t x) {
  uint64_t lo = 0, hi = L;  // the first head above x lies in [lo, hi]
  const uint32_t lane = (uint32_t)lane_id();
  while (lo < hi) {
    const uint64_t step = (hi - lo + kWave - 1) / kWave;
    const uint64_t idx = lo + lane * step;
    const bool le = idx < hi && head[idx] <= x;
    const uint32_t t = (uint32_t)__popcll(__ballot(le));  // pivots at or below x form a prefix
    if (t == 0) {
      hi = lo;
    } else {
      const uint64_t last = lo + (uint64_t)(t - 1) * step;
      lo = last + 1;
      hi = min(hi, last + step);
    }
  }
  return lo ? lo - 1 : 0;
}

__device__ __forceinline__ LeafSum wave_leaf_sum_range(const uint8_t* __restrict__ leaf, uint32_t used, uint64_t lo,
                                                       uint64_t hi) {
  uint64_t s = 0, n = 0;
  wave_decode_leaf(leaf, used, [&](uint32_t, uint64_t k, uint64_t) {
    if (k >= lo && k < hi) {
      s += k;
      n++;
    }
  });
  return LeafSum{wave_sum(s), wave_sum(n)};
}

__global__ void __launch_bounds__(kWave) k_rm_ends_wave(QueryArgs a, uint64_t* __restrict__ first_int,
                                                        uint64_t* __restrict__ nint,
                                                        unsigned long long* __restrict__ sum,
                                                        unsigned long long* __restrict__ count,
                                                        unsigned long long* __restrict__ alg) {
  uint64_t visited = 0;
  for (uint64_t i = blockIdx.x; i < a.q; i += gridDim.x) {
    const uint64_t lo = a.lo[i], hi = a.hi[i];
    uint64_t f = 0, n = 0;
    LeafSum r{0, 0};
    if (lo < hi) {
      f = wave_locate_leaf(a.head, a.L, lo);
      const uint64_t l = wave_locate_leaf(a.head, a.L, hi - 1);
      const uint32_t uf = a.used[f];
      r = a.raw ? wave_raw_sum_range(a.bytes + f * (uint64_t)a.S, uf, lo, hi)
                : wave_leaf_sum_range(a.bytes + f * (uint64_t)a.S, uf, lo, hi);
      visited += uf;
      if (l != f) {
        const uint32_t ul = a.used[l];
        const LeafSum r2 = a.raw ? wave_raw_sum_range(a.bytes + l * (uint64_t)a.S, ul, lo, hi)
                                 : wave_leaf_sum_range(a.bytes + l * (uint64_t)a.S, ul, lo, hi);
        r.sum += r2.sum;
        r.count += r2.count;
        visited += ul;
      }
      n = (l > f + 1) ? l - f - 1 : 0;
    }
    if (lane_id() == 0) {
      first_int[i] = f + 1;
      nint[i] = n;
      sum[i] = r.sum;
      count[i] = r.count;
    }
  }
  if (alg && lane_id() == 0) alg[blockIdx.x] = visited;
}

// Sum and count of one interior leaf (a leaf every key of which is in its
// query's range), for any leaf format.
template <bool kPlain>
__device__ __forceinline__ LeafSum interior_leaf(const QueryArgs& a, uint64_t leaf, uint32_t u) {
  const uint8_t* lp = a.bytes + leaf * (uint64_t)a.S;
  const uint64_t h = a.head[leaf];
  const uint64_t span = a.head[leaf + 1] - h;  // interior leaves always have a successor
  if constexpr (kPlain) {
    return span < (1ull << 28) ? leaf_sum_zf(lp, u, h) : leaf_sum_range(lp, u, 0, kNoKey);
  } else {
    if (a.vals) {
      // the values: m 8-byte words ending at the leaf's end (8-byte aligned)
      const uint32_t m = (a.fill[leaf] - u) / 8;
      const uint64_t* w = reinterpret_cast<const uint64_t*>(lp + a.S - 8u * m);
      uint64_t s0 = 0, s1 = 0;
      uint32_t i = 0;
      for (; i + 2 <= m; i += 2) {
        s0 += w[i];
        s1 += w[i + 1];
      }
      if (i < m) s0 += w[i];
      return LeafSum{s0 + s1, m};
    }
    return a.raw                ? raw_sum_all(lp, u)
           : span >= (1ull << 28) ? leaf_sum_range(lp, u, 0, kNoKey)
                                  : leaf_sum_fast(lp, u, h);
  }
}

// Interior visits, flattened over all queries.  The visits are cut into steps
// of 64, and waves take groups of `chunk` consecutive steps, group g by wave
// g mod (number of waves).  At a step, lane l decodes visit base + l, so the
// wave's loads fall on 64 neighbouring leaves, and the waves running at the
// same time sweep one region of the leaf array together.  (Giving each lane
// `chunk` consecutive leaves instead spreads one load instruction over 64 *
// chunk leaves, and the memory system delivers markedly fewer bytes per second
// for that pattern.)  The query of a step's first visit is found by one binary
// search over the visit offsets, with wave-uniform (scalar) loads; each lane
// then walks forward to its own visit's query.  Partial sums are exact
// integers, so they may be combined in any order:
//  * while every lane's visit belongs to the same query, each lane adds its
//    leaf to a running share; the shares are summed across the wave and
//    flushed with one pair of 64-bit atomics when the query changes;
//  * a step whose lanes span several queries is reduced at once by query
//    (visits ascend with the lane, so equal queries sit in runs of lanes), one
//    pair of atomics per run -- a query spanning millions of leaves would
//    otherwise serialise on one address.
//
// kPlain: compressed leaves without values (zero past `used`), decoded with
// leaf_sum_zf; this instance also keeps the register count of the other
// formats' decoders out of the hot kernel.
template <bool kPlain>
__global__ void __launch_bounds__(256) k_rm_interior(QueryArgs a, const uint64_t* __restrict__ ioff,
                                                     const uint64_t* __restrict__ first_int, uint32_t chunk,
                                                     unsigned long long* __restrict__ sum,
                                                     unsigned long long* __restrict__ count,
                                                     unsigned long long* __restrict__ alg) {
  const uint64_t V = ioff[a.q];
  const uint64_t G = (uint64_t)kWave * chunk;
  const uint64_t ngroups = (V + G - 1) / G;
  const uint64_t nwaves = (uint64_t)gridDim.x * blockDim.x / kWave;
  const uint64_t wave = (uint64_t)__builtin_amdgcn_readfirstlane((int)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave));
  const int lane = lane_id();
  uint64_t visited = 0;
  uint64_t cq = ~0ull, cs = 0, cn = 0;  // carried query (wave-uniform) and this lane's share
  auto flush_carry = [&]() {
    if (cq != ~0ull) {
      const uint64_t ts = wave_sum<uint64_t>(cs), tn = wave_sum<uint64_t>(cn);
      if (lane == 0 && tn) {
        atomicAdd(&sum[cq], (unsigned long long)ts);
        atomicAdd(&count[cq], (unsigned long long)tn);
      }
    }
    cq = ~0ull;
    cs = cn = 0;
  };
  for (uint64_t g = wave; g < ngroups; g += nwaves) {
    const uint64_t Wend = min((g + 1) * G, V);
    for (uint64_t base = g * G; base < Wend; base += kWave) {
      const uint64_t v = base + lane;
      uint64_t vq = ~0ull, s = 0, n = 0;
      if (v < Wend) {
        uint64_t qi = upper_bound_u64(ioff, a.q + 1, base) - 1;
        while (ioff[qi + 1] <= v) qi++;
        vq = qi;
        const uint64_t leaf = first_int[qi] + (v - ioff[qi]);
        const uint32_t u = a.used[leaf];
        const LeafSum r = interior_leaf<kPlain>(a, leaf, u);
        s = r.sum;
        n = r.count;
        visited += u;
      }
      const uint64_t q0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(vq >> 32)) << 32) |
                          (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)vq);
      const bool uni = __ballot(vq != q0) == 0;
      if (uni && q0 == cq) {
        cs += s;
        cn += n;
        continue;
      }
      flush_carry();
      if (uni) {
        cq = q0;
        cs = s;
        cn = n;
        continue;
      }
      // several queries in this step: segmented inclusive scan over runs of equal vq
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t qu = __shfl_up(vq, d, kWave);
        const uint64_t su = __shfl_up(s, d, kWave);
        const uint64_t nu = __shfl_up(n, d, kWave);
        if (lane >= d && qu == vq) {
          s += su;
          n += nu;
        }
      }
      const uint64_t qn = __shfl_down(vq, 1, kWave);
      const bool run_end = lane == kWave - 1 || qn != vq;
      if (run_end && vq != ~0ull && n) {
        atomicAdd(&sum[vq], (unsigned long long)s);
        atomicAdd(&count[vq], (unsigned long long)n);
      }
    }
  }
  flush_carry();
  if (alg) {
    const uint64_t t = wave_sum(visited);
    if (lane_id() == 0) alg[((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave] = t;
  }
}

// Sum of n per-wave statistics slots, added to *out (one block).
__global__ void __launch_bounds__(1024) k_fold_sum(const unsigned long long* __restrict__ part, uint64_t n,
                                                   unsigned long long* out) {
  __shared__ uint64_t red[1024 / kWave];
  uint64_t t = 0;
  for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) t += part[i];
  t = wave_sum(t);
  if (lane_id() == 0) red[threadIdx.x / kWave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x / kWave); i++) t += red[i];
    atomicAdd(out, (unsigned long long)t);
  }
}

// Values of key-value leaves: one lane per key -- locate the leaf, walk its
// codes to the key; found[i] = whether it is present, val[i] its value (0 if not).
__global__ void __launch_bounds__(256) k_kv_get(QueryArgs a, const uint64_t* __restrict__ keys,
                                                uint64_t* __restrict__ val, uint8_t* __restrict__ found) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.q;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = keys[i];
    const uint64_t leaf = locate_leaf(a.head, a.L, x);
    const uint32_t codes = a.used[leaf];
    const LeafSum r = kv_leaf_values(a.bytes + leaf * (uint64_t)a.S, codes, leaf_vals(a, leaf, codes), x, x + 1);
    val[i] = r.sum;
    found[i] = r.count ? 1 : 0;
  }
}

// Membership: one lane per key -- locate the leaf, scan it for [x, x + 1).
__global__ void __launch_bounds__(256) k_contains(QueryArgs a, const uint64_t* __restrict__ keys,
                                                  uint8_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.q;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = keys[i];
    const uint64_t leaf = locate_leaf(a.head, a.L, x);
    const LeafSum r = leaf_range_any(a, leaf, a.used[leaf], x, x + 1);
    out[i] = r.count ? 1 : 0;
  }
}

}  // namespace cpma_dev
