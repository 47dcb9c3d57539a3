// One-wave merge of a long insert slice into its leaf (the batch-merge phase of
// Section "Parallel Batch Updates in a PMA" for slices too long for the
// one-key-per-lane wave merge or for one lane).
#pragma once
#include "update.hpp"

namespace cpma_dev {

// Heavy inserts: one wave merges one long insert slice into its leaf.  Each
// batch key is ranked among the old keys by binary search in LDS; an old key's
// output position is its index plus the number of new batch keys ranked at or
// below it (an LDS histogram of those ranks, scanned), so the slice is only
// streamed, twice.  The merged keys are built in LDS when at most ccap of them
// result, else in the HBM staging buffer, then encoded in place or into the
// arena.
constexpr uint32_t kHeavyLds = 2048;  // merged keys held in LDS beyond a full leaf's

// LDS of k_merge_heavy for leaf size S and merged-key room cap beyond a full
// leaf (byte offsets, each 16-byte aligned for even S): old keys A (a leaf
// holds at most S - 7 keys: an 8-byte head and one byte per further key),
// their presence flags F, the histogram N of the new batch keys' ranks, the
// encode buffer and, with cap > 0, ccap = S - 7 + cap merged keys.
struct HeavyLayout {
  uint32_t f, n, buf, c, ccap, total;
  __host__ __device__ HeavyLayout(uint32_t S, uint32_t cap) {
    const uint32_t maxA = S - 7;
    f = 8u * (maxA + 1);
    n = f + 4u * ((maxA + 4) & ~3u);
    buf = n + 4u * ((maxA + 4) & ~3u);
    c = buf + ((S + 15u) & ~15u);
    ccap = cap ? maxA + cap : 0u;
    total = c + 8u * ccap;
  }
};

// Places the new batch keys and the old keys into C (LDS or staging), then
// encodes C into the leaf.
__device__ __forceinline__ void heavy_place(const MergeArgs& a, uint32_t s, uint64_t leaf, const uint64_t* Bs,
                                            uint32_t nb, const uint64_t* A, const uint32_t* F, const uint32_t* N,
                                            uint32_t nA, uint64_t* C, uint32_t nC, uint8_t* buf, uint32_t used0,
                                            unsigned long long& alg) {
  const int lane = lane_id();
  for (uint32_t j = lane; j < nb; j += kWave) {
    const uint64_t x = Bs[j];
    const uint32_t r = lds_lower_bound(A, nA, x);
    if (!(r < nA && A[r] == x)) C[r + j - F[r]] = x;
  }
  // new batch keys before A[i]: those ranked at most i
  for (uint32_t i = lane; i < nA; i += kWave) C[i + N[i + 1]] = A[i];
  __threadfence_block();
  __syncthreads();
  const uint64_t written = wave_store_leaf(a, s, leaf, [&](uint32_t i) { return C[i]; }, nC, buf, used0);
  alg += used0 + written + 8ull * nb + 20;
}

__device__ __forceinline__ void heavy_slice(const MergeArgs& a, uint32_t s, uint8_t* smem, const HeavyLayout& lay,
                                            unsigned long long& delta, unsigned long long& alg) {
  const uint32_t S = a.S;
  const int lane = lane_id();
  uint64_t* A = reinterpret_cast<uint64_t*>(smem);
  uint32_t* F = reinterpret_cast<uint32_t*>(smem + lay.f);
  uint32_t* N = reinterpret_cast<uint32_t*>(smem + lay.n);
  uint8_t* buf = smem + lay.buf;
  const uint64_t leaf = a.seg_leaf[s];
  const uint32_t b = a.seg_begin[s];
  const uint32_t nb = a.seg_begin[s + 1] - b;
  const uint8_t* src = a.bytes + leaf * (uint64_t)S;
  const uint32_t used0 = a.used[leaf];
  const uint64_t* Bs = a.B + b;
  const uint32_t nA = wave_decode_leaf(src, used0, [&](uint32_t i, uint64_t x, uint64_t) { A[i] = x; });
  for (uint32_t i = lane; i <= nA; i += kWave) {
    F[i] = 0;
    N[i] = 0;
  }
  __syncthreads();
  for (uint32_t j = lane; j < nb; j += kWave) {
    const uint64_t x = Bs[j];
    const uint32_t r = lds_lower_bound(A, nA, x);
    if (r < nA && A[r] == x)
      F[r] = 1;
    else
      atomicAdd(&N[r], 1u);
  }
  __syncthreads();
  // exclusive scans: F[i] = batch keys already present among A[0, i),
  // N[i] = new batch keys whose rank among the old keys is below i
  wave_scan_inplace(F, nA + 1);
  wave_scan_inplace(N, nA + 1);
  __syncthreads();
  const uint32_t present = F[nA];
  const uint32_t nC = nA + nb - present;
  if (nC <= lay.ccap) {
    heavy_place(a, s, leaf, Bs, nb, A, F, N, nA, reinterpret_cast<uint64_t*>(smem + lay.c), nC, buf, used0, alg);
  } else {
    uint64_t off = 0;
    if (lane == 0) off = atomicAdd(&a.ctr->stage_cursor, (unsigned long long)nC);
    off = __shfl(off, 0, kWave);
    if (off + nC > a.stage_cap) {
      if (lane == 0) atomicOr(&a.ctr->error, 2u);
      return;
    }
    heavy_place(a, s, leaf, Bs, nb, A, F, N, nA, a.stage + off, nC, buf, used0, alg);
  }
  delta += nb - present;
  __syncthreads();
}

// Merges the slices of the heavy list (the lane merge's longest), or with
// from_spill those of the spill list (the wave merge's long inserts).
// Up to S - 7 + cap merged keys stay in LDS; the launch's dynamic LDS is
// HeavyLayout(S, cap).total.  Every block writes its {keys added, algorithmic
// bytes} slot of a.part.
__global__ void __launch_bounds__(kWave) k_merge_heavy(MergeArgs a, uint32_t cap, int from_spill) {
  extern __shared__ __align__(16) uint8_t smem[];
  const HeavyLayout lay(a.S, cap);
  const uint32_t n = from_spill ? a.ctr->nspill : a.ctr->heavy;
  const uint32_t* list = from_spill ? a.spill_list : a.heavy_list;
  unsigned long long delta = 0, alg = 0;
  for (uint32_t h = blockIdx.x; h < n; h += gridDim.x) {
    const uint32_t s = list[h];
    heavy_slice(a, s, smem, lay, delta, alg);
  }
  if (lane_id() == 0) {
    a.part[2 * blockIdx.x] = delta;
    a.part[2 * blockIdx.x + 1] = alg;
  }
}

}  // namespace cpma_dev
