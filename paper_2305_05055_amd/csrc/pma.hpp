// Batch merge of the uncompressed variant (the plain PMA): one wave per touched
// leaf, any slice length (the batch-merge phase of Section "Parallel Batch
// Updates in a PMA" on leaves of raw 8-byte keys packed to the left).
//
// The wave copies the leaf's keys to LDS.  Insert: every batch key of the
// slice finds its rank among the old keys by binary search; a key already
// present is dropped; a new key lands at rank + (new keys before it), and each
// new key adds one to the shift of the old keys from its rank on (LDS counts,
// then one prefix sum), so old key i lands at i + shift(i).  Delete: every
// batch key found flags its old key; kept keys move down by the flags before
// them.  The merged leaf is written in place when it fits S bytes, else to the
// segment's overflow-arena region, which the redistribution then reads.
#pragma once
#include "update.hpp"

namespace cpma_dev {

constexpr uint32_t kPmaMaxKeys = 4096 / 8;  // keys of the largest leaf (4 KiB)

__global__ void __launch_bounds__(kWave) k_pma_merge(MergeArgs a) {
  __shared__ uint64_t A[kPmaMaxKeys];        // old keys
  __shared__ uint32_t C[kPmaMaxKeys + 1];    // insert: new keys per rank; delete: removal flags
  const int lane = lane_id();
  const uint32_t S = a.S;
  const uint64_t T = a.ctr->T;
  unsigned long long delta = 0, alg = 0;
  for (uint64_t t = blockIdx.x; t < T; t += gridDim.x) {
    const uint4 d = a.seg_desc[t];
    const uint64_t leaf = d.x;
    const uint32_t b = d.y, e = a.seg_begin[t + 1];
    const uint32_t nb = e - b;
    const uint32_t used0 = d.z, nA = used0 / 8;
    const uint64_t* src = reinterpret_cast<const uint64_t*>(a.bytes + leaf * (uint64_t)S);
    for (uint32_t i = lane; i < nA; i += kWave) A[i] = src[i];
    for (uint32_t i = lane; i <= nA; i += kWave) C[i] = 0;
    __syncthreads();
    const uint64_t* Bs = a.B + b;
    uint32_t nout = 0;
    uint64_t first_key = kNoKey;
    if (a.is_insert) {
      // count the new keys first: the destination depends on the total
      uint32_t nnew = 0;
      for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
        const uint32_t j = c0 + lane;
        bool isnew = false;
        if (j < nb) {
          const uint64_t x = Bs[j];
          const uint32_t r = lds_lower_bound<uint64_t>(A, nA, x);
          isnew = !(r < nA && A[r] == x);
          if (isnew) atomicAdd(&C[r], 1u);
        }
        nnew += (uint32_t)__popcll(__ballot(isnew));
      }
      nout = nA + nnew;
      __syncthreads();
      const uint32_t U = 8 * nout;
      uint64_t* dst = reinterpret_cast<uint64_t*>(a.bytes + leaf * (uint64_t)S);
      bool to_arena = false;
      uint64_t off = 0;
      if (U > S) {
        off = arena_region(a, t);
        if (off + U > a.arena_cap) {
          if (lane == 0) atomicOr(&a.ctr->error, 1u);
          __syncthreads();
          continue;
        }
        dst = reinterpret_cast<uint64_t*>(a.arena + off);
        to_arena = true;
      }
      // new keys: rank + new keys before them (a running count across chunks)
      uint32_t before = 0;
      uint64_t firstnew = kNoKey;
      for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
        const uint32_t j = c0 + lane;
        bool isnew = false;
        uint64_t x = 0;
        uint32_t r = 0;
        if (j < nb) {
          x = Bs[j];
          r = lds_lower_bound<uint64_t>(A, nA, x);
          isnew = !(r < nA && A[r] == x);
        }
        const uint64_t m = __ballot(isnew);
        if (isnew) dst[r + before + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = x;
        if (m && firstnew == kNoKey) {
          const int fl = __ffsll((unsigned long long)m) - 1;
          firstnew = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), fl) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, fl);
        }
        before += (uint32_t)__popcll(m);
      }
      // old keys: i + (new keys at ranks <= i), from a running prefix over C
      uint32_t carry = 0;
      for (uint32_t c0 = 0; c0 < nA; c0 += kWave) {
        const uint32_t i = c0 + lane;
        const uint32_t cv = i < nA ? C[i] : 0u;
        const uint32_t incl = wave_incl_scan(cv);
        if (i < nA) dst[i + carry + incl] = A[i];
        carry += lane63_u32(incl);
      }
      first_key = nA ? min(A[0], firstnew) : firstnew;
      delta += nnew;
      if (lane == 0) {
        if (to_arena) a.ovf[leaf] = off;
        a.used[leaf] = U;
        a.head[leaf] = U ? first_key : kNoKey;
      }
      alg += used0 + U + 8ull * nb + 20;
    } else {
      for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
        const uint32_t j = c0 + lane;
        if (j < nb) {
          const uint64_t x = Bs[j];
          const uint32_t r = lds_lower_bound<uint64_t>(A, nA, x);
          if (r < nA && A[r] == x) C[r] = 1u;  // slices are repeat-free: one writer per key
        }
      }
      __syncthreads();
      uint64_t* dst = reinterpret_cast<uint64_t*>(a.bytes + leaf * (uint64_t)S);
      uint32_t gone = 0;
      for (uint32_t c0 = 0; c0 < nA; c0 += kWave) {
        const uint32_t i = c0 + lane;
        const bool g = i < nA && C[i];
        const uint64_t gm = __ballot(g);
        const bool keep = i < nA && !g;
        const uint64_t km = __ballot(keep);
        if (keep) dst[i - gone - (uint32_t)__popcll(gm & ((1ull << lane) - 1ull))] = A[i];
        if (km && first_key == kNoKey) first_key = A[c0 + (uint32_t)(__ffsll((unsigned long long)km) - 1)];
        gone += (uint32_t)__popcll(gm);
      }
      nout = nA - gone;
      // zero the freed tail of the leaf
      for (uint32_t i = nout + lane; i < nA; i += kWave) dst[i] = 0;
      delta += gone;
      if (lane == 0) {
        a.used[leaf] = 8 * nout;
        a.head[leaf] = nout ? first_key : kNoKey;
      }
      alg += 2ull * used0 + 8ull * nb + 20;
    }
    __syncthreads();  // A and C are refilled by the next segment
  }
  if (lane == 0) {
    a.part[2 * blockIdx.x] = delta;
    a.part[2 * blockIdx.x + 1] = alg;
  }
}

}  // namespace cpma_dev
