// One pass over a sequence of insert / delete requests (serving).
//
// The paper applies one batch of inserts or of deletes at a time (Section
// "Parallel Batch Updates in a PMA"), and a single writer applies its batches
// in order (Section "Evaluation on graph workloads").  A sequence of requests
// reduces to at most one delete batch and one insert batch with the same final
// set, and every request's count (keys it added or removed, as its own call
// would return) follows from one stable sort of all their keys:
//   * after a key's first operation in the sequence its state no longer depends
//     on the set: an insert leaves it present, a delete absent;
//   * so a later occurrence changes the key iff its kind differs from the
//     previous occurrence's, and the first changes it iff its kind differs from
//     the key's membership before the sequence;
//   * the final state follows the last occurrence's kind.
// Items are (key, value) with value = position in the concatenated requests |
// delete bit << 31; a stable sort by key keeps each key's occurrences in
// request order.
#pragma once
#include "query.hpp"

namespace cpma_dev {

// Kind byte (0 insert, 1 delete) of every position; one block per request.
__global__ void __launch_bounds__(256) k_fuse_kinds(const uint64_t* __restrict__ off,
                                                    const uint8_t* __restrict__ rdel, uint32_t nreq,
                                                    uint8_t* __restrict__ kinds) {
  for (uint32_t r = blockIdx.x; r < nreq; r += gridDim.x) {
    const uint8_t k = rdel[r];
    const uint64_t e = off[r + 1];
    for (uint64_t i = off[r] + threadIdx.x; i < e; i += blockDim.x) kinds[i] = k;
  }
}

// Membership before the sequence of each distinct key (nd of them, on the device).
__global__ void __launch_bounds__(256) k_fuse_member(QueryArgs a, const uint64_t* __restrict__ keys,
                                                     const unsigned long long* __restrict__ nd,
                                                     uint8_t* __restrict__ member) {
  const uint64_t q = *nd;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = keys[i];
    const uint64_t leaf = locate_leaf(a.head, a.L, x);
    const LeafSum r = leaf_sum_range(a.bytes + leaf * (uint64_t)a.S, a.used[leaf], x, x + 1);
    member[i] = r.count ? 1 : 0;
  }
}

// The same per leaf for large batches: leaf f's distinct keys are
// keys[sbeg[f] .. sbeg[f + 1]); one wave decodes the leaf once into LDS
// (dynamic, 8 bytes per possible key: S - 7 codes plus the head) and binary-
// searches each of them there.
__global__ void __launch_bounds__(kWave) k_fuse_member_leaf(QueryArgs a, const uint64_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ sbeg,
                                                            uint8_t* __restrict__ member) {
  extern __shared__ uint64_t K[];
  for (uint64_t f = blockIdx.x; f < a.L; f += gridDim.x) {
    const uint32_t b = sbeg[f], e = sbeg[f + 1];
    if (b == e) continue;
    const uint32_t u = a.used[f];
    const uint32_t nk =
        wave_decode_leaf(a.bytes + f * (uint64_t)a.S, u, [&](uint32_t i, uint64_t x, uint64_t) { K[i] = x; });
    __syncthreads();
    for (uint32_t j = b + lane_id(); j < e; j += kWave) {
      const uint64_t x = keys[j];
      uint32_t lo = 0, hi = nk;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (K[mid] < x)
          lo = mid + 1;
        else
          hi = mid;
      }
      member[j] = (lo < nk && K[lo] == x) ? 1 : 0;
    }
    __syncthreads();
  }
}

// Gather of requests that live in device memory: request r's n keys from src
// to out[dst ..); one block per request.
struct GatherReq {
  const uint64_t* src;
  uint64_t dst;
  uint64_t n;
};

__global__ void __launch_bounds__(256) k_fuse_gather(const GatherReq* __restrict__ t, uint32_t nreq,
                                                     uint64_t* __restrict__ out) {
  for (uint32_t r = blockIdx.x; r < nreq; r += gridDim.x) {
    const GatherReq g = t[r];
    for (uint64_t i = threadIdx.x; i < g.n; i += blockDim.x) out[g.dst + i] = g.src[i];
  }
}

// Per sorted item: whether its request changes the key (credit, stored at the
// item's position), and per distinct key the net change of the whole sequence
// (code 1: absent before, present after; 2: present before, absent after; 0:
// unchanged).  dpos is the exclusive count of first occurrences.
__global__ void __launch_bounds__(256) k_fuse_credit(const uint64_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ vals, uint64_t m,
                                                     const uint32_t* __restrict__ dpos,
                                                     const uint8_t* __restrict__ member,
                                                     uint8_t* __restrict__ credit, uint8_t* __restrict__ code) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = keys[i];
    const uint32_t v = vals[i];
    const uint32_t del = v >> 31;
    const bool first = i == 0 || keys[i - 1] != x;
    const uint32_t d = first ? dpos[i] : dpos[i] - 1u;
    const uint32_t was = member[d];
    // state before this item, as "absent" (the delete bit a previous item
    // would have had)
    const uint32_t prev_del = first ? (was ^ 1u) : (vals[i - 1] >> 31);
    credit[v & 0x7fffffffu] = (uint8_t)(del != prev_del);
    if (i + 1 == m || keys[i + 1] != x) code[d] = (uint8_t)(del ? (was ? 2 : 0) : (was ? 0 : 1));
  }
}

// Packed (insert, delete) flags of distinct key i: low word insert, high word
// delete; zero past nd.
struct FuseSplitFn {
  const uint8_t* code;
  const unsigned long long* nd;
  __device__ uint64_t operator()(uint64_t i) const {
    if (i >= *nd) return 0;
    const uint32_t c = code[i];
    return (uint64_t)(c == 1) | ((uint64_t)(c == 2) << 32);
  }
};

// Writes the net insert and delete batches (sorted, repeat-free) and their
// sizes (cnt[1] inserts, cnt[2] deletes).
__global__ void __launch_bounds__(256) k_fuse_split(const uint64_t* __restrict__ dkeys,
                                                    const uint8_t* __restrict__ code,
                                                    const uint64_t* __restrict__ pos,
                                                    uint64_t* __restrict__ ins, uint64_t* __restrict__ del,
                                                    unsigned long long* __restrict__ cnt) {
  const uint64_t nd = cnt[0];
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t c = code[i];
    if (c == 1) ins[(uint32_t)pos[i]] = dkeys[i];
    if (c == 2) del[pos[i] >> 32] = dkeys[i];
    if (i == 0) {
      cnt[1] = (uint32_t)pos[nd];
      cnt[2] = pos[nd] >> 32;
    }
  }
}

// Request owning position p: the r with off[r] <= p < off[r + 1].
__device__ __forceinline__ uint32_t fuse_req_of(const uint64_t* off, uint32_t nreq, uint64_t p) {
  uint32_t lo = 0, hi = nreq + 1;  // first index with off[idx] > p, minus one
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= p)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo - 1;
}

// Sum of the credit bytes of every request (positions are request-contiguous).
// A wave takes 1024 consecutive positions: one wave sum and one atomic when
// they belong to one request, else a run-length walk per lane over its 16.
__global__ void __launch_bounds__(256) k_fuse_reduce(const uint8_t* __restrict__ credit, uint64_t m,
                                                     const uint64_t* __restrict__ off, uint32_t nreq,
                                                     unsigned long long* __restrict__ res) {
  constexpr uint32_t kChunk = 16 * kWave;
  const int lane = lane_id();
  const uint64_t nchunks = (m + kChunk - 1) / kChunk;
  const uint64_t wstride = (uint64_t)gridDim.x * (blockDim.x / kWave);
  for (uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; w < nchunks; w += wstride) {
    const uint64_t b = w * kChunk, e = min(b + kChunk, m);
    const uint32_t r0 = fuse_req_of(off, nreq, b), r1 = fuse_req_of(off, nreq, e - 1);
    if (r0 == r1) {
      uint32_t c = 0;
#pragma unroll
      for (uint32_t j = 0; j < 16; j++) {
        const uint64_t p = b + j * kWave + lane;
        if (p < e) c += credit[p];
      }
      c = wave_sum(c);
      if (lane == 0 && c) atomicAdd(&res[r0], (unsigned long long)c);
    } else {
      const uint64_t p0 = b + (uint64_t)lane * 16;
      if (p0 < e) {
        const uint64_t p1 = min(p0 + 16, e);
        uint32_t r = fuse_req_of(off, nreq, p0);
        uint64_t end = off[r + 1];
        uint32_t acc = 0;
        for (uint64_t p = p0; p < p1; p++) {
          while (p >= end) {
            if (acc) atomicAdd(&res[r], (unsigned long long)acc);
            acc = 0;
            r++;
            end = off[r + 1];
          }
          acc += credit[p];
        }
        if (acc) atomicAdd(&res[r], (unsigned long long)acc);
      }
    }
  }
}

}  // namespace cpma_dev
