// Resize by a direct split of the old leaves (Section "Packed Memory Array",
// "Resizing a PMA", with the even spread of the redistribution phase in
// "Parallel Batch Updates in a PMA"): the whole key sequence moves into a fresh
// array of Lt leaves straight from the old leaf images, with no staged keys.
//
// The old leaves hold the key sequence as one delta chain that restarts at each
// leaf head.  The chain cost of a key is the code length of its distance to the
// previous key (8 bytes for the very first key).  A leaf's chain bytes are its
// used bytes with the 8-byte head replaced by the head's chain cost hc; their
// exclusive prefix CP over leaf ids (empty leaves add 0) gives the chain prefix
// P of any key without decoding: CP[f] for the head of leaf f, and
// CP[f] + hc_f + p - 8 for the code that starts at byte p of leaf f.
//
// Destination leaf j takes the keys with floor(P * Lt / total) == j, so it
// starts at the first key with P >= T_j = ceil(j * total / Lt).  Its image is
// the old bytes from that key up to the next destination leaf's first key, with
// the first key rewritten as an 8-byte head and every old head in between
// rewritten as the code of its distance to the key before it: a spliced byte
// copy, the same layout as the staged spread produces.
#pragma once
#include "leaf.hpp"
#include "update.hpp"

namespace cpma_dev {

// First key of a destination leaf.
struct SplitRec {
  uint64_t leaf;  // old leaf holding it; L marks the end of the sequence
  uint64_t x;     // the key
  uint64_t P;     // its chain prefix (total at the end)
  uint32_t p;     // byte where its code starts in the old leaf (0: the old head)
  uint32_t cost;  // its chain cost
};

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, d, kWave));
  return v;
}

// lastk[f] = last key of every non-empty old leaf (the sum of all its deltas).
__global__ void __launch_bounds__(kWave) k_leaf_last(SrcLeaves src, uint64_t L, uint64_t* __restrict__ lastk) {
  for (uint64_t f = blockIdx.x; f < L; f += gridDim.x) {
    const uint32_t u = src.used[f];
    if (u == 0) continue;
    uint64_t sum = 0;
    wave_decode_leaf(src.ptr(f, u), u, [&](uint32_t, uint64_t, uint64_t d) { sum += d; });
    sum = wave_sum(sum);
    if (lane_id() == 0) lastk[f] = sum;
  }
}

struct NonEmptyFn {
  const uint32_t* used;
  __device__ uint32_t operator()(uint64_t f) const { return used[f] != 0 ? 1u : 0u; }
};

// ne[r] = id of the r-th non-empty old leaf; ne[M] = L closes the list.
__global__ void k_ne_compact(const uint32_t* __restrict__ used, const uint32_t* __restrict__ rank, uint64_t L,
                             uint32_t* __restrict__ ne) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f <= L;
       f += (uint64_t)gridDim.x * blockDim.x) {
    if (f == L)
      ne[rank[L]] = (uint32_t)L;
    else if (used[f] != 0)
      ne[rank[f]] = (uint32_t)f;
  }
}

// Chain bytes of old leaf f (0 when empty).
struct ChainFn {
  const uint32_t* used;
  const uint64_t* head;
  const uint64_t* lastk;
  const uint32_t* rank;
  const uint32_t* ne;
  __device__ uint64_t operator()(uint64_t f) const {
    const uint32_t u = used[f];
    if (u == 0) return 0;
    const uint32_t r = rank[f];
    const uint32_t hc = r == 0 ? 8u : vlen(head[f] - lastk[ne[r - 1]]);
    return (uint64_t)hc + u - 8u;
  }
};

struct SplitArgs {
  SrcLeaves src;
  const uint64_t* head;   // old heads
  const uint64_t* lastk;  // old last keys
  const uint32_t* rank;   // non-empty rank of each old leaf
  const uint32_t* ne;     // non-empty old leaf ids, closed by L
  const uint64_t* CP;     // L + 1 entries
  uint64_t L;             // old leaves
  uint64_t Lt;            // destination leaves
};

// rec[j] for j in [0, Lt]: the first key of destination leaf j (rec[Lt] = end).
__global__ void __launch_bounds__(kWave) k_split_locate(SplitArgs a, SplitRec* __restrict__ rec) {
  const uint64_t total = a.CP[a.L];
  const uint64_t q = total / a.Lt, rem = total % a.Lt;
  for (uint64_t j = blockIdx.x; j <= a.Lt; j += gridDim.x) {
    SplitRec R;
    R.leaf = a.L;
    R.x = 0;
    R.P = total;
    R.p = 0;
    R.cost = 0;
    bool mine = lane_id() == 0;
    // T = ceil(j * total / Lt) without a 128-bit product (j * rem < Lt^2)
    const uint64_t T = (j == a.Lt) ? total : j * q + (j * rem + a.Lt - 1) / a.Lt;
    if (T < total) {
      // CP[f] <= T < CP[f + 1]: leaf f is not empty
      const uint64_t f = upper_bound_u64(a.CP, a.L + 1, T) - 1;
      const uint32_t u = a.src.used[f];
      const uint64_t hc = a.CP[f + 1] - a.CP[f] - (u - 8u);
      uint64_t hf = f;  // leaf whose head is the key, if it is a head
      if (a.CP[f] != T) {
        hf = a.L;
        // first code that starts at byte >= b
        const uint64_t over = T - a.CP[f];
        const uint32_t b = over <= hc ? 8u : (uint32_t)(over - hc + 8u);
        uint32_t best = 0xffffffffu, bc = 0;
        uint64_t bx = 0;
        wave_decode_leaf(a.src.ptr(f, u), u, [&](uint32_t idx, uint64_t key, uint64_t d, uint32_t end) {
          if (idx == 0) return;
          const uint32_t len = vlen(d);
          const uint32_t start = end + 1u - len;
          if (start >= b && start < best) {
            best = start;
            bx = key;
            bc = len;
          }
        });
        const uint32_t bmin = wave_min_u32(best);
        if (bmin != 0xffffffffu) {
          mine = best == bmin;
          R.leaf = f;
          R.x = bx;
          R.P = a.CP[f] + hc + bmin - 8u;
          R.p = bmin;
          R.cost = bc;
        } else if (a.CP[f + 1] < total) {
          // no code of leaf f qualifies: the head of the next non-empty leaf
          hf = a.ne[a.rank[f] + 1];
        }
      }
      if (hf < a.L) {
        const uint32_t uf = a.src.used[hf];
        R.leaf = hf;
        R.x = a.head[hf];
        R.P = a.CP[hf];
        R.p = 0;
        R.cost = (uint32_t)(a.CP[hf + 1] - a.CP[hf] - (uf - 8u));
      }
    }
    if (mine) rec[j] = R;
  }
}

// Planned bytes of every destination leaf and its leaf-level check (an empty
// destination leaf fails as below its lower bound).
__global__ void k_split_plan(Bounds dstb, uint64_t Lt, const SplitRec* __restrict__ rec,
                             uint32_t* __restrict__ plan_used, uint32_t* __restrict__ fail) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < Lt;
       j += (uint64_t)gridDim.x * blockDim.x) {
    const SplitRec& A = rec[j];
    const uint64_t Pb = rec[j + 1].P;
    uint64_t U = 0;
    uint32_t v = 2u;
    if (A.P < Pb) {
      U = 8u + (Pb - A.P - A.cost);
      v = violation(dstb, 0, U, 1);
      if (U > dstb.S) v |= 1u;
    }
    if (v) atomicOr(fail, v);
    plan_used[j] = (uint32_t)(U > 0xffffffffull ? 0xffffffffull : U);
  }
}

// dst[i - bs] = src[i] for i in [bs, be), one wave; src is 16-byte aligned and
// readable in whole 16-byte chunks below round16(be); writes stop at dst_cap.
__device__ __forceinline__ void wave_copy_bytes(uint8_t* dst, uint32_t dst_cap, const uint8_t* __restrict__ src,
                                                uint32_t bs, uint32_t be) {
  for (uint32_t base = bs & ~15u; base < be; base += 16u * kWave) {
    const uint32_t p0 = base + 16u * lane_id();
    if (p0 < be) {
      const uint4 w = *reinterpret_cast<const uint4*>(src + p0);
      const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int k = 0; k < 16; k++) {
        const uint32_t i = p0 + (uint32_t)k;
        if (i >= bs && i < be && i - bs < dst_cap) dst[i - bs] = (uint8_t)(words[k >> 2] >> (8 * (k & 3)));
      }
    }
  }
}

// Writes destination leaf j from the old images (a planned split: no leaf is
// empty or above S bytes).  A length that disagrees with the plan sets the
// error counter.
__global__ void __launch_bounds__(kWave) k_split_write(SplitArgs a, uint32_t S, const SplitRec* __restrict__ rec,
                                                       uint8_t* __restrict__ dbytes, uint32_t* __restrict__ dused,
                                                       uint64_t* __restrict__ dhead, Counters* ctr) {
  extern __shared__ __align__(16) uint8_t buf[];
  for (uint64_t j = blockIdx.x; j < a.Lt; j += gridDim.x) {
    const SplitRec A = rec[j], B = rec[j + 1];
    wave_zero(buf, S);
    __syncthreads();
    if (lane_id() == 0) put_le64(buf, A.x);
    uint32_t pos = 8;
    uint64_t f = A.leaf;
    uint32_t bs = A.p == 0 ? 8u : A.p + A.cost;
    bool bad = f >= a.L;
    while (!bad) {
      const uint32_t u = a.src.used[f];
      const bool last = f == B.leaf;  // the end lies inside leaf f (B.p >= 8)
      const uint32_t be = last ? B.p : u;
      if (be < bs || be > u) {
        bad = true;
        break;
      }
      wave_copy_bytes(buf + min(pos, S), S - min(pos, S), a.src.ptr(f, u), bs, be);
      pos += be - bs;
      if (last) break;
      const uint64_t fn = a.ne[a.rank[f] + 1];
      if (fn >= a.L || (fn == B.leaf && B.p == 0)) break;
      const uint64_t d = a.head[fn] - a.lastk[f];
      const uint32_t len = vlen(d);
      if (lane_id() == 0 && pos + len <= S) vput(buf + pos, d);
      pos += len;
      f = fn;
      bs = 8;
    }
    __syncthreads();
    const uint64_t want = 8u + (B.P - A.P - A.cost);
    if (bad || pos != want || pos > S) {
      if (lane_id() == 0) atomicOr(&ctr->error, 1u);
    } else {
      wave_copy16(dbytes + j * (uint64_t)S, buf, S);
      if (lane_id() == 0) {
        dused[j] = pos;
        dhead[j] = A.x;
      }
    }
    __syncthreads();
  }
}

}  // namespace cpma_dev
