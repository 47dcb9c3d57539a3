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
#include "scan_lane.hpp"
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

// Last key of a leaf: the head plus every delta.  Narrow form (every delta below
// 2^28): the range scan's lane decoder, which ends on the last key.
__device__ __forceinline__ uint64_t leaf_last_narrow(const uint8_t* __restrict__ leaf, uint32_t used,
                                                     uint64_t head) {
  uint64_t last = head;
  leaf_sum_fast(leaf, used, head, &last);
  return last;
}

__device__ __forceinline__ uint64_t leaf_last_wide(const uint8_t* __restrict__ leaf, uint32_t used, uint64_t head) {
  uint64_t last = head;
  uint32_t sh = 0;
  for (uint32_t c = 0; c < used; c += 16) {
    const uint4 cur = load16(leaf + c);
    const uint32_t words[4] = {cur.x, cur.y, cur.z, cur.w};
    const uint32_t nvalid = min(16u, used - c);
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t b = (words[i >> 2] >> (8 * (i & 3))) & 0xffu;
      const bool valid = (uint32_t)i < nvalid && !(c == 0 && i < 8);
      if (valid) {
        if (sh < 64) last += (uint64_t)(b & 0x7fu) << sh;
        sh = (b & 0x80u) ? sh + 7u : 0u;
      }
    }
  }
  return last;
}

// lastk[f] = last key of every non-empty old leaf.  head[f + 1] bounds the keys
// of leaf f from above (an empty leaf keeps a head above every earlier key), so
// a span below 2^28 selects the narrow decoder.
__global__ void __launch_bounds__(256) k_leaf_last(SrcLeaves src, const uint64_t* __restrict__ head, uint64_t L,
                                                   uint64_t* __restrict__ lastk) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < L;
       f += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = src.used[f];
    if (u == 0) continue;
    const uint64_t h = head[f];
    const uint64_t nx = f + 1 < L ? head[f + 1] : ~0ull;
    const uint8_t* p = src.ptr(f, u);
    lastk[f] = (nx > h && nx - h < (1ull << 28)) ? leaf_last_narrow(p, u, h) : leaf_last_wide(p, u, h);
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

// Per old leaf, what the writer needs when it walks from one source leaf to the
// next: one 32-byte load per hop instead of a chain of dependent loads.
struct SrcInfo {
  uint64_t head;
  uint64_t lastk;
  uint32_t used;
  uint32_t next;  // next non-empty old leaf (L after the last)
  uint64_t pad;
};

__global__ void k_src_info(const uint32_t* __restrict__ used, const uint64_t* __restrict__ head,
                           const uint64_t* __restrict__ lastk, const uint32_t* __restrict__ rank,
                           const uint32_t* __restrict__ ne, uint64_t L, SrcInfo* __restrict__ info) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < L;
       f += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = used[f];
    if (u == 0) continue;
    SrcInfo I;
    I.head = head[f];
    I.lastk = lastk[f];
    I.used = u;
    I.next = ne[rank[f] + 1];
    I.pad = 0;
    info[f] = I;
  }
}

struct SplitArgs {
  SrcLeaves src;
  const SrcInfo* info;
  const uint64_t* head;   // old heads
  const uint64_t* lastk;  // old last keys
  const uint32_t* rank;   // non-empty rank of each old leaf
  const uint32_t* ne;     // non-empty old leaf ids, closed by L
  const uint64_t* CP;     // L + 1 entries
  uint64_t L;             // old leaves
  uint64_t Lt;            // destination leaves
};

// ceil(j * total / Lt); the caller guarantees total * Lt < 2^63.
__device__ __forceinline__ uint64_t split_threshold(uint64_t j, uint64_t total, uint64_t Lt) {
  return (j * total + Lt - 1) / Lt;
}

__device__ __forceinline__ void put_rec(SplitRec* rec, uint64_t j, uint64_t leaf, uint64_t x, uint64_t P, uint32_t p,
                                        uint32_t cost) {
  SplitRec R;
  R.leaf = leaf;
  R.x = x;
  R.P = P;
  R.p = p;
  R.cost = cost;
  rec[j] = R;
}

// rec[j] for j in [0, Lt]: the first key of destination leaf j (rec[Lt] = end).
// One lane per old leaf f writes the records of the thresholds in
// [CP[f], CP[f + 1]): j from floor((CP[f] - 1) Lt / total) + 1 (0 when
// CP[f] = 0) up to, excluding, the same bound for CP[f + 1].  Thresholds past
// the last code of f fall on the head of the next non-empty leaf.
__global__ void __launch_bounds__(256) k_split_locate(SplitArgs a, SplitRec* __restrict__ rec) {
  const uint64_t total = a.CP[a.L];
  const uint64_t Lt = a.Lt;
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < a.L;
       f += (uint64_t)gridDim.x * blockDim.x) {
    if (f == 0) {
      // thresholds at or past the total: the end record
      for (uint64_t j = (total - 1) * Lt / total + 1; j <= Lt; j++) put_rec(rec, j, a.L, 0, total, 0, 0);
    }
    const uint32_t u = a.src.used[f];
    if (u == 0) continue;
    const uint64_t c0 = a.CP[f], c1 = a.CP[f + 1];
    uint64_t j = c0 == 0 ? 0 : (c0 - 1) * Lt / total + 1;
    const uint64_t jend = (c1 - 1) * Lt / total + 1;
    if (j >= jend) continue;
    const uint32_t hc = (uint32_t)(c1 - c0 - (u - 8u));
    const uint64_t h = a.head[f];
    uint64_t T = split_threshold(j, total, Lt);
    if (T == c0) {
      put_rec(rec, j, f, h, c0, 0, hc);
      j++;
      T = split_threshold(j, total, Lt);
    }
    if (j >= jend) continue;
    const uint8_t* leaf = a.src.ptr(f, u);
    const uint64_t nx = f + 1 < a.L ? a.head[f + 1] : ~0ull;
    if (nx > h && nx - h < (1ull << 28)) {
      // narrow leaf (every delta below 2^28): 32-bit walk with the next chunk in
      // flight; bytes past `used` become payload-free continuation bytes and the
      // head a zero terminator, as in the range scan's decoder.  The code that
      // starts at byte s (s >= 8) reaches threshold T when s >= T - c0 - hc + 8.
      auto first_byte = [&](uint64_t t) -> uint32_t {
        const uint64_t over = t - c0;
        return over <= hc ? 8u : (uint32_t)min<uint64_t>(over - hc + 8u, 0xffffffffull);
      };
      uint32_t bp = first_byte(T);
      uint32_t key32 = 0, acc = 0, sh = 0, start = 0;
      uint4 nxt = load16(leaf);
      for (uint32_t c = 0; c < u && j < jend; c += 16) {
        const uint4 cur = nxt;
        if (c + 16 < u) nxt = load16(leaf + c + 16);
        uint32_t w[4] = {cur.x, cur.y, cur.z, cur.w};
        if (c == 0) {
          w[0] = 0x80808080u;
          w[1] = 0x00808080u;
        }
        const int32_t nv = (int32_t)u - (int32_t)c;
        if (nv < 16) {
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const int32_t v = nv - 4 * k;
            const uint32_t keep = v >= 4 ? 0xffffffffu : (v <= 0 ? 0u : ((1u << (8 * v)) - 1u));
            w[k] = (w[k] & keep) | (0x80808080u & ~keep);
          }
        }
#pragma unroll
        for (int i = 0; i < 16; i++) {
          const uint32_t x = w[i >> 2];
          const int o = 8 * (i & 3);
          const uint32_t cm = 0u - ((x >> (o + 7)) & 1u);  // all ones on a continuation byte
          acc |= ((x >> o) & 0x7fu) << (sh & 31u);
          key32 += acc & ~cm;
          if (!cm && start >= 8u && start >= bp && j < jend) {
            const uint32_t end = c + (uint32_t)i;
            const uint64_t P = c0 + hc + start - 8u;
            do {
              put_rec(rec, j, f, h + key32, P, start, end + 1u - start);
              j++;
              T = split_threshold(j, total, Lt);
              bp = first_byte(T);
            } while (j < jend && start >= bp);
          }
          acc &= cm;
          start = cm ? start : c + (uint32_t)i + 1u;
          sh = (sh + 7u) & cm;
        }
      }
    } else {
    // walk the codes of f: the code starting at byte s has chain prefix c0 + hc + s - 8
    uint64_t key = h, acc = 0;
    uint32_t sh = 0, start = 8;
    for (uint32_t c = 0; c < u && j < jend; c += 16) {
      const uint4 cur = load16(leaf + c);
      const uint32_t words[4] = {cur.x, cur.y, cur.z, cur.w};
      const uint32_t nvalid = min(16u, u - c);
#pragma unroll
      for (int i = 0; i < 16; i++) {
        const uint32_t b = (words[i >> 2] >> (8 * (i & 3))) & 0xffu;
        const bool valid = (uint32_t)i < nvalid && !(c == 0 && i < 8);
        if (valid && j < jend) {
          if (sh < 64) acc |= (uint64_t)(b & 0x7fu) << sh;
          sh += 7;
          if (!(b & 0x80u)) {
            key += acc;
            const uint64_t P = c0 + hc + start - 8u;
            const uint32_t end = c + (uint32_t)i;
            while (j < jend && P >= T) {
              put_rec(rec, j, f, key, P, start, end + 1u - start);
              j++;
              T = split_threshold(j, total, Lt);
            }
            acc = 0;
            sh = 0;
            start = end + 1u;
          }
        }
      }
    }
    }
    if (j < jend) {
      const uint64_t hf = a.ne[a.rank[f] + 1];
      if (hf < a.L) {
        const uint32_t uf = a.src.used[hf];
        const uint64_t cf = a.CP[hf];
        const uint32_t hcf = (uint32_t)(a.CP[hf + 1] - cf - (uf - 8u));
        for (; j < jend; j++) put_rec(rec, j, hf, a.head[hf], cf, 0, hcf);
      } else {
        for (; j < jend; j++) put_rec(rec, j, a.L, 0, total, 0, 0);
      }
    }
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
// error counter.  The next source leaf's record loads while the current
// leaf's bytes are copied.
__global__ void __launch_bounds__(kWave) k_split_write(SplitArgs a, uint32_t S, const SplitRec* __restrict__ rec,
                                                       uint8_t* __restrict__ dbytes, uint32_t* __restrict__ dused,
                                                       uint64_t* __restrict__ dhead, Counters* ctr) {
  extern __shared__ __align__(16) uint8_t buf[];
  for (uint64_t j = blockIdx.x; j < a.Lt; j += gridDim.x) {
    const SplitRec A = rec[j], B = rec[j + 1];
    bool bad = A.leaf >= a.L;
    uint64_t f = bad ? 0 : A.leaf;
    SrcInfo I = a.info[f];
    wave_zero(buf, S);
    __syncthreads();
    if (lane_id() == 0) put_le64(buf, A.x);
    uint32_t pos = 8;
    uint32_t bs = A.p == 0 ? 8u : A.p + A.cost;
    while (!bad) {
      const uint32_t u = I.used;
      const bool last = f == B.leaf;  // the end lies inside leaf f (B.p >= 8)
      const uint64_t fn = I.next;
      const bool hop = !last && fn < a.L && !(fn == B.leaf && B.p == 0);
      SrcInfo In;
      if (hop) In = a.info[fn];
      const uint32_t be = last ? B.p : u;
      if (be < bs || be > u) {
        bad = true;
        break;
      }
      wave_copy_bytes(buf + min(pos, S), S - min(pos, S), a.src.ptr(f, u), bs, be);
      pos += be - bs;
      if (!hop) break;
      const uint64_t d = In.head - I.lastk;
      const uint32_t len = vlen(d);
      if (lane_id() == 0 && pos + len <= S) vput(buf + pos, d);
      pos += len;
      f = fn;
      I = In;
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
