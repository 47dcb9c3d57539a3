// Lane-per-leaf batch merge (the batch-merge phase of Section "Parallel Batch
// Updates in a PMA", with the CPMA's single-pass leaf updates of Section
// "Compressed Packed Memory Array", "Point updates").
//
// Each lane owns one touched leaf and its slice of the sorted batch and streams
// through them like the serial two-finger merge, so a wave merges 64 leaves at
// once with no LDS and no cross-lane traffic.
//
//  * insert: pass 1 runs the merge forward without writing, to learn the new
//    encoded size and the leaf's last key; pass 2 runs it backward and writes
//    the new codes from the end.  Writing backward in place is safe: the bytes
//    still to be written always cover at least the bytes still to be read,
//    because splitting a gap into several deltas never takes fewer bytes than
//    the single delta it replaces.  A result larger than the leaf goes to the
//    overflow arena instead.
//  * delete: one forward pass writes the kept keys in place (the output never
//    overtakes the input, for the same reason) and zero-fills the freed tail.
#pragma once
#include "update.hpp"

namespace cpma_dev {

// Byte streams over a leaf image.  Bytes are fetched with 16-byte loads only
// when a byte of that chunk is needed, so a stream never reads past the byte
// range it is asked for.
struct ChunkCache {
  const uint8_t* base;
  uint4 q;
  uint32_t qpos;  // chunk start held in q (0xffffffff: none)
  __device__ __forceinline__ void init(const uint8_t* b) {
    base = b;
    qpos = 0xffffffffu;
  }
  __device__ __forceinline__ uint32_t byte_at(uint32_t p) {
    const uint32_t c = p & ~15u;
    if (c != qpos) {
      q = *reinterpret_cast<const uint4*>(base + c);
      qpos = c;
    }
    const uint32_t wi = (p >> 2) & 3u;
    const uint32_t w = wi == 0 ? q.x : wi == 1 ? q.y : wi == 2 ? q.z : q.w;
    return (w >> (8 * (p & 3u))) & 0xffu;
  }
};

struct FwdBytes {
  ChunkCache cc;
  uint32_t pos;  // next byte position
  __device__ __forceinline__ void start(const uint8_t* b, uint32_t p) {
    cc.init(b);
    pos = p;
  }
  __device__ __forceinline__ uint32_t next() { return cc.byte_at(pos++); }
};

// Backward byte stream: next() returns the byte at pos-1 and moves down.
struct BwdBytes {
  ChunkCache cc;
  uint32_t pos;  // bytes below pos are unread
  __device__ __forceinline__ void start(const uint8_t* b, uint32_t p) {
    cc.init(b);
    pos = p;
  }
  __device__ __forceinline__ uint32_t peek() { return cc.byte_at(pos - 1); }
  __device__ __forceinline__ uint32_t next() { return cc.byte_at(--pos); }
};

// Forward reader of a leaf's keys.
struct FwdKeys {
  FwdBytes by;
  uint32_t used;
  uint64_t key;
  __device__ __forceinline__ void start(const uint8_t* leaf, uint32_t u) {
    used = u;
    if (u >= 8) {
      by.start(leaf, 0);
      uint64_t h = 0;
#pragma unroll
      for (int i = 0; i < 8; i++) h |= (uint64_t)by.next() << (8 * i);
      key = h;
    }
  }
  // Advances to the next key; false at the end.
  __device__ __forceinline__ bool advance() {
    if (by.pos >= used) return false;
    uint64_t acc = 0;
    uint32_t sh = 0, b;
    do {
      b = by.next();
      acc |= (uint64_t)(b & 0x7fu) << sh;
      sh += 7;
    } while ((b & 0x80u) && sh < 64);
    key += acc;
    return true;
  }
};

// Backward reader: starts at the last key and walks down to the head.
struct BwdKeys {
  BwdBytes by;
  uint64_t key;
  __device__ __forceinline__ void start(const uint8_t* leaf, uint32_t u, uint64_t last) {
    key = last;
    by.start(leaf, u);
  }
  __device__ __forceinline__ bool advance() {
    if (by.pos <= 8) return false;
    // The code ending at pos-1: its top group first, lower groups below it.
    uint64_t v = by.next() & 0x7fu;
    while (by.pos > 8) {
      const uint32_t b = by.peek();
      if (!(b & 0x80u)) break;
      by.next();
      v = (v << 7) | (b & 0x7fu);
    }
    key -= v;
    return true;
  }
};

// Forward writer with dword stores.
struct FwdWriter {
  uint8_t* base;
  uint32_t p;
  uint32_t acc;
  uint32_t cap;  // guard: never write at or past cap
  __device__ __forceinline__ void start(uint8_t* b, uint32_t c) {
    base = b;
    p = 0;
    acc = 0;
    cap = c;
  }
  __device__ __forceinline__ void put(uint32_t byte) {
    if (p >= cap) return;
    acc |= byte << (8 * (p & 3u));
    p++;
    if ((p & 3u) == 0) {
      *reinterpret_cast<uint32_t*>(base + p - 4) = acc;
      acc = 0;
    }
  }
  __device__ __forceinline__ void put_head(uint64_t x) {
#pragma unroll
    for (int i = 0; i < 8; i++) put((uint32_t)(x >> (8 * i)) & 0xffu);
  }
  __device__ __forceinline__ void put_code(uint64_t d) {
    while (d >= 0x80) {
      put((uint32_t)(d & 0x7f) | 0x80u);
      d >>= 7;
    }
    put((uint32_t)d);
  }
  // Writes the last partial word (its upper bytes zero).
  __device__ __forceinline__ void finish() {
    if (p & 3u) *reinterpret_cast<uint32_t*>(base + (p & ~3u)) = acc;
  }
};

// Backward writer with dword stores: fills [p, end) from the top down.
struct BwdWriter {
  uint8_t* base;
  uint32_t p;
  uint32_t acc;
  __device__ __forceinline__ void start(uint8_t* b, uint32_t end) {
    base = b;
    p = end;
    acc = 0;
  }
  __device__ __forceinline__ void put(uint32_t byte) {
    if (p == 0) return;  // guard: never write below the region
    p--;
    acc |= byte << (8 * (p & 3u));
    if ((p & 3u) == 0) {
      *reinterpret_cast<uint32_t*>(base + p) = acc;
      acc = 0;
    }
  }
  // Code of d, written from its last byte down to its first.
  __device__ __forceinline__ void put_code(uint64_t d) {
    const uint32_t n = vlen(d);
    put((uint32_t)(d >> (7 * (n - 1))) & 0x7fu);
    for (int t = (int)n - 2; t >= 0; t--) put(((uint32_t)(d >> (7 * t)) & 0x7fu) | 0x80u);
  }
  __device__ __forceinline__ void put_head(uint64_t x) {
#pragma unroll
    for (int i = 7; i >= 0; i--) put((uint32_t)(x >> (8 * i)) & 0xffu);
  }
};

// Insert slices longer than this take the one-wave heavy merge.  One lane
// walking a slice key by key is latency-bound (about 2 us per key), so a
// single long slice would set the batch's latency: at 2 and 4 KiB leaves a
// slice of 300 / 4000 keys in one leaf took 0.9 / 3.1 ms here and 0.07 /
// 0.43 ms on the heavy merge.  Uniform batches give these leaves slices of
// ~50-110 keys, which stay on the lane.
constexpr uint32_t kLaneHeavy = 256;

// The main merge for leaves larger than the wave merge takes: every segment
// except the long insert slices above.  (Long insert slices of smaller leaves
// go to the heavy merge too.)
__global__ void __launch_bounds__(256) k_merge_lane(MergeArgs a) {
  const uint64_t T = a.ctr->T;
  const uint64_t lanes = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long delta = 0, alg = 0;
  const uint32_t S = a.S;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += lanes) {
    const uint64_t s = t;
    const uint64_t leaf = a.seg_leaf[s];
    const uint32_t b = a.seg_begin[s], e = a.seg_begin[s + 1];
    const uint32_t nb = e - b;
    const uint64_t* B = a.B + b;
    uint8_t* lp = a.bytes + leaf * (uint64_t)S;
    const uint32_t used0 = a.used[leaf];
    if (a.is_insert) {
      if (nb > kLaneHeavy) {
        a.heavy_list[atomicAdd(&a.ctr->heavy, 1u)] = (uint32_t)s;
        continue;
      }
      // ---- pass 1: forward merge, sizes only ---------------------------------
      FwdKeys rd;
      rd.start(lp, used0);
      bool have_old = used0 >= 8;
      uint32_t j = 0;
      uint64_t bj = B[0];
      uint64_t prev = 0, last_old = 0;
      bool have_prev = false;
      uint64_t size = 0;
      uint32_t added = 0;
      while (have_old || j < nb) {
        uint64_t x;
        if (have_old && (j >= nb || rd.key <= bj)) {
          x = rd.key;
          last_old = x;
          if (j < nb && bj == x) {
            j++;
            if (j < nb) bj = B[j];
          }
          have_old = rd.advance();
        } else {
          x = bj;
          added++;
          j++;
          if (j < nb) bj = B[j];
        }
        size += have_prev ? vlen(x - prev) : 8u;
        prev = x;
        have_prev = true;
      }
      // ---- destination ----------------------------------------------------------
      uint8_t* dst = lp;
      if (size > S) {
        const uint64_t need = (size + 15) & ~15ull;
        const uint64_t off = arena_region(a, s);
        if (off + need > a.arena_cap) {
          atomicOr(&a.ctr->error, 1u);
          continue;
        }
        dst = a.arena + off;
        a.ovf[leaf] = off;
      }
      // ---- pass 2: backward merge, writing from the end -------------------------
      BwdKeys br;
      br.start(lp, used0, last_old);
      have_old = used0 >= 8;
      int64_t jj = (int64_t)nb - 1;
      uint64_t bjj = B[jj];
      BwdWriter wr;
      wr.start(dst, (uint32_t)size);
      bool have_cur = false;
      uint64_t cur = 0;
      while (have_old || jj >= 0) {
        uint64_t x;
        if (have_old && (jj < 0 || br.key >= bjj)) {
          x = br.key;
          if (jj >= 0 && bjj == x) {
            jj--;
            if (jj >= 0) bjj = B[jj];
          }
          have_old = br.advance();
        } else {
          x = bjj;
          jj--;
          if (jj >= 0) bjj = B[jj];
        }
        if (have_cur) wr.put_code(cur - x);
        cur = x;
        have_cur = true;
      }
      wr.put_head(cur);
      a.used[leaf] = (uint32_t)size;
      a.head[leaf] = cur;
      delta += added;
      alg += used0 + size + 8ull * nb + 20;
    } else {
      // ---- delete: one forward pass, in place ------------------------------------
      FwdKeys rd;
      rd.start(lp, used0);
      bool have_old = used0 >= 8;
      uint32_t j = 0;
      uint64_t bj = nb ? B[0] : 0;
      FwdWriter wr;
      wr.start(lp, used0);
      bool have_prev = false;
      uint64_t prev = 0, first = kNoKey;
      uint32_t removed = 0;
      while (have_old) {
        const uint64_t x = rd.key;
        while (j < nb && bj < x) {
          j++;
          if (j < nb) bj = B[j];
        }
        if (j < nb && bj == x) {
          removed++;
        } else {
          if (have_prev) {
            wr.put_code(x - prev);
          } else {
            wr.put_head(x);
            first = x;
          }
          prev = x;
          have_prev = true;
        }
        have_old = rd.advance();
      }
      wr.finish();
      const uint32_t size = wr.p;
      for (uint32_t z = (size + 3u) & ~3u; z < ((used0 + 3u) & ~3u); z += 4)
        *reinterpret_cast<uint32_t*>(lp + z) = 0u;
      a.used[leaf] = size;
      a.head[leaf] = have_prev ? first : kNoKey;
      delta += removed;
      alg += used0 + used0 + 8ull * nb + 20;
    }
  }
  delta = wave_sum((uint64_t)delta);
  alg = wave_sum((uint64_t)alg);
  // per-wave slot, summed by k_fold_parts
  const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (lane_id() == 0) {
    a.part[2 * w] = delta;
    a.part[2 * w + 1] = alg;
  }
}

}  // namespace cpma_dev
