// Lane-per-leaf decoders for range_map and contains.
//
// A range query is a search followed by a scan (Section "Packed Memory Array",
// "Design and operations").  Leaves strictly inside a query's leaf span hold only
// keys of the range, so they need a sum and a count but no comparisons; the two
// end leaves (and a point query's single leaf) compare every key.
//
// Each lane decodes a whole leaf on its own.  All lanes of a wave walk their
// leaves one byte per step from offset 0, so their 16-byte chunk loads happen
// in the same step (coalesced in time, no divergent stalls), and no cross-lane
// operation is needed.
#pragma once
#include "common.hpp"

namespace cpma_dev {

struct LeafSum {
  uint64_t sum;    // wrapping sum of keys
  uint64_t count;  // number of keys
};

__device__ __forceinline__ uint4 load16(const uint8_t* p) { return *reinterpret_cast<const uint4*>(p); }

// Interior fast path: sum and count of every key of a leaf whose key span is
// below 2^28 (so every delta code is at most 4 bytes and fits 32-bit shifts).
//
// Per byte: p = payload bits, the running chunk-relative delta Dc grows by
// p << sh; at a terminator byte Dc equals (key - key at chunk start), so the
// chunk's keys sum to cnt * base + sum of Dc at terminators.  The leaf streams
// in 64-byte rounds with the next round's four loads in flight.
__device__ __forceinline__ void fast_chunk(const uint4 q, uint32_t c, uint32_t used, uint64_t& base, uint32_t& sh,
                                           LeafSum& r) {
  const uint32_t words[4] = {q.x, q.y, q.z, q.w};
  const uint32_t nvalid = c < used ? min(16u, used - c) : 0u;
  uint32_t Dc = 0, Sc = 0, cnt = 0;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const uint32_t w = words[i >> 2];
    const int o = 8 * (i & 3);
    const bool valid = (uint32_t)i < nvalid && !(c == 0 && i < 8);
    const uint32_t p = valid ? ((w >> o) & 0x7fu) : 0u;
    const bool term = valid && !((w >> (o + 7)) & 1u);
    Dc += p << sh;
    sh = term ? 0u : (valid ? sh + 7u : sh);
    Sc += term ? Dc : 0u;
    cnt += term ? 1u : 0u;
  }
  r.sum += (uint64_t)cnt * base + Sc;
  r.count += cnt;
  base += Dc;
}

__device__ __forceinline__ LeafSum leaf_sum_fast(const uint8_t* __restrict__ leaf, uint32_t used,
                                                 uint64_t head) {
  LeafSum r{head, 1};
  uint64_t base = head;  // key value reached by the running delta so far
  uint32_t sh = 0;
  const uint4 z = make_uint4(0, 0, 0, 0);
  uint4 a0 = load16(leaf);
  uint4 a1 = 16 < used ? load16(leaf + 16) : z;
  uint4 a2 = 32 < used ? load16(leaf + 32) : z;
  uint4 a3 = 48 < used ? load16(leaf + 48) : z;
  for (uint32_t c = 0; c < used; c += 64) {
    uint4 b0 = z, b1 = z, b2 = z, b3 = z;
    if (c + 64 < used) b0 = load16(leaf + c + 64);
    if (c + 80 < used) b1 = load16(leaf + c + 80);
    if (c + 96 < used) b2 = load16(leaf + c + 96);
    if (c + 112 < used) b3 = load16(leaf + c + 112);
    fast_chunk(a0, c, used, base, sh, r);
    fast_chunk(a1, c + 16, used, base, sh, r);
    fast_chunk(a2, c + 32, used, base, sh, r);
    fast_chunk(a3, c + 48, used, base, sh, r);
    a0 = b0;
    a1 = b1;
    a2 = b2;
    a3 = b3;
  }
  return r;
}

// The same in 128-byte rounds: a lane's eight loads of one round cover one whole
// cache line, so a line is consumed before any other lane's stream can evict it
// (many lanes stream separate leaves at once, far more lines than L2 holds).
__device__ __forceinline__ LeafSum leaf_sum_fast_line(const uint8_t* __restrict__ leaf, uint32_t used,
                                                      uint64_t head) {
  LeafSum r{head, 1};
  uint64_t base = head;
  uint32_t sh = 0;
  const uint4 z = make_uint4(0, 0, 0, 0);
  for (uint32_t c = 0; c < used; c += 128) {
    uint4 q[8];
#pragma unroll
    for (int k = 0; k < 8; k++) q[k] = (c + 16u * k < used) ? load16(leaf + c + 16u * k) : z;
#pragma unroll
    for (int k = 0; k < 8; k++) fast_chunk(q[k], c + 16u * k, used, base, sh, r);
  }
  return r;
}

// General path: 64-bit decode; counts and sums keys in [lo, hi).  Stops early
// once a key reaches hi.
__device__ __forceinline__ LeafSum leaf_sum_range(const uint8_t* __restrict__ leaf, uint32_t used,
                                                  uint64_t lo, uint64_t hi) {
  LeafSum r{0, 0};
  if (used < 8) return r;
  uint4 cur = load16(leaf);
  uint64_t key = ((uint64_t)cur.y << 32) | cur.x;
  if (key >= hi) return r;
  if (key >= lo) {
    r.sum += key;
    r.count++;
  }
  uint64_t acc = 0;
  uint32_t sh = 0;
  bool done = false;
  for (uint32_t c = 0; c < used && !done; c += 16) {
    if (c) cur = load16(leaf + c);
    const uint32_t words[4] = {cur.x, cur.y, cur.z, cur.w};
    const uint32_t nvalid = min(16u, used - c);
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t b = (words[i >> 2] >> (8 * (i & 3))) & 0xffu;
      const bool valid = (uint32_t)i < nvalid && !(c == 0 && i < 8) && !done;
      if (valid) {
        if (sh < 64) acc |= (uint64_t)(b & 0x7fu) << sh;
        sh += 7;
        if (!(b & 0x80u)) {
          key += acc;
          acc = 0;
          sh = 0;
          if (key >= hi) {
            done = true;
          } else if (key >= lo) {
            r.sum += key;
            r.count++;
          }
        }
      }
    }
  }
  return r;
}

}  // namespace cpma_dev
