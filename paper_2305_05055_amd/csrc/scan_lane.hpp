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
// chunk's keys sum to cnt * base + sum of Dc at terminators.  The byte loop has
// no validity tests: bytes at or past `used` are rewritten to 0x80, continuation
// bytes without payload (one masked merge per word, in the last chunk only); the head's eight
// bytes become seven such bytes and a zero terminator, so the head counts as a
// key at offset 0 from the chunk base (the head itself).  The terminator count
// is one popcount per word.  The leaf streams in 64-byte rounds with the next
// round's four loads in flight.
__device__ __forceinline__ void fast_chunk(const uint4 q, uint32_t c, uint32_t used, uint64_t& base, uint32_t& sh,
                                           LeafSum& r) {
  uint32_t w[4] = {q.x, q.y, q.z, q.w};
  if (c == 0) {
    w[0] = 0x80808080u;
    w[1] = 0x00808080u;
  }
  const int32_t nv = (int32_t)used - (int32_t)c;
  if (nv < 16) {
    // bytes at or past `used` (zero fill in place; arbitrary in an overflow
    // copy) become exactly 0x80
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int32_t v = nv - 4 * k;
      const uint32_t keep = v >= 4 ? 0xffffffffu : (v <= 0 ? 0u : ((1u << (8 * v)) - 1u));
      w[k] = (w[k] & keep) | (0x80808080u & ~keep);
    }
  }
  const uint32_t cnt = (uint32_t)(__popc(~w[0] & 0x80808080u) + __popc(~w[1] & 0x80808080u) +
                                  __popc(~w[2] & 0x80808080u) + __popc(~w[3] & 0x80808080u));
  uint32_t Dc = 0, Sc = 0;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const uint32_t x = w[i >> 2];
    const int o = 8 * (i & 3);
    const uint32_t p = (x >> o) & 0x7fu;
    const uint32_t cm = 0u - ((x >> (o + 7)) & 1u);  // all ones on a continuation byte
    Dc += p << (sh & 31u);
    Sc += Dc & ~cm;
    sh = (sh + 7u) & cm;
  }
  r.sum += (uint64_t)cnt * base + Sc;
  r.count += cnt;
  base += Dc;
}

// Also returns the leaf's last key through *last.
__device__ __forceinline__ LeafSum leaf_sum_fast(const uint8_t* __restrict__ leaf, uint32_t used,
                                                 uint64_t head, uint64_t* last = nullptr) {
  LeafSum r{0, 0};
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
  if (last) *last = base;
  return r;
}

// Keeps the loads above it above it: without this the compiler sinks each
// round's loads down to their use in the next round, so that every round waits
// for its own loads instead of finding them done.
__device__ __forceinline__ void issue_now() { asm volatile("" ::: "memory"); }

// One byte (byte J of word x) of leaf_sum_zf: the running offset D (key minus
// head) grows by the byte's payload at its shift; a terminator's D is returned
// for the sum, a continuation byte returns 0.  The continuation mask is one
// sign-extending extract, written so that the compiler keeps it: left to
// itself it rebuilds the mask from a compare and two selects per byte.
template <int J>
__device__ __forceinline__ uint32_t zf_byte(uint32_t x, uint32_t& D, uint32_t& sh) {
  uint32_t cm;  // all ones on a continuation byte
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(cm) : "v"(x), "i"(8 * J + 7));
  D += __builtin_amdgcn_ubfe(x, 8 * J, 7) << (sh & 31u);
  sh = (sh + 7u) & cm;
  return D & ~cm;
}

// One 16-byte chunk of leaf_sum_zf.  Offsets stay below 2^28, so the chunk's
// 16 terminator offsets sum below 2^32 and are folded into the 64-bit total
// once.  `cont` counts continuation bytes.
__device__ __forceinline__ void zf_chunk(const uint4 q, uint32_t& D, uint32_t& sh, uint64_t& Sc, uint32_t& cont) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t x = w[k];
    const uint32_t t0 = zf_byte<0>(x, D, sh);
    const uint32_t t1 = zf_byte<1>(x, D, sh);
    const uint32_t t2 = zf_byte<2>(x, D, sh);
    const uint32_t t3 = zf_byte<3>(x, D, sh);
    s += (t0 + t1) + (t2 + t3);
    cont += (uint32_t)__popc(x & 0x80808080u);
  }
  Sc += s;
}

// Sum and count of every key of a leaf read in place, for leaves whose key span
// is below 2^28 and whose bytes past `used` are zero (the leaf layout's zero
// fill; not key-value leaves, whose values sit at the leaf's end).  The leaf is
// read in whole 64-byte rounds (S is a multiple of 64) with no bounds tests:
//  * each zero byte past `used` decodes as a zero delta, one more copy of the
//    last key; there are exactly 64 * rounds - used of them, taken back out of
//    the sum at the end;
//  * the key count is `used` minus the continuation bytes, once the head's
//    eight bytes are replaced by seven payload-free continuation bytes and a
//    terminator (the head: one key at offset 0);
//  * every round's four loads are issued unconditionally (past the last round
//    they reread it), so the next round is in flight while one is decoded.
__device__ __forceinline__ LeafSum leaf_sum_zf(const uint8_t* __restrict__ leaf, uint32_t used, uint64_t head) {
  if (used == 0) return LeafSum{0, 0};
  const uint32_t lastr = (used - 1u) & ~63u;  // first byte of the last round
  uint32_t D = 0, sh = 0, cont = 0;
  uint64_t Sc = 0;
  const uint4* pa = reinterpret_cast<const uint4*>(leaf);
  uint4 a0 = pa[0], a1 = pa[1], a2 = pa[2], a3 = pa[3];
  const uint4* pb = reinterpret_cast<const uint4*>(leaf + min(64u, lastr));
  uint4 b0 = pb[0], b1 = pb[1], b2 = pb[2], b3 = pb[3];
  issue_now();
  a0.x = 0x80808080u;
  a0.y = 0x00808080u;
  zf_chunk(a0, D, sh, Sc, cont);
  zf_chunk(a1, D, sh, Sc, cont);
  zf_chunk(a2, D, sh, Sc, cont);
  zf_chunk(a3, D, sh, Sc, cont);
  // ping-pong between two register sets: no copies between rounds
  for (uint32_t c = 64; c < used;) {
    pa = reinterpret_cast<const uint4*>(leaf + min(c + 64u, lastr));
    a0 = pa[0];
    a1 = pa[1];
    a2 = pa[2];
    a3 = pa[3];
    issue_now();
    zf_chunk(b0, D, sh, Sc, cont);
    zf_chunk(b1, D, sh, Sc, cont);
    zf_chunk(b2, D, sh, Sc, cont);
    zf_chunk(b3, D, sh, Sc, cont);
    c += 64;
    if (c >= used) break;
    pb = reinterpret_cast<const uint4*>(leaf + min(c + 64u, lastr));
    b0 = pb[0];
    b1 = pb[1];
    b2 = pb[2];
    b3 = pb[3];
    issue_now();
    zf_chunk(a0, D, sh, Sc, cont);
    zf_chunk(a1, D, sh, Sc, cont);
    zf_chunk(a2, D, sh, Sc, cont);
    zf_chunk(a3, D, sh, Sc, cont);
    c += 64;
  }
  const uint32_t zeros = ((used + 63u) & ~63u) - used;
  const uint64_t cnt = used - cont;
  return LeafSum{cnt * head + (Sc - (uint64_t)zeros * D), cnt};
}

// General path: 64-bit decode; counts and sums keys in [lo, hi).  Stops early
// once a key reaches hi.
__device__ __forceinline__ LeafSum leaf_sum_range(const uint8_t* __restrict__ leaf, uint32_t used,
                                                  uint64_t lo, uint64_t hi) {
  LeafSum r{0, 0};
  if (used < 8) return r;
  // 64-byte rounds with the next round's four loads in flight (a lane walks
  // its leaf alone, so every load would otherwise be a full round trip)
  const uint4 z = make_uint4(0, 0, 0, 0);
  uint4 a0 = load16(leaf);
  uint4 a1 = 16 < used ? load16(leaf + 16) : z;
  uint4 a2 = 32 < used ? load16(leaf + 32) : z;
  uint4 a3 = 48 < used ? load16(leaf + 48) : z;
  uint64_t key = ((uint64_t)a0.y << 32) | a0.x;
  if (key >= hi) return r;
  if (key >= lo) {
    r.sum += key;
    r.count++;
  }
  uint64_t acc = 0;
  uint32_t sh = 0;
  bool done = false;
  auto chunk = [&](const uint4 cur, uint32_t c) {
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
  };
  for (uint32_t c = 0; c < used && !done; c += 64) {
    uint4 b0 = z, b1 = z, b2 = z, b3 = z;
    if (c + 64 < used) b0 = load16(leaf + c + 64);
    if (c + 80 < used) b1 = load16(leaf + c + 80);
    if (c + 96 < used) b2 = load16(leaf + c + 96);
    if (c + 112 < used) b3 = load16(leaf + c + 112);
    chunk(a0, c);
    if (c + 16 < used && !done) chunk(a1, c + 16);
    if (c + 32 < used && !done) chunk(a2, c + 32);
    if (c + 48 < used && !done) chunk(a3, c + 48);
    a0 = b0;
    a1 = b1;
    a2 = b2;
    a3 = b3;
  }
  return r;
}

// ---- uncompressed leaves (the plain PMA) ---------------------------------------
// The uncompressed variant keeps the same leaves, tree and byte-density bounds,
// but a leaf holds its keys as raw little-endian 8-byte words packed to the
// left (used = 8 x keys, zero fill after them), with no delta codes (Section
// "Packed Memory Array"; the ablation of Section "Evaluation on
// microbenchmarks" that isolates what compression buys).

// Sum and count of the keys in [lo, hi) of an uncompressed leaf, one lane.
__device__ __forceinline__ LeafSum raw_sum_range(const uint8_t* __restrict__ leaf, uint32_t used, uint64_t lo,
                                                 uint64_t hi) {
  LeafSum r{0, 0};
  const uint64_t* k = reinterpret_cast<const uint64_t*>(leaf);
  const uint32_t m = used / 8;
  for (uint32_t i = 0; i < m; i += 2) {
    const uint4 w = *reinterpret_cast<const uint4*>(k + i);
    const uint64_t a = ((uint64_t)w.y << 32) | w.x;
    const uint64_t b = ((uint64_t)w.w << 32) | w.z;
    if (a >= hi) break;
    if (a >= lo) {
      r.sum += a;
      r.count++;
    }
    if (i + 1 < m) {
      if (b >= hi) break;
      if (b >= lo) {
        r.sum += b;
        r.count++;
      }
    }
  }
  return r;
}

// Sum and count of every key of an uncompressed leaf, one lane (16-byte loads,
// four in flight).
__device__ __forceinline__ LeafSum raw_sum_all(const uint8_t* __restrict__ leaf, uint32_t used) {
  const uint4* w = reinterpret_cast<const uint4*>(leaf);
  const uint32_t m = used / 8, nw = m / 2;
  uint64_t s0 = 0, s1 = 0;
  uint32_t i = 0;
  for (; i + 4 <= nw; i += 4) {
    const uint4 a = w[i], b = w[i + 1], c = w[i + 2], d = w[i + 3];
    s0 += (((uint64_t)a.y << 32) | a.x) + (((uint64_t)a.w << 32) | a.z) + (((uint64_t)b.y << 32) | b.x) +
          (((uint64_t)b.w << 32) | b.z);
    s1 += (((uint64_t)c.y << 32) | c.x) + (((uint64_t)c.w << 32) | c.z) + (((uint64_t)d.y << 32) | d.x) +
          (((uint64_t)d.w << 32) | d.z);
  }
  for (; i < nw; i++) {
    const uint4 a = w[i];
    s0 += (((uint64_t)a.y << 32) | a.x) + (((uint64_t)a.w << 32) | a.z);
  }
  if (m & 1u) s1 += reinterpret_cast<const uint64_t*>(leaf)[m - 1];
  return LeafSum{s0 + s1, m};
}

// The same for a whole wave on one leaf (keys i = lane, lane + 64, ...).
__device__ __forceinline__ LeafSum wave_raw_sum_range(const uint8_t* __restrict__ leaf, uint32_t used, uint64_t lo,
                                                      uint64_t hi) {
  const uint64_t* k = reinterpret_cast<const uint64_t*>(leaf);
  uint64_t s = 0, n = 0;
  for (uint32_t i = lane_id(); i < used / 8; i += kWave) {
    const uint64_t x = k[i];
    if (x >= lo && x < hi) {
      s += x;
      n++;
    }
  }
  return LeafSum{wave_sum(s), wave_sum(n)};
}

}  // namespace cpma_dev
