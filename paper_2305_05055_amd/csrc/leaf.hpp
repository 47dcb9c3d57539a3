// Wave-level leaf codec.
//
// Leaf layout (Section "Compressed Packed Memory Array", "CPMA structure"): the
// head key in bytes [0, 8) little-endian, then the deltas to the following keys
// as byte codes packed to the left, then zero fill up to the leaf size.  A key is
// the running sum of the head and the deltas before it (delta encoding,
// "Data compression techniques").
//
// Decoding runs one wave over 1024-byte chunks: lane l owns bytes
// [16 l, 16 l + 16) of the chunk and parses the byte codes that END in its bytes;
// a code that starts in the previous lane arrives as a carried partial value
// (at most one lane back, since a code is at most 10 bytes long).  Keys then come
// from a wave prefix sum of the per-lane delta totals.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace cpma_dev {

struct LaneCodes {
  uint64_t v[16];      // value of the code ending at byte i (raw, before the carry fix)
  uint32_t tmask;      // bit i: a code (or the head) ends at byte i
  uint64_t first_raw;  // raw value of the first code ending in this lane
  uint64_t tail_acc;   // bits of a code still open at the end of the lane
  uint32_t tail_sh;    // its bit length so far (multiple of 7)
};

// Parses the lane's 16 bytes w (positions pos0 .. pos0+15 of the leaf, valid below
// `used`).  The head occupies positions 0..7 and is reported as a value ending at
// byte 7.
__device__ __forceinline__ void lane_parse(const uint4 w, uint32_t pos0, uint32_t used,
                                           LaneCodes& c) {
  const uint32_t words[4] = {w.x, w.y, w.z, w.w};
  const uint32_t nvalid = pos0 < used ? min(16u, used - pos0) : 0u;
  const bool head_lane = (pos0 == 0);
  uint64_t acc = 0;
  uint32_t sh = 0;
  bool seen = false;
  c.tmask = 0;
  c.first_raw = 0;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const uint32_t b = (words[i >> 2] >> (8 * (i & 3))) & 0xffu;
    const bool valid = (uint32_t)i < nvalid && !(head_lane && i < 8);
    if (valid && sh < 64) acc |= (uint64_t)(b & 0x7fu) << sh;
    const bool term = valid && !(b & 0x80u);
    c.v[i] = term ? acc : 0ull;
    if (term) {
      if (!seen) c.first_raw = acc;
      seen = true;
      c.tmask |= 1u << i;
      acc = 0;
      sh = 0;
    } else if (valid) {
      sh += 7;
    }
  }
  if (head_lane && nvalid >= 8) {
    c.v[7] = ((uint64_t)words[1] << 32) | words[0];
    c.tmask |= 1u << 7;
  }
  c.tail_acc = acc;
  c.tail_sh = sh;
}

// Decodes the leaf at src (16-byte aligned, `used` valid bytes) with one wave and
// calls emit(index, key, delta) for every key in order (the head's delta is the
// head itself); an emit taking a fourth argument also gets the byte where the
// key's code ends.  Returns the key count (uniform).
template <class Emit>
__device__ __forceinline__ uint32_t wave_decode_leaf(const uint8_t* __restrict__ src, uint32_t used,
                                                     Emit&& emit) {
  const int lane = lane_id();
  uint64_t run_key = 0, carry_acc = 0;
  uint32_t run_cnt = 0, carry_sh = 0;
  for (uint32_t base = 0; base < used; base += 16u * kWave) {
    const uint32_t pos0 = base + 16u * lane;
    uint4 w = make_uint4(0, 0, 0, 0);
    if (pos0 < used) w = *reinterpret_cast<const uint4*>(src + pos0);
    LaneCodes c;
    lane_parse(w, pos0, used, c);
    uint64_t cin_acc = dpp_prev64(c.tail_acc);
    uint32_t cin_sh = dpp_prev32(c.tail_sh);
    if (lane == 0) {
      cin_acc = carry_acc;
      cin_sh = carry_sh;
    }
    uint64_t corr = 0;
    if (c.tmask != 0 && pos0 != 0) {
      uint64_t fixed = cin_acc | (cin_sh < 64 ? (c.first_raw << cin_sh) : 0ull);
      corr = fixed - c.first_raw;
    }
    uint64_t lsum = corr;
#pragma unroll
    for (int i = 0; i < 16; i++) lsum += c.v[i];
    const uint32_t lcnt = (uint32_t)__popc(c.tmask);
    const uint64_t incl_sum = wave_incl_scan(lsum);
    const uint32_t incl_cnt = wave_incl_scan(lcnt);
    uint64_t key = run_key + (incl_sum - lsum);
    uint64_t pend = corr;  // the carry fix belongs to the lane's first code
    uint32_t idx = run_cnt + (incl_cnt - lcnt);
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (c.tmask & (1u << i)) {
        const uint64_t d = c.v[i] + pend;
        pend = 0;
        key += d;
        if constexpr (std::is_invocable<Emit&, uint32_t, uint64_t, uint64_t, uint32_t>::value)
          emit(idx, key, d, pos0 + (uint32_t)i);
        else
          emit(idx, key, d);
        idx++;
      }
    }
    run_key += lane63_u64(incl_sum);
    run_cnt += lane63_u32(incl_cnt);
    carry_acc = lane63_u64(c.tail_acc);
    carry_sh = lane63_u32(c.tail_sh);
  }
  return run_cnt;
}

// Single-chunk variant (leaf size <= 1024): the caller has already loaded the
// lane's 16 bytes w (zeros past `used`).
template <class Emit>
__device__ __forceinline__ uint32_t wave_decode_regs(const uint4 w, uint32_t used, Emit&& emit) {
  const int lane = lane_id();
  const uint32_t pos0 = 16u * lane;
  LaneCodes c;
  lane_parse(w, pos0, used, c);
  uint64_t cin_acc = dpp_prev64(c.tail_acc);
  uint32_t cin_sh = dpp_prev32(c.tail_sh);
  uint64_t corr = 0;
  if (c.tmask != 0 && pos0 != 0) {
    const uint64_t fixed = cin_acc | (cin_sh < 64 ? (c.first_raw << cin_sh) : 0ull);
    corr = fixed - c.first_raw;
  }
  uint64_t lsum = corr;
#pragma unroll
  for (int i = 0; i < 16; i++) lsum += c.v[i];
  const uint32_t lcnt = (uint32_t)__popc(c.tmask);
  const uint64_t incl_sum = wave_incl_scan(lsum);
  const uint32_t incl_cnt = wave_incl_scan(lcnt);
  uint64_t key = incl_sum - lsum;
  uint64_t pend = corr;
  uint32_t idx = incl_cnt - lcnt;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    if (c.tmask & (1u << i)) {
      const uint64_t d = c.v[i] + pend;
      pend = 0;
      key += d;
      emit(idx, key, d);
      idx++;
    }
  }
  return lane63_u32(incl_cnt);
}

// Narrow single-chunk decode (leaf size <= 1024): every key lies within 2^32 of
// `base`, so every delta fits 32 bits and a code has at most 5 bytes.  Keys are
// produced as 32-bit offsets from base (head_rel = head - base).
//
// A key is the head plus the payload of every code byte before it, each byte's
// 7 bits shifted by 7 times its place in its code; so a running sum of shifted
// payloads over the bytes, read at a code's last byte, is that key's offset.
// Per lane: the running sum over its 16 bytes (the shift a code carries in
// from the previous lane is 7 times that lane's run of trailing continuation
// bytes, known before parsing), then one wave scan of the lane totals gives
// every lane its starting offset, codes that straddle lanes included.  The
// head and bytes past `used` carry no payload.  emit(index, key offset) runs
// for every key in order; returns the key count.
__device__ __forceinline__ uint32_t msb_nibble(uint32_t x) {
  x = (x >> 7) & 0x01010101u;
  return (x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xfu;
}

template <class Emit>
__device__ __forceinline__ uint32_t wave_decode_narrow(uint4 w, uint32_t used, uint32_t head_rel, Emit&& emit) {
  const int lane = lane_id();
  const uint32_t pos0 = 16u * lane;
  const uint32_t nvalid = pos0 < used ? min(16u, used - pos0) : 0u;
  uint32_t vm = nvalid >= 16u ? 0xffffu : ((1u << nvalid) - 1u);
  const bool hl = lane == 0 && used >= 8u;
  if (lane == 0) {
    vm &= 0xff00u;  // the head is not a code
    w.x = 0;
    w.y = 0;
  }
  uint32_t words[4] = {w.x, w.y, w.z, w.w};
  if (nvalid < 16u) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int32_t v = (int32_t)nvalid - 4 * k;
      words[k] &= v >= 4 ? 0xffffffffu : (v <= 0 ? 0u : ((1u << (8 * v)) - 1u));
    }
  }
  const uint32_t msb = msb_nibble(words[0]) | (msb_nibble(words[1]) << 4) | (msb_nibble(words[2]) << 8) |
                       (msb_nibble(words[3]) << 12);
  const uint32_t tm = vm & ~msb;  // code ends
  const uint32_t cm = vm & msb;   // continuation bytes
  const uint32_t tc = __clz(~(cm << 16));
  uint32_t sh = 7u * dpp_prev32(tc);
  uint32_t run = 0;
  uint32_t kv[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    run += ((words[j >> 2] >> (8 * (j & 3))) & 0x7fu) << sh;
    kv[j] = run;
    sh = (sh + 7u) & (0u - ((cm >> j) & 1u));
  }
  const uint32_t lead = hl ? head_rel : 0u;
  const uint32_t tot = run + lead;
  const uint32_t lcnt = (uint32_t)__popc(tm) + (hl ? 1u : 0u);
  const uint32_t ex = wave_incl_scan(tot) - tot;
  const uint32_t icl = wave_incl_scan(lcnt);
  uint32_t idx = icl - lcnt;
  if (hl) emit(idx++, head_rel);
  const uint32_t off = ex + lead;
#pragma unroll
  for (int j = 0; j < 16; j++)
    if ((tm >> j) & 1u) emit(idx++, off + kv[j]);
  return lane63_u32(icl);
}

// Number of keys in a leaf image: the head plus one per byte with a clear high bit.
__device__ __forceinline__ uint32_t wave_count_keys(const uint8_t* __restrict__ src, uint32_t used) {
  const int lane = lane_id();
  uint32_t cnt = 0;
  for (uint32_t base = 0; base < used; base += 16u * kWave) {
    const uint32_t pos0 = base + 16u * lane;
    if (pos0 < used) {
      const uint4 w = *reinterpret_cast<const uint4*>(src + pos0);
      const uint32_t words[4] = {w.x, w.y, w.z, w.w};
      const uint32_t nvalid = min(16u, used - pos0);
#pragma unroll
      for (int i = 0; i < 16; i++) {
        const uint32_t b = (words[i >> 2] >> (8 * (i & 3))) & 0xffu;
        const bool head_byte = (pos0 == 0) && i < 8;
        cnt += ((uint32_t)i < nvalid && !head_byte && !(b & 0x80u)) ? 1u : 0u;
      }
      if (pos0 == 0) cnt += 1;  // the head
    }
  }
  return wave_sum(cnt);
}

// Encoded size of keys get(0..m): 8 bytes for the head, then one code per delta.
template <class Get>
__device__ __forceinline__ uint64_t wave_encoded_size(Get&& get, uint32_t m) {
  const int lane = lane_id();
  uint64_t tot = 0;
  for (uint32_t base = 0; base < m; base += kWave) {
    const uint32_t i = base + lane;
    uint32_t c = 0;
    if (i < m) c = (i == 0) ? 8u : vlen(get(i) - get(i - 1));
    tot += wave_sum(c);
  }
  return tot;
}

// Writes the encoding of get(0..m) to dst (LDS or global, byte granular).
template <class Get>
__device__ __forceinline__ void wave_encode_bytes(Get&& get, uint32_t m, uint8_t* dst) {
  const int lane = lane_id();
  uint64_t off0 = 0;
  for (uint32_t base = 0; base < m; base += kWave) {
    const uint32_t i = base + lane;
    uint32_t c = 0;
    uint64_t x = 0, prev = 0;
    if (i < m) {
      x = get(i);
      if (i > 0) prev = get(i - 1);
      c = (i == 0) ? 8u : vlen(x - prev);
    }
    const uint64_t incl = wave_incl_scan((uint64_t)c);
    if (i < m) {
      uint8_t* p = dst + off0 + incl - c;
      if (i == 0)
        put_le64(p, x);
      else
        vput(p, x - prev);
    }
    off0 += lane63_u64(incl);
  }
}

// Zero-fills lds_buf[0, S) (S a multiple of 16) with one wave.
__device__ __forceinline__ void wave_zero(uint8_t* buf, uint32_t S) {
  for (uint32_t o = 16u * lane_id(); o < S; o += 16u * kWave)
    *reinterpret_cast<uint4*>(buf + o) = make_uint4(0, 0, 0, 0);
}

// Copies S bytes (multiple of 16) from src to dst with 16-byte accesses.
__device__ __forceinline__ void wave_copy16(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src,
                                            uint32_t S) {
  for (uint32_t o = 16u * lane_id(); o < S; o += 16u * kWave)
    *reinterpret_cast<uint4*>(dst + o) = *reinterpret_cast<const uint4*>(src + o);
}

}  // namespace cpma_dev
