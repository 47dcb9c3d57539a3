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

// Decoder state at a 16-byte chunk boundary c of a narrow leaf, for walks that
// start there instead of at the head: K = payload contributions of the bytes in
// [8, c) (each byte's 7 bits shifted by its place in its code), and the code
// still open at c: its run of continuation bytes before c and their
// contributions (partial).  The last complete key before c is head + K -
// partial; the open code started at c - run.  c = ~0: none.
struct LeafCkpt {
  uint32_t c, K, partial, shrun;  // shrun: shift (7 run) | run << 8
};

// lastk[f] = last key of every non-empty old leaf, and for narrow leaves (key
// span below 2^28: every code at most 4 bytes, every sum in 32 bits) the
// decoder state at the starts of the second, third and fourth quarters.  Four
// lanes share a leaf: lane q sums the contributions of its quarter's bytes,
// starting from the shift that the continuation bytes just before its quarter
// imply, and a prefix over the four lanes gives the checkpoints and the total.
// head[f + 1] bounds the keys of leaf f from above (an empty leaf keeps a head
// above every earlier key), so it selects the narrow form.
__global__ void __launch_bounds__(256) k_leaf_last(SrcLeaves src, const uint64_t* __restrict__ head, uint64_t L,
                                                   uint64_t* __restrict__ lastk, LeafCkpt* __restrict__ ck) {
  const uint32_t q = threadIdx.x & 3u;
  const uint64_t quads = ((uint64_t)gridDim.x * blockDim.x) >> 2;
  for (uint64_t f = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2; f < L; f += quads) {
    const uint32_t u = src.used[f];
    if (u == 0) continue;  // the same for the four lanes of a leaf
    const uint64_t h = head[f];
    const uint64_t nx = f + 1 < L ? head[f + 1] : ~0ull;
    const uint8_t* p = src.ptr(f, u);
    if (!(nx > h && nx - h < (1ull << 28))) {
      if (q == 0) lastk[f] = leaf_last_wide(p, u, h);
      else ck[f * 3 + q - 1] = LeafCkpt{~0u, 0, 0, 0};
      continue;
    }
    const uint32_t Q = ((u + 3) / 4 + 15) & ~15u;
    const uint32_t b = q * Q, e = min(u, b + Q);
    uint32_t D = 0, sh = 0, run = 0, partial = 0;
    if (b < u) {
      if (q > 0) {
        // continuation bytes that end the previous chunk (never the head's)
        const uint4 pc = load16(p + b - 16);
        const uint32_t pw[4] = {pc.x, pc.y, pc.z, pc.w};
        uint32_t m = 0;  // high bits of the chunk's bytes (the head's bytes count as clear)
#pragma unroll
        for (int i = 0; i < 16; i++)
          if (b - 16 + (uint32_t)i >= 8) m |= ((pw[i >> 2] >> (8 * (i & 3) + 7)) & 1u) << i;
        run = min((uint32_t)__clz((int)~(m << 16)), 3u);  // a narrow code has at most 3 continuation bytes
#pragma unroll
        for (int i = 0; i < 16; i++)
          if ((uint32_t)i + run >= 16) partial += ((pw[i >> 2] >> (8 * (i & 3))) & 0x7fu) << (7 * (i + run - 16));
        sh = 7 * run;
      }
      auto chunk = [&](const uint4 cur, uint32_t c) {
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
          const uint32_t cm = 0u - ((x >> (o + 7)) & 1u);
          D += ((x >> o) & 0x7fu) << (sh & 31u);
          sh = (sh + 7u) & cm;
        }
      };
      // 64-byte rounds with the next round's four loads in flight
      const uint4 z = make_uint4(0, 0, 0, 0);
      uint4 a0 = load16(p + b);
      uint4 a1 = b + 16 < e ? load16(p + b + 16) : z;
      uint4 a2 = b + 32 < e ? load16(p + b + 32) : z;
      uint4 a3 = b + 48 < e ? load16(p + b + 48) : z;
      for (uint32_t c = b; c < e; c += 64) {
        uint4 b0 = z, b1 = z, b2 = z, b3 = z;
        if (c + 64 < e) b0 = load16(p + c + 64);
        if (c + 80 < e) b1 = load16(p + c + 80);
        if (c + 96 < e) b2 = load16(p + c + 96);
        if (c + 112 < e) b3 = load16(p + c + 112);
        chunk(a0, c);
        if (c + 16 < e) chunk(a1, c + 16);
        if (c + 32 < e) chunk(a2, c + 32);
        if (c + 48 < e) chunk(a3, c + 48);
        a0 = b0;
        a1 = b1;
        a2 = b2;
        a3 = b3;
      }
    }
    // prefix over the four lanes of the leaf
    uint32_t incl = D;
    uint32_t v = (uint32_t)__shfl_up((int)incl, 1, 4);
    if (q >= 1) incl += v;
    v = (uint32_t)__shfl_up((int)incl, 2, 4);
    if (q >= 2) incl += v;
    const uint32_t total = (uint32_t)__shfl((int)incl, 3, 4);
    if (q == 0)
      lastk[f] = h + total;
    else
      ck[f * 3 + q - 1] = b < u ? LeafCkpt{b, incl - D, partial, (7 * run) | (run << 8)} : LeafCkpt{~0u, 0, 0, 0};
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
  uint64_t img;   // byte offset of the leaf's image: main array, or overflow arena with kImgArena set
};
constexpr uint64_t kImgArena = 1ull << 63;

__global__ void k_src_info(SrcLeaves src, const uint64_t* __restrict__ head, const uint64_t* __restrict__ lastk,
                           const uint32_t* __restrict__ rank, const uint32_t* __restrict__ ne, uint64_t L,
                           SrcInfo* __restrict__ info) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < L;
       f += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = src.used[f];
    if (u == 0) continue;
    SrcInfo I;
    I.head = head[f];
    I.lastk = lastk[f];
    I.used = u;
    I.next = ne[rank[f] + 1];
    I.img = u > src.S ? (src.ovf[f] | kImgArena) : f * (uint64_t)src.S;
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
  const LeafCkpt* ck;     // three per old leaf (narrow leaves)
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
      // Each threshold's walk starts at the last quarter checkpoint at or
      // before that byte (the head for the first quarter).
      auto first_byte = [&](uint64_t t) -> uint32_t {
        const uint64_t over = t - c0;
        return over <= hc ? 8u : (uint32_t)min<uint64_t>(over - hc + 8u, 0xffffffffull);
      };
      const LeafCkpt K1 = a.ck[f * 3], K2 = a.ck[f * 3 + 1], K3 = a.ck[f * 3 + 2];
      uint32_t bp = first_byte(T);
      while (j < jend) {
        uint32_t cs = 0, key32 = 0, acc = 0, sh = 0, start = 0;
        auto take = [&](const LeafCkpt& k) {
          if (k.c != ~0u && k.c <= bp) {
            cs = k.c;
            key32 = k.K - k.partial;
            acc = k.partial;
            sh = k.shrun & 0xffu;
            start = k.c - (k.shrun >> 8);
          }
        };
        take(K1);
        take(K2);
        take(K3);
        bool hit = false;
        uint4 nxt = load16(leaf + cs);
        for (uint32_t c = cs; c < u && !hit; c += 16) {
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
            if (!cm && !hit && start >= 8u && start >= bp) {
              const uint32_t end = c + (uint32_t)i;
              const uint64_t P = c0 + hc + start - 8u;
              do {
                put_rec(rec, j, f, h + key32, P, start, end + 1u - start);
                j++;
                T = split_threshold(j, total, Lt);
                bp = first_byte(T);
              } while (j < jend && start >= bp);
              hit = true;
            }
            acc &= cm;
            start = cm ? start : c + (uint32_t)i + 1u;
            sh = (sh + 7u) & cm;
          }
        }
        if (!hit) break;  // no code of f starts at or past bp
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

// Destination image in registers: lane l holds bytes [16 l + 1024 t, + 16) of
// stripe t (kStripes stripes: leaves up to 1024 * kStripes bytes).  Pieces are
// ORed in, so a piece only has to zero the bytes outside its own range.
template <int kStripes>
struct SplitImage {
  uint4 o[kStripes];
};

// Bytes [a, b) of a dword as a mask (a, b clamped to [0, 4]).
__device__ __forceinline__ uint32_t byte_mask(int32_t a, int32_t b) {
  a = max(a, 0);
  b = min(b, 4);
  if (a >= b) return 0u;
  const uint32_t hi = b == 4 ? 0xffffffffu : (1u << (8 * b)) - 1u;
  return hi & ~((1u << (8 * a)) - 1u);
}

// Output bytes [ob, ob + n) take source bytes [sb, sb + n) of src, which is
// 16-byte aligned and readable in whole 16-byte chunks that hold any of those
// bytes.  Each lane loads the (at most two) aligned source chunks under its
// output chunk and shifts them into place with byte aligns; the shift is the
// same for every lane.
template <int kStripes>
__device__ __forceinline__ void image_or_run(SplitImage<kStripes>& im, uint32_t S, const uint8_t* __restrict__ src,
                                             uint32_t sb, uint32_t ob, uint32_t n) {
  const int32_t lane = lane_id();
  const int32_t lo = (int32_t)sb, hi = (int32_t)(sb + n);
  const uint32_t R = (sb - ob) & 15u;
  const uint32_t qw = R >> 2, r = R & 3u;
#pragma unroll
  for (int t = 0; t < kStripes; t++) {
    const int32_t q16 = 1024 * t + 16 * lane;
    if (q16 >= (int32_t)S || q16 + 16 <= (int32_t)ob || q16 >= (int32_t)(ob + n)) continue;
    const int32_t s0 = q16 - (int32_t)ob + (int32_t)sb;  // may be below 0 by up to 15
    const int32_t c0 = (s0 >> 4) * 16, c1 = c0 + 16;
    uint4 A = make_uint4(0, 0, 0, 0), B = A;
    if (c0 < hi && c0 + 16 > lo) A = load16(src + c0);
    if (c1 < hi && c1 + 16 > lo) B = load16(src + c1);
    const uint32_t w[8] = {A.x, A.y, A.z, A.w, B.x, B.y, B.z, B.w};
    uint32_t x[5];
#pragma unroll
    for (int k = 0; k < 5; k++) x[k] = qw == 0 ? w[k] : qw == 1 ? w[k + 1] : qw == 2 ? w[k + 2] : w[k + 3];
    const int32_t a = (int32_t)ob - q16, b = (int32_t)(ob + n) - q16;
    im.o[t].x |= __builtin_amdgcn_alignbyte(x[1], x[0], r) & byte_mask(a, b);
    im.o[t].y |= __builtin_amdgcn_alignbyte(x[2], x[1], r) & byte_mask(a - 4, b - 4);
    im.o[t].z |= __builtin_amdgcn_alignbyte(x[3], x[2], r) & byte_mask(a - 8, b - 8);
    im.o[t].w |= __builtin_amdgcn_alignbyte(x[4], x[3], r) & byte_mask(a - 12, b - 12);
  }
}

// The code of d (len bytes) at output byte cp.
template <int kStripes>
__device__ __forceinline__ void image_or_code(SplitImage<kStripes>& im, uint32_t S, uint32_t cp, uint64_t d, uint32_t len) {
  const int32_t lane = lane_id();
#pragma unroll
  for (int t = 0; t < kStripes; t++) {
    const int32_t q16 = 1024 * t + 16 * lane;
    if (q16 >= (int32_t)S || q16 + 16 <= (int32_t)cp || q16 >= (int32_t)(cp + len)) continue;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int i = 0; i < 16; i++) {
      const uint32_t k = (uint32_t)(q16 + i) - cp;
      if (k < len) {
        const uint32_t byte = (uint32_t)((d >> (7 * k)) & 0x7fu) | (k + 1 < len ? 0x80u : 0u);
        w[i >> 2] |= byte << (8 * (i & 3));
      }
    }
    im.o[t].x |= w[0];
    im.o[t].y |= w[1];
    im.o[t].z |= w[2];
    im.o[t].w |= w[3];
  }
}

// Value of lane t (uniform t) of a per-lane struct of whole dwords.
template <class T>
__device__ __forceinline__ T lane_value(const T& v, uint32_t t) {
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
  uint32_t w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (uint32_t k = 0; k < sizeof(T) / 4; k++) w[k] = (uint32_t)__builtin_amdgcn_readlane((int)w[k], (int)t);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Address of an image offset (global memory: both bases are kernel arguments).
__device__ __forceinline__ const uint8_t* img_ptr(const SrcLeaves& src, uint64_t img) {
  return (img & kImgArena) ? src.arena + (img & ~kImgArena) : src.bytes + img;
}

// One run of old bytes in a destination image: output bytes [ob, ob + n) are
// source bytes [sb, sb + n) of the image at src.
struct RunDesc {
  uint64_t img;  // image offset (img_ptr)
  uint32_t sb, ob, n;
};

// The two aligned source chunks under the lane's output chunk q16 (stripe 0).
// Loads are unconditional: a chunk that holds no byte of the run is clamped to
// one that does (n = 0: the image's first chunk), and its bytes are masked off.
struct RunChunks {
  uint4 A, B;
};

__device__ __forceinline__ RunChunks run_load(const SrcLeaves& src, const RunDesc& r, int32_t q16) {
  int32_t c0 = 0, c1 = 0;
  if (r.n) {
    const int32_t s0 = q16 - (int32_t)r.ob + (int32_t)r.sb;
    const int32_t cf = ((int32_t)r.sb >> 4) * 16, cl = ((int32_t)(r.sb + r.n - 1) >> 4) * 16;
    c0 = min(max((s0 >> 4) * 16, cf), cl);
    c1 = min(max((s0 >> 4) * 16 + 16, cf), cl);
  }
  const uint8_t* p = img_ptr(src, r.img);
  RunChunks c;
  c.A = load16(p + c0);
  c.B = load16(p + c1);
  return c;
}

__device__ __forceinline__ void run_apply(uint4& o, const RunChunks& c, const RunDesc& r, int32_t q16) {
  if (r.n == 0 || q16 + 16 <= (int32_t)r.ob || q16 >= (int32_t)(r.ob + r.n)) return;
  const uint32_t R = (r.sb - r.ob) & 15u;
  const uint32_t qw = R >> 2, rr = R & 3u;
  const uint32_t w[8] = {c.A.x, c.A.y, c.A.z, c.A.w, c.B.x, c.B.y, c.B.z, c.B.w};
  uint32_t x[5];
#pragma unroll
  for (int k = 0; k < 5; k++) x[k] = qw == 0 ? w[k] : qw == 1 ? w[k + 1] : qw == 2 ? w[k + 2] : w[k + 3];
  const int32_t a = (int32_t)r.ob - q16, b = (int32_t)(r.ob + r.n) - q16;
  o.x |= __builtin_amdgcn_alignbyte(x[1], x[0], rr) & byte_mask(a, b);
  o.y |= __builtin_amdgcn_alignbyte(x[2], x[1], rr) & byte_mask(a - 4, b - 4);
  o.z |= __builtin_amdgcn_alignbyte(x[3], x[2], rr) & byte_mask(a - 8, b - 8);
  o.w |= __builtin_amdgcn_alignbyte(x[4], x[3], rr) & byte_mask(a - 12, b - 12);
}

// A destination leaf made of at most two runs of old bytes with one spliced
// code between them (the common case: the leaf starts inside one old leaf and
// ends in it or in the next non-empty one).  fast = false: more runs follow,
// the writer walks them.
struct LeafPlan {
  RunDesc r1, r2;       // r2.n = 0 when absent
  uint64_t clo, chi;    // bytes of the spliced code, little-endian (zero past its length)
  uint32_t cpos, clen;  // its output position and length (clen = 0: none)
  uint32_t end;         // output length after r2
  uint32_t fast, bad;
};

__device__ __forceinline__ bool split_hops(const SplitArgs& a, uint64_t f, const SrcInfo& I, const SplitRec& B) {
  return f != B.leaf && I.next < a.L && !(I.next == B.leaf && B.p == 0);
}

__device__ __forceinline__ LeafPlan make_plan(const SplitArgs& a, uint32_t S, const SplitRec& A, const SplitRec& B,
                                              const SrcInfo& I, const SrcInfo& N) {
  LeafPlan P;
  P.r1 = RunDesc{0, 0, 0, 0};
  P.r2 = P.r1;
  P.clo = P.chi = 0;
  P.cpos = P.clen = 0;
  P.end = 8;
  P.fast = false;
  P.bad = A.leaf >= a.L;
  if (P.bad) return P;
  const uint64_t f = A.leaf;
  const uint32_t bs = A.p == 0 ? 8u : A.p + A.cost;
  const uint32_t be = f == B.leaf ? B.p : I.used;
  if (be < bs || be > I.used || 8u + (be - bs) > S) {
    P.bad = true;
    return P;
  }
  P.r1 = RunDesc{I.img, bs, 8u, be - bs};
  uint32_t pos = 8u + (be - bs);
  P.end = pos;
  P.fast = true;
  if (!split_hops(a, f, I, B)) return P;
  const uint64_t d = N.head - I.lastk;
  const uint32_t len = vlen(d);
  if (pos + len > S) {
    P.bad = true;
    return P;
  }
  uint64_t v = d;
  for (uint32_t k = 0; k < len; k++) {
    const uint64_t byte = (v & 0x7fu) | (k + 1 < len ? 0x80u : 0u);
    v >>= 7;
    if (k < 8)
      P.clo |= byte << (8 * k);
    else
      P.chi |= byte << (8 * (k - 8));
  }
  P.cpos = pos;
  P.clen = len;
  pos += len;
  P.end = pos;
  const uint64_t f2 = I.next;
  if (split_hops(a, f2, N, B)) {
    P.fast = false;
    return P;
  }
  const uint32_t be2 = f2 == B.leaf ? B.p : N.used;
  if (be2 < 8u || be2 > N.used || pos + (be2 - 8u) > S) {
    P.bad = true;
    return P;
  }
  P.r2 = RunDesc{N.img, 8u, pos, be2 - 8u};
  P.end = pos + (be2 - 8u);
  return P;
}

// The spliced code into the lane's output chunk q16: the code's bytes shifted
// into place (bytes past its length are zero).
__device__ __forceinline__ void code_apply(uint4& o, const LeafPlan& P, int32_t q16) {
  if (P.clen == 0 || q16 + 16 <= (int32_t)P.cpos || q16 >= (int32_t)(P.cpos + P.clen)) return;
  const unsigned __int128 C = ((unsigned __int128)P.chi << 64) | P.clo;
  const int32_t sh = q16 - (int32_t)P.cpos;  // in (-16, 10)
  const unsigned __int128 W = sh >= 0 ? (C >> (8 * sh)) : (C << (8 * -sh));
  o.x |= (uint32_t)W;
  o.y |= (uint32_t)(W >> 32);
  o.z |= (uint32_t)(W >> 64);
  o.w |= (uint32_t)(W >> 96);
}

// Writes the destination leaves (a planned split: no leaf is empty or above S
// bytes).  A wave takes 64 consecutive destination leaves.  For leaves up to
// 1024 bytes, lane l first plans leaf j0 + l (its records, the descriptors of
// its first two source leaves, runs and spliced code), so the dependent
// metadata loads of 64 leaves overlap; the wave then builds each leaf's image
// in registers (head, runs of old bytes shifted into place, the code) and
// stores it with one 16-byte store per lane, zero fill included, loading the
// next leaf's source chunks before it stores the current one.  Leaves of more
// than two runs, and larger leaves, walk their source leaves one by one.  A
// leaf whose length disagrees with the plan sets the error counter and is not
// written.  Nothing is written when the plan's check failed (*fail != 0).
template <int kStripes>
__global__ void __launch_bounds__(kWave) k_split_write(SplitArgs a, uint32_t S, const SplitRec* __restrict__ rec,
                                                       uint8_t* __restrict__ dbytes, uint32_t* __restrict__ dused,
                                                       uint64_t* __restrict__ dhead, Counters* ctr,
                                                       const uint32_t* __restrict__ fail) {
  if (*fail) return;  // the plan failed its check: nothing to write
  const int lane = lane_id();
  const int32_t q16 = 16 * lane;
  // any number of runs, descriptors and source chunks loaded on demand
  auto walk = [&](SplitImage<kStripes>& im, const SplitRec& A, const SplitRec& B, uint32_t& pos) -> bool {
    uint64_t f = A.leaf;
    SrcInfo I = a.info[f];
    uint32_t bs = A.p == 0 ? 8u : A.p + A.cost;
    for (;;) {
      const uint32_t u = I.used;
      const bool last = f == B.leaf;  // the end lies inside leaf f (B.p >= 8)
      const uint64_t fn = I.next;
      const bool hop = split_hops(a, f, I, B);
      SrcInfo In{};
      if (hop) In = a.info[fn];
      const uint32_t be = last ? B.p : u;
      if (be < bs || be > u || pos + (be - bs) > S) return false;
      image_or_run(im, S, img_ptr(a.src, I.img), bs, pos, be - bs);
      pos += be - bs;
      if (!hop) return true;
      const uint64_t d = In.head - I.lastk;
      const uint32_t len = vlen(d);
      if (pos + len > S) return false;
      image_or_code(im, S, pos, d, len);
      pos += len;
      f = fn;
      I = In;
      bs = 8;
    }
  };
  auto finish = [&](uint64_t j, uint64_t x, uint64_t want, bool ok, uint32_t pos, const SplitImage<kStripes>& im) {
    if (!ok || pos != want) {
      if (lane == 0) atomicOr(&ctr->error, 1u);
      return;
    }
    uint8_t* dst = dbytes + j * (uint64_t)S;
#pragma unroll
    for (int s = 0; s < kStripes; s++) {
      const uint32_t q = 1024u * s + 16u * (uint32_t)lane;
      if (q < S) *reinterpret_cast<uint4*>(dst + q) = im.o[s];
    }
    if (lane == 0) {
      dused[j] = pos;
      dhead[j] = x;
    }
  };
  for (uint64_t j0 = (uint64_t)blockIdx.x * kWave; j0 < a.Lt; j0 += (uint64_t)gridDim.x * kWave) {
    const uint32_t nj = (uint32_t)min<uint64_t>(kWave, a.Lt - j0);
    if constexpr (kStripes == 1) {
      struct LeafWork {
        LeafPlan P;
        uint64_t x, want;
      };
      LeafWork Wl;
      {
        const SplitRec A = rec[j0 + min<uint32_t>((uint32_t)lane, nj - 1)];
        const SplitRec B = rec[j0 + min<uint32_t>((uint32_t)lane, nj - 1) + 1];
        SrcInfo I{}, N{};
        if (A.leaf < a.L) {
          I = a.info[A.leaf];
          if (split_hops(a, A.leaf, I, B)) N = a.info[I.next];
        }
        Wl.P = make_plan(a, S, A, B, I, N);
        Wl.x = A.x;
        Wl.want = 8u + (B.P - A.P - A.cost);
      }
      // two buffers of source chunks, used in turn (no register copies
      // between steps, so waiting for one never waits for the other)
      auto step = [&](uint32_t t, const LeafWork& W, const RunChunks& C1, const RunChunks& C2, LeafWork& Wn,
                      RunChunks& D1, RunChunks& D2) {
        // next leaf's source chunks first (the last leaf reloads its own)
        Wn = lane_value(Wl, t + 1 < nj ? t + 1 : t);
        D1 = run_load(a.src, Wn.P.r1, q16);
        D2 = run_load(a.src, Wn.P.r2, q16);
        SplitImage<1> im;
        im.o[0] = make_uint4(0, 0, 0, 0);
        if (lane == 0) {
          im.o[0].x = (uint32_t)W.x;
          im.o[0].y = (uint32_t)(W.x >> 32);
        }
        bool ok = !W.P.bad;
        uint32_t pos = W.P.end;
        if (ok) {
          if (W.P.fast) {
            run_apply(im.o[0], C1, W.P.r1, q16);
            run_apply(im.o[0], C2, W.P.r2, q16);
            code_apply(im.o[0], W.P, q16);
          } else {
            pos = 8;
            ok = walk(im, rec[j0 + t], rec[j0 + t + 1], pos);
          }
        }
        finish(j0 + t, W.x, W.want, ok, pos, im);
      };
      LeafWork W0 = lane_value(Wl, 0), W1;
      RunChunks C1 = run_load(a.src, W0.P.r1, q16), C2 = run_load(a.src, W0.P.r2, q16), D1, D2;
      for (uint32_t t = 0; t < nj; t += 2) {
        step(t, W0, C1, C2, W1, D1, D2);
        if (t + 1 < nj) step(t + 1, W1, D1, D2, W0, C1, C2);
      }
    } else {
      for (uint32_t t = 0; t < nj; t++) {
        const SplitRec A = rec[j0 + t], B = rec[j0 + t + 1];
        SplitImage<kStripes> im;
#pragma unroll
        for (int s = 0; s < kStripes; s++) im.o[s] = make_uint4(0, 0, 0, 0);
        if (lane == 0) {
          im.o[0].x = (uint32_t)A.x;
          im.o[0].y = (uint32_t)(A.x >> 32);
        }
        uint32_t pos = 8;
        const bool ok = A.leaf < a.L && walk(im, A, B, pos);
        finish(j0 + t, A.x, 8u + (B.P - A.P - A.cost), ok, pos, im);
      }
    }
  }
}

}  // namespace cpma_dev
