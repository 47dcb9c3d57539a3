// Wave-cooperative batch merge: one wave per touched leaf (the batch-merge phase
// of Section "Parallel Batch Updates in a PMA").  The wave decodes the leaf's
// keys into LDS, ranks the slice's batch keys among them, and writes the merged
// encoding with byte offsets from wave prefix sums (DPP), so every step is a
// handful of parallel passes over at most S / 16 lanes' worth of data.
//
// Insert (slice of at most 64 keys, one per lane): new keys with the same rank r
// (the number of old keys below them) form the group inserted before old key r.
// Each old key's code is recomputed against its new predecessor (the last key of
// its group, else the previous old key).  Groups are runs of lanes, so their
// ranks, byte totals and last keys go to 64-entry tables from DPP scans, and a
// lane walking its block of old keys meets them in rank order.  Delete (any
// slice length): present keys are flagged by rank in a bit mask, and each kept
// key's code is recomputed against the previous kept key.  LDS per wave stays
// near 10 KB (the decoded keys dominate), which keeps several waves per SIMD.
#pragma once
#include "leaf.hpp"
#include "update.hpp"

namespace cpma_dev {

constexpr uint32_t kWaveSlice = 64;   // insert slice handled per wave
constexpr uint32_t kWaveMaxS = 1024;  // leaf size handled per wave (16 bytes per lane)

// Code length and code bytes of a delta held in the key type (32-bit offsets
// in the narrow instance).
__device__ __forceinline__ uint32_t vlen_t(uint32_t d) { return (32u - (uint32_t)__clz((int)(d | 1u)) + 6u) / 7u; }
__device__ __forceinline__ uint32_t vlen_t(uint64_t d) { return vlen(d); }
template <typename T>
__device__ __forceinline__ void vput_t(uint8_t* dst, T d) {
  uint32_t n = 0;
  while (d >= 0x80) {
    dst[n++] = (uint8_t)(d | 0x80);
    d >>= 7;
  }
  dst[n] = (uint8_t)d;
}
__device__ __forceinline__ uint32_t dpp_prev_t(uint32_t v) { return dpp_prev32(v); }
__device__ __forceinline__ uint64_t dpp_prev_t(uint64_t v) { return dpp_prev64(v); }
__device__ __forceinline__ uint32_t readlane_t(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t readlane_t(uint64_t v, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}

// Key x (offset from base) as a leaf head (8 bytes) or as the code of x - pred.
template <typename KT>
__device__ __forceinline__ void put_key_bytes(uint8_t* dst, bool head, KT x, KT pred, uint64_t base) {
  if (head)
    put_le64(dst, base + (uint64_t)x);
  else
    vput_t<KT>(dst, (KT)(x - pred));
}

// KT = uint32_t: keys are stored in LDS as offsets from the segment's smallest
// possible key (segments flagged wide are handed to the 64-bit instance), which
// halves the dominant LDS array.  KT = uint64_t: processes the handed-over list,
// or with all_segments every segment not routed to the heavy merge (small
// batches: one launch instead of two).
//
// The body runs as one wave with its own LDS (MergeLds); the merge kernel is one
// wave per block, and the fused small-batch kernel runs several such waves in
// one block, each on its own segments.  The wave's first segment is t0, it
// takes every tstep-th one after it, and it leaves its totals in slot `slot`.
template <typename KT>
struct MergeLds {
  alignas(16) uint8_t out[kWaveMaxS];  // the merged leaf image
  KT K[kWaveMaxS];                     // decoded old keys
  KT GK[kWaveSlice];                   // group g: its last key (new predecessor of old key GR[g])
  uint32_t GR[kWaveSlice + 1];         // group g: rank; GR[ng] closes the table
  uint32_t GB[kWaveSlice];             // group g: bytes of its codes
  uint32_t GS[kWaveSlice];             // group g: output offset
  uint32_t DF[kWaveMaxS / 32];         // delete flags by old index
};

// Orders the LDS traffic of the lanes sharing one MergeLds: the whole (one-wave)
// block in the merge kernel, one wave of a larger block otherwise -- the same
// workgroup-scope fences, without the block-wide barrier.
template <bool kWaveOnly>
__device__ __forceinline__ void merge_sync() {
  if constexpr (kWaveOnly) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

template <typename KT, bool kWaveOnly>
__device__ __forceinline__ void merge_wave_body(MergeArgs a, int all_segments, MergeLds<KT>& L, uint64_t t0,
                                                uint64_t tstep, uint64_t slot) {
  constexpr bool kNarrow = sizeof(KT) == 4;
  KT* const K = L.K;
  KT* const GK = L.GK;
  uint32_t* const GR = L.GR;
  uint32_t* const GB = L.GB;
  uint32_t* const GS = L.GS;
  uint32_t* const DF = L.DF;
  uint8_t* const out = L.out;
  const int lane = lane_id();
  const uint32_t S = a.S;
  const bool listed = !kNarrow && !all_segments;
  const uint64_t T = listed ? (uint64_t)a.ctr->nwide : (uint64_t)a.ctr->T;
  const uint32_t pos0 = 16u * lane;
  unsigned long long delta = 0, alg = 0;
  auto seg_of = [&](uint64_t t) -> uint64_t { return listed ? (uint64_t)a.wide_list[t] : t; };
  auto skip = [&](const uint4& d) { return kNarrow ? d.w != 0 : (all_segments && d.w == 2); };
  // Software pipeline: the next segment's descriptor, leaf bytes and batch keys
  // are loaded while the current one is merged.
  uint4 d_cur = make_uint4(0, 0, 0, 0), d_nxt = d_cur;
  uint32_t e_cur = 0, e_nxt = 0;
  uint64_t s_cur = 0, s_nxt = 0;
  uint4 w_cur = make_uint4(0, 0, 0, 0), w_nxt = w_cur;
  uint64_t b_cur = 0, b_nxt = 0;
  uint64_t t = t0;
  if (t < T) {
    s_cur = seg_of(t);
    d_cur = a.seg_desc[s_cur];
    e_cur = a.seg_begin[s_cur + 1];
    if (!skip(d_cur)) {
      if (pos0 < d_cur.z) w_cur = *reinterpret_cast<const uint4*>(a.bytes + (uint64_t)d_cur.x * S + pos0);
      if ((uint32_t)lane < e_cur - d_cur.y) b_cur = a.B[d_cur.y + lane];
    }
  }
  for (; t < T; t += tstep) {
    const uint64_t tn = t + tstep;
    if (tn < T) {
      s_nxt = seg_of(tn);
      d_nxt = a.seg_desc[s_nxt];
      e_nxt = a.seg_begin[s_nxt + 1];
    }
    const uint64_t s = s_cur;
    const uint64_t leaf = d_cur.x;
    const uint32_t b = d_cur.y, e = e_cur;
    const uint32_t nb = e - b;
    const uint32_t used0 = d_cur.z;
    const bool wide = skip(d_cur);
    const uint4 w = w_cur;
    const uint64_t bj0 = b_cur;
    if (tn < T) {
      w_nxt = make_uint4(0, 0, 0, 0);
      b_nxt = 0;
      if (!skip(d_nxt)) {
        if (pos0 < d_nxt.z) w_nxt = *reinterpret_cast<const uint4*>(a.bytes + (uint64_t)d_nxt.x * S + pos0);
        if ((uint32_t)lane < e_nxt - d_nxt.y) b_nxt = a.B[d_nxt.y + lane];
      }
    }
    s_cur = s_nxt;
    d_cur = d_nxt;
    e_cur = e_nxt;
    w_cur = w_nxt;
    b_cur = b_nxt;
    if (wide) continue;  // routed to the wide or spill list
    // smallest possible key of the segment: the old head or the first slice key
    uint64_t base = 0;
    if (kNarrow) {
      const uint64_t hd = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)w.y, 0) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)w.x, 0);
      const uint64_t b0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bj0 >> 32), 0) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bj0, 0);
      base = used0 ? min(hd, b0) : b0;
    }
    const uint64_t* Bg = a.B + b;
    uint8_t* lp = a.bytes + leaf * (uint64_t)S;
    uint32_t nA;
    if constexpr (kNarrow) {
      const uint64_t hd = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)w.y, 0) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)w.x, 0);
      nA = wave_decode_narrow(w, used0, (uint32_t)(hd - base), [&](uint32_t i, uint32_t x) { K[i] = (KT)x; });
    } else {
      nA = wave_decode_regs(w, used0, [&](uint32_t i, uint64_t x, uint64_t) { K[i] = (KT)x; });
    }
    wave_zero(out, S);
    // lane-contiguous block of old-key indices [i0, i1) over [0, nA] (index nA: trailing group)
    const uint32_t m = (nA + 1 + kWave - 1) / kWave;
    const uint32_t i0 = min(nA + 1, (uint32_t)lane * m), i1 = min(nA + 1, i0 + m);
    uint32_t U = 0;
    uint64_t first_key = kNoKey;
    uint64_t arena_off = 0;
    bool to_arena = false;
    if (a.is_insert) {
      // keys below are offsets from base (the key type of this instance)
      const bool has_b = (uint32_t)lane < nb;
      const KT bj = has_b ? (KT)(bj0 - base) : (KT)0;
      uint32_t r = 0xffffffffu;
      bool isnew = false;
      if (has_b) {
        r = lds_lower_bound<KT>(K, nA, bj);
        isnew = !(r < nA && K[r] == bj);
      }
      const KT b_prev = dpp_prev_t(bj);
      const uint32_t r_prev = dpp_prev32(r);
      const uint32_t new_prev = dpp_prev32(isnew ? 1u : 0u);
      const uint32_t r_next = dpp_next32(r);
      const uint32_t new_next = dpp_next32(isnew ? 1u : 0u);
      const bool same_prev = lane > 0 && new_prev && r_prev == r;
      const bool same_next = lane < kWave - 1 && new_next && r_next == r;
      bool has_pred = false;
      KT pred = 0;
      if (isnew) {
        if (same_prev) {
          pred = b_prev;
          has_pred = true;
        } else if (r > 0) {
          pred = K[r - 1];
          has_pred = true;
        }
      }
      const uint32_t cost = isnew ? (has_pred ? vlen_t((KT)(bj - pred)) : 8u) : 0u;
      const uint32_t incl = dpp_incl_scan<uint32_t>(cost);
      const uint32_t ex = incl - cost;
      const bool gstart = isnew && !same_prev;
      const uint64_t smask = __ballot(gstart);
      const uint32_t ng = (uint32_t)__popcll(smask);
      const uint32_t gid = (uint32_t)__popcll(smask & ((2ull << lane) - 1ull)) - 1u;
      const uint32_t exfirst = dpp_incl_max(gstart ? ex : 0u);  // ex of the group's first lane
      if (gstart) GR[gid] = r;
      if (isnew && !same_next) {
        GB[gid] = incl - exfirst;
        GK[gid] = bj;
      }
      if (lane == 0) GR[ng] = 0xffffffffu;
      const uint64_t newmask = __ballot(isnew);
      const uint32_t nnew = (uint32_t)__popcll(newmask);
      merge_sync<kWaveOnly>();
      // first group at or after this lane's block
      uint32_t p0 = 0;
      {
        uint32_t hi = ng;
        while (p0 < hi) {
          const uint32_t mid = (p0 + hi) >> 1;
          if (GR[mid] < i0)
            p0 = mid + 1;
          else
            hi = mid;
        }
      }
      const KT k_before = (i0 > 0 && i0 <= nA) ? K[i0 - 1] : (KT)0;  // old key before the block
      // sweep 1: bytes per index (group before old key i, then old key i)
      uint32_t lt = 0;
      uint32_t p = p0;
      KT kp = k_before;
      for (uint32_t i = i0; i < i1; i++) {
        const bool gh = GR[p] == i;
        uint32_t t = gh ? GB[p] : 0u;
        if (i < nA) {
          const KT x = K[i];
          const bool hp = gh || i > 0;
          const KT np = gh ? GK[p] : kp;
          t += hp ? vlen_t((KT)(x - np)) : 8u;
          kp = x;
        }
        lt += t;
        p += gh ? 1u : 0u;
      }
      const uint32_t lincl = dpp_incl_scan<uint32_t>(lt);
      U = lane63_u32(lincl);
      if (U > S) {
        const uint64_t need = ((uint64_t)U + 15) & ~15ull;
        const uint64_t off = arena_region(a, s);
        if (off + need > a.arena_cap) {
          if (lane == 0) atomicOr(&a.ctr->error, 1u);
          continue;
        }
        arena_off = off;
        to_arena = true;
      }
      // sweep 2: write old keys, record group starts; then the new keys at
      // their group's start + their offset inside the group.  Instantiated
      // once for the LDS image and once for the arena, so that each copy's
      // stores have a known address space (a pointer that may be either
      // compiles to generic stores, far slower for LDS).
      auto write_merged = [&](auto dst) {
        uint32_t run = lincl - lt;
        uint32_t p = p0;
        KT kp = k_before;
        for (uint32_t i = i0; i < i1; i++) {
          const bool gh = GR[p] == i;
          const uint32_t gb = gh ? GB[p] : 0u;
          if (gh) GS[p] = run;
          if (i < nA) {
            const KT x = K[i];
            const bool hp = gh || i > 0;
            const KT np = gh ? GK[p] : kp;
            const uint32_t c = hp ? vlen_t((KT)(x - np)) : 8u;
            put_key_bytes<KT>(dst + run + gb, !hp, x, np, base);
            run += gb + c;
            kp = x;
          } else {
            run += gb;
          }
          p += gh ? 1u : 0u;
        }
        merge_sync<kWaveOnly>();
        if (isnew) put_key_bytes<KT>(dst + GS[gid] + (ex - exfirst), !has_pred, bj, pred, base);
      };
      if (to_arena)
        write_merged(a.arena + arena_off);
      else
        write_merged(out);
      uint64_t firstnew = kNoKey;
      if (nnew) firstnew = base + (uint64_t)readlane_t(bj, __ffsll((unsigned long long)newmask) - 1);
      first_key = nA ? min(base + (uint64_t)K[0], firstnew) : firstnew;
      delta += nnew;
    } else {
      for (uint32_t i = lane; i < kWaveMaxS / 32; i += kWave) DF[i] = 0;
      merge_sync<kWaveOnly>();
      for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
        const uint32_t j = c0 + lane;
        if (j < nb) {
          const KT xr = (KT)(Bg[j] - base);
          const uint32_t r = lds_lower_bound<KT>(K, nA, xr);
          if (r < nA && K[r] == xr) atomicOr(&DF[r >> 5], 1u << (r & 31));
        }
      }
      merge_sync<kWaveOnly>();
      auto gone = [&](uint32_t i) { return (DF[i >> 5] >> (i & 31)) & 1u; };
      // last kept index (+1) inside this lane's block, then across lanes
      uint32_t lastk = 0, lt = 0, nrem = 0;
      for (uint32_t i = i0; i < min(i1, nA); i++) {
        if (!gone(i)) lastk = i + 1;
        else nrem++;
      }
      const uint32_t pk_in = dpp_prev32(dpp_incl_max(lastk));  // 0 = none before this block
      const KT kin = pk_in ? K[pk_in - 1] : (KT)0;
      uint32_t pk = pk_in;
      KT kp = kin;
      for (uint32_t i = i0; i < min(i1, nA); i++) {
        if (gone(i)) continue;
        const KT x = K[i];
        lt += pk ? vlen_t((KT)(x - kp)) : 8u;
        pk = i + 1;
        kp = x;
      }
      const uint32_t lincl = dpp_incl_scan<uint32_t>(lt);
      U = lane63_u32(lincl);
      uint32_t run = lincl - lt;
      pk = pk_in;
      kp = kin;
      for (uint32_t i = i0; i < min(i1, nA); i++) {
        if (gone(i)) continue;
        const KT x = K[i];
        put_key_bytes<KT>(out + run, pk == 0, x, kp, base);
        run += pk ? vlen_t((KT)(x - kp)) : 8u;
        pk = i + 1;
        kp = x;
      }
      // smallest kept key: the key at the first index whose flag is clear
      uint32_t fk = 0xffffffffu;
      for (uint32_t i = i0; i < min(i1, nA); i++)
        if (!gone(i)) {
          fk = i;
          break;
        }
      uint32_t fkmin = fk;
      for (int d = 32; d > 0; d >>= 1) fkmin = min(fkmin, (uint32_t)__shfl_xor((int)fkmin, d, kWave));
      first_key = (fkmin != 0xffffffffu) ? base + (uint64_t)K[fkmin] : kNoKey;
      delta += wave_sum(nrem);
    }
    merge_sync<kWaveOnly>();
    if (!to_arena) {
      const uint32_t len = ((max(used0, U) + 15u) & ~15u);
      wave_copy16(lp, out, len);
      alg += used0 + len + 8ull * nb + 20;
    } else {
      if (lane == 0) a.ovf[leaf] = arena_off;
      alg += used0 + U + 8ull * nb + 20;
    }
    if (lane == 0) {
      a.used[leaf] = U;
      a.head[leaf] = U ? first_key : kNoKey;
    }
    merge_sync<kWaveOnly>();
  }
  // no atomics on shared counters (thousands of waves would serialise on
  // them): each wave leaves its totals in its own slot, summed by k_fold_parts
  if (lane == 0) {
    a.part[2 * slot] = delta;
    a.part[2 * slot + 1] = alg;
  }
}

template <typename KT>
__global__ void __launch_bounds__(kWave) k_merge_wave(MergeArgs a, int all_segments = 0) {
  __shared__ MergeLds<KT> L;
  merge_wave_body<KT, false>(a, all_segments, L, blockIdx.x, gridDim.x, blockIdx.x);
}

}  // namespace cpma_dev
