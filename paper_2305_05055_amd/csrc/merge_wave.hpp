// Wave-cooperative batch merge: one wave per touched leaf (the batch-merge phase
// of Section "Parallel Batch Updates in a PMA").  The wave decodes the leaf's
// keys into LDS, ranks the slice's batch keys among them, and writes the merged
// encoding with byte offsets from wave prefix sums (DPP), so every step is a
// handful of parallel passes over at most S / 16 lanes' worth of data.
//
// Insert (slice of at most 64 keys, one per lane): new keys with the same rank r
// (the number of old keys below them) form the group inserted before old key r.
// Each old key's code is recomputed against its new predecessor (the last key of
// its group, else the previous old key); group bytes and offsets come from LDS
// atomics and prefix sums.  Delete (any slice length): present keys are flagged
// by rank, and each kept key's code is recomputed against the previous kept key.
#pragma once
#include "leaf.hpp"
#include "update.hpp"

namespace cpma_dev {

constexpr uint32_t kWaveSlice = 64;   // insert slice handled per wave
constexpr uint32_t kWaveMaxS = 1024;  // leaf size handled per wave (16 bytes per lane)

__device__ __forceinline__ void put_key_bytes(uint8_t* dst, bool head, uint64_t x, uint64_t pred) {
  if (head)
    put_le64(dst, x);
  else
    vput(dst, x - pred);
}

__global__ void __launch_bounds__(kWave) k_merge_wave(MergeArgs a) {
  __shared__ uint64_t K[kWaveMaxS];
  __shared__ uint64_t Bs[kWaveSlice];
  __shared__ uint32_t G[kWaveMaxS + 1];
  __shared__ uint16_t OFF[kWaveMaxS + 1];
  __shared__ __align__(16) uint8_t out[kWaveMaxS];
  const int lane = lane_id();
  const uint32_t S = a.S;
  const uint64_t T = a.ctr->T;
  const uint32_t pos0 = 16u * lane;
  unsigned long long delta = 0, alg = 0;
  // Software pipeline: the next segment's descriptor, leaf bytes and batch keys
  // are loaded while the current one is merged.
  uint4 d_cur = make_uint4(0, 0, 0, 0), d_nxt = d_cur;
  uint32_t e_cur = 0, e_nxt = 0;
  uint4 w_cur = make_uint4(0, 0, 0, 0), w_nxt = w_cur;
  uint64_t b_cur = 0, b_nxt = 0;
  uint64_t s = blockIdx.x;
  if (s < T) {
    d_cur = a.seg_desc[s];
    e_cur = a.seg_begin[s + 1];
    if (pos0 < d_cur.z) w_cur = *reinterpret_cast<const uint4*>(a.bytes + (uint64_t)d_cur.x * S + pos0);
    if ((uint32_t)lane < e_cur - d_cur.y) b_cur = a.B[d_cur.y + lane];
  }
  for (; s < T; s += gridDim.x) {
    const uint64_t sn = s + gridDim.x;
    if (sn < T) {
      d_nxt = a.seg_desc[sn];
      e_nxt = a.seg_begin[sn + 1];
    }
    const uint64_t leaf = d_cur.x;
    const uint32_t b = d_cur.y, e = e_cur;
    const uint32_t nb = e - b;
    const uint32_t used0 = d_cur.z;
    const uint4 w = w_cur;
    const uint64_t bj0 = b_cur;
    if (sn < T) {
      w_nxt = make_uint4(0, 0, 0, 0);
      if (pos0 < d_nxt.z) w_nxt = *reinterpret_cast<const uint4*>(a.bytes + (uint64_t)d_nxt.x * S + pos0);
      b_nxt = ((uint32_t)lane < e_nxt - d_nxt.y) ? a.B[d_nxt.y + lane] : 0;
    }
    d_cur = d_nxt;
    e_cur = e_nxt;
    w_cur = w_nxt;
    b_cur = b_nxt;
    if (a.is_insert && nb > kWaveSlice) {
      if (lane == 0) a.spill_list[atomicAdd(&a.ctr->nspill, 1u)] = (uint32_t)s;
      continue;
    }
    const uint64_t* Bg = a.B + b;
    uint8_t* lp = a.bytes + leaf * (uint64_t)S;
    const uint32_t nA = wave_decode_regs(w, used0, [&](uint32_t i, uint64_t x, uint64_t) { K[i] = x; });
    wave_zero(out, S);
    // lane-contiguous block of old-key indices [i0, i1) over [0, nA] (index nA: trailing group)
    const uint32_t m = (nA + 1 + kWave - 1) / kWave;
    const uint32_t i0 = min(nA + 1, (uint32_t)lane * m), i1 = min(nA + 1, i0 + m);
    uint32_t U = 0;
    uint64_t first_key = kNoKey;
    uint8_t* dst = out;
    uint64_t arena_off = 0;
    bool to_arena = false;
    if (a.is_insert) {
      const bool has_b = (uint32_t)lane < nb;
      const uint64_t bj = has_b ? bj0 : 0;
      if (has_b) Bs[lane] = bj;
      for (uint32_t i = lane; i <= nA; i += kWave) G[i] = 0xffu;
      __syncthreads();
      uint32_t r = 0xffffffffu;
      bool isnew = false;
      if (has_b) {
        r = (uint32_t)lds_lower_bound(K, nA, bj);
        isnew = !(r < nA && K[r] == bj);
      }
      const uint64_t b_prev = dpp_prev64(bj);
      const uint32_t r_prev = dpp_prev32(r);
      const uint32_t new_prev = dpp_prev32(isnew ? 1u : 0u);
      const uint32_t r_next = dpp_next32(r);
      const uint32_t new_next = dpp_next32(isnew ? 1u : 0u);
      const bool same_prev = lane > 0 && new_prev && r_prev == r;
      const bool same_next = lane < kWave - 1 && new_next && r_next == r;
      bool has_pred = false;
      uint64_t pred = 0;
      if (isnew) {
        if (same_prev) {
          pred = b_prev;
          has_pred = true;
        } else if (r > 0) {
          pred = K[r - 1];
          has_pred = true;
        }
      }
      const uint32_t cost = isnew ? (has_pred ? vlen(bj - pred) : 8u) : 0u;
      const uint32_t incl = dpp_incl_scan<uint32_t>(cost);
      const uint32_t ex = incl - cost;
      if (isnew) {
        atomicAdd(&G[r], cost << 8);
        if (!same_next) atomicAnd(&G[r], 0xffffff00u | (uint32_t)lane);
        if (!same_prev) atomicOr(&G[r], ex << 20);
      }
      const uint64_t newmask = __ballot(isnew);
      const uint32_t nnew = (uint32_t)__popcll(newmask);
      __syncthreads();
      // sweep 1: bytes per index (group before old key i, then old key i)
      uint32_t lt = 0;
      for (uint32_t i = i0; i < i1; i++) {
        const uint32_t g = G[i];
        uint32_t t = (g >> 8) & 0xfffu;
        if (i < nA) {
          const uint32_t lj = g & 0xffu;
          const bool hp = lj != 0xffu || i > 0;
          const uint64_t np = lj != 0xffu ? Bs[lj] : (i > 0 ? K[i - 1] : 0);
          t += hp ? vlen(K[i] - np) : 8u;
        }
        lt += t;
      }
      const uint32_t lincl = dpp_incl_scan<uint32_t>(lt);
      U = lane63_u32(lincl);
      if (U > S) {
        const uint64_t need = ((uint64_t)U + 15) & ~15ull;
        uint64_t off = 0;
        if (lane == 0) off = atomicAdd(&a.ctr->arena_cursor, (unsigned long long)need);
        off = __shfl(off, 0, kWave);
        if (off + need > a.arena_cap) {
          if (lane == 0) atomicOr(&a.ctr->error, 1u);
          continue;
        }
        arena_off = off;
        dst = a.arena + off;
        to_arena = true;
      }
      // sweep 2: write old keys, record group starts
      uint32_t run = lincl - lt;
      for (uint32_t i = i0; i < i1; i++) {
        const uint32_t g = G[i];
        const uint32_t gb = (g >> 8) & 0xfffu;
        OFF[i] = (uint16_t)min(run, 0xffffu);
        if (i < nA) {
          const uint32_t lj = g & 0xffu;
          const bool hp = lj != 0xffu || i > 0;
          const uint64_t np = lj != 0xffu ? Bs[lj] : (i > 0 ? K[i - 1] : 0);
          const uint64_t x = K[i];
          const uint32_t c = hp ? vlen(x - np) : 8u;
          put_key_bytes(dst + run + gb, !hp, x, np);
          run += gb + c;
        } else {
          run += gb;
        }
      }
      __syncthreads();
      // new keys: group start + offset inside the group
      if (isnew) {
        const uint32_t gstart = OFF[r];
        const uint32_t exfirst = G[r] >> 20;
        put_key_bytes(dst + gstart + (ex - exfirst), !has_pred, bj, pred);
      }
      const uint64_t firstnew = nnew ? Bs[__ffsll((unsigned long long)newmask) - 1] : kNoKey;
      first_key = nA ? min(K[0], firstnew) : firstnew;
      delta += nnew;
    } else {
      for (uint32_t i = lane; i < nA; i += kWave) G[i] = 0;
      __syncthreads();
      for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
        const uint32_t j = c0 + lane;
        if (j < nb) {
          const uint64_t x = Bg[j];
          const uint32_t r = (uint32_t)lds_lower_bound(K, nA, x);
          if (r < nA && K[r] == x) G[r] = 1;
        }
      }
      __syncthreads();
      // last kept index (+1) inside this lane's block, then across lanes
      uint32_t lastk = 0, lt = 0, nrem = 0;
      for (uint32_t i = i0; i < min(i1, nA); i++) {
        if (!G[i]) lastk = i + 1;
        else nrem++;
      }
      const uint32_t pk_in = dpp_prev32(dpp_incl_max(lastk));  // 0 = none before this block
      uint32_t pk = pk_in;
      for (uint32_t i = i0; i < min(i1, nA); i++) {
        if (G[i]) continue;
        lt += pk ? vlen(K[i] - K[pk - 1]) : 8u;
        pk = i + 1;
      }
      const uint32_t lincl = dpp_incl_scan<uint32_t>(lt);
      U = lane63_u32(lincl);
      uint32_t run = lincl - lt;
      pk = pk_in;
      for (uint32_t i = i0; i < min(i1, nA); i++) {
        if (G[i]) continue;
        const uint64_t x = K[i];
        const uint64_t np = pk ? K[pk - 1] : 0;
        put_key_bytes(out + run, pk == 0, x, np);
        run += pk ? vlen(x - np) : 8u;
        pk = i + 1;
      }
      // smallest kept key: the key at the first index whose flag is clear
      uint32_t fk = 0xffffffffu;
      for (uint32_t i = i0; i < min(i1, nA); i++)
        if (!G[i]) {
          fk = i;
          break;
        }
      uint32_t fkmin = fk;
      for (int d = 32; d > 0; d >>= 1) fkmin = min(fkmin, (uint32_t)__shfl_xor((int)fkmin, d, kWave));
      first_key = (fkmin != 0xffffffffu) ? K[fkmin] : kNoKey;
      delta += wave_sum(nrem);
    }
    __syncthreads();
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
    __syncthreads();
  }
  if (lane == 0) {
    if (delta) atomicAdd(&a.ctr->delta, delta);
    if (alg) atomicAdd(&a.ctr->alg_bytes, alg);
  }
}

}  // namespace cpma_dev
