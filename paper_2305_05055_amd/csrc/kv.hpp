// Key-value leaves (the key-value CPMA the paper names as future work for
// weighted graphs, Section "Evaluation on graph workloads").  Every key
// carries an 8-byte value.  A leaf keeps its keys exactly as the CPMA does --
// the head and the delta codes from byte 0, clen bytes -- and the values as
// 8-byte words in key order at the end of the leaf.  Its filled bytes (used,
// which the density bounds count) are clen + 8 per key, so every key costs its
// code plus 8 and at most S / 9 keys fit a leaf.
#pragma once
#include "leaf.hpp"
#include "update.hpp"

namespace cpma_dev {

// LDS of the key-value merge, sized by the leaf size: the old keys and values
// (at most S / 9 + 1 keys fit a leaf), the merged keys and values (a merged
// leaf of more than `cap` keys is staged in HBM instead), the new leaf image
// and the per-rank counts.
struct KvLayout {
  uint32_t nold, cap;
  uint32_t k, v, mk, mv, img, c, total;
  __host__ __device__ explicit KvLayout(uint32_t S) {
    nold = S / 9 + 2;
    cap = 2 * nold + 64;
    k = 0;
    v = k + 8 * nold;
    mk = v + 8 * nold;
    mv = mk + 8 * cap;
    img = (mv + 8 * cap + 15) & ~15u;
    c = img + S;
    total = c + 4 * (nold + 1) + 16;
  }
};

// Batch merge on key-value leaves: one wave per touched leaf, any slice length.
// The wave decodes the old keys and copies the old values to LDS.  Insert:
// each batch key's rank by binary search; a present key takes the batch value
// (when values are given); a new key lands at rank + new keys before it, and
// counts one at its rank, whose prefix sum shifts the old keys.  Delete: found
// keys flag their slot; kept keys move down.  The merged keys and values are
// then re-encoded: a leaf that fits is built in LDS and copied over the old
// one, a larger one goes to the segment's overflow-arena region (codes, then
// the values from the next 8-byte boundary).
__global__ void __launch_bounds__(kWave) k_kv_merge(MergeArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ unsigned long long stage_off;
  const uint32_t S = a.S;
  const KvLayout lay(S);
  uint64_t* K = reinterpret_cast<uint64_t*>(smem + lay.k);
  uint64_t* V = reinterpret_cast<uint64_t*>(smem + lay.v);
  uint64_t* MK = reinterpret_cast<uint64_t*>(smem + lay.mk);
  uint64_t* MV = reinterpret_cast<uint64_t*>(smem + lay.mv);
  uint8_t* img = smem + lay.img;  // S bytes: the new leaf
  uint32_t* C = reinterpret_cast<uint32_t*>(smem + lay.c);
  const int lane = lane_id();
  const uint64_t T = a.ctr->T;
  const uint64_t below = (1ull << lane) - 1ull;
  unsigned long long delta = 0, alg = 0;
  for (uint64_t t = blockIdx.x; t < T; t += gridDim.x) {
    const uint4 d = a.seg_desc[t];
    const uint64_t leaf = d.x;
    const uint32_t b = d.y, e = a.seg_begin[t + 1];
    const uint32_t nb = e - b;
    const uint32_t used0 = d.z;
    const uint32_t cl0 = used0 ? a.clen[leaf] : 0u;
    const uint32_t m0 = (used0 - cl0) / 8;
    uint8_t* lp = a.bytes + leaf * (uint64_t)S;
    wave_decode_leaf(lp, cl0, [&](uint32_t i, uint64_t x, uint64_t) { K[i] = x; });
    const uint64_t* ov = reinterpret_cast<const uint64_t*>(lp + S - 8u * m0);
    for (uint32_t i = lane; i < m0; i += kWave) V[i] = ov[i];
    for (uint32_t i = lane; i <= m0; i += kWave) C[i] = 0;
    __syncthreads();
    const uint64_t* Bs = a.B + b;
    uint32_t mn = 0;
    uint64_t* M = MK;
    uint64_t* MVp = MV;
    bool ok = true;
    if (a.is_insert) {
      uint32_t nnew = 0;
      for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
        const uint32_t j = c0 + lane;
        bool isnew = false;
        if (j < nb) {
          const uint64_t x = Bs[j];
          const uint32_t r = lds_lower_bound<uint64_t>(K, m0, x);
          isnew = !(r < m0 && K[r] == x);
          if (isnew)
            atomicAdd(&C[r], 1u);
          else if (a.Bv)
            V[r] = a.Bv[b + j];  // slices hold distinct keys: one writer per slot
        }
        nnew += (uint32_t)__popcll(__ballot(isnew));
      }
      mn = m0 + nnew;
      if (mn > lay.cap) {
        if (lane == 0) stage_off = atomicAdd(&a.ctr->stage_cursor, (unsigned long long)mn);
        __syncthreads();
        const uint64_t off = stage_off;
        if (off + mn > a.stage_cap) {
          ok = false;
        } else {
          M = a.stage + off;
          MVp = a.vstage + off;
        }
      }
      __syncthreads();
      if (ok) {
        uint32_t before = 0;
        for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
          const uint32_t j = c0 + lane;
          bool isnew = false;
          uint64_t x = 0;
          uint32_t r = 0;
          if (j < nb) {
            x = Bs[j];
            r = lds_lower_bound<uint64_t>(K, m0, x);
            isnew = !(r < m0 && K[r] == x);
          }
          const uint64_t nm = __ballot(isnew);
          if (isnew) {
            const uint32_t p = r + before + (uint32_t)__popcll(nm & below);
            M[p] = x;
            MVp[p] = a.Bv ? a.Bv[b + j] : 0ull;
          }
          before += (uint32_t)__popcll(nm);
        }
        uint32_t carry = 0;
        for (uint32_t c0 = 0; c0 < m0; c0 += kWave) {
          const uint32_t i = c0 + lane;
          const uint32_t cv = i < m0 ? C[i] : 0u;
          const uint32_t incl = wave_incl_scan(cv);
          if (i < m0) {
            M[i + carry + incl] = K[i];
            MVp[i + carry + incl] = V[i];
          }
          carry += lane63_u32(incl);
        }
        delta += nnew;
      }
    } else {
      for (uint32_t c0 = 0; c0 < nb; c0 += kWave) {
        const uint32_t j = c0 + lane;
        if (j < nb) {
          const uint64_t x = Bs[j];
          const uint32_t r = lds_lower_bound<uint64_t>(K, m0, x);
          if (r < m0 && K[r] == x) C[r] = 1u;
        }
      }
      __syncthreads();
      uint32_t gone = 0;
      for (uint32_t c0 = 0; c0 < m0; c0 += kWave) {
        const uint32_t i = c0 + lane;
        const bool g = i < m0 && C[i];
        const uint64_t gm = __ballot(g);
        if (i < m0 && !g) {
          const uint32_t p = i - gone - (uint32_t)__popcll(gm & below);
          M[p] = K[i];
          MVp[p] = V[i];
        }
        gone += (uint32_t)__popcll(gm);
      }
      mn = m0 - gone;
      delta += gone;
    }
    if (!ok) {
      if (lane == 0) atomicOr(&a.ctr->error, 1u);
      __syncthreads();
      continue;
    }
    __syncthreads();
    // code bytes of the merged keys (the head 8, then each delta's code)
    auto cost = [&](uint32_t p) -> uint32_t { return p == 0 ? 8u : vlen(M[p] - M[p - 1]); };
    uint32_t cl = 0;
    for (uint32_t c0 = 0; c0 < mn; c0 += kWave) {
      const uint32_t p = c0 + lane;
      cl += p < mn ? cost(p) : 0u;
    }
    cl = wave_sum(cl);
    const uint32_t U = cl + 8u * mn;
    uint64_t aoff = 0;
    const bool to_arena = U > S;
    if (to_arena) {
      aoff = arena_region(a, t);
      if (aoff + (((uint64_t)cl + 7) & ~7ull) + 8ull * mn > a.arena_cap) {
        if (lane == 0) atomicOr(&a.ctr->error, 1u);
        __syncthreads();
        continue;
      }
    } else {
      wave_zero(img, S);
      __syncthreads();
    }
    // codes from dst, values at vdst; instantiated once for the LDS image and
    // once for the arena, so that each copy's stores have a known address
    // space (a pointer that may be either compiles to generic stores)
    auto write_leaf = [&](auto dst, auto vdst) {
      uint32_t run = 0;
      for (uint32_t c0 = 0; c0 < mn; c0 += kWave) {
        const uint32_t p = c0 + lane;
        const uint32_t c = p < mn ? cost(p) : 0u;
        const uint32_t incl = wave_incl_scan(c);
        if (p < mn) {
          auto q = dst + run + incl - c;
          if (p == 0)
            put_le64(q, M[0]);
          else
            vput(q, M[p] - M[p - 1]);
          vdst[p] = MVp[p];
        }
        run += lane63_u32(incl);
      }
    };
    if (to_arena)
      write_leaf(a.arena + aoff, reinterpret_cast<uint64_t*>(a.arena + aoff + ((cl + 7u) & ~7u)));
    else
      write_leaf(img, reinterpret_cast<uint64_t*>(img + S - 8u * mn));
    __syncthreads();
    if (!to_arena) wave_copy16(lp, img, S);
    if (lane == 0) {
      if (to_arena) a.ovf[leaf] = aoff;
      a.used[leaf] = U;
      a.clen[leaf] = cl;
      a.head[leaf] = mn ? M[0] : kNoKey;
    }
    alg += used0 + U + 16ull * nb + 24;
    __syncthreads();
  }
  if (lane == 0) {
    a.part[2 * blockIdx.x] = delta;
    a.part[2 * blockIdx.x + 1] = alg;
  }
}

// Keys of a sorted batch with their values: the first occurrence of each key
// (the smallest input position: the sort is stable) with the value at its
// input position.  pos: exclusive scan of first-occurrence flags.
__global__ void k_kv_compact(const uint64_t* __restrict__ a, const uint32_t* __restrict__ idx, uint64_t n,
                             const uint32_t* __restrict__ pos, const uint64_t* __restrict__ vals,
                             uint64_t* __restrict__ kout, uint64_t* __restrict__ vout,
                             unsigned long long* __restrict__ n_out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (i == 0 || a[i] != a[i - 1]) {
      kout[pos[i]] = a[i];
      vout[pos[i]] = vals ? vals[idx[i] & 0x7fffffffu] : 0ull;
    }
    if (i == 0) *n_out = pos[n];
  }
}

// One lane walks a key-value leaf's codes (clen bytes) and returns, for the
// keys in [lo, hi), the sum of their values (mod 2^64) and their count; with
// hi = lo + 1 and `found`, the value of key lo.
__device__ __forceinline__ LeafSum kv_leaf_values(const uint8_t* __restrict__ leaf, uint32_t clen,
                                                  const uint64_t* __restrict__ vals, uint64_t lo, uint64_t hi) {
  LeafSum r{0, 0};
  if (clen < 8) return r;
  uint64_t key = 0;
  for (int i = 7; i >= 0; i--) key = (key << 8) | leaf[i];
  uint32_t idx = 0, pos = 8;
  while (true) {
    if (key >= hi) break;
    if (key >= lo) {
      r.sum += vals[idx];
      r.count++;
    }
    if (pos >= clen) break;
    uint64_t d = 0;
    uint32_t sh = 0;
    uint8_t c;
    do {
      c = leaf[pos++];
      if (sh < 64) d |= (uint64_t)(c & 0x7fu) << sh;
      sh += 7;
    } while (c & 0x80u);
    key += d;
    idx++;
  }
  return r;
}

}  // namespace cpma_dev
