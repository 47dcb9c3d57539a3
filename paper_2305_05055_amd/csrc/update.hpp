// Batch-update kernels: leaf location, per-leaf merge, density counting up the
// implicit tree and window redistribution (Section "Parallel Batch Updates in a
// PMA": batch-merge phase, counting phase, redistribution phase).
#pragma once
#include "leaf.hpp"
#include "scan.hpp"

namespace cpma_dev {


// Device-side counters of one update, read back by the host at its sync points.
struct Counters {
  unsigned long long delta;         // keys added (insert) or removed (delete)
  unsigned long long stage_cursor;  // keys used in the staging buffer by heavy merges
  unsigned long long kprime;        // batch size after removing repeats
  unsigned long long T;             // touched leaves (segments)
  unsigned long long root_sum;      // filled bytes of the whole structure
  unsigned int heavy;               // segments routed to the heavy merge
  unsigned int nwin;                // windows selected for redistribution
  unsigned int root_viol;           // violation bits of the root
  unsigned int error;               // internal capacity overflow (bug guard)
  unsigned int nspill;              // segments the wave merge hands to the heavy merge
  unsigned int nwide;               // segments whose key span needs 64-bit merge keys
  unsigned long long alg_bytes;     // algorithmic HBM bytes of the merge (statistics)
  unsigned long long alg_bytes_q;   // algorithmic HBM bytes of range scans (statistics)
  unsigned long long alg_bytes_h;   // algorithmic HBM bytes of the follow-up merges (statistics)
  unsigned int reserved;            // a small batch held the reserved key (nothing was changed)
  unsigned int path_unsafe;         // a node on a touched path left its bounds (small-batch count)
};

__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t x) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint64_t upper_bound_u64(const uint64_t* a, uint64_t n, uint64_t x) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (a[mid] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Leaf that holds (or would hold) key x: the last leaf whose head is <= x, leaf 0
// for keys below every head (Section "Compressed Packed Memory Array", "Point
// queries": binary search on the uncompressed leaf heads).
__device__ __forceinline__ uint64_t locate_leaf(const uint64_t* head, uint64_t L, uint64_t x) {
  uint64_t ub = upper_bound_u64(head, L, x);
  return ub ? ub - 1 : 0;
}

__global__ void k_locate(const uint64_t* __restrict__ B, const unsigned long long* kprime,
                         const uint64_t* __restrict__ head, uint64_t L, uint32_t* __restrict__ leafid) {
  const uint64_t k = *kprime;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
       i += (uint64_t)gridDim.x * blockDim.x)
    leafid[i] = (uint32_t)locate_leaf(head, L, B[i]);
}

struct SegFlag {
  const uint32_t* leafid;
  const unsigned long long* kprime;
  __device__ uint32_t operator()(uint64_t i) const {
    return (i < *kprime && (i == 0 || leafid[i] != leafid[i - 1])) ? 1u : 0u;
  }
};

// Touched leaves: one segment per run of equal leaf ids (the batch slice bound
// for each leaf, which the paper finds with two exponential searches).
// A segment is wide when its old keys and slice keys can span more than 2^32:
// they lie in [min(head, first slice key), head of the next leaf).
__device__ __forceinline__ uint32_t seg_wide(const uint32_t* used, const uint64_t* head, uint64_t L, uint32_t lf,
                                             uint64_t bfirst) {
  const uint64_t lo = used[lf] ? min(head[lf], bfirst) : bfirst;
  const uint64_t hi = lf + 1 < L ? head[lf + 1] : ~0ull;
  return (hi - lo > (1ull << 32)) ? 1u : 0u;
}

__global__ void k_segments(const uint32_t* __restrict__ leafid, const unsigned long long* kprime,
                           const uint32_t* __restrict__ segpos, uint64_t kbound,
                           uint32_t* __restrict__ seg_leaf, uint32_t* __restrict__ seg_begin,
                           uint4* __restrict__ seg_desc, const uint32_t* __restrict__ used,
                           const uint64_t* __restrict__ head, uint64_t L, const uint64_t* __restrict__ B,
                           Counters* ctr) {
  const uint64_t k = *kprime;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (i == 0 || leafid[i] != leafid[i - 1]) {
      const uint32_t lf = leafid[i];
      seg_leaf[segpos[i]] = lf;
      seg_begin[segpos[i]] = (uint32_t)i;
      seg_desc[segpos[i]] = make_uint4(lf, (uint32_t)i, used[lf], seg_wide(used, head, L, lf, B[i]));
    }
    if (i == 0) {
      uint32_t T = segpos[kbound];
      seg_begin[T] = (uint32_t)k;
      ctr->T = T;
    }
  }
}

// Large batches: the same segments found per leaf instead of per key.  Leaf f
// owns the batch keys in [head[f], head[f + 1]) (leaf 0 also those below every
// head, the last leaf those above), so its slice starts at the first batch key
// >= head[f]: L searches in the batch instead of k' searches in the heads.
__global__ void k_leaf_slices(const uint64_t* __restrict__ B, const unsigned long long* kprime,
                              const uint64_t* __restrict__ head, uint64_t L, uint32_t* __restrict__ sbeg) {
  const uint64_t k = *kprime;
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f <= L;
       f += (uint64_t)gridDim.x * blockDim.x)
    sbeg[f] = (uint32_t)(f == 0 ? 0 : (f == L ? k : lower_bound_u64(B, k, head[f])));
}

struct SliceFlag {
  const uint32_t* sbeg;
  __device__ uint32_t operator()(uint64_t f) const { return sbeg[f + 1] > sbeg[f] ? 1u : 0u; }
};

__global__ void k_segments_by_leaf(const uint32_t* __restrict__ sbeg, const unsigned long long* kprime,
                                   const uint32_t* __restrict__ segpos, uint64_t L,
                                   uint32_t* __restrict__ seg_leaf, uint32_t* __restrict__ seg_begin,
                                   uint4* __restrict__ seg_desc, const uint32_t* __restrict__ used,
                                   const uint64_t* __restrict__ head, const uint64_t* __restrict__ B,
                                   Counters* ctr) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f <= L;
       f += (uint64_t)gridDim.x * blockDim.x) {
    if (f == L) {
      const uint32_t T = segpos[L];
      seg_begin[T] = (uint32_t)*kprime;
      ctr->T = T;
    } else if (sbeg[f + 1] > sbeg[f]) {
      const uint32_t b = sbeg[f], p = segpos[f];
      seg_leaf[p] = (uint32_t)f;
      seg_begin[p] = b;
      seg_desc[p] = make_uint4((uint32_t)f, b, used[f], seg_wide(used, head, L, (uint32_t)f, B[b]));
    }
  }
}

// Appends `value` for every active lane with pred set: one atomic per wave.
__device__ __forceinline__ void wave_append(uint32_t* __restrict__ list, unsigned int* counter, bool pred,
                                            uint32_t value) {
  const uint64_t m = __ballot(pred);
  if (!m) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (unsigned int)__popcll(m));
  base = __shfl(base, leader, kWave);
  if (pred) list[base + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull))] = value;
}

// Segment routing for the wave merge: inserts with more keys than one wave takes
// go to the heavy merge (spill list), segments of wide key span to the 64-bit
// instance (wide list); desc.w becomes 0 (narrow instance), 1 (wide) or 2 (spill).
__global__ void k_classify(uint4* __restrict__ seg_desc, const uint32_t* __restrict__ seg_begin, uint32_t slice,
                           int is_insert, uint32_t* __restrict__ wide_list, uint32_t* __restrict__ spill_list,
                           Counters* ctr, uint64_t bound) {
  const uint64_t T = ctr->T;
  const uint64_t n = (bound + kWave - 1) / kWave * kWave;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (uint64_t)gridDim.x * blockDim.x) {
    bool spill = false, wide = false;
    if (s < T) {
      uint4 d = seg_desc[s];
      const uint32_t nb = seg_begin[s + 1] - d.y;
      spill = is_insert && nb > slice;
      wide = !spill && d.w != 0;
      d.w = spill ? 2u : (wide ? 1u : 0u);
      seg_desc[s] = d;
    }
    wave_append(spill_list, &ctr->nspill, spill, (uint32_t)s);
    wave_append(wide_list, &ctr->nwide, wide, (uint32_t)s);
  }
}

// ---- per-leaf merge -------------------------------------------------------------
struct MergeArgs {
  uint8_t* bytes;
  uint32_t* used;
  uint64_t* head;
  uint64_t* ovf;          // arena offset of an overflowing leaf
  uint8_t* arena;
  uint64_t arena_cap;
  uint64_t* stage;        // heavy-merge output keys
  uint64_t stage_cap;
  const uint64_t* B;      // sorted, repeat-free batch
  const uint32_t* seg_leaf;
  const uint32_t* seg_begin;
  const uint4* seg_desc;  // {leaf, slice begin, used before the merge, wide span}
  uint32_t* heavy_list;
  uint32_t* spill_list;   // segments routed from the wave merge to the heavy merge
  uint32_t* wide_list;    // segments whose keys span more than 2^32
  Counters* ctr;
  unsigned long long* part;  // per wave of the launch: {keys added / removed, algorithmic bytes}
  uint32_t S;
  int is_insert;
  // key-value leaves
  uint32_t kv;               // every key carries an 8-byte value
  uint32_t* clen;            // code bytes of every leaf
  const uint64_t* Bv;        // the batch keys' values (insert; NULL: new keys get 0, present keys keep theirs)
  uint64_t* vstage;          // values of staged merged leaves (beside stage)
};

// Arena region of segment s: s * (S + 16) + 16 * (its first batch index).  A
// merge grows a leaf by at most 10 bytes per new key (the new key's code; the
// old key after it only gets a smaller delta), so segment s needs at most
// S + 10 * nb + 15 bytes: the regions are disjoint, 16-byte aligned and need
// no shared cursor.
__device__ __forceinline__ uint64_t arena_region(const MergeArgs& a, uint64_t s) {
  // a key-value leaf grows by at most 18 bytes per new key (code and value);
  // 32 per key keeps the regions 16-byte aligned
  return s * (uint64_t)(a.S + 16) + (a.kv ? 32ull : 16ull) * a.seg_begin[s];
}

// Sums the per-wave parts of the merge launches into the counters: the first
// n_narrow pairs count as main-merge bytes, the next n_wide as follow-up bytes.
// A few blocks, each adding its partial sums with three atomics.
__global__ void __launch_bounds__(1024) k_fold_parts(const unsigned long long* __restrict__ part,
                                                     uint32_t n_narrow, uint32_t n_wide, Counters* ctr) {
  __shared__ uint64_t red[3][1024 / kWave];
  uint64_t d = 0, an = 0, aw = 0;
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < n_narrow + n_wide; w += gridDim.x * blockDim.x) {
    d += part[2 * w];
    if (w < n_narrow)
      an += part[2 * w + 1];
    else
      aw += part[2 * w + 1];
  }
  d = wave_sum(d);
  an = wave_sum(an);
  aw = wave_sum(aw);
  const int wid = threadIdx.x / kWave;
  if (lane_id() == 0) {
    red[0][wid] = d;
    red[1][wid] = an;
    red[2][wid] = aw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x / kWave); i++) {
      d += red[0][i];
      an += red[1][i];
      aw += red[2][i];
    }
    if (d) atomicAdd(&ctr->delta, (unsigned long long)d);
    if (an) atomicAdd(&ctr->alg_bytes, (unsigned long long)an);
    if (aw) atomicAdd(&ctr->alg_bytes_h, (unsigned long long)aw);
  }
}

template <typename KT>
__device__ __forceinline__ uint32_t lds_lower_bound(const KT* A, uint32_t n, KT x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (A[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Exclusive prefix sum in place over F[0..n) (one wave).
__device__ __forceinline__ void wave_scan_inplace(uint32_t* F, uint32_t n) {
  uint32_t run = 0;
  for (uint32_t base = 0; base < n; base += kWave) {
    const uint32_t i = base + lane_id();
    const uint32_t v = i < n ? F[i] : 0u;
    const uint32_t incl = wave_incl_scan(v);
    if (i < n) F[i] = run + incl - v;
    run += lane63_u32(incl);
  }
}

// Writes keys get(0..m) into leaf `leaf`: in place if they fit, else into the
// overflow arena (the paper's out-of-place memory for an overflowing leaf,
// cleaned up by the redistribution).  Only the first max(old_used, new size)
// bytes are rewritten: the rest of the leaf is already zero.  Updates used /
// head / ovf and returns the bytes written.
template <class Get>
__device__ uint64_t wave_store_leaf(const MergeArgs& a, uint64_t seg, uint64_t leaf, Get&& get, uint32_t m,
                                    uint8_t* buf, uint32_t old_used) {
  const int lane = lane_id();
  uint8_t* dst = a.bytes + leaf * (uint64_t)a.S;
  if (m == 0) {
    wave_zero(dst, (old_used + 15u) & ~15u);
    if (lane == 0) {
      a.used[leaf] = 0;
      a.head[leaf] = kNoKey;
    }
    return old_used;
  }
  const uint64_t T = wave_encoded_size(get, m);
  uint64_t written;
  if (T <= a.S) {
    const uint32_t len = ((uint32_t)max((uint64_t)old_used, T) + 15u) & ~15u;
    wave_zero(buf, len);
    __syncthreads();
    wave_encode_bytes(get, m, buf);
    __syncthreads();
    wave_copy16(dst, buf, len);
    written = len;
  } else {
    const uint64_t need = (T + 15) & ~15ull;
    const uint64_t off = arena_region(a, seg);
    if (off + need > a.arena_cap) {
      if (lane == 0) atomicOr(&a.ctr->error, 1u);
      return 0;
    }
    wave_encode_bytes(get, m, a.arena + off);
    if (lane == 0) a.ovf[leaf] = off;
    written = T;
  }
  if (lane == 0) {
    a.used[leaf] = (uint32_t)T;
    a.head[leaf] = get(0);
  }
  return written;
}

// ---- counting phase: byte sums of every node of the implicit tree ----------------
constexpr int kPyrThreads = 256;
constexpr int kPyrLowLevels = 9;  // levels 1..9 per block of 512 leaves

__global__ void __launch_bounds__(kPyrThreads) k_pyr_low(const uint32_t* __restrict__ used, uint64_t L,
                                                         Pyramid P, int top) {
  __shared__ uint64_t s[kPyrThreads];
  const int t = threadIdx.x;
  const uint64_t n1 = (uint64_t)blockIdx.x * kPyrThreads + t;  // level-1 node
  uint64_t v = 0;
  if (2 * n1 < L) v += used[2 * n1];
  if (2 * n1 + 1 < L) v += used[2 * n1 + 1];
  s[t] = v;
  if (n1 < P.cnt[1]) P.base[P.off[1] + n1] = v;
  __syncthreads();
  for (int h = 2; h <= top; h++) {
    const int active = kPyrThreads >> (h - 1);
    uint64_t x = 0;
    if (t < active) x = s[2 * t] + s[2 * t + 1];
    __syncthreads();
    if (t < active) {
      s[t] = x;
      const uint64_t node = (uint64_t)blockIdx.x * active + t;
      if (node < P.cnt[h]) P.base[P.off[h] + node] = x;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_pyr_high(Pyramid P, int from) {
  for (int h = from + 1; h <= P.H; h++) {
    const uint64_t* lower = P.base + P.off[h - 1];
    const uint64_t nlow = P.cnt[h - 1];
    for (uint64_t i = threadIdx.x; i < P.cnt[h]; i += blockDim.x) {
      uint64_t v = lower[2 * i];
      if (2 * i + 1 < nlow) v += lower[2 * i + 1];
      P.base[P.off[h] + i] = v;
    }
    __threadfence_block();
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t node_viol(const Bounds& bd, const Pyramid& P, const uint32_t* used,
                                              int h, uint64_t i) {
  return violation(bd, h, node_sum(P, used, h, i), node_leaves(bd.L, h, i));
}

// A node is redistributed when it is within its bounds but a child is not (the
// walk up from a violating node stops at the first ancestor within bounds).
__device__ __forceinline__ bool node_redist(const Bounds& bd, const Pyramid& P, const uint32_t* used,
                                            int h, uint64_t i) {
  if (h == 0 || node_viol(bd, P, used, h, i)) return false;
  const uint64_t c0 = 2 * i, c1 = 2 * i + 1;
  const uint64_t nchild = (h - 1 == 0) ? bd.L : P.cnt[h - 1];
  if (node_viol(bd, P, used, h - 1, c0)) return true;
  return c1 < nchild && node_viol(bd, P, used, h - 1, c1) != 0;
}

// Window selection: every node that must be redistributed and has no ancestor
// that is itself redistributed (maximal windows).  Root violation -> resize.
__global__ void k_select(Bounds bd, Pyramid P, const uint32_t* __restrict__ used,
                         uint64_t* __restrict__ win, Counters* ctr) {
  const uint64_t total = (bd.H == 0) ? 1 : P.off[bd.H] + P.cnt[bd.H] - P.off[1];
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    if (bd.H == 0) {
      ctr->root_sum = used[0];
      ctr->root_viol = violation(bd, 0, used[0], 1);
      return;
    }
    int h = 1;
    uint64_t g = t + P.off[1];
    while (!(g >= P.off[h] && g < P.off[h] + P.cnt[h])) h++;
    const uint64_t i = g - P.off[h];
    if (h == bd.H) {
      ctr->root_sum = P.base[P.off[h]];
      ctr->root_viol = node_viol(bd, P, used, h, 0);
    }
    if (!node_redist(bd, P, used, h, i)) continue;
    bool covered = false;
    for (int h2 = h + 1; h2 <= bd.H && !covered; h2++)
      covered = node_redist(bd, P, used, h2, i >> (h2 - h));
    if (covered) continue;
    const uint32_t slot = atomicAdd(&ctr->nwin, 1u);
    win[slot] = ((uint64_t)h << 48) | i;
  }
}

// ---- redistribution: pack (copy 1) then spread evenly (copy 2) -------------------
// Windows are described by flat index ranges: window w owns source leaves
// src_begin[w] .. +src_n[w] (flat ids src_flat[w] ..) and destination leaves
// dst_begin[w] .. +dst_n[w] (flat ids dst_flat[w] ..).
struct WinArgs {
  uint32_t W;
  const uint64_t* src_begin;
  const uint64_t* src_flat;  // W + 1
  const uint64_t* dst_begin;
  const uint64_t* dst_n;
  const uint64_t* dst_flat;  // W + 1
  const uint32_t* level;     // window height (subtree check bound)
  uint32_t raw;              // uncompressed leaves (raw 8-byte keys)
  uint32_t vbytes;           // 8 when every key carries a value, else 0
};

__device__ __forceinline__ uint32_t find_window(const uint64_t* flat, uint32_t W, uint64_t f) {
  return (uint32_t)(upper_bound_u64(flat, (uint64_t)W + 1, f) - 1);
}

struct SrcLeaves {
  const uint8_t* bytes;
  const uint32_t* used;
  const uint64_t* ovf;
  const uint8_t* arena;
  uint32_t S;
  const uint32_t* clen;  // key-value leaves: code bytes (used counts codes and values)
  __device__ const uint8_t* ptr(uint64_t leaf, uint32_t u) const {
    return u > S ? arena + ovf[leaf] : bytes + leaf * (uint64_t)S;
  }
};

// Key-value leaves: the key codes from byte 0 (clen bytes), the m values as
// 8-byte words in key order at the end of the leaf (an overflow copy in the
// arena keeps them right after the codes, from the next 8-byte boundary).
__device__ __forceinline__ const uint8_t* kv_values(const uint8_t* base, uint32_t u, uint32_t clen, uint32_t S) {
  return u > S ? base + ((clen + 7u) & ~7u) : base + S - (u - clen);
}

__global__ void __launch_bounds__(kWave) k_win_count(WinArgs wa, SrcLeaves src, uint64_t nflat,
                                                     uint64_t* __restrict__ cnt) {
  for (uint64_t f = blockIdx.x; f < nflat; f += gridDim.x) {
    const uint32_t w = find_window(wa.src_flat, wa.W, f);
    const uint64_t leaf = wa.src_begin[w] + (f - wa.src_flat[w]);
    const uint32_t u = src.used[leaf];
    const uint32_t c = wa.raw ? u / 8 : (wa.vbytes ? (u - src.clen[leaf]) / 8 : wave_count_keys(src.ptr(leaf, u), u));
    if (lane_id() == 0) cnt[f] = c;
  }
}

// Also records every staged key's byte cost in the old delta chain: its code
// length, 8 for a leaf head (fixed up by k_head_costs when the head is not the
// first key of its window).
__global__ void __launch_bounds__(kWave) k_win_pack(WinArgs wa, SrcLeaves src, uint64_t nflat,
                                                    const uint64_t* __restrict__ koff,
                                                    uint64_t* __restrict__ stage,
                                                    uint32_t* __restrict__ win_id,
                                                    uint8_t* __restrict__ ccost,
                                                    uint64_t* __restrict__ vstage = nullptr) {
  for (uint64_t f = blockIdx.x; f < nflat; f += gridDim.x) {
    const uint32_t w = find_window(wa.src_flat, wa.W, f);
    const uint64_t leaf = wa.src_begin[w] + (f - wa.src_flat[w]);
    const uint32_t u = src.used[leaf];
    uint64_t* out = stage + koff[f];
    uint32_t* wid = win_id + koff[f];
    uint8_t* cc = ccost + koff[f];
    if (wa.raw) {
      const uint64_t* k = reinterpret_cast<const uint64_t*>(src.ptr(leaf, u));
      for (uint32_t i = lane_id(); i < u / 8; i += kWave) {
        out[i] = k[i];
        wid[i] = w;
        cc[i] = 8;
      }
      continue;
    }
    if (wa.vbytes) {
      const uint32_t cl = src.clen[leaf];
      const uint8_t* base = src.ptr(leaf, u);
      const uint64_t* vals = reinterpret_cast<const uint64_t*>(kv_values(base, u, cl, src.S));
      uint64_t* vo = vstage + koff[f];
      for (uint32_t i = lane_id(); i < (u - cl) / 8; i += kWave) vo[i] = vals[i];
      wave_decode_leaf(base, cl, [&](uint32_t i, uint64_t x, uint64_t d) {
        out[i] = x;
        wid[i] = w;
        cc[i] = (uint8_t)((i == 0 ? 8u : vlen(d)) + 8u);
      });
      continue;
    }
    wave_decode_leaf(src.ptr(leaf, u), u, [&](uint32_t i, uint64_t x, uint64_t d) {
      out[i] = x;
      wid[i] = w;
      cc[i] = i == 0 ? (uint8_t)8 : (uint8_t)vlen(d);
    });
  }
}

// Head of a non-first source leaf: its chain cost is the code of its distance
// to the previous staged key.
__global__ void k_head_costs(WinArgs wa, uint64_t nflat, const uint64_t* __restrict__ koff,
                             const uint64_t* __restrict__ welem, const uint64_t* __restrict__ x,
                             uint8_t* __restrict__ ccost) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nflat;
       f += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t e = koff[f];
    if (koff[f + 1] == e) continue;
    const uint32_t w = find_window(wa.src_flat, wa.W, f);
    if (e != welem[w]) ccost[e] = (uint8_t)(vlen(x[e] - x[e - 1]) + wa.vbytes);
  }
}

// Chain costs of a sorted key array that forms a single window.
__global__ void k_chain_costs(const uint64_t* __restrict__ x, uint64_t K, uint8_t* __restrict__ ccost,
                              uint32_t vbytes = 0) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < K;
       e += (uint64_t)gridDim.x * blockDim.x)
    ccost[e] = (uint8_t)((e == 0 ? 8u : vlen(x[e] - x[e - 1])) + vbytes);
}

struct U8Fn {
  const uint8_t* p;
  __device__ uint64_t operator()(uint64_t i) const { return p[i]; }
};

// welem[w] = first staged key of window w (W + 1 entries).
__global__ void k_win_elems(WinArgs wa, const uint64_t* __restrict__ koff, uint64_t* __restrict__ welem,
                            uint32_t* __restrict__ fail) {
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w <= wa.W; w += gridDim.x * blockDim.x) {
    welem[w] = koff[wa.src_flat[w]];
    if (w < wa.W) fail[w] = 0;
  }
}

// Even split by bytes: key e goes to destination leaf j = floor(P_e * n / total),
// where P_e is the window's byte prefix before e (chain costs).  A key that
// starts a leaf becomes its head (8 bytes); the others keep their code.  Gaps
// (empty leaves) fail the window.
__global__ void k_assign(WinArgs wa, uint64_t K, const uint8_t* __restrict__ ccost,
                         const uint32_t* __restrict__ win_id, const uint64_t* __restrict__ welem,
                         const uint64_t* __restrict__ P, uint8_t* __restrict__ ncost,
                         uint64_t* __restrict__ lstart, uint32_t* __restrict__ fail) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < K;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t w = win_id[e];
    const uint64_t first = welem[w], end = welem[w + 1];
    const uint64_t n = wa.dst_n[w];
    const uint64_t p0 = P[first];
    const uint64_t tot = P[end] - p0;
    const uint64_t pe = P[e] - p0;
    const uint64_t j = (pe * n) / tot;
    bool head = (e == first);
    if (!head) {
      const uint64_t jp = ((pe - ccost[e - 1]) * n) / tot;
      head = j != jp;
      if (j > jp + 1) atomicOr(&fail[w], 2u);
    }
    if (e + 1 == end && j != n - 1) atomicOr(&fail[w], 2u);
    ncost[e] = head ? (uint8_t)(8 + wa.vbytes) : ccost[e];
    if (head) lstart[wa.dst_flat[w] + j] = e;
  }
}

__device__ __forceinline__ bool leaf_range(const WinArgs& wa, const uint64_t* welem, const uint64_t* lstart,
                                           uint64_t fd, uint32_t& w, uint64_t& d, uint64_t& s,
                                           uint64_t& e) {
  w = find_window(wa.dst_flat, wa.W, fd);
  const uint64_t j = fd - wa.dst_flat[w];
  d = wa.dst_begin[w] + j;
  s = lstart[fd];
  e = (j + 1 == wa.dst_n[w]) ? welem[w + 1] : lstart[fd + 1];
  return s != ~0ull && e != ~0ull && s < e && s >= welem[w] && e <= welem[w + 1];
}

// Planned byte count of every destination leaf, checked against the leaf bounds.
__global__ void __launch_bounds__(kWave) k_leaf_bytes(WinArgs wa, Bounds dstb, uint64_t nflat,
                                                      const uint64_t* __restrict__ welem,
                                                      const uint64_t* __restrict__ lstart,
                                                      const uint8_t* __restrict__ ncost,
                                                      uint32_t* __restrict__ planU,
                                                      uint32_t* __restrict__ plan_used,
                                                      int32_t* __restrict__ win_of_leaf,
                                                      uint32_t* __restrict__ fail) {
  for (uint64_t fd = blockIdx.x; fd < nflat; fd += gridDim.x) {
    uint32_t w;
    uint64_t d, s, e;
    const bool ok = leaf_range(wa, welem, lstart, fd, w, d, s, e);
    uint64_t U = 0;
    if (ok)
      for (uint64_t i = s + lane_id(); i < e; i += kWave) U += ncost[i];
    U = wave_sum(U);
    if (lane_id() == 0) {
      uint32_t v = ok ? violation(dstb, 0, U, 1) : 2u;
      if (U > dstb.S) v |= 1u;
      if (v) atomicOr(&fail[w], v);
      planU[fd] = (uint32_t)(U > 0xffffffffull ? 0xffffffffull : U);
      plan_used[d] = planU[fd];
      if (win_of_leaf) win_of_leaf[d] = (int32_t)w;
    }
  }
}

// Subtree check of the planned layout: a node strictly inside a window (lower than
// the window's own height) must satisfy its bounds, else the window escalates.
// check_all: every node of the destination tree counts (fresh layouts).
__global__ void k_check_plan(Bounds bd, Pyramid P, const uint32_t* __restrict__ plan_used,
                             const int32_t* __restrict__ win_of_leaf, const uint32_t* __restrict__ level,
                             int check_all, uint32_t* __restrict__ fail) {
  const uint64_t total = (bd.H == 0) ? 1 : P.off[bd.H] + P.cnt[bd.H] - P.off[1];
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    int h = 0;
    uint64_t i = 0;
    if (bd.H > 0) {
      h = 1;
      const uint64_t g = t + P.off[1];
      while (!(g >= P.off[h] && g < P.off[h] + P.cnt[h])) h++;
      i = g - P.off[h];
    }
    const uint32_t v = violation(bd, h, node_sum(P, plan_used, h, i), node_leaves(bd.L, h, i));
    if (!v) continue;
    if (check_all) {
      atomicOr(&fail[0], v);
    } else {
      const int32_t w = win_of_leaf[i << h];
      if (w >= 0 && (uint32_t)h < level[w]) atomicOr(&fail[w], v);
    }
  }
}

__global__ void k_clear_win_map(WinArgs wa, uint64_t nflat, int32_t* __restrict__ win_of_leaf) {
  for (uint64_t fd = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; fd < nflat;
       fd += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t w = find_window(wa.dst_flat, wa.W, fd);
    win_of_leaf[wa.dst_begin[w] + (fd - wa.dst_flat[w])] = -1;
  }
}

// Spread: encode every destination leaf from the staged keys (copy 2).
__global__ void __launch_bounds__(kWave) k_leaf_encode(WinArgs wa, uint64_t nflat, uint32_t S,
                                                       const uint64_t* __restrict__ welem,
                                                       const uint64_t* __restrict__ lstart,
                                                       const uint64_t* __restrict__ x,
                                                       const uint32_t* __restrict__ planU,
                                                       uint8_t* __restrict__ dst_bytes,
                                                       uint32_t* __restrict__ dst_used,
                                                       uint64_t* __restrict__ dst_head,
                                                       const uint64_t* __restrict__ xv = nullptr,
                                                       uint32_t* __restrict__ dst_clen = nullptr) {
  extern __shared__ __align__(16) uint8_t buf[];
  for (uint64_t fd = blockIdx.x; fd < nflat; fd += gridDim.x) {
    uint32_t w;
    uint64_t d, s, e;
    leaf_range(wa, welem, lstart, fd, w, d, s, e);
    wave_zero(buf, S);
    __syncthreads();
    const uint64_t* xs = x + s;
    const uint32_t m = (uint32_t)(e - s);
    if (wa.raw) {
      for (uint32_t i = lane_id(); i < m; i += kWave) reinterpret_cast<uint64_t*>(buf)[i] = xs[i];
    } else {
      wave_encode_bytes([&](uint32_t i) { return xs[i]; }, m, buf);
      if (wa.vbytes) {  // the values at the end of the leaf, in key order
        uint64_t* vb = reinterpret_cast<uint64_t*>(buf + S - 8u * m);
        for (uint32_t i = lane_id(); i < m; i += kWave) vb[i] = xv[s + i];
      }
    }
    __syncthreads();
    wave_copy16(dst_bytes + d * (uint64_t)S, buf, S);
    if (lane_id() == 0) {
      dst_used[d] = planU[fd];
      dst_head[d] = xs[0];
      if (wa.vbytes) dst_clen[d] = planU[fd] - 8u * m;
    }
    __syncthreads();
  }
}

}  // namespace cpma_dev
