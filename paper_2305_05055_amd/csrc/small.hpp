// Small batches (at most kSmallBatch keys): one workgroup does the whole batch
// preparation that large batches spread over some thirty launches -- the
// reserved-key check, a bitonic sort in LDS, removal of repeats, the leaf of
// every key (binary search on the heads; a 64-ary search by a whole wave when
// there are few keys), the touched-leaf segments and their routing -- so a
// small update is bound by a handful of launches instead of dozens.  It also
// zeroes the update's counters (it is the update's first kernel).
#pragma once
#include "merge_wave.hpp"
#include "query.hpp"
#include "update.hpp"

namespace cpma_dev {

constexpr uint32_t kSmallBatch = 4096;
constexpr uint32_t kSmallThreads = 1024;

// Up to kArgKeys host keys travel in the launch's arguments instead of a
// separate copy to the device (one launch fewer on the small-batch path).
constexpr uint32_t kArgKeys = 256;
struct ArgKeys {
  uint64_t k[kArgKeys];
};

// Exclusive scan of one value per thread over the workgroup; returns the
// thread's offset, *total the sum.
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = lane_id(), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < nw; w++) {
    const uint32_t x = wsum[w];
    before += w < wid ? x : 0u;
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// Also routes the segments: an insert slice longer than `slice` keys goes to the
// spill list (desc.w = 2), which the heavy merge takes; every other segment is
// merged by the 64-bit wave instance (desc.w = 0).
struct SmallPrepLds {
  uint64_t A[kSmallBatch];
  uint32_t LF[kSmallBatch];  // leaf of each key, then segment starts
  uint32_t wsum[kSmallThreads / kWave];
  uint32_t bad;
};

__device__ __forceinline__ void small_prep_body(const uint64_t* __restrict__ in, const ArgKeys& ak, uint32_t k,
                                                const uint64_t* __restrict__ head, uint64_t L,
                                                const uint32_t* __restrict__ used, uint64_t* __restrict__ B,
                                                uint32_t* __restrict__ seg_leaf, uint32_t* __restrict__ seg_begin,
                                                uint4* __restrict__ seg_desc, int is_insert, uint32_t slice,
                                                uint32_t* __restrict__ spill_list, Counters* ctr, SmallPrepLds& sm) {
  uint64_t* const A = sm.A;
  uint32_t* const LF = sm.LF;
  uint32_t* const wsum = sm.wsum;
  uint32_t& bad = sm.bad;
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t kPer = kSmallBatch / kSmallThreads;
  uint32_t n = 1;
  while (n < k) n <<= 1;
  if (tid == 0) bad = 0;
  for (uint32_t i = tid; i < (uint32_t)(sizeof(Counters) / 4); i += kSmallThreads)
    reinterpret_cast<uint32_t*>(ctr)[i] = 0u;
  __syncthreads();
  for (uint32_t i = tid; i < n; i += kSmallThreads) {
    const uint64_t x = i < k ? (in ? in[i] : ak.k[i]) : kNoKey;  // padding sorts last; no `in`: keys in ak
    if (i < k && x == kNoKey) bad = 1;
    A[i] = x;
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) {
      ctr->reserved = 1;
      ctr->kprime = 0;
      ctr->T = 0;
      seg_begin[0] = 0;
    }
    return;
  }
  // bitonic sort of n (a power of two) keys.  Up to one key per thread, a
  // thread keeps key `tid` in a register: a stage whose partner index differs
  // in the low 6 bits is a shuffle inside the wave, and only strides of 64 and
  // more go through LDS (one barrier per stage).
  if (n <= kSmallThreads) {
    uint64_t x = tid < n ? A[tid] : kNoKey;
    uint32_t lds_stages = 0;
    for (uint32_t size = 2; size <= n; size <<= 1) {
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
        uint64_t y;
        if (stride >= kWave) {
          // A[0, 1024) and A[1024, 2048) serve consecutive LDS stages in turn:
          // a write to one follows the barrier of the stage that read the
          // other, which every thread passed after its last read of this one
          uint64_t* buf = A + ((lds_stages++ & 1u) ? kSmallThreads : 0u);
          buf[tid] = x;
          __syncthreads();
          y = buf[tid ^ stride];
        } else {
          y = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), (int)stride, kWave) << 32) |
              (uint32_t)__shfl_xor((int)(uint32_t)x, (int)stride, kWave);
        }
        const bool up = (tid & size) == 0;
        const bool lower = (tid & stride) == 0;
        x = (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
      }
    }
    __syncthreads();
    if (tid < n) A[tid] = x;
    __syncthreads();
  } else {
  for (uint32_t size = 2; size <= n; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = tid; t < n / 2; t += kSmallThreads) {
        const uint32_t i = 2 * t - (t & (stride - 1));
        const uint32_t j = i + stride;
        const uint64_t a = A[i], b = A[j];
        const bool up = (i & size) == 0;
        if ((a > b) == up) {
          A[i] = b;
          A[j] = a;
        }
      }
      __syncthreads();
    }
  }
  }
  // drop repeats: each thread owns kPer consecutive positions
  const uint32_t i0 = tid * kPer;
  uint32_t mine = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    const uint32_t i = i0 + q;
    mine += (i < k && (i == 0 || A[i] != A[i - 1])) ? 1u : 0u;
  }
  uint32_t kp;
  uint32_t pos = block_scan_u32(mine, wsum, &kp);
  uint64_t mykeys[kPer];
  uint32_t mypos[kPer];
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    const uint32_t i = i0 + q;
    const bool first = i < k && (i == 0 || A[i] != A[i - 1]);
    mykeys[q] = first ? A[i] : 0;
    mypos[q] = first ? pos : ~0u;
    pos += first ? 1u : 0u;
  }
  __syncthreads();
  // unique keys to B and their leaves to LF.  With few keys: one 64-ary wave
  // search per key (a few dependent steps instead of ~log2 L; the keys go
  // back to A for it).  Otherwise one binary search per key, whose first
  // levels run in LDS: A (no longer needed) takes every st-th head, and only
  // the last ~log2 st steps read the heads in HBM.
  constexpr uint32_t kWaves = kSmallThreads / kWave;
  const bool by_wave = kp <= 2 * kWaves;
  if (by_wave) {
#pragma unroll
    for (uint32_t q = 0; q < kPer; q++) {
      if (mypos[q] != ~0u) {
        A[mypos[q]] = mykeys[q];
        B[mypos[q]] = mykeys[q];
      }
    }
  } else {
    const uint64_t st = (L + kSmallBatch - 1) / kSmallBatch;
    const uint32_t ns = (uint32_t)((L + st - 1) / st);  // samples head[i st], i < ns <= kSmallBatch
    for (uint32_t i = tid; i < ns; i += kSmallThreads) A[i] = head[(uint64_t)i * st];
#pragma unroll
    for (uint32_t q = 0; q < kPer; q++)
      if (mypos[q] != ~0u) B[mypos[q]] = mykeys[q];
    __threadfence_block();
    __syncthreads();
    // one key per thread (round robin): each search is a chain of dependent
    // loads, so the keys' chains run side by side rather than kPer in a row
    for (uint32_t u = tid; u < kp; u += kSmallThreads) {
      const uint64_t x = B[u];
      uint32_t lo = 0, hi = ns;  // first sample above x
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A[mid] <= x)
          lo = mid + 1;
        else
          hi = mid;
      }
      // the first head above x has an index in ((lo - 1) st, lo st], within [0, L]
      uint64_t a = lo == 0 ? 0 : (uint64_t)(lo - 1) * st + 1;
      uint64_t b = min((uint64_t)lo * st, L);
      while (a < b) {
        const uint64_t mid = (a + b) >> 1;
        if (head[mid] <= x)
          a = mid + 1;
        else
          b = mid;
      }
      LF[u] = (uint32_t)(a ? a - 1 : 0);
    }
  }
  __syncthreads();
  if (by_wave) {
    for (uint32_t i = tid / kWave; i < kp; i += kWaves) {
      const uint32_t lf = (uint32_t)wave_locate_leaf(head, L, A[i]);
      if (lane_id() == 0) LF[i] = lf;
    }
    __syncthreads();
  }
  // segments: runs of equal leaf ids
  uint32_t starts = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    const uint32_t i = i0 + q;
    starts += (i < kp && (i == 0 || LF[i] != LF[i - 1])) ? 1u : 0u;
  }
  uint32_t T;
  uint32_t sp = block_scan_u32(starts, wsum, &T);
  uint32_t segl[kPer], segi[kPer];
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    const uint32_t i = i0 + q;
    const bool st = i < kp && (i == 0 || LF[i] != LF[i - 1]);
    segl[q] = st ? LF[i] : ~0u;
    segi[q] = st ? sp : ~0u;
    sp += st ? 1u : 0u;
  }
  __syncthreads();
  // segment starts into LF[0, T]
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++)
    if (segi[q] != ~0u) LF[segi[q]] = i0 + q;
  if (tid == 0) LF[T] = kp;
  __syncthreads();
  uint32_t nsp = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    if (segi[q] == ~0u) continue;
    const uint32_t s = segi[q], b = LF[s], lf = segl[q];
    const bool spill = is_insert && LF[s + 1] - b > slice;
    seg_leaf[s] = lf;
    seg_begin[s] = b;
    seg_desc[s] = make_uint4(lf, b, used[lf], spill ? 2u : 0u);
    nsp += spill ? 1u : 0u;
  }
  uint32_t nspill;
  uint32_t pos2 = block_scan_u32(nsp, wsum, &nspill);
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    if (segi[q] == ~0u) continue;
    const uint32_t s = segi[q];
    if (is_insert && LF[s + 1] - LF[s] > slice) spill_list[pos2++] = s;
  }
  if (tid == 0) {
    seg_begin[T] = kp;
    ctr->kprime = kp;
    ctr->T = T;
    ctr->nspill = nspill;
  }
}

__global__ void __launch_bounds__(kSmallThreads) k_small_prep(const uint64_t* __restrict__ in, ArgKeys ak, uint32_t k,
                                                              const uint64_t* __restrict__ head, uint64_t L,
                                                              const uint32_t* __restrict__ used,
                                                              uint64_t* __restrict__ B, uint32_t* __restrict__ seg_leaf,
                                                              uint32_t* __restrict__ seg_begin,
                                                              uint4* __restrict__ seg_desc, int is_insert,
                                                              uint32_t slice, uint32_t* __restrict__ spill_list,
                                                              Counters* ctr) {
  __shared__ SmallPrepLds sm;
  small_prep_body(in, ak, k, head, L, used, B, seg_leaf, seg_begin, seg_desc, is_insert, slice, spill_list, ctr, sm);
}

// ---- counting for a small batch: the paths of the touched leaves only ----------
// A rebalance ends only when its count finds no node to redistribute, so then
// every node of the implicit tree is within its density bounds (a violating
// node below a root within bounds has a highest violating ancestor, whose
// parent would have been selected), and the pyramid holds every node's byte
// sum.  A small batch changes only the leaves it touched, so only their
// ancestors can leave their bounds.  This one-block kernel gives each of them
// its exact new sum (old sum plus the byte growth of the touched leaves below
// it, from a prefix sum over the segments, which are in leaf order), writes it
// into the pyramid and checks it against the bounds of its level.  Any
// violation sets ctr->path_unsafe, and the full count runs instead.  Every
// block builds the prefix sum (at most kSmallBatch segments) and takes its
// share of the (level, segment) pairs.
constexpr uint32_t kPathThreads = 1024;


// Launched as a single block it can also finish the update (part and hout not
// null): it first folds the merge's per-wave totals (what k_fold_parts does;
// `part` holds n_narrow then n_wide slot pairs), and at the end copies the
// counters to host memory `hout`, so the host reads them after one stream
// synchronisation with no copy launch in between.
struct PathLds {
  uint32_t lf[kSmallBatch];
  uint64_t G[kSmallBatch + 1];  // G[t]: growth of the segments before t (mod 2^64)
  uint64_t wsum[kPathThreads / kWave];
  uint64_t red[3][kPathThreads / kWave];
  uint32_t bad;
};

__device__ __forceinline__ void path_check_body(Bounds bd, Pyramid P, const uint32_t* __restrict__ used,
                                                const uint32_t* __restrict__ seg_leaf,
                                                const uint4* __restrict__ seg_desc, Counters* ctr,
                                                const unsigned long long* __restrict__ part, uint32_t n_narrow,
                                                uint32_t n_wide, Counters* hout, PathLds& pl) {
  uint32_t* const lf = pl.lf;
  uint64_t* const G = pl.G;
  uint64_t* const wsum = pl.wsum;
  auto& red = pl.red;
  uint32_t& bad = pl.bad;
  constexpr uint32_t kPer = kSmallBatch / kPathThreads;
  const uint32_t tid = threadIdx.x;
  if (part) {
    uint64_t d = 0, an = 0, aw = 0;
    for (uint32_t w = tid; w < n_narrow + n_wide; w += kPathThreads) {
      d += part[2 * w];
      (w < n_narrow ? an : aw) += part[2 * w + 1];
    }
    d = wave_sum(d);
    an = wave_sum(an);
    aw = wave_sum(aw);
    if (lane_id() == 0) {
      red[0][tid / kWave] = d;
      red[1][tid / kWave] = an;
      red[2][tid / kWave] = aw;
    }
    __syncthreads();
    if (tid == 0) {
      for (uint32_t i = 1; i < kPathThreads / kWave; i++) {
        d += red[0][i];
        an += red[1][i];
        aw += red[2][i];
      }
      ctr->delta += d;
      ctr->alg_bytes += an;
      ctr->alg_bytes_h += aw;
    }
  }
  const uint32_t T = (uint32_t)ctr->T;
  if (tid == 0) bad = T > kSmallBatch;  // not a small batch: let the full count decide
  if (T > 0 && T <= kSmallBatch) {
  uint64_t g[kPer];
  uint64_t mine = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    const uint32_t t = tid * kPer + q;
    g[q] = 0;
    if (t < T) {
      const uint32_t f = seg_leaf[t];
      lf[t] = f;
      g[q] = (uint64_t)used[f] - (uint64_t)seg_desc[t].z;
    }
    mine += g[q];
  }
  const uint64_t incl = wave_incl_scan<uint64_t>(mine);
  if (lane_id() == kWave - 1) wsum[tid / kWave] = incl;
  __syncthreads();
  uint64_t run = incl - mine;
  for (uint32_t w = 0; w < tid / kWave; w++) run += wsum[w];
#pragma unroll
  for (uint32_t q = 0; q < kPer; q++) {
    const uint32_t t = tid * kPer + q;
    if (t < T) {
      G[t] = run;
      run += g[q];
      if (t == T - 1) G[T] = run;
    }
  }
  __syncthreads();
  // (level, segment) pairs spread over the grid; each thread first issues the
  // loads of a chunk of pairs, then checks and stores them, so the chunk's
  // pyramid reads are in flight together.  Only a node's first segment works.
  constexpr uint32_t kChunk = 8;
  const uint32_t npairs = T * (uint32_t)(bd.H + 1);
  const uint32_t stride = gridDim.x * kPathThreads;
  uint32_t v = 0;
  for (uint32_t base = blockIdx.x * kPathThreads; base < npairs; base += stride * kChunk) {
    uint64_t old[kChunk];
    uint32_t pt[kChunk], ph[kChunk];
#pragma unroll
    for (uint32_t c = 0; c < kChunk; c++) {
      const uint32_t j = base + c * stride + tid;
      ph[c] = ~0u;
      old[c] = 0;
      if (j >= npairs) continue;
      const uint32_t h = j / T, t = j - h * T;
      const uint64_t node = (uint64_t)lf[t] >> h;
      if (t > 0 && ((uint64_t)lf[t - 1] >> h) == node) continue;  // not the node's first segment
      ph[c] = h;
      pt[c] = t;
      old[c] = h == 0 ? (uint64_t)used[node] : P.base[P.off[h] + node];  // a leaf: its new size
    }
#pragma unroll
    for (uint32_t c = 0; c < kChunk; c++) {
      if (ph[c] == ~0u) continue;
      const uint32_t h = ph[c], t = pt[c];
      const uint64_t node = (uint64_t)lf[t] >> h;
      uint64_t sum = old[c];
      if (h > 0) {
        const uint64_t lim = (node + 1) << h;  // first leaf past the node
        uint32_t lo = t + 1, hi = T;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if ((uint64_t)lf[mid] < lim)
            lo = mid + 1;
          else
            hi = mid;
        }
        sum += G[lo] - G[t];
        P.base[P.off[h] + node] = sum;
      }
      v |= violation(bd, (int)h, sum, node_leaves(bd.L, (int)h, node));
    }
  }
  if (v) bad = 1;
  }
  __syncthreads();
  if (tid == 0) {
    if (bad) ctr->path_unsafe = 1;
    if (hout) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(ctr);
      uint32_t* dst = reinterpret_cast<uint32_t*>(hout);
      for (uint32_t i = 0; i < sizeof(Counters) / 4; i++)
        dst[i] = __hip_atomic_load(&src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence_system();
    }
  }
}

__global__ void __launch_bounds__(kPathThreads) k_path_check(Bounds bd, Pyramid P, const uint32_t* __restrict__ used,
                                                             const uint32_t* __restrict__ seg_leaf,
                                                             const uint4* __restrict__ seg_desc, Counters* ctr,
                                                             const unsigned long long* __restrict__ part,
                                                             uint32_t n_narrow, uint32_t n_wide, Counters* hout) {
  __shared__ PathLds pl;
  path_check_body(bd, P, used, seg_leaf, seg_desc, ctr, part, n_narrow, n_wide, hout, pl);
}

// ---- a whole small update in one launch --------------------------------------
// For batches of at most kWaveSlice keys (no insert slice can then spill): the
// preparation above, the merge of every touched leaf (kFusedMergeWaves waves of
// the block, one leaf at a time each, as the merge kernel's waves do), and the
// path check of the touched leaves, which also folds the merge's totals and
// writes the counters to host memory.  The three phases run back to back on
// one block, their intermediate results read from where the phase before
// wrote them (block barriers in between), instead of as three launches.
constexpr uint32_t kFusedMergeWaves = 12;

__global__ void __launch_bounds__(kSmallThreads) k_small_update(const uint64_t* __restrict__ in, ArgKeys ak,
                                                                uint32_t k, const uint64_t* __restrict__ head,
                                                                uint64_t L, uint64_t* __restrict__ B,
                                                                int is_insert, MergeArgs ma, Bounds bd, Pyramid P,
                                                                Counters* hout) {
  static_assert(kFusedMergeWaves * kWave <= kSmallThreads, "merge waves fit in the block");
  __shared__ union {
    SmallPrepLds prep;
    MergeLds<uint64_t> merge[kFusedMergeWaves];
    PathLds path;
  } lds;
  // the segment arrays the merge reads are the ones the preparation writes
  small_prep_body(in, ak, k, head, L, ma.used, B, const_cast<uint32_t*>(ma.seg_leaf),
                  const_cast<uint32_t*>(ma.seg_begin), const_cast<uint4*>(ma.seg_desc), is_insert, kWaveSlice,
                  ma.spill_list, ma.ctr, lds.prep);
  __syncthreads();
  const uint32_t w = threadIdx.x / kWave;
  if (w < kFusedMergeWaves) merge_wave_body<uint64_t, true>(ma, 1, lds.merge[w], w, kFusedMergeWaves, w);
  __syncthreads();
  path_check_body(bd, P, ma.used, ma.seg_leaf, ma.seg_desc, ma.ctr, ma.part, 0, kFusedMergeWaves, hout, lds.path);
}

}  // namespace cpma_dev
