// F-Graph on the CPMA (Section "Evaluation on graph workloads"): one CPMA holds
// every edge (u, v) of a graph as the key u<<32 | v, so a vertex's neighbours are
// the keys of [u<<32, (u+1)<<32) and a pass over all leaves visits every edge
// grouped by source.  Delta coding elides the source except at leaf heads and
// at each vertex's first edge.
//
// The kernels below are full passes: one wave decodes one leaf (keys land in lane
// registers), gathers the per-neighbour values for all of its keys at once, then
// each lane folds its keys into runs of equal source and flushes a run with one
// atomic.  PageRank (a fixed number of iterations) runs in pull form, which on
// a symmetric edge set (an undirected graph, the case F-Graph supports) equals
// pushing p(u)/deg(u) along every edge.  BFS is level synchronous and
// direction optimising: each level passes over the leaves holding the current
// level's vertices (top-down) or the unvisited ones (bottom-up).
#pragma once
#include "leaf.hpp"

namespace cpma_dev {

struct FgArgs {
  const uint8_t* bytes;
  const uint32_t* used;
  const uint64_t* head;
  uint64_t L;
  uint32_t S;   // at most 1024: one 16-byte chunk per lane
  uint32_t nv;  // vertex ids are < nv; keys with a larger id are ignored
};

// Keys of one leaf in the lane's registers: kk[i] is valid where bit i of tmask
// is set (the code ending at byte i of the lane's 16 bytes).
__device__ __forceinline__ uint32_t wave_leaf_keys(const uint8_t* __restrict__ src, uint32_t used,
                                                   uint64_t (&kk)[16]) {
  const int lane = lane_id();
  const uint32_t pos0 = 16u * lane;
  uint4 w = make_uint4(0, 0, 0, 0);
  if (pos0 < used) w = *reinterpret_cast<const uint4*>(src + pos0);
  LaneCodes c;
  lane_parse(w, pos0, used, c);
  const uint64_t cin_acc = dpp_prev64(c.tail_acc);
  const uint32_t cin_sh = dpp_prev32(c.tail_sh);
  uint64_t corr = 0;
  if (c.tmask != 0 && pos0 != 0) {
    const uint64_t fixed = cin_acc | (cin_sh < 64 ? (c.first_raw << cin_sh) : 0ull);
    corr = fixed - c.first_raw;
  }
  uint64_t lsum = corr;
#pragma unroll
  for (int i = 0; i < 16; i++) lsum += c.v[i];
  const uint64_t incl = wave_incl_scan(lsum);
  uint64_t key = incl - lsum + corr;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    key += c.v[i];
    kk[i] = key;
  }
  return c.tmask;
}

__device__ __forceinline__ uint32_t src_of(uint64_t k) { return (uint32_t)(k >> 32); }
__device__ __forceinline__ uint32_t dst_of(uint64_t k) { return (uint32_t)k; }

// The leaf's first source if every key of the leaf has it (a high-degree
// vertex whose edges fill whole leaves), else UINT32_MAX.  Such leaves reduce
// across the wave first: per-lane atomics would all hit that one vertex.
__device__ __forceinline__ uint32_t fg_single_source(const FgArgs& g, uint64_t leaf, const uint64_t (&kk)[16],
                                                    uint32_t tm) {
  if (!__ballot(tm != 0)) return 0xffffffffu;  // no keys
  const uint32_t first = src_of(g.head[leaf]);  // the head is the leaf's first key
  bool other = false;
#pragma unroll
  for (int i = 0; i < 16; i++) other |= (tm & (1u << i)) && src_of(kk[i]) != first;
  return __ballot(other) ? 0xffffffffu : first;
}

__device__ __forceinline__ float wave_sum_f32(float x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// deg[u] += number of edges with source u.
__global__ void __launch_bounds__(256) k_fg_degree(FgArgs g, uint32_t* __restrict__ deg) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  for (uint64_t leaf = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; leaf < g.L;
       leaf += waves) {
    uint64_t kk[16];
    const uint32_t tm = wave_leaf_keys(g.bytes + leaf * (uint64_t)g.S, g.used[leaf], kk);
    const uint32_t one = fg_single_source(g, leaf, kk, tm);
    if (one != 0xffffffffu) {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < 16; i++) c += ((tm & (1u << i)) && dst_of(kk[i]) < g.nv) ? 1u : 0u;
      c = wave_sum(c);
      if (lane_id() == 0 && one < g.nv && c) atomicAdd(&deg[one], c);
      continue;
    }
    uint32_t run = 0xffffffffu, cnt = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (tm & (1u << i)) {
        const uint32_t s = src_of(kk[i]);
        if (s != run) {
          if (run < g.nv && cnt) atomicAdd(&deg[run], cnt);
          run = s;
          cnt = 0;
        }
        cnt += dst_of(kk[i]) < g.nv ? 1u : 0u;
      }
    }
    if (run < g.nv && cnt) atomicAdd(&deg[run], cnt);
  }
}

// acc[u] += sum over edges (u, v) of contrib[v]   (FP32).
__global__ void __launch_bounds__(256) k_fg_pull(FgArgs g, const float* __restrict__ contrib,
                                                 float* __restrict__ acc) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  for (uint64_t leaf = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; leaf < g.L;
       leaf += waves) {
    uint64_t kk[16];
    const uint32_t tm = wave_leaf_keys(g.bytes + leaf * (uint64_t)g.S, g.used[leaf], kk);
    float val[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t d = dst_of(kk[i]);
      val[i] = ((tm & (1u << i)) && d < g.nv) ? contrib[d] : 0.f;
    }
    const uint32_t one = fg_single_source(g, leaf, kk, tm);
    if (one != 0xffffffffu) {
      float t = 0.f;
#pragma unroll
      for (int i = 0; i < 16; i++) t += val[i];
      t = wave_sum_f32(t);
      if (lane_id() == 0 && one < g.nv) atomicAdd(&acc[one], t);
      continue;
    }
    uint32_t run = 0xffffffffu;
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (tm & (1u << i)) {
        const uint32_t s = src_of(kk[i]);
        if (s != run) {
          if (run < g.nv) atomicAdd(&acc[run], sum);
          run = s;
          sum = 0.f;
        }
        sum += val[i];
      }
    }
    if (run < g.nv) atomicAdd(&acc[run], sum);
  }
}

// BFS state besides the levels: two bitmaps over the vertices, rebuilt from the
// levels after every level (2 MB each at 2^24 vertices, so the random tests of
// a step hit L2 instead of the 4-byte level entries):
//   front: level == cur (the vertices being expanded);
//   seen:  level != unvisited.
constexpr uint32_t kUnvisited = 0xffffffffu;

struct BfsBits {
  const uint32_t* front;
  const uint32_t* seen;
};

__device__ __forceinline__ bool bit_of(const uint32_t* b, uint32_t v) { return (b[v >> 5] >> (v & 31)) & 1u; }

// Whether bits [s0, s1] of b (xor `flip`) hold a one.
__device__ __forceinline__ bool any_bit(const uint32_t* b, uint32_t flip, uint32_t s0, uint32_t s1) {
  const uint32_t w0 = s0 >> 5, w1 = s1 >> 5;
  uint32_t acc = 0;
  for (uint32_t w = w0; w <= w1; w++) {
    uint32_t x = b[w] ^ flip;
    if (w == w0) x &= ~0u << (s0 & 31);
    if (w == w1) x &= ~0u >> (31 - (s1 & 31));
    acc |= x;
  }
  return acc != 0;
}

// Whether leaf f holds a source whose bit in b (xor `flip`) is set (one lane).
// The leaf's keys lie in [head[f], head[f + 1]), so its sources lie in
// [src(head[f]), src(head[f + 1])]: a few bitmap words instead of a decode.
// Spans wider than kFgSkipSpan vertices (the last leaf, sparse id ranges) are
// not tested and count as holding one.
constexpr uint32_t kFgSkipSpan = 256;

__device__ __forceinline__ bool fg_leaf_has(const FgArgs& g, const uint32_t* b, uint32_t flip, uint64_t f) {
  const uint64_t h = g.head[f];
  if (h == kNoKey) return false;  // the empty leaf of an empty set
  const uint32_t s0 = src_of(h);
  if (s0 >= g.nv) return false;  // every key of the leaf is ignored
  if (f + 1 >= g.L) return true;
  const uint32_t s1 = min(src_of(g.head[f + 1]), g.nv - 1);
  if (s1 - s0 >= kFgSkipSpan) return true;
  return any_bit(b, flip, s0, s1);
}

// One level of a level-synchronous BFS (the hop distance of every vertex
// reached from the source).  On a symmetric edge set a vertex v joins level
// cur + 1 iff it is unvisited and some neighbour u has level cur, which can be
// found from either end of the edge (u, v):
//   top-down:  for edges (u, v) with u at level cur, mark v if unvisited;
//   bottom-up: for edges (v, u) with v unvisited, mark v if u is at level cur.
// Each direction decodes only the leaves holding a source it needs (level cur,
// resp. unvisited): a wave takes 64 leaves, each lane tests one, and the wave
// then decodes the needed ones one after another.  A mark is a plain store of
// cur + 1 into the levels: every writer stores the same value, and the tests
// read only the bitmaps, which this level does not change.
template <bool kBottomUp>
__global__ void __launch_bounds__(256) k_fg_bfs_step(FgArgs g, BfsBits bb, uint32_t* __restrict__ level,
                                                     uint32_t cur) {
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  for (uint64_t base = wave * kWave; base < g.L; base += nwaves * kWave) {
    const uint64_t f = base + (uint64_t)lane_id();
    const bool need = f < g.L && (kBottomUp ? fg_leaf_has(g, bb.seen, ~0u, f) : fg_leaf_has(g, bb.front, 0u, f));
    uint64_t m = __ballot(need);
    while (m) {
      const uint64_t leaf = base + (uint64_t)(__ffsll((unsigned long long)m) - 1);
      m &= m - 1;
      uint64_t kk[16];
      const uint32_t tm = wave_leaf_keys(g.bytes + leaf * (uint64_t)g.S, g.used[leaf], kk);
#pragma unroll
      for (int i = 0; i < 16; i++) {
        const uint32_t s = src_of(kk[i]), d = dst_of(kk[i]);
        const bool ok = (tm & (1u << i)) && s < g.nv && d < g.nv;
        if (kBottomUp) {
          if (ok && !bit_of(bb.seen, s) && bit_of(bb.front, d)) level[s] = cur + 1;
        } else {
          if (ok && bit_of(bb.front, s) && !bit_of(bb.seen, d)) level[d] = cur + 1;
        }
      }
    }
  }
}

// After a level: the bitmaps for the next one (front: level == next; seen:
// level != unvisited), one 32-bit word per thread, and per block the number of
// vertices at level `next` and of unvisited vertices as one slot pair (summed by
// k_fg_fold_counts; no counter shared by all blocks).
__global__ void __launch_bounds__(256) k_fg_level_bits(const uint32_t* __restrict__ level, uint32_t nv, uint32_t next,
                                                       uint32_t* __restrict__ front, uint32_t* __restrict__ seen,
                                                       unsigned long long* __restrict__ part) {
  __shared__ uint64_t red[2][256 / kWave];
  uint64_t a = 0, b = 0;
  const uint32_t nw = (nv + 31) / 32;
  const bool vec = (reinterpret_cast<uintptr_t>(level) & 15) == 0;  // 16-byte loads of 4 levels
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
    uint32_t fw = 0, sw = 0;
    const uint32_t v0 = w * 32;
    if (v0 + 32 <= nv && vec) {
      const uint4* p = reinterpret_cast<const uint4*>(level + v0);
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const uint4 x = p[q];
        const uint32_t l[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int j = 0; j < 4; j++) {
          fw |= (uint32_t)(l[j] == next) << (4 * q + j);
          sw |= (uint32_t)(l[j] != kUnvisited) << (4 * q + j);
        }
      }
    } else {
      for (uint32_t j = 0; v0 + j < nv; j++) {
        const uint32_t l = level[v0 + j];
        fw |= (uint32_t)(l == next) << j;
        sw |= (uint32_t)(l != kUnvisited) << j;
      }
    }
    front[w] = fw;
    seen[w] = sw;
    a += (uint32_t)__popc(fw);
    b += (uint32_t)(min(32u, nv - v0) - (uint32_t)__popc(sw));
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = a;
    red[1][threadIdx.x / kWave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; w++) {
      a += red[0][w];
      b += red[1][w];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// Sums n slot pairs into out[0], out[1] (one block; out is overwritten).
__global__ void __launch_bounds__(1024) k_fg_fold_counts(const unsigned long long* __restrict__ part, uint32_t n,
                                                         unsigned long long* __restrict__ out) {
  __shared__ uint64_t red[2][1024 / kWave];
  uint64_t a = 0, b = 0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = a;
    red[1][threadIdx.x / kWave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 1024 / kWave; w++) {
      a += red[0][w];
      b += red[1][w];
    }
    out[0] = a;
    out[1] = b;
  }
}

// Degree counts widened for a 64-bit prefix sum (the vertex offset array).
struct U32AsU64Fn {
  const uint32_t* p;
  __device__ uint64_t operator()(uint64_t i) const { return p[i]; }
};

// ---- connected components (label propagation with pointer jumping) -----------
// lab[u] = min(lab[u], min over edges (u, v) of lab[v]), one atomic per run of
// equal source; *changed is set when a label fell.  Labels only fall, and only
// to the label of a vertex of the same component, so the component's smallest
// id keeps its own label and, once no label falls, every vertex holds it.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, off, kWave));
  return x;
}

__global__ void __launch_bounds__(256) k_fg_cc_prop(FgArgs g, uint32_t* __restrict__ lab,
                                                    uint32_t* __restrict__ changed) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  bool ch = false;
  for (uint64_t leaf = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; leaf < g.L;
       leaf += waves) {
    uint64_t kk[16];
    const uint32_t tm = wave_leaf_keys(g.bytes + leaf * (uint64_t)g.S, g.used[leaf], kk);
    uint32_t val[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t sv = src_of(kk[i]), d = dst_of(kk[i]);
      val[i] = ((tm & (1u << i)) && d < g.nv && sv < g.nv) ? lab[d] : 0xffffffffu;
    }
    const uint32_t one = fg_single_source(g, leaf, kk, tm);
    if (one != 0xffffffffu) {
      uint32_t m = 0xffffffffu;
#pragma unroll
      for (int i = 0; i < 16; i++) m = min(m, val[i]);
      m = wave_min_u32(m);
      if (lane_id() == 0 && one < g.nv && m != 0xffffffffu) ch |= atomicMin(&lab[one], m) > m;
      continue;
    }
    uint32_t run = 0xffffffffu, rmin = 0xffffffffu;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (tm & (1u << i)) {
        const uint32_t sv = src_of(kk[i]);
        if (sv != run) {
          if (run < g.nv && rmin != 0xffffffffu) ch |= atomicMin(&lab[run], rmin) > rmin;
          run = sv;
          rmin = 0xffffffffu;
        }
        rmin = min(rmin, val[i]);
      }
    }
    if (run < g.nv && rmin != 0xffffffffu) ch |= atomicMin(&lab[run], rmin) > rmin;
  }
  if (__ballot(ch) && lane_id() == 0) *changed = 1u;  // every writer stores the same value
}

// Pointer jumping: lab[v] = lab[lab[v]] until it stops falling (every label
// on the chain is a vertex of v's component, so the result is too).
__global__ void k_fg_cc_jump(uint32_t* __restrict__ lab, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    uint32_t l = lab[v];
    for (;;) {
      const uint32_t ll = lab[l];
      if (ll >= l) break;
      l = ll;
    }
    lab[v] = l;
  }
}

__global__ void k_fg_iota(uint32_t* __restrict__ lab, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) lab[v] = v;
}

// ---- single-source betweenness (Brandes), level by level --------------------
// With BFS levels from the source known, on a symmetric edge set:
//   sigma[v] = sum over edges (v, u) with level[u] = level[v] - 1 of sigma[u]
//   delta[v] = sigma[v] * sum over edges (v, w) with level[w] = level[v] + 1 of
//              (1 + delta[w]) / sigma[w]
// A level's pass decodes only the leaves holding a source of that level (the
// `front` bitmap), folds each run of equal source and adds it with one FP64
// atomic.  kDelta selects the second formula.
template <bool kDelta>
__global__ void __launch_bounds__(256) k_fg_bc_level(FgArgs g, BfsBits bb, const uint32_t* __restrict__ level,
                                                     uint32_t cur, const double* sigma_in, const double* delta_in,
                                                     double* out) {
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint32_t want = kDelta ? cur + 1 : cur - 1;  // the neighbours' level
  for (uint64_t base = wave * kWave; base < g.L; base += nwaves * kWave) {
    const uint64_t f = base + (uint64_t)lane_id();
    const bool need = f < g.L && fg_leaf_has(g, bb.front, 0u, f);
    uint64_t m = __ballot(need);
    while (m) {
      const uint64_t leaf = base + (uint64_t)(__ffsll((unsigned long long)m) - 1);
      m &= m - 1;
      uint64_t kk[16];
      const uint32_t tm = wave_leaf_keys(g.bytes + leaf * (uint64_t)g.S, g.used[leaf], kk);
      uint32_t run = 0xffffffffu;
      double acc = 0.0;
      bool any = false;
#pragma unroll
      for (int i = 0; i < 16; i++) {
        if (!(tm & (1u << i))) continue;
        const uint32_t sv = src_of(kk[i]), d = dst_of(kk[i]);
        if (sv != run) {
          if (any) atomicAdd(&out[run], kDelta ? sigma_in[run] * acc : acc);
          run = sv;
          acc = 0.0;
          any = false;
        }
        if (sv < g.nv && d < g.nv && bit_of(bb.front, sv) && level[d] == want) {
          acc += kDelta ? (1.0 + delta_in[d]) / sigma_in[d] : sigma_in[d];
          any = true;
        }
      }
      if (any) atomicAdd(&out[run], kDelta ? sigma_in[run] * acc : acc);
    }
  }
}

// PageRank vertex kernels: contrib[u] = p[u] / deg[u] (0 for isolated vertices),
// and the update p[v] = (1 - d) / N + d * acc[v].
__global__ void k_pr_contrib(const float* __restrict__ p, const uint32_t* __restrict__ deg, uint32_t nv,
                             float* __restrict__ contrib, float* __restrict__ acc) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    contrib[v] = deg[v] ? p[v] / (float)deg[v] : 0.f;
    acc[v] = 0.f;
  }
}

__global__ void k_pr_update(const float* __restrict__ acc, uint32_t nv, float base, float damping,
                            float* __restrict__ p) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x)
    p[v] = base + damping * acc[v];
}

}  // namespace cpma_dev
