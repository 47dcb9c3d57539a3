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
// pushing p(u)/deg(u) along every edge.  BFS is level synchronous: a pass over
// all edges claims the unvisited targets of the current level's vertices.
#pragma once
#include "leaf.hpp"

namespace cpma_dev {

struct FgArgs {
  const uint8_t* bytes;
  const uint32_t* used;
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

// deg[u] += number of edges with source u.
__global__ void __launch_bounds__(256) k_fg_degree(FgArgs g, uint32_t* __restrict__ deg) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  for (uint64_t leaf = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; leaf < g.L;
       leaf += waves) {
    uint64_t kk[16];
    const uint32_t tm = wave_leaf_keys(g.bytes + leaf * (uint64_t)g.S, g.used[leaf], kk);
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

// Level-synchronous BFS step as a full pass: for every edge (u, v) with u at
// level `cur` and v unvisited, v is claimed for level cur + 1 (compare-and-swap,
// so each vertex is counted once); *found counts the claims.
__global__ void __launch_bounds__(256) k_fg_bfs_step(FgArgs g, uint32_t* __restrict__ level, uint32_t cur,
                                                     unsigned int* __restrict__ found) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  uint32_t claimed = 0;
  for (uint64_t leaf = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; leaf < g.L;
       leaf += waves) {
    uint64_t kk[16];
    const uint32_t tm = wave_leaf_keys(g.bytes + leaf * (uint64_t)g.S, g.used[leaf], kk);
    bool hit[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t s = src_of(kk[i]), d = dst_of(kk[i]);
      const bool ok = (tm & (1u << i)) && s < g.nv && d < g.nv;
      hit[i] = ok && level[s] == cur && level[d] == 0xffffffffu;
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (hit[i]) {
        const uint32_t d = dst_of(kk[i]);
        if (atomicCAS(&level[d], 0xffffffffu, cur + 1) == 0xffffffffu) claimed++;
      }
    }
  }
  // the host only tests for zero: a plain store of 1, not a counter every
  // wave would serialise on
  if (__ballot(claimed != 0) && lane_id() == 0)
    __hip_atomic_store(found, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
