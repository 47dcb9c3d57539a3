// Device-side building blocks shared by every CPMA kernel on gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpma_dev {

constexpr int kWave = 64;
constexpr uint64_t kNoKey = ~0ull;   // reserved key: head of an empty single-leaf set
constexpr int64_t kQ = 65536;        // fixed-point unit of the density bounds
constexpr int kMaxLevels = 48;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// ---- DPP wave primitives (GFX9 row shifts, row broadcasts, wave shifts) -------------
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf, bool BOUND_ZERO = true>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO);
}
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf, bool BOUND_ZERO = true>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t lo = dpp32<CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO>((uint32_t)v);
  const uint32_t hi = dpp32<CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum over the 64 lanes: in-row Hillis-Steele steps of 1, 2, 4, 8
// lanes, then the row broadcasts of lanes 15 and 31.
template <typename T>
__device__ __forceinline__ T dpp_incl_scan(T v);
template <>
__device__ __forceinline__ uint32_t dpp_incl_scan<uint32_t>(uint32_t v) {
  v += dpp32<0x111>(v);
  v += dpp32<0x112>(v);
  v += dpp32<0x114>(v);
  v += dpp32<0x118>(v);
  v += dpp32<0x142, 0xa, 0xf, false>(v);
  v += dpp32<0x143, 0xc, 0xf, false>(v);
  return v;
}
template <>
__device__ __forceinline__ uint64_t dpp_incl_scan<uint64_t>(uint64_t v) {
  v += dpp64<0x111>(v);
  v += dpp64<0x112>(v);
  v += dpp64<0x114>(v);
  v += dpp64<0x118>(v);
  v += dpp64<0x142, 0xa, 0xf, false>(v);
  v += dpp64<0x143, 0xc, 0xf, false>(v);
  return v;
}

// Inclusive prefix maximum over the 64 lanes (same step pattern).
__device__ __forceinline__ uint32_t dpp_incl_max(uint32_t v) {
  v = max(v, dpp32<0x111>(v));
  v = max(v, dpp32<0x112>(v));
  v = max(v, dpp32<0x114>(v));
  v = max(v, dpp32<0x118>(v));
  v = max(v, dpp32<0x142, 0xa, 0xf, false>(v));
  v = max(v, dpp32<0x143, 0xc, 0xf, false>(v));
  return v;
}

// Value of lane l-1 (0 for lane 0) and of lane l+1 (0 for lane 63).
__device__ __forceinline__ uint32_t dpp_prev32(uint32_t v) { return dpp32<0x138>(v); }
__device__ __forceinline__ uint64_t dpp_prev64(uint64_t v) { return dpp64<0x138>(v); }
__device__ __forceinline__ uint32_t dpp_next32(uint32_t v) { return dpp32<0x130>(v); }
__device__ __forceinline__ uint64_t dpp_next64(uint64_t v) { return dpp64<0x130>(v); }

__device__ __forceinline__ uint32_t lane63_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint64_t lane63_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// ---- wave-level scans / reductions (64 lanes, DPP) ---------------------------------
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  return dpp_incl_scan<T>(v);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v);
template <>
__device__ __forceinline__ uint32_t wave_sum<uint32_t>(uint32_t v) {
  return lane63_u32(dpp_incl_scan<uint32_t>(v));
}
template <>
__device__ __forceinline__ uint64_t wave_sum<uint64_t>(uint64_t v) {
  return lane63_u64(dpp_incl_scan<uint64_t>(v));
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v |= __shfl_xor(v, d, kWave);
  return v;
}

// ---- byte codes ------------------------------------------------------------------
// A delta d >= 1 takes ceil(bitlen(d) / 7) bytes: 7 payload bits per byte, least
// significant group first, high bit set while more bytes follow.
__host__ __device__ __forceinline__ uint32_t vlen(uint64_t d) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t bits = 64u - (uint32_t)__clzll((long long)(d | 1));
#else
  uint32_t bits = 64u - (uint32_t)__builtin_clzll(d | 1);
#endif
  return (bits + 6u) / 7u;
}

// Writes the code of d at dst (dst may be LDS or global); returns its length.
__device__ __forceinline__ uint32_t vput(uint8_t* dst, uint64_t d) {
  uint32_t n = 0;
  while (d >= 0x80) {
    dst[n++] = (uint8_t)(d | 0x80);
    d >>= 7;
  }
  dst[n++] = (uint8_t)d;
  return n;
}

__device__ __forceinline__ void put_le64(uint8_t* dst, uint64_t x) {
#pragma unroll
  for (int i = 0; i < 8; i++) dst[i] = (uint8_t)(x >> (8 * i));
}

// ---- density bounds ----------------------------------------------------------------
// Upper / lower byte-density bound at height h of a tree of height H, fixed point
// 1/65536, interpolated linearly between the leaf and the root values.
struct Bounds {
  int64_t up_leaf, up_root, lo_leaf, lo_root;
  int H;          // ceil(log2 L)
  uint64_t L;     // leaves
  uint32_t S;     // leaf bytes
};

__host__ __device__ __forceinline__ int64_t bound_up(const Bounds& b, int h) {
  return b.H == 0 ? b.up_leaf : b.up_leaf - ((b.up_leaf - b.up_root) * h) / b.H;
}
__host__ __device__ __forceinline__ int64_t bound_lo(const Bounds& b, int h) {
  return b.H == 0 ? b.lo_leaf : b.lo_leaf + ((b.lo_root - b.lo_leaf) * h) / b.H;
}

// Violation of node (h, i) holding `sum` filled bytes over `nleaves` leaves:
// bit 0 = above its upper bound, bit 1 = below its lower bound.  The root of a
// single-leaf structure has no lower bound.
__host__ __device__ __forceinline__ uint32_t violation(const Bounds& b, int h, uint64_t sum,
                                                       uint64_t nleaves) {
  const uint64_t cap = nleaves * (uint64_t)b.S;
  const uint64_t lhs = sum * (uint64_t)kQ;
  uint32_t v = 0;
  if (lhs > (uint64_t)bound_up(b, h) * cap) v |= 1u;
  const bool exempt = (h == b.H) && (b.L == 1);
  if (!exempt && lhs < (uint64_t)bound_lo(b, h) * cap) v |= 2u;
  return v;
}

// Implicit-tree level table: level h (1..H) of a tree over L leaves has
// ceil(L / 2^h) nodes stored at base + off[h]; level 0 is the used[] array.
struct Pyramid {
  uint64_t* base;
  uint64_t off[kMaxLevels];
  uint64_t cnt[kMaxLevels];
  int H;
};

__device__ __forceinline__ uint64_t node_sum(const Pyramid& p, const uint32_t* used, int h,
                                             uint64_t i) {
  return h == 0 ? (uint64_t)used[i] : p.base[p.off[h] + i];
}
__device__ __forceinline__ uint64_t node_leaves(uint64_t L, int h, uint64_t i) {
  uint64_t first = i << h;
  uint64_t last = first + (1ull << h);
  return (last > L ? L : last) - first;
}

// Plain fill kernel (used instead of memset nodes so the work can be graph-captured).
template <typename T>
__global__ void k_fill(T* p, uint64_t n, T v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Two small regions cleared in one launch of one block (an update's counters
// and its batch flags): one launch less on a queue that is often idle.
__global__ void k_clear2(uint32_t* a, uint32_t na, uint32_t* b, uint32_t nb) {
  for (uint32_t i = threadIdx.x; i < na + nb; i += blockDim.x) {
    if (i < na)
      a[i] = 0u;
    else
      b[i - na] = 0u;
  }
}

}  // namespace cpma_dev
