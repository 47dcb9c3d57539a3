// Host orchestration and C ABI of the MI355X CPMA (declarations: include/cpma.h).
//
// One handle owns a device-resident CPMA: leaves (L * S bytes), leaf heads and
// used byte counts, plus scratch kept across calls.  A batch update runs the
// paper's three phases (Section "Parallel Batch Updates in a PMA") as device
// kernels: merge into leaves (with out-of-place overflow), counting of node
// densities up the implicit tree, and redistribution of the violating regions;
// the host only reads a few counters at the sync points between phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "cpma.h"
#include "query.hpp"
#include "sort.hpp"
#include "update.hpp"
#include "merge_lane.hpp"
#include "merge_heavy.hpp"
#include "merge_wave.hpp"
#include "fgraph.hpp"
#include "resize.hpp"
#include "tune.hpp"
#include "small.hpp"
#include "fuse.hpp"
#include "pma.hpp"
#include "kv.hpp"

using namespace cpma_dev;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  const cpma_config* al = nullptr;  // the owner's allocator hooks (NULL hooks: hipMalloc)
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

struct Fail {
  cpma_status st;
};

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) throw Fail{CPMA_ERR_DEVICE}; \
  } while (0)

// Device memory through the owner's hooks, else hipMalloc / hipFree.
void* dev_alloc(const cpma_config* al, size_t bytes) {
  if (al && al->alloc) {
    void* p = al->alloc(bytes, al->ctx);
    if (p && (reinterpret_cast<uintptr_t>(p) & 255)) {  // the hooks promise 256-byte alignment
      al->free(p, al->ctx);
      throw Fail{CPMA_ERR_INVALID};
    }
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(const cpma_config* al, void* p) {
  if (!p) return;
  if (al && al->free)
    al->free(p, al->ctx);
  else
    hipFree(p);
}

// Grows b to at least `bytes` (contents are not kept), with `slack` extra room.
void ensure(DevBuf& b, size_t bytes, double slack = 0.5) {
  if (bytes == 0) bytes = 16;
  if (b.cap >= bytes) return;
  if (b.p) {
    dev_free(b.al, b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + (size_t)((double)bytes * slack) + 256;
  b.p = dev_alloc(b.al, want);
  if (!b.p) {
    b.p = dev_alloc(b.al, bytes);
    if (!b.p) throw Fail{CPMA_ERR_NOMEM};
    want = bytes;
  }
  b.cap = want;
}

void release(DevBuf& b) {
  dev_free(b.al, b.p);
  b.p = nullptr;
  b.cap = 0;
}

uint32_t grid_for(uint64_t n, uint32_t block, uint32_t cap = 65535u * 4) {
  uint64_t g = (n + block - 1) / block;
  if (g == 0) g = 1;
  return (uint32_t)std::min<uint64_t>(g, cap);
}

int tree_height(uint64_t L) {
  int H = 0;
  while ((1ull << H) < L) H++;
  return H;
}

}  // namespace

struct cpma {
  int device = 0;
  int num_cus = 256;
  uint32_t rm_blocks[2] = {2048, 2048};  // resident blocks of k_rm_interior<false>, <true>
  int msd_bits = 0;  // bit length of the last unsorted batch of the MSD split's size (0: none yet)
  // a small batch's merge totals, left for the single-block path check to fold
  const unsigned long long* fin_parts = nullptr;
  uint32_t fin_nn = 0, fin_nw = 0;
  cpma_config cfg{};
  uint32_t S = 1024;
  uint64_t L = 0, n = 0;
  int64_t q_up_leaf = 0, q_up_root = 0, q_lo_leaf = 0, q_lo_root = 0;
  DevBuf bytes, used, head;
  // the pyramid holds every node's byte sum of the current layout: set by a
  // count that found every node within bounds, cleared by any other use of
  // the pyramid's memory
  bool pyr_valid = false;
  // scratch
  DevBuf kin, kb0, kb1, kdedup, leafid, segpos, seg_leaf, seg_begin, seg_desc, heavy, spill, scan_tmp, ovf, arena,
      stage, pyr, win, wargs, cnt, koff, win_id, welem, P, ccost, ncost, lstart, planU, plan_used,
      spare_bytes, spare_used, spare_head, fg_level, fg_deg, fg_p, fg_c, fg_acc,
      win_of_leaf, fail, qa, qb, qfirst, qnvis, qvoff, qsum, qcount, qout, lastk, lckpt, ne_rank, ne_list, chain_pfx,
      srec, wide, srcinfo, parts, qparts, fz_meta, fz_v0, fz_v1, fz_byte, fz_member, fz_code, fz_ctr, fz_res,
      ctr_buf, info_buf, qalg_buf, clen, spare_clen, vstage, kvals, kvdedup;
  // key-value sets: the current update batch's values (device, repeat-free and
  // in batch order), NULL for key-only updates
  const uint64_t* batch_vals = nullptr;
  bool kv() const { return cfg.values != 0; }
  // the leaf array the key decoders read as "used": the code bytes of a
  // key-value set, else the filled bytes
  const uint32_t* code_bytes() const { return (const uint32_t*)(cfg.values ? clen.p : used.p); }
  Counters* dctr = nullptr;
  Counters* hctr = nullptr;
  BatchInfo* dinfo = nullptr;
  BatchInfo* hinfo = nullptr;
  void* hpin = nullptr;  // pinned host staging for small uploads
  size_t hpin_cap = 0;
  uint64_t wol_L = 0;    // leaves covered by win_of_leaf's -1 initialisation
  bool broken = false;
  // set when the current call has started writing the structure: an
  // allocation failure after that point cannot leave the set unchanged
  bool mutating = false;
  // phase statistics (cpma_stats_*)
  bool stats_on = false;
  uint32_t stats_mask = 0;  // phases timed while stats_on: bit (1 << phase)
  cpma_phase_stat stats[CPMA_PHASE_NUM];
  struct Pending {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> evpool;
  unsigned long long* dqalg = nullptr;  // range-scan byte counter

  // every device buffer the handle owns (allocator hooks, release)
  std::vector<DevBuf*> bufs() {
    return {&bytes,     &used,      &head,      &kin,         &kb0,        &kb1,         &kdedup,     &leafid,
            &segpos,    &seg_leaf,  &seg_begin, &seg_desc,    &heavy,      &spill,       &scan_tmp,   &ovf,
            &arena,     &stage,     &pyr,       &win,         &wargs,      &cnt,         &koff,       &win_id,
            &welem,     &P,         &ccost,     &ncost,       &lstart,     &planU,       &plan_used,  &spare_bytes,
            &spare_used, &spare_head, &fg_level, &fg_deg,     &fg_p,       &fg_c,        &fg_acc,     &win_of_leaf,
            &fail,      &qa,        &qb,        &qfirst,      &qnvis,      &qvoff,       &qsum,       &qcount,
            &qout,      &lastk,     &ne_rank,   &ne_list,     &chain_pfx,  &srec,        &wide,       &srcinfo,
            &parts,     &qparts,    &fz_meta,   &fz_v0,       &fz_v1,      &fz_byte,     &fz_member,  &fz_code,
            &fz_ctr,    &fz_res,    &ctr_buf,   &info_buf,    &qalg_buf,   &lckpt,      &clen,        &spare_clen,
            &vstage,    &kvals,     &kvdedup};
  }

  Bounds bounds(uint64_t Lx) const {
    Bounds b;
    b.up_leaf = q_up_leaf;
    b.up_root = q_up_root;
    b.lo_leaf = q_lo_leaf;
    b.lo_root = q_lo_root;
    b.H = tree_height(Lx);
    b.L = Lx;
    b.S = S;
    return b;
  }
};

namespace {

Pyramid pyramid_layout(uint64_t L) {
  Pyramid P;
  memset(&P, 0, sizeof(P));
  P.H = tree_height(L);
  uint64_t off = 0;
  P.cnt[0] = L;
  for (int h = 1; h <= P.H; h++) {
    P.cnt[h] = (L + (1ull << h) - 1) >> h;
    P.off[h] = off;
    off += P.cnt[h];
  }
  return P;
}

// Layout of the pyramid of L leaves with its memory; the memory's contents are
// the caller's from here on.
Pyramid make_pyramid(cpma* s, uint64_t L) {
  Pyramid P = pyramid_layout(L);
  s->pyr_valid = false;
  const uint64_t nodes = P.H == 0 ? 0 : P.off[P.H] + P.cnt[P.H];  // above the leaves
  ensure(s->pyr, (nodes + 1) * sizeof(uint64_t));
  P.base = s->pyr.as<uint64_t>();
  return P;
}

void build_pyramid(cpma* s, const Pyramid& P, const uint32_t* used, uint64_t L, hipStream_t st) {
  if (P.H == 0) return;
  const int top = std::min(P.H, kPyrLowLevels);
  const uint64_t blocks = (P.cnt[1] + kPyrThreads - 1) / kPyrThreads;
  hipLaunchKernelGGL(k_pyr_low, dim3((uint32_t)blocks), dim3(kPyrThreads), 0, st, used, L, P, top);
  if (P.H > top) hipLaunchKernelGGL(k_pyr_high, dim3(1), dim3(1024), 0, st, P, top);
  HIPCHK(hipGetLastError());
}

void* host_pin(cpma* s, size_t bytes) {
  if (s->hpin_cap < bytes) {
    if (s->hpin) {
      HIPCHK(hipDeviceSynchronize());  // no copy may still read the old buffer
      hipHostFree(s->hpin);
    }
    s->hpin = nullptr;
    size_t want = std::max<size_t>(2 * bytes, 1 << 16);  // room, so a slowly growing need reallocates rarely
    HIPCHK(hipHostMalloc(&s->hpin, want, hipHostMallocDefault));
    s->hpin_cap = want;
  }
  return s->hpin;
}

void zero_counters(cpma* s, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(s->dctr),
                     (uint64_t)(sizeof(Counters) / 4), 0u);
  HIPCHK(hipGetLastError());
}

// ---- phase timing with HIP events (only while statistics are enabled) ----------
struct PhaseMark {
  int phase;
  hipEvent_t a;
};

hipEvent_t get_event(cpma* s) {
  if (!s->evpool.empty()) {
    hipEvent_t e = s->evpool.back();
    s->evpool.pop_back();
    return e;
  }
  // timing only: results always come back through stream synchronisation,
  // so the record needs no system-scope fence (whose cache writeback and
  // invalidation would idle the GPU between the timed kernels)
  hipEvent_t e;
  HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}

PhaseMark phase_begin(cpma* s, int phase, hipStream_t st) {
  if (!s->stats_on || !((s->stats_mask >> phase) & 1u)) return PhaseMark{-1, nullptr};
  hipEvent_t e = get_event(s);
  HIPCHK(hipEventRecord(e, st));
  return PhaseMark{phase, e};
}

void phase_end(cpma* s, const PhaseMark& m, hipStream_t st, uint64_t alg_bytes = 0) {
  if (m.phase < 0) return;
  hipEvent_t e = get_event(s);
  HIPCHK(hipEventRecord(e, st));
  s->pending.push_back({m.phase, m.a, e});
  s->stats[m.phase].alg_bytes += alg_bytes;
}

// Folds the recorded event pairs into the statistics (waits for each pair's
// end event: a phase may end after the call's last synchronisation).
void resolve_phases(cpma* s) {
  for (const auto& p : s->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      s->stats[p.phase].ms += ms;
      s->stats[p.phase].launches += 1;
    }
    s->evpool.push_back(p.a);
    s->evpool.push_back(p.b);
  }
  s->pending.clear();
}

void read_counters(cpma* s, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(s->hctr, s->dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  resolve_phases(s);
  if (s->hctr->error) throw Fail{CPMA_ERR_DEVICE};
}

template <typename T, typename F>
void scan(cpma* s, T* out, uint64_t n, hipStream_t st, F fn) {
  ensure(s->scan_tmp, scan_scratch_elems(n) * sizeof(T));
  HIPCHK(scan_exclusive<T>(fn, n, out, s->scan_tmp.as<T>(), st));
}

// MSD split of an unsorted batch into buckets small enough for one block's
// LDS, then every bucket sorted there with its repeats removed (src -> kb0 ->
// kb1), then the buckets' first occurrences packed into kdedup (their number
// in dctr->kprime).  The bucket count makes an average bucket about 0.8
// kBktCap keys; the low bits sorted inside a bucket must fit 32 bits.
struct MsdPlan {
  int r = 0;          // low bits sorted inside a bucket
  uint32_t nd = 0;    // buckets
  uint32_t nt = 0;    // split tiles
  uint64_t nc() const { return (uint64_t)nd * nt; }
};

bool msd_plan(uint64_t k, int bits, MsdPlan* p) {
  int b = kMsdMinBits;
  while (b < kMsdMaxBits && (k >> b) > kBktTarget) b++;
  b = std::min(b, bits);
  if (bits - b > 32 || (k >> b) > kBktTarget) return false;
  p->r = bits - b;
  p->nd = 1u << b;
  p->nt = (uint32_t)((k + kMsdTile - 1) / kMsdTile);
  return true;
}

void msd_buffers(cpma* s, uint64_t k, const MsdPlan& p) {
  ensure(s->cnt, (p.nc() + 1) * sizeof(uint32_t));
  ensure(s->koff, (p.nc() + 1) * sizeof(uint32_t));
  ensure(s->kb0, k * sizeof(uint64_t));
  ensure(s->kb1, k * sizeof(uint64_t));
  ensure(s->kdedup, k * sizeof(uint64_t));
}

// Bucket starts from the per-tile counts in s->cnt, and the largest bucket
// into dinfo->max_bucket; with publish, the BatchInfo also goes to s->hinfo
// (see wait_published).
void msd_offsets(cpma* s, const MsdPlan& p, hipStream_t st, bool publish = false) {
  scan<uint32_t>(s, s->koff.as<uint32_t>(), p.nc(), st, LoadFn<uint32_t>{s->cnt.as<uint32_t>()});
  if (publish) __atomic_store_n(&s->hinfo->ready, 0u, __ATOMIC_RELEASE);
  hipLaunchKernelGGL(k_msd_max, dim3(1), dim3(kMsdThreads), 0, st, (const uint32_t*)s->koff.as<uint32_t>(), p.nt,
                     p.nd, s->dinfo, publish ? s->hinfo : nullptr);
  HIPCHK(hipGetLastError());
}

// Waits until a kernel has published the BatchInfo to s->hinfo (its ready
// field), polling host memory instead of synchronising the stream, whose
// later work may already be queued.  Bounded: after a second the stream is
// synchronised, which reports a device error if there was one.
void wait_published(cpma* s, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t it = 1;; it++) {
    if (__atomic_load_n(&s->hinfo->ready, __ATOMIC_ACQUIRE)) return;
    if ((it & 4095u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) break;
    __builtin_ia32_pause();
  }
  HIPCHK(hipStreamSynchronize(st));
  if (!__atomic_load_n(&s->hinfo->ready, __ATOMIC_ACQUIRE)) throw Fail{CPMA_ERR_DEVICE};
}

// Split, bucket sorts and packing, once the bucket starts are known and no
// bucket exceeds kBktCap.
void msd_finish(cpma* s, const uint64_t* src, uint64_t k, const MsdPlan& p, hipStream_t st) {
  const uint32_t* koff = s->koff.as<uint32_t>();
  hipLaunchKernelGGL(k_msd_scatter, dim3(p.nt), dim3(kMsdThreads), 0, st, src, s->kb0.as<uint32_t>(), (uint32_t)k,
                     p.r, p.nd, koff);
  HIPCHK(hipGetLastError());
  // the per-tile counts are consumed: their buffer takes the buckets' first
  // occurrence counts and those counts' scan (nc >= 32 nd)
  uint32_t* ucnt = s->cnt.as<uint32_t>();
  uint32_t* uoff = ucnt + p.nd + 1;
  hipLaunchKernelGGL(k_bucket_sort, dim3(p.nd), dim3(kBktThreads), 0, st, (const uint32_t*)s->kb0.as<uint32_t>(),
                     s->kb1.as<uint64_t>(), koff, p.nt, p.r, ucnt, &s->dctr->error);
  HIPCHK(hipGetLastError());
  scan<uint32_t>(s, uoff, p.nd, st, LoadFn<uint32_t>{ucnt});
  hipLaunchKernelGGL(k_bucket_compact, dim3(p.nd), dim3(256), 0, st, (const uint64_t*)s->kb1.as<uint64_t>(), koff,
                     p.nt, (const uint32_t*)uoff, p.nd, s->kdedup.as<uint64_t>(), &s->dctr->kprime);
  HIPCHK(hipGetLastError());
}

// The split for a batch whose bit length is known: counts, then the largest
// bucket read back before anything is written.  False if a bucket exceeds
// kBktCap (skewed batches) or the plan does not apply; the caller then sorts
// with LSD passes.
bool msd_split_sort(cpma* s, const uint64_t* src, uint64_t k, int bits, hipStream_t st) {
  MsdPlan p;
  if (!msd_plan(k, bits, &p)) return false;
  msd_buffers(s, k, p);
  hipLaunchKernelGGL(k_msd_hist, dim3(p.nt), dim3(kMsdThreads), 0, st, src, (uint32_t)k, p.r, p.nd,
                     s->cnt.as<uint32_t>());
  HIPCHK(hipGetLastError());
  // a count for a wrong bit length may have left its maximum
  hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, &s->dinfo->max_bucket, (uint64_t)1, 0u);
  msd_offsets(s, p, st);
  HIPCHK(hipMemcpyAsync(s->hinfo, s->dinfo, sizeof(BatchInfo), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (s->hinfo->max_bucket > kBktCap) return false;
  msd_finish(s, src, k, p, st);
  return true;
}

// ---------------------------------------------------------------------------
// Batch prep: device copy, validation, radix sort, removal of repeats.
// Returns the device pointer of the sorted repeat-free batch; its length is in
// dctr->kprime (device).  Throws CPMA_ERR_RESERVED_KEY before any mutation.
// ---------------------------------------------------------------------------
const uint64_t* prepare_batch(cpma* s, const uint64_t* keys, uint64_t k, cpma_mem mem, hipStream_t st,
                              bool clear_counters = false) {
  if (k >= (1ull << 32)) throw Fail{CPMA_ERR_INVALID};
  const uint64_t* src = keys;
  if (mem == CPMA_MEM_HOST) {
    ensure(s->kin, k * sizeof(uint64_t));
    HIPCHK(hipMemcpyAsync(s->kin.p, keys, k * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    src = s->kin.as<uint64_t>();
  }
  if (clear_counters)  // the update's counters too, in the same launch
    hipLaunchKernelGGL(k_clear2, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(s->dctr),
                       (uint32_t)(sizeof(Counters) / 4), reinterpret_cast<uint32_t*>(s->dinfo),
                       (uint32_t)(sizeof(BatchInfo) / 4));
  else
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(s->dinfo),
                       (uint64_t)(sizeof(BatchInfo) / 4), 0u);
  // validation reads every key once; below the MSD split's size it also
  // counts the first radix digit per sort tile (used if the batch turns out
  // unsorted)
  const uint32_t nblk = (uint32_t)((k + kSortTile - 1) / kSortTile);
  ensure(s->cnt, ((uint64_t)nblk * 256 + 1) * sizeof(uint32_t));
  ensure(s->koff, ((uint64_t)nblk * 256 + 1) * sizeof(uint32_t));
  // batches of the MSD split's size: with the bit length of the last such
  // batch, validation also counts the split's buckets and the bucket starts
  // are scanned before the one read-back
  const bool msd_size = k >= kMsdMinKeys && k <= kMsdMaxKeys;
  MsdPlan guess;
  const bool fused = msd_size && s->msd_bits > 0 && msd_plan(k, s->msd_bits, &guess);
  // the validation counts the first LSD digit when the split is out of reach
  // (batch size, or the last large batch's bit length); hist0 says whether
  // those counts are still in s->cnt
  bool hist0 = !msd_size || (s->msd_bits > 0 && !fused);
  if (fused) {
    msd_buffers(s, k, guess);
    hipLaunchKernelGGL(k_validate_msd, dim3(guess.nt), dim3(kMsdThreads), 0, st, src, (uint32_t)k, guess.r, guess.nd,
                       s->dinfo, s->cnt.as<uint32_t>());
    HIPCHK(hipGetLastError());
    msd_offsets(s, guess, st, true);
  } else if (!hist0) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(k, 256, 4096)), dim3(256), 0, st, src, k, s->dinfo);
  } else {
    hipLaunchKernelGGL(k_validate_hist, dim3(nblk), dim3(kSortThreads), 0, st, src, (uint32_t)k, s->dinfo,
                       s->cnt.as<uint32_t>());
  }
  HIPCHK(hipGetLastError());
  if (fused) {
    wait_published(s, st);
  } else {
    HIPCHK(hipMemcpyAsync(s->hinfo, s->dinfo, sizeof(BatchInfo), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (s->hinfo->has_reserved) throw Fail{CPMA_ERR_RESERVED_KEY};

  const uint64_t* sorted = src;
  PhaseMark pm = phase_begin(s, CPMA_PHASE_SORT, st);
  uint64_t sort_bytes = 0;
  if (s->hinfo->unsorted) {
    const uint64_t orv = s->hinfo->or_all;
    int bits = 64 - __builtin_clzll(orv | 1);
    int passes = (bits + 7) / 8;
    ensure(s->kb0, k * sizeof(uint64_t));
    ensure(s->kb1, k * sizeof(uint64_t));
    if (msd_size) {
      // the validation's counts hold if this batch has no more bits than the
      // one they were counted for (fewer only leaves high buckets empty)
      const bool counted = fused && bits <= s->msd_bits && s->hinfo->max_bucket <= kBktCap;
      s->msd_bits = bits;
      if (counted) {
        msd_finish(s, src, k, guess, st);
        // split (read 8, write 4), bucket sort (read 4, write 8), packing
        // (read + write 16); the counts came with the validation, repeats are
        // removed
        phase_end(s, pm, st, 40ull * k);
        return s->kdedup.as<uint64_t>();
      }
      MsdPlan own;
      if (msd_plan(k, bits, &own)) {
        hist0 = false;  // the recount overwrites them
        if (msd_split_sort(s, src, k, bits, st)) {
          // count (read 8), then as above
          phase_end(s, pm, st, 48ull * k);
          return s->kdedup.as<uint64_t>();
        }
      }
    }
    const uint64_t* in = src;
    for (int p = 0; p < passes; p++) {
      uint64_t* out = (p & 1) ? s->kb1.as<uint64_t>() : s->kb0.as<uint64_t>();
      if (p > 0 || !hist0)  // else the first pass's counts came with the validation
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, st, in, (uint32_t)k, 8 * p,
                           s->cnt.as<uint32_t>());
      HIPCHK(hipGetLastError());
      scan<uint32_t>(s, s->koff.as<uint32_t>(), (uint64_t)nblk * 256, st,
                     LoadFn<uint32_t>{s->cnt.as<uint32_t>()});
      hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, st, in, out, (uint32_t)k,
                         8 * p, (const uint32_t*)s->koff.as<uint32_t>());
      HIPCHK(hipGetLastError());
      in = out;
    }
    if (passes) {
      sorted = in;
      sort_bytes = 24ull * k * (uint64_t)passes;
    }
  }
  ensure(s->kdedup, k * sizeof(uint64_t));
  {
    const uint32_t nt = (uint32_t)std::max<uint64_t>(1, (k + kSortTile - 1) / kSortTile);
    ensure(s->cnt, ((uint64_t)nt + 1) * sizeof(uint32_t));
    ensure(s->koff, ((uint64_t)nt + 1) * sizeof(uint32_t));
    hipLaunchKernelGGL(k_unique_count, dim3(nt), dim3(kSortThreads), 0, st, sorted, k, s->cnt.as<uint32_t>());
    HIPCHK(hipGetLastError());
    scan<uint32_t>(s, s->koff.as<uint32_t>(), nt, st, LoadFn<uint32_t>{s->cnt.as<uint32_t>()});
    hipLaunchKernelGGL(k_unique_write, dim3(nt), dim3(kSortThreads), 0, st, sorted, k,
                       (const uint32_t*)s->koff.as<uint32_t>(), nt, s->kdedup.as<uint64_t>(), &s->dctr->kprime);
    HIPCHK(hipGetLastError());
  }
  phase_end(s, pm, st, sort_bytes + 24ull * k);
  return s->kdedup.as<uint64_t>();
}

// Batch prep with values: validation, a stable radix sort of the keys carrying
// their input positions, then the first occurrence of every key with the value
// at its position (vals NULL: values 0).  Returns the repeat-free keys; their
// values are in s->kvdedup and their number in dctr->kprime.  Throws
// CPMA_ERR_RESERVED_KEY before any mutation.
const uint64_t* kv_prepare(cpma* s, const uint64_t* keys, const uint64_t* vals, uint64_t k, cpma_mem mem,
                           hipStream_t st) {
  if (k >= (1ull << 31)) throw Fail{CPMA_ERR_INVALID};  // positions travel in 31 bits
  const uint64_t* src = keys;
  const uint64_t* vsrc = vals;
  if (mem == CPMA_MEM_HOST) {
    ensure(s->kin, k * sizeof(uint64_t));
    HIPCHK(hipMemcpyAsync(s->kin.p, keys, k * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    src = s->kin.as<uint64_t>();
    if (vals) {
      ensure(s->kvals, k * sizeof(uint64_t));
      HIPCHK(hipMemcpyAsync(s->kvals.p, vals, k * sizeof(uint64_t), hipMemcpyHostToDevice, st));
      vsrc = s->kvals.as<uint64_t>();
    }
  }
  hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(s->dinfo),
                     (uint64_t)(sizeof(BatchInfo) / 4), 0u);
  hipLaunchKernelGGL(k_validate, dim3(grid_for(k, 256, 4096)), dim3(256), 0, st, src, k, s->dinfo);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(s->hinfo, s->dinfo, sizeof(BatchInfo), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (s->hinfo->has_reserved) throw Fail{CPMA_ERR_RESERVED_KEY};
  PhaseMark pm = phase_begin(s, CPMA_PHASE_SORT, st);
  const int bits = 64 - __builtin_clzll(s->hinfo->or_all | 1);
  const int passes = (bits + 7) / 8;
  ensure(s->kb0, k * sizeof(uint64_t));
  ensure(s->kb1, k * sizeof(uint64_t));
  ensure(s->fz_v0, k * sizeof(uint32_t));
  ensure(s->fz_v1, k * sizeof(uint32_t));
  ensure(s->fz_byte, k);
  hipLaunchKernelGGL((k_fill<uint8_t>), dim3(grid_for(k, 256, 4096)), dim3(256), 0, st, s->fz_byte.as<uint8_t>(), k,
                     (uint8_t)0);  // the first pass's values are the positions
  const uint32_t nblk = (uint32_t)((k + kSortTile - 1) / kSortTile);
  ensure(s->cnt, ((uint64_t)nblk * 256 + 1) * sizeof(uint32_t));
  ensure(s->koff, ((uint64_t)nblk * 256 + 1) * sizeof(uint32_t));
  const uint64_t* kin = src;
  const uint32_t* vin = nullptr;
  for (int p = 0; p < passes; p++) {
    uint64_t* kout = (p & 1) ? s->kb1.as<uint64_t>() : s->kb0.as<uint64_t>();
    uint32_t* vout = (p & 1) ? s->fz_v1.as<uint32_t>() : s->fz_v0.as<uint32_t>();
    hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, st, kin, (uint32_t)k, 8 * p,
                       s->cnt.as<uint32_t>());
    HIPCHK(hipGetLastError());
    scan<uint32_t>(s, s->koff.as<uint32_t>(), (uint64_t)nblk * 256, st, LoadFn<uint32_t>{s->cnt.as<uint32_t>()});
    hipLaunchKernelGGL(k_radix_scatter_kv, dim3(nblk), dim3(kSortThreads), 0, st, kin, kout, (uint32_t)k, 8 * p,
                       (const uint32_t*)s->koff.as<uint32_t>(), vin, (const uint8_t*)s->fz_byte.as<uint8_t>(), vout);
    HIPCHK(hipGetLastError());
    kin = kout;
    vin = vout;
  }
  ensure(s->segpos, (k + 1) * sizeof(uint32_t));
  ensure(s->kdedup, k * sizeof(uint64_t));
  ensure(s->kvdedup, k * sizeof(uint64_t));
  scan<uint32_t>(s, s->segpos.as<uint32_t>(), k, st, FirstFlag{kin});
  hipLaunchKernelGGL(k_kv_compact, dim3(grid_for(k, 256)), dim3(256), 0, st, kin, vin, k,
                     (const uint32_t*)s->segpos.as<uint32_t>(), vsrc, s->kdedup.as<uint64_t>(),
                     s->kvdedup.as<uint64_t>(), &s->dctr->kprime);
  HIPCHK(hipGetLastError());
  phase_end(s, pm, st, (16ull * passes + 28) * k);
  return s->kdedup.as<uint64_t>();
}

size_t heavy_smem(uint32_t S, uint32_t cap) { return HeavyLayout(S, cap).total; }

// ---------------------------------------------------------------------------
// Redistribution of a set of windows (level, index) in place.  Returns false if
// some window had to escalate past the root (caller resizes).
// ---------------------------------------------------------------------------
struct Win {
  int h;
  uint64_t i;
};

void normalize(std::vector<Win>& w) {
  std::sort(w.begin(), w.end(), [](const Win& a, const Win& b) {
    uint64_t fa = a.i << a.h, fb = b.i << b.h;
    if (fa != fb) return fa < fb;
    return a.h > b.h;
  });
  std::vector<Win> out;
  uint64_t cover_end = 0;
  bool have = false;
  for (const Win& x : w) {
    uint64_t f = x.i << x.h, e = (x.i + 1) << x.h;
    if (have && f < cover_end) continue;  // nested in the previous kept window
    out.push_back(x);
    cover_end = e;
    have = true;
  }
  w.swap(out);
}

// Uploads the window description; returns device WinArgs.
WinArgs upload_windows(cpma* s, const std::vector<uint64_t>& src_begin, const std::vector<uint64_t>& src_n,
                       const std::vector<uint64_t>& dst_begin, const std::vector<uint64_t>& dst_n,
                       const std::vector<uint32_t>& level, hipStream_t st, uint64_t& nsrc, uint64_t& ndst) {
  const uint32_t W = (uint32_t)src_begin.size();
  const size_t n64 = 6ull * (W + 1);
  const size_t bytes = n64 * 8 + (W + 1) * 4ull;
  uint64_t* h = reinterpret_cast<uint64_t*>(host_pin(s, bytes));
  uint64_t* sb = h;
  uint64_t* sf = sb + (W + 1);
  uint64_t* db = sf + (W + 1);
  uint64_t* dn = db + (W + 1);
  uint64_t* df = dn + (W + 1);
  uint32_t* lv = reinterpret_cast<uint32_t*>(df + (W + 1) + (W + 1));
  nsrc = ndst = 0;
  for (uint32_t w = 0; w < W; w++) {
    sb[w] = src_begin[w];
    sf[w] = nsrc;
    nsrc += src_n[w];
    db[w] = dst_begin[w];
    dn[w] = dst_n[w];
    df[w] = ndst;
    ndst += dst_n[w];
    lv[w] = level[w];
  }
  sb[W] = 0;
  sf[W] = nsrc;
  db[W] = 0;
  dn[W] = 0;
  df[W] = ndst;
  lv[W] = 0;
  ensure(s->wargs, bytes);
  HIPCHK(hipMemcpyAsync(s->wargs.p, h, bytes, hipMemcpyHostToDevice, st));
  uint64_t* d = s->wargs.as<uint64_t>();
  WinArgs wa;
  wa.W = W;
  wa.src_begin = d;
  wa.src_flat = d + (W + 1);
  wa.dst_begin = d + 2 * (W + 1);
  wa.dst_n = d + 3 * (W + 1);
  wa.dst_flat = d + 4 * (W + 1);
  wa.level = reinterpret_cast<const uint32_t*>(d + 6 * (W + 1));
  wa.raw = s->cfg.uncompressed ? 1u : 0u;
  wa.vbytes = s->kv() ? 8u : 0u;
  return wa;
}

SrcLeaves src_leaves(cpma* s) {
  SrcLeaves sl;
  sl.bytes = s->bytes.as<uint8_t>();
  sl.used = s->used.as<uint32_t>();
  sl.ovf = s->ovf.as<uint64_t>();
  sl.arena = s->arena.as<uint8_t>();
  sl.S = s->S;
  sl.clen = s->clen.as<uint32_t>();
  return sl;
}

// Pack (copy 1): decode the source leaves of every window into the staging
// buffer.  Returns the number of staged keys K.
uint64_t pack_windows(cpma* s, const WinArgs& wa, uint64_t nsrc, hipStream_t st) {
  ensure(s->cnt, nsrc * sizeof(uint64_t));
  ensure(s->koff, (nsrc + 1) * sizeof(uint64_t));
  const SrcLeaves sl = src_leaves(s);
  hipLaunchKernelGGL(k_win_count, dim3(grid_for(nsrc, 1, 1u << 20)), dim3(kWave), 0, st, wa, sl, nsrc,
                     s->cnt.as<uint64_t>());
  HIPCHK(hipGetLastError());
  scan<uint64_t>(s, s->koff.as<uint64_t>(), nsrc, st, LoadFn<uint64_t>{s->cnt.as<uint64_t>()});
  uint64_t K = 0;
  HIPCHK(hipMemcpyAsync(&s->hctr->root_sum, s->koff.as<uint64_t>() + nsrc, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  K = s->hctr->root_sum;
  ensure(s->stage, std::max<uint64_t>(K, 1) * sizeof(uint64_t));
  ensure(s->win_id, std::max<uint64_t>(K, 1) * sizeof(uint32_t));
  ensure(s->ccost, std::max<uint64_t>(K, 1));
  if (s->kv()) ensure(s->vstage, std::max<uint64_t>(K, 1) * sizeof(uint64_t));
  hipLaunchKernelGGL(k_win_pack, dim3(grid_for(nsrc, 1, 1u << 20)), dim3(kWave), 0, st, wa, sl, nsrc,
                     (const uint64_t*)s->koff.as<uint64_t>(), s->stage.as<uint64_t>(), s->win_id.as<uint32_t>(),
                     s->ccost.as<uint8_t>(), s->kv() ? s->vstage.as<uint64_t>() : (uint64_t*)nullptr);
  HIPCHK(hipGetLastError());
  return K;
}

// Plans the even spread of the staged keys into the destination leaves and checks
// it.  Returns per-window failure bits in `fails`.
// nsrc > 0: the staged keys come from pack_windows (fix the heads' chain costs);
// nsrc == 0: the caller prepared the chain costs.
void plan_spread(cpma* s, const WinArgs& wa, uint64_t nsrc, uint64_t K, uint64_t ndst, const Bounds& dstb,
                 uint32_t* plan_used, uint64_t Ldst, bool fresh, hipStream_t st, std::vector<uint32_t>& fails) {
  const uint32_t W = wa.W;
  ensure(s->welem, (W + 1) * sizeof(uint64_t));
  ensure(s->fail, std::max<uint32_t>(W, 1) * sizeof(uint32_t));
  ensure(s->P, (K + 1) * sizeof(uint64_t));
  ensure(s->ncost, std::max<uint64_t>(K, 1));
  ensure(s->lstart, (ndst + 1) * sizeof(uint64_t));
  ensure(s->planU, (ndst + 1) * sizeof(uint32_t));
  hipLaunchKernelGGL(k_win_elems, dim3(grid_for(W + 1, 256)), dim3(256), 0, st, wa,
                     (const uint64_t*)s->koff.as<uint64_t>(), s->welem.as<uint64_t>(), s->fail.as<uint32_t>());
  HIPCHK(hipGetLastError());
  if (nsrc > 0 && !s->cfg.uncompressed)
    hipLaunchKernelGGL(k_head_costs, dim3(grid_for(nsrc, 256, 1u << 16)), dim3(256), 0, st, wa, nsrc,
                       (const uint64_t*)s->koff.as<uint64_t>(), (const uint64_t*)s->welem.as<uint64_t>(),
                       (const uint64_t*)s->stage.as<uint64_t>(), s->ccost.as<uint8_t>());
  scan<uint64_t>(s, s->P.as<uint64_t>(), K, st, U8Fn{s->ccost.as<uint8_t>()});
  hipLaunchKernelGGL((k_fill<uint64_t>), dim3(grid_for(ndst + 1, 256, 4096)), dim3(256), 0, st,
                     s->lstart.as<uint64_t>(), ndst + 1, ~0ull);
  hipLaunchKernelGGL(k_assign, dim3(grid_for(K, 256, 1u << 16)), dim3(256), 0, st, wa, K,
                     (const uint8_t*)s->ccost.as<uint8_t>(), (const uint32_t*)s->win_id.as<uint32_t>(),
                     (const uint64_t*)s->welem.as<uint64_t>(), (const uint64_t*)s->P.as<uint64_t>(),
                     s->ncost.as<uint8_t>(), s->lstart.as<uint64_t>(), s->fail.as<uint32_t>());
  HIPCHK(hipGetLastError());
  int32_t* wol = fresh ? nullptr : s->win_of_leaf.as<int32_t>();
  hipLaunchKernelGGL(k_leaf_bytes, dim3(grid_for(ndst, 1, 1u << 20)), dim3(kWave), 0, st, wa, dstb, ndst,
                     (const uint64_t*)s->welem.as<uint64_t>(), (const uint64_t*)s->lstart.as<uint64_t>(),
                     (const uint8_t*)s->ncost.as<uint8_t>(), s->planU.as<uint32_t>(), plan_used, wol,
                     s->fail.as<uint32_t>());
  HIPCHK(hipGetLastError());
  Pyramid P = make_pyramid(s, Ldst);
  build_pyramid(s, P, plan_used, Ldst, st);
  const uint64_t nodes = (P.H == 0) ? 1 : P.off[P.H] + P.cnt[P.H];
  hipLaunchKernelGGL(k_check_plan, dim3(grid_for(nodes, 256, 1u << 16)), dim3(256), 0, st, dstb, P,
                     (const uint32_t*)plan_used, (const int32_t*)wol, wa.level, fresh ? 1 : 0,
                     s->fail.as<uint32_t>());
  HIPCHK(hipGetLastError());
  if (!fresh)
    hipLaunchKernelGGL(k_clear_win_map, dim3(grid_for(ndst, 256, 1u << 16)), dim3(256), 0, st, wa, ndst,
                       s->win_of_leaf.as<int32_t>());
  HIPCHK(hipGetLastError());
  fails.resize(W);
  uint32_t* hf = reinterpret_cast<uint32_t*>(host_pin(s, W * 4ull + 16));
  HIPCHK(hipMemcpyAsync(hf, s->fail.p, W * 4ull, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::copy(hf, hf + W, fails.begin());
}

void encode_spread(cpma* s, const WinArgs& wa, uint64_t ndst, uint8_t* dbytes, uint32_t* dused, uint64_t* dhead,
                   hipStream_t st, uint32_t* dclen = nullptr) {
  hipLaunchKernelGGL(k_leaf_encode, dim3(grid_for(ndst, 1, 1u << 20)), dim3(kWave), s->S, st, wa, ndst, s->S,
                     (const uint64_t*)s->welem.as<uint64_t>(), (const uint64_t*)s->lstart.as<uint64_t>(),
                     (const uint64_t*)s->stage.as<uint64_t>(), (const uint32_t*)s->planU.as<uint32_t>(), dbytes,
                     dused, dhead, s->kv() ? (const uint64_t*)s->vstage.as<uint64_t>() : (const uint64_t*)nullptr,
                     dclen);
  HIPCHK(hipGetLastError());
}

void ensure_win_map(cpma* s) {
  if (s->wol_L >= s->L && s->win_of_leaf.cap >= s->L * 4) return;
  ensure(s->win_of_leaf, s->L * sizeof(int32_t));
  hipLaunchKernelGGL((k_fill<int32_t>), dim3(grid_for(s->win_of_leaf.cap / 4, 256, 4096)), dim3(256), 0, 0,
                     s->win_of_leaf.as<int32_t>(), (uint64_t)(s->win_of_leaf.cap / 4), -1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipDeviceSynchronize());
  s->wol_L = s->win_of_leaf.cap / 4;
}

// Returns true when done, false when a window escalated past the root.
bool redistribute(cpma* s, std::vector<Win> wins, hipStream_t st, uint64_t* moved) {
  const int H = tree_height(s->L);
  ensure_win_map(s);
  for (int attempt = 0; attempt < 4 * (H + 2); attempt++) {
    normalize(wins);
    std::vector<uint64_t> sb, sn;
    std::vector<uint32_t> lv;
    for (const Win& w : wins) {
      uint64_t f = w.i << w.h;
      uint64_t e = std::min<uint64_t>(s->L, (w.i + 1) << w.h);
      sb.push_back(f);
      sn.push_back(e - f);
      lv.push_back((uint32_t)w.h);
    }
    uint64_t nsrc, ndst;
    WinArgs wa = upload_windows(s, sb, sn, sb, sn, lv, st, nsrc, ndst);
    const uint64_t K = pack_windows(s, wa, nsrc, st);
    ensure(s->plan_used, s->L * sizeof(uint32_t));
    HIPCHK(hipMemcpyAsync(s->plan_used.p, s->used.p, s->L * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    std::vector<uint32_t> fails;
    plan_spread(s, wa, nsrc, K, ndst, s->bounds(s->L), s->plan_used.as<uint32_t>(), s->L, false, st, fails);
    bool any = false;
    for (uint32_t f : fails) any |= (f != 0);
    if (!any) {
      encode_spread(s, wa, ndst, s->bytes.as<uint8_t>(), s->used.as<uint32_t>(), s->head.as<uint64_t>(), st,
                    s->kv() ? s->clen.as<uint32_t>() : nullptr);
      // algorithmic bytes: every window leaf read (at most S) and rewritten
      // whole with its used count and head
      *moved = ndst * (2ull * s->S + 12);
      return true;
    }
    for (size_t w = 0; w < wins.size(); w++) {
      if (!fails[w]) continue;
      wins[w].h += 1;
      wins[w].i >>= 1;
      if (wins[w].h > H) return false;
    }
  }
  throw Fail{CPMA_ERR_DEVICE};
}

// The spare leaf arrays become the structure (the old ones become the spares,
// so repeated resizes reuse memory instead of freeing and allocating it).
void swap_in_spare(cpma* s, uint64_t Lt) {
  std::swap(s->bytes, s->spare_bytes);
  std::swap(s->used, s->spare_used);
  std::swap(s->head, s->spare_head);
  if (s->kv()) std::swap(s->clen, s->spare_clen);
  s->L = Lt;
}

// Spreads the K staged keys (sorted, one window) evenly over a fresh array of Lt
// leaves; adjusts Lt by the growing factor until every node is within bounds,
// then replaces the structure.  costs_ready: s->ccost already holds the chain
// costs of the staged keys.
void spread_fresh(cpma* s, uint64_t K, uint64_t Lt, hipStream_t st, bool costs_ready = false) {
  if (K == 0) {
    ensure(s->spare_bytes, s->S);
    ensure(s->spare_used, 4);
    ensure(s->spare_head, 8);
    if (s->kv()) {
      ensure(s->spare_clen, 4);
      hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, s->spare_clen.as<uint32_t>(), (uint64_t)1, 0u);
    }
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(256), 0, st, s->spare_bytes.as<uint32_t>(),
                       (uint64_t)(s->S / 4), 0u);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, s->spare_used.as<uint32_t>(), (uint64_t)1, 0u);
    hipLaunchKernelGGL((k_fill<uint64_t>), dim3(1), dim3(64), 0, st, s->spare_head.as<uint64_t>(), (uint64_t)1,
                       kNoKey);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    swap_in_spare(s, 1);
    return;
  }
  const double g = s->cfg.grow;
  ensure(s->win_id, K * sizeof(uint32_t));
  hipLaunchKernelGGL((k_fill<uint32_t>), dim3(grid_for(K, 256, 4096)), dim3(256), 0, st, s->win_id.as<uint32_t>(),
                     K, 0u);
  if (!costs_ready) {
    ensure(s->ccost, K);
    if (s->cfg.uncompressed)
      hipLaunchKernelGGL((k_fill<uint8_t>), dim3(grid_for(K, 256, 4096)), dim3(256), 0, st, s->ccost.as<uint8_t>(), K,
                         (uint8_t)8);
    else
      hipLaunchKernelGGL(k_chain_costs, dim3(grid_for(K, 256, 1u << 16)), dim3(256), 0, st,
                         (const uint64_t*)s->stage.as<uint64_t>(), K, s->ccost.as<uint8_t>(), s->kv() ? 8u : 0u);
    HIPCHK(hipGetLastError());
  }
  // One window over all staged keys: its source is one flat entry, so the
  // window's key range comes from koff = {0, K}.
  ensure(s->koff, 2 * sizeof(uint64_t));
  uint64_t* hk = reinterpret_cast<uint64_t*>(host_pin(s, 16));
  hk[0] = 0;
  hk[1] = K;
  HIPCHK(hipMemcpyAsync(s->koff.p, hk, 16, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  int last_dir = 0;
  for (int attempt = 0; attempt < 64; attempt++) {
    uint64_t nsrc, ndst;
    std::vector<uint64_t> sb{0}, sn{1}, db{0}, dn{Lt};
    std::vector<uint32_t> lv{(uint32_t)(tree_height(Lt) + 1)};
    WinArgs wa = upload_windows(s, sb, sn, db, dn, lv, st, nsrc, ndst);
    ensure(s->spare_used, Lt * sizeof(uint32_t));
    std::vector<uint32_t> fails;
    plan_spread(s, wa, 0, K, ndst, s->bounds(Lt), s->spare_used.as<uint32_t>(), Lt, true, st, fails);
    if (fails[0] == 0) {
      ensure(s->spare_bytes, Lt * (uint64_t)s->S);
      ensure(s->spare_head, Lt * sizeof(uint64_t));
      if (s->kv()) ensure(s->spare_clen, Lt * sizeof(uint32_t));
      encode_spread(s, wa, ndst, s->spare_bytes.as<uint8_t>(), s->spare_used.as<uint32_t>(),
                    s->spare_head.as<uint64_t>(), st, s->kv() ? s->spare_clen.as<uint32_t>() : nullptr);
      HIPCHK(hipStreamSynchronize(st));
      swap_in_spare(s, Lt);
      return;
    }
    int dir = (fails[0] & 1u) ? +1 : -1;
    if (dir == -1 && Lt == 1) throw Fail{CPMA_ERR_DEVICE};
    if (last_dir != 0 && dir != last_dir) {
      // Bounds pull both ways: settle on the larger layout's neighbour.
      Lt = Lt + 1;
    } else if (dir > 0) {
      Lt = std::max<uint64_t>(Lt + 1, (uint64_t)std::ceil(g * (double)Lt));
    } else {
      Lt = std::max<uint64_t>(1, (uint64_t)std::floor((double)Lt / g));
    }
    last_dir = dir;
  }
  throw Fail{CPMA_ERR_DEVICE};
}

// Grows or shrinks to Lt leaves (Lt then moves by the growing factor until every
// node of the new tree is within its bounds) by a direct split of the old leaf
// images into the spare arrays.  Returns the algorithmic bytes moved.
// total_used: sum of the old used bytes (bounds the chain total from above).
// Returns false, with nothing changed, when thresholds would overflow 64 bits.
// Uncompressed and key-value leaves: a resize stages every key (and value;
// one window over all leaves)
// and spreads them over a fresh array of about Lt leaves, which steps by the
// growing factor until every node is within its bounds.  Returns the
// algorithmic bytes moved through *moved.
bool raw_resize(cpma* s, uint64_t Lt, hipStream_t st, uint64_t* moved) {
  uint64_t nsrc = 0, ndst = 0;
  std::vector<uint64_t> sb{0}, sn{s->L};
  std::vector<uint32_t> lv{(uint32_t)tree_height(s->L)};
  WinArgs wa = upload_windows(s, sb, sn, sb, sn, lv, st, nsrc, ndst);
  const uint64_t K = pack_windows(s, wa, nsrc, st);
  const uint64_t L0 = s->L;
  if (s->kv() && K > 0) {
    // the staged keys form one chain: every source leaf's head but the first
    // costs its delta's code, not a head's 8 bytes
    hipLaunchKernelGGL(k_chain_costs, dim3(grid_for(K, 256, 1u << 16)), dim3(256), 0, st,
                       (const uint64_t*)s->stage.as<uint64_t>(), K, s->ccost.as<uint8_t>(), 8u);
    HIPCHK(hipGetLastError());
  }
  spread_fresh(s, K, std::max<uint64_t>(Lt, 1), st, true);
  *moved = 16ull * K + 12ull * (L0 + s->L);
  return true;
}

bool split_resize(cpma* s, uint64_t Lt, uint64_t total_used, hipStream_t st, uint64_t* moved) {
  if (s->cfg.uncompressed || s->kv()) return raw_resize(s, Lt, st, moved);
  const uint64_t L = s->L;
  // a head's chain cost can exceed its 8 bytes by 2 (64-bit distances)
  auto fits = [&](uint64_t lt) { return (__int128)(total_used + 2 * L + 16) * (lt + 1) < ((__int128)1 << 62); };
  if (!fits(Lt)) return false;
  ensure(s->lastk, L * sizeof(uint64_t));
  ensure(s->lckpt, L * 3 * sizeof(LeafCkpt));
  ensure(s->ne_rank, (L + 1) * sizeof(uint32_t));
  ensure(s->ne_list, (L + 1) * sizeof(uint32_t));
  ensure(s->chain_pfx, (L + 1) * sizeof(uint64_t));
  const SrcLeaves sl = src_leaves(s);
  hipLaunchKernelGGL(k_leaf_last, dim3(grid_for(4 * L, 256, 1u << 16)), dim3(256), 0, st, sl,
                     (const uint64_t*)s->head.as<uint64_t>(), L, s->lastk.as<uint64_t>(), s->lckpt.as<LeafCkpt>());
  HIPCHK(hipGetLastError());
  scan<uint32_t>(s, s->ne_rank.as<uint32_t>(), L, st, NonEmptyFn{sl.used});
  hipLaunchKernelGGL(k_ne_compact, dim3(grid_for(L + 1, 256, 1u << 16)), dim3(256), 0, st, sl.used,
                     (const uint32_t*)s->ne_rank.as<uint32_t>(), L, s->ne_list.as<uint32_t>());
  HIPCHK(hipGetLastError());
  SplitArgs a;
  a.src = sl;
  a.head = s->head.as<uint64_t>();
  a.lastk = s->lastk.as<uint64_t>();
  a.ck = s->lckpt.as<LeafCkpt>();
  a.rank = s->ne_rank.as<uint32_t>();
  a.ne = s->ne_list.as<uint32_t>();
  a.CP = s->chain_pfx.as<uint64_t>();
  a.L = L;
  scan<uint64_t>(s, s->chain_pfx.as<uint64_t>(), L, st, ChainFn{sl.used, a.head, a.lastk, a.rank, a.ne});
  ensure(s->srcinfo, std::max<uint64_t>(L, 1) * sizeof(SrcInfo));
  hipLaunchKernelGGL(k_src_info, dim3(grid_for(L, 256, 1u << 16)), dim3(256), 0, st, sl, a.head, a.lastk,
                     a.rank, a.ne, L, s->srcinfo.as<SrcInfo>());
  HIPCHK(hipGetLastError());
  a.info = s->srcinfo.as<SrcInfo>();
  const double g = s->cfg.grow;
  int last_dir = 0;
  for (int attempt = 0; attempt < 64; attempt++) {
    if (!fits(Lt)) throw Fail{CPMA_ERR_DEVICE};
    a.Lt = Lt;
    ensure(s->srec, (Lt + 1) * sizeof(SplitRec));
    ensure(s->spare_used, Lt * sizeof(uint32_t), std::max(0.25, s->cfg.grow * s->cfg.grow - 1.0 + 0.05));
    ensure(s->fail, 16);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, s->fail.as<uint32_t>(), (uint64_t)1, 0u);
    hipLaunchKernelGGL(k_split_locate, dim3(grid_for(L, 256, 1u << 16)), dim3(256), 0, st, a,
                       s->srec.as<SplitRec>());
    HIPCHK(hipGetLastError());
    const Bounds db = s->bounds(Lt);
    hipLaunchKernelGGL(k_split_plan, dim3(grid_for(Lt, 256, 1u << 16)), dim3(256), 0, st, db, Lt,
                       (const SplitRec*)s->srec.as<SplitRec>(), s->spare_used.as<uint32_t>(),
                       s->fail.as<uint32_t>());
    HIPCHK(hipGetLastError());
    Pyramid P = make_pyramid(s, Lt);
    build_pyramid(s, P, s->spare_used.as<uint32_t>(), Lt, st);
    const uint64_t nodes = (P.H == 0) ? 1 : P.off[P.H] + P.cnt[P.H];
    hipLaunchKernelGGL(k_check_plan, dim3(grid_for(nodes, 256, 1u << 16)), dim3(256), 0, st, db, P,
                       (const uint32_t*)s->spare_used.as<uint32_t>(), (const int32_t*)nullptr,
                       (const uint32_t*)nullptr, 1, s->fail.as<uint32_t>());
    HIPCHK(hipGetLastError());
    // the write is queued behind the check and does nothing if the check
    // failed, so one read-back serves both
    const double room = std::max(0.25, s->cfg.grow * s->cfg.grow - 1.0 + 0.05);
    ensure(s->spare_bytes, Lt * (uint64_t)s->S, room);
    ensure(s->spare_head, Lt * sizeof(uint64_t), room);
    zero_counters(s, st);
    auto wr = s->S <= 1024 ? k_split_write<1> : k_split_write<4>;
    hipLaunchKernelGGL(wr, dim3(grid_for(Lt, kWave, 1u << 16)), dim3(kWave), 0, st, a, s->S,
                       (const SplitRec*)s->srec.as<SplitRec>(), s->spare_bytes.as<uint8_t>(),
                       s->spare_used.as<uint32_t>(), s->spare_head.as<uint64_t>(), s->dctr,
                       (const uint32_t*)s->fail.as<uint32_t>());
    HIPCHK(hipGetLastError());
    uint32_t* hf = reinterpret_cast<uint32_t*>(host_pin(s, 16));
    HIPCHK(hipMemcpyAsync(hf, s->fail.p, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(s->hctr, s->dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    resolve_phases(s);
    const uint32_t fail = hf[0];
    if (fail == 0) {
      if (s->hctr->error) throw Fail{CPMA_ERR_DEVICE};
      swap_in_spare(s, Lt);
      *moved = Lt * ((uint64_t)s->S + 12);
      return true;
    }
    const int dir = (fail & 1u) ? +1 : -1;
    if (dir == -1 && Lt == 1) throw Fail{CPMA_ERR_DEVICE};
    if (last_dir != 0 && dir != last_dir) {
      Lt = Lt + 1;  // bounds pull both ways: settle on the larger layout's neighbour
    } else if (dir > 0) {
      Lt = std::max<uint64_t>(Lt + 1, (uint64_t)std::ceil(g * (double)Lt));
    } else {
      Lt = std::max<uint64_t>(1, (uint64_t)std::floor((double)Lt / g));
    }
    last_dir = dir;
  }
  throw Fail{CPMA_ERR_DEVICE};
}

// Device memory for the next growth steps, taken when a set is built: the
// resize's scratch arrays for three growing factors ahead, and the spare leaf
// arrays (which trade places with the live ones at every resize) for the next
// growth with the same room a resize leaves.  A resize then allocates nothing
// until the set has grown well past its built size; each allocation
// synchronises the device and takes tens to hundreds of microseconds.
void reserve_growth(cpma* s) {
  const double g = s->cfg.grow;
  const uint64_t L = s->L;
  const uint64_t Lr = (uint64_t)std::ceil((double)L * g * g * g) + 1;
  ensure(s->lastk, Lr * sizeof(uint64_t));
  ensure(s->lckpt, Lr * 3 * sizeof(LeafCkpt));
  ensure(s->ne_rank, (Lr + 1) * sizeof(uint32_t));
  ensure(s->ne_list, (Lr + 1) * sizeof(uint32_t));
  ensure(s->chain_pfx, (Lr + 1) * sizeof(uint64_t));
  ensure(s->srcinfo, Lr * sizeof(SrcInfo));
  ensure(s->srec, (Lr + 1) * sizeof(SplitRec));
  ensure(s->fail, 16);
  make_pyramid(s, Lr);
  const uint64_t Ln = (uint64_t)std::ceil((double)L * g) + 1;
  const double room = std::max(0.25, g * g - 1.0 + 0.05);
  ensure(s->spare_used, Ln * sizeof(uint32_t), room);
  ensure(s->spare_head, Ln * sizeof(uint64_t), room);
  ensure(s->spare_bytes, Ln * (uint64_t)s->S, room);
  if (s->kv()) ensure(s->spare_clen, Ln * sizeof(uint32_t), room);
}

// Pyramid memory for Lx leaves; contents survive unless the buffer has to grow.
void reserve_pyramid(cpma* s, uint64_t Lx) {
  const Pyramid P = pyramid_layout(Lx);
  const uint64_t nodes = P.H == 0 ? 0 : P.off[P.H] + P.cnt[P.H];
  const size_t need = (nodes + 1) * sizeof(uint64_t);
  if (s->pyr.cap < need) {
    s->pyr_valid = false;
    ensure(s->pyr, need);
  }
}

// Everything the density count, a resize and the redistribution fallback can
// need once a batch of k keys has been merged into the leaves.  Before the
// batch the root is within its upper bound (bytes <= tau_H * L * S), and a new
// key adds at most 10 code bytes (bytes(x - a) + bytes(b - x) - bytes(b - a)
// <= bytes(b - x)), so after the merge the structure fits in the leaves that
// the growth steps reach once tau_H * L * S + 10 k bytes, and 8 per leaf,
// are under the root bound; one step more covers a fresh layout that fails a
// bound and steps again.  A shrink needs no more than L leaves.
void reserve_after_merge(cpma* s, uint64_t k, bool insert) {
  const double g = s->cfg.grow;
  const uint64_t L = s->L;
  const __int128 total = (__int128)s->q_up_root * L * s->S / kQ + 1 + (insert ? 10 * (__int128)k : 0);
  uint64_t Lmax = L;
  while ((total + 8 * (__int128)Lmax) * kQ > (__int128)s->q_up_root * Lmax * s->S)
    Lmax = std::max<uint64_t>(Lmax + 1, (uint64_t)std::ceil(g * (double)Lmax));
  Lmax = std::max<uint64_t>(Lmax + 1, (uint64_t)std::ceil(g * (double)Lmax));
  // a rebuild lays the keys out at build density, one step more if that fails
  const uint64_t Lb = (uint64_t)std::ceil((double)total / (s->cfg.build_density * (double)s->S)) + 1;
  Lmax = std::max<uint64_t>(Lmax, std::max<uint64_t>(Lb + 1, (uint64_t)std::ceil(g * (double)Lb)));
  const double room = std::max(0.25, g * g - 1.0 + 0.05);
  // resize: tables over the source leaves, split records and spare arrays of
  // the destination (the same room split_resize asks for)
  ensure(s->lastk, std::max<uint64_t>(L, 1) * sizeof(uint64_t));
  ensure(s->lckpt, std::max<uint64_t>(L, 1) * 3 * sizeof(LeafCkpt));
  ensure(s->ne_rank, (L + 1) * sizeof(uint32_t));
  ensure(s->ne_list, (L + 1) * sizeof(uint32_t));
  ensure(s->chain_pfx, (L + 1) * sizeof(uint64_t));
  ensure(s->srcinfo, std::max<uint64_t>(L, 1) * sizeof(SrcInfo));
  ensure(s->srec, (Lmax + 1) * sizeof(SplitRec));
  ensure(s->fail, 16);
  ensure(s->spare_used, Lmax * sizeof(uint32_t), room);
  ensure(s->spare_head, Lmax * sizeof(uint64_t), room);
  ensure(s->spare_bytes, Lmax * (uint64_t)s->S, room);
  // counting: the pyramid and the window list; prefix sums over leaves
  reserve_pyramid(s, Lmax);
  ensure(s->win, Lmax * sizeof(uint64_t));
  ensure(s->scan_tmp, scan_scratch_elems(Lmax + 1) * sizeof(uint64_t));
  if (s->cfg.uncompressed || s->kv()) {
    // an uncompressed or key-value resize stages every key and spreads it afresh
    const uint64_t K = std::max<uint64_t>(1, s->n + (insert ? k : 0));
    if (s->kv()) {
      ensure(s->vstage, K * sizeof(uint64_t));
      ensure(s->spare_clen, Lmax * sizeof(uint32_t), room);
    }
    ensure(s->cnt, std::max<uint64_t>(L, 1) * sizeof(uint64_t));
    ensure(s->koff, (L + 1) * sizeof(uint64_t));
    ensure(s->stage, K * sizeof(uint64_t));
    ensure(s->win_id, K * sizeof(uint32_t));
    ensure(s->ccost, K);
    ensure(s->P, (K + 1) * sizeof(uint64_t));
    ensure(s->ncost, K);
    ensure(s->lstart, (Lmax + 1) * sizeof(uint64_t));
    ensure(s->planU, (Lmax + 1) * sizeof(uint32_t));
    ensure(s->welem, 2 * sizeof(uint64_t));
    ensure(s->scan_tmp, scan_scratch_elems(std::max<uint64_t>(K, Lmax) + 1) * sizeof(uint64_t));
  }
}

// Root out of bounds: move everything to an array grown (or shrunk) by the
// growing factor, spread evenly (Section "Packed Memory Array", "Resizing a
// PMA").  Returns the algorithmic bytes moved (old used bytes read, new array
// written).
uint64_t resize(cpma* s, uint64_t total, uint32_t viol, hipStream_t st) {
  const double g = s->cfg.grow;
  const int64_t Q = kQ;
  uint64_t Lt = s->L;
  if (viol & 1u) {
    do {
      Lt = std::max<uint64_t>(Lt + 1, (uint64_t)std::ceil(g * (double)Lt));
    } while ((__int128)(total + 8 * Lt) * Q > (__int128)s->q_up_root * Lt * s->S);
  } else {
    while (Lt > 1 && (__int128)total * Q < (__int128)s->q_lo_root * Lt * s->S)
      Lt = std::max<uint64_t>(1, (uint64_t)std::floor((double)Lt / g));
  }
  if (s->n == 0) {
    spread_fresh(s, 0, 1, st);
    return 0;
  }
  uint64_t moved = 0;
  if (split_resize(s, Lt, total, st, &moved)) return total + moved;
  // staged fallback for structures whose split thresholds exceed 64 bits
  uint64_t nsrc, ndst;
  std::vector<uint64_t> sb{0}, sn{s->L};
  std::vector<uint32_t> lv{(uint32_t)(tree_height(s->L) + 1)};
  WinArgs wa = upload_windows(s, sb, sn, sb, sn, lv, st, nsrc, ndst);
  const uint64_t K = pack_windows(s, wa, nsrc, st);
  if (K != s->n) throw Fail{CPMA_ERR_DEVICE};
  spread_fresh(s, K, Lt, st);
  return total + Lt * ((uint64_t)s->S + 12);
}

// The merge's totals from the counters read back after it: the keys it added
// or removed, and its algorithmic bytes for the statistics.
uint64_t take_merge(cpma* s, const Counters& c, int merged) {
  if (c.reserved) throw Fail{CPMA_ERR_RESERVED_KEY};  // small batch: nothing was merged
  if (s->stats_on) {
    if ((s->stats_mask >> CPMA_PHASE_MERGE) & 1u) s->stats[CPMA_PHASE_MERGE].alg_bytes += c.alg_bytes;
    if ((s->stats_mask >> CPMA_PHASE_HEAVY) & 1u) s->stats[CPMA_PHASE_HEAVY].alg_bytes += c.alg_bytes_h;
  }
  if (merged)
    s->n += c.delta;
  else
    s->n -= c.delta;
  return c.delta;
}

// Counting + redistribution until every node of the implicit tree is within its
// bounds.
// merged: -1 after a build; 0 / 1 right after a delete / insert merge, whose
// counters are still on the device: the first count only reads the structure,
// so one read-back serves both (the merge's errors are checked before anything
// is redistributed).  Returns the merge's delta.
// small_k: the keys of a small batch (0: not one).
uint64_t rebalance(cpma* s, hipStream_t st, int merged = -1, uint64_t small_k = 0) {
  uint64_t delta = 0;
  bool taken = false;
  if (small_k && merged >= 0 && s->pyr_valid) {
    // every node was within bounds before this batch and the pyramid is
    // current: check only the paths of the touched leaves
    Pyramid P = pyramid_layout(s->L);
    P.base = s->pyr.as<uint64_t>();
    PhaseMark pc = phase_begin(s, CPMA_PHASE_COUNT, st);
    // (level, segment) pairs: at most min(k, L) segments on H + 1 levels
    const uint64_t pairs = std::min<uint64_t>(small_k, s->L) * (uint64_t)(P.H + 1);
    const bool fin = s->fin_parts != nullptr;  // one block: fold the merge and return the counters too
    const uint32_t pgrid = fin ? 1u : (uint32_t)std::min<uint64_t>((pairs + kPathThreads - 1) / kPathThreads, 128);
    hipLaunchKernelGGL(k_path_check, dim3(std::max(1u, pgrid)), dim3(kPathThreads), 0, st, s->bounds(s->L), P,
                       (const uint32_t*)s->used.as<uint32_t>(), (const uint32_t*)s->seg_leaf.as<uint32_t>(),
                       (const uint4*)s->seg_desc.as<uint4>(), s->dctr, s->fin_parts, s->fin_nn, s->fin_nw,
                       fin ? s->hctr : nullptr);
    s->fin_parts = nullptr;
    HIPCHK(hipGetLastError());
    phase_end(s, pc, st);
    if (fin) {
      HIPCHK(hipStreamSynchronize(st));
      resolve_phases(s);
      if (s->hctr->error) throw Fail{CPMA_ERR_DEVICE};
    } else {
      read_counters(s, st);
    }
    const Counters c = *s->hctr;
    delta = take_merge(s, c, merged);
    taken = true;
    if (!c.path_unsafe) return delta;  // the pyramid now holds the new sums
    s->pyr_valid = false;
  }
  for (int round = 0; round < 256; round++) {
    const bool after_merge = round == 0 && merged >= 0 && !taken;
    PhaseMark pc = phase_begin(s, CPMA_PHASE_COUNT, st);
    Pyramid P = make_pyramid(s, s->L);
    build_pyramid(s, P, s->used.as<uint32_t>(), s->L, st);
    ensure(s->win, std::max<uint64_t>(s->L, 1) * sizeof(uint64_t));
    // after a merge the counters are those cleared when the update began (its
    // window count is still zero) plus the merge's totals, which are kept
    if (!after_merge) zero_counters(s, st);
    const uint64_t nodes = (P.H == 0) ? 1 : P.off[P.H] + P.cnt[P.H];
    hipLaunchKernelGGL(k_select, dim3(grid_for(nodes, 256, 1u << 16)), dim3(256), 0, st, s->bounds(s->L), P,
                       (const uint32_t*)s->used.as<uint32_t>(), s->win.as<uint64_t>(), s->dctr);
    HIPCHK(hipGetLastError());
    phase_end(s, pc, st, 4ull * s->L + 16ull * nodes);
    read_counters(s, st);
    const Counters c = *s->hctr;
    if (after_merge) delta = take_merge(s, c, merged);
    if (c.root_viol) {
      PhaseMark pr = phase_begin(s, CPMA_PHASE_REDIST, st);
      const uint64_t moved = resize(s, c.root_sum, c.root_viol, st);
      phase_end(s, pr, st, moved);
      // a resize checks every node of the new tree (leaves at planning, the
      // rest on its pyramid) before it writes, so another count would find
      // nothing
      return delta;
    }
    if (c.nwin == 0) {
      s->pyr_valid = true;  // built this round from the current sizes, all within bounds
      return delta;
    }
    uint64_t* hw = reinterpret_cast<uint64_t*>(host_pin(s, c.nwin * 8ull));
    HIPCHK(hipMemcpyAsync(hw, s->win.p, c.nwin * 8ull, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<Win> wins(c.nwin);
    for (uint32_t w = 0; w < c.nwin; w++) wins[w] = Win{(int)(hw[w] >> 48), hw[w] & ((1ull << 48) - 1)};
    PhaseMark pr = phase_begin(s, CPMA_PHASE_REDIST, st);
    uint64_t moved = 0;
    bool done;
    try {
      done = redistribute(s, wins, st, &moved);
    } catch (const Fail& f) {
      if (f.st != CPMA_ERR_NOMEM) throw;
      // no memory for the windows' staging (it allocates before it writes):
      // spread the whole structure over its own leaf count instead, with the
      // memory reserved before the merge
      if (!split_resize(s, s->L, c.root_sum, st, &moved)) throw Fail{CPMA_ERR_DEVICE};
      phase_end(s, pr, st, moved);
      return delta;
    }
    phase_end(s, pr, st, moved);
    if (!done) {
      // Escalation past the root: grow if the structure is dense, else shrink.
      const uint64_t total = c.root_sum;
      const bool dense = (__int128)total * kQ * 2 >
                         (__int128)(s->q_up_root + s->q_lo_root) * s->L * s->S;
      resize(s, total, dense ? 1u : 2u, st);
    }
  }
  throw Fail{CPMA_ERR_DEVICE};
}

// Full rebuild after a batch of at least rebuild_frac * n keys has been merged
// into every leaf it touches: the whole structure is spread over a fresh array
// sized for the build density (Section "Parallel Batch Updates in a PMA":
// large batches rebuild the structure by merging the batch with all its
// elements).  One count reads the merge's totals and the byte total; the
// split writer then lays everything out with the same even byte split as a
// resize, checking every node of the new tree before it writes.  Returns the
// merge's delta.
uint64_t rebuild(cpma* s, hipStream_t st, int merged) {
  PhaseMark pc = phase_begin(s, CPMA_PHASE_COUNT, st);
  Pyramid P = make_pyramid(s, s->L);
  build_pyramid(s, P, s->used.as<uint32_t>(), s->L, st);
  ensure(s->win, std::max<uint64_t>(s->L, 1) * sizeof(uint64_t));
  const uint64_t nodes = (P.H == 0) ? 1 : P.off[P.H] + P.cnt[P.H];
  hipLaunchKernelGGL(k_select, dim3(grid_for(nodes, 256, 1u << 16)), dim3(256), 0, st, s->bounds(s->L), P,
                     (const uint32_t*)s->used.as<uint32_t>(), s->win.as<uint64_t>(), s->dctr);
  HIPCHK(hipGetLastError());
  phase_end(s, pc, st, 4ull * s->L + 16ull * nodes);
  read_counters(s, st);
  const Counters c = *s->hctr;
  const uint64_t delta = take_merge(s, c, merged);
  PhaseMark pr = phase_begin(s, CPMA_PHASE_REDIST, st);
  if (s->n == 0) {
    spread_fresh(s, 0, 1, st);
    phase_end(s, pr, st);
    return delta;
  }
  const uint64_t total = c.root_sum;
  const uint64_t Lt =
      std::max<uint64_t>(1, (uint64_t)std::ceil((double)total / (s->cfg.build_density * (double)s->S)));
  uint64_t moved = 0;
  if (!split_resize(s, Lt, total, st, &moved)) {
    phase_end(s, pr, st);
    rebalance(s, st);  // thresholds beyond 64 bits: the counted path
    return delta;
  }
  phase_end(s, pr, st, total + moved);
  return delta;
}

// Launch shapes of the merge kernels for a batch of at most kbound keys.
struct MergeGrids {
  uint32_t lgrid, wgrid, lwaves, hgrid_spill;
  uint64_t part_slots;  // (keys changed, bytes) slot pairs of every launch
};

MergeGrids merge_grids(const cpma* s, uint64_t kbound) {
  MergeGrids m;
  const uint64_t segs = std::min<uint64_t>(kbound, s->L);
  m.lgrid = (uint32_t)std::min<uint64_t>((segs + 255) / 256, (uint64_t)s->num_cus * 16);
  // many more waves than fit at once: a wave takes a few segments, and the
  // dispatcher hands out the rest as waves finish, which evens out segments of
  // unequal work (4-5 % faster at 1e7 into 1e8 than 40 waves per CU)
  m.wgrid = std::max(1u, (uint32_t)std::min<uint64_t>(segs, (uint64_t)s->num_cus * 320));
  m.lwaves = std::max(1u, m.lgrid) * (256 / kWave);
  // heavy merge of spilled slices: at most kbound / (kWaveSlice + 1) of them,
  // a few LDS-bound waves per CU
  m.hgrid_spill =
      (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, kbound / (kWaveSlice + 1)), (uint64_t)s->num_cus * 4);
  m.part_slots = 2ull * m.wgrid + 2ull * m.lwaves + std::max(m.hgrid_spill, 1024u);
  return m;
}

// Every allocation a batch of at most kbound keys can need, taken before the
// batch writes the structure: batch preparation and segments, the merge's
// overflow arena and staging, and what follows the merge.
void reserve_batch(cpma* s, uint64_t kbound, bool insert) {
  const uint64_t L = s->L;
  const uint64_t kl = std::max(kbound, L);
  ensure(s->kdedup, kbound * sizeof(uint64_t));
  ensure(s->leafid, (kl + 1) * sizeof(uint32_t));
  ensure(s->segpos, (kl + 1) * sizeof(uint32_t));
  ensure(s->seg_leaf, kbound * sizeof(uint32_t));
  ensure(s->seg_begin, (kbound + 1) * sizeof(uint32_t));
  ensure(s->seg_desc, (kbound + 1) * sizeof(uint4));
  ensure(s->heavy, kbound * sizeof(uint32_t));
  ensure(s->spill, kbound * sizeof(uint32_t));
  ensure(s->wide, kbound * sizeof(uint32_t));
  ensure(s->ovf, std::max<uint64_t>(L, 1) * sizeof(uint64_t));
  // overflow arena: segment s owns s * (S + 16) + 16 * (its first batch index)
  // onwards (a leaf that outgrows S holds at most S + 10 bytes per new key)
  const uint64_t arena_cap =
      insert ? std::min<uint64_t>(L, kbound) * (uint64_t)(s->S + 16) + (s->kv() ? 32 : 16) * kbound + 256 : 256;
  ensure(s->arena, arena_cap, 1.0);
  // heavy-merge staging: only slices of more than kHeavyLds keys stage, each at
  // most its own keys plus one leaf's keys
  uint64_t stage_cap = insert ? kbound + (kbound / kHeavyLds + 1) * (uint64_t)s->S + 64 : 64;
  if (s->kv()) {
    // key-value merges stage a merged leaf of more than KvLayout::cap keys:
    // its new keys (more than its old ones) and its old ones
    stage_cap = insert ? 2 * kbound + 64 : 64;
    ensure(s->vstage, stage_cap * sizeof(uint64_t));
  }
  ensure(s->stage, stage_cap * sizeof(uint64_t));
  ensure(s->parts, 16ull * merge_grids(s, kbound).part_slots);
  ensure(s->scan_tmp, scan_scratch_elems(kl + 1) * sizeof(uint64_t));
  reserve_after_merge(s, kbound, insert);
}

// small: the small-batch kernel already wrote kprime, the segments, their routing and T.
// rebuild: the batch is large enough for a full rebuild instead of counting.
// Arguments of the merge kernels for the batch B (sorted, repeat-free) and the
// segments of the current update.
MergeArgs merge_args(cpma* s, const uint64_t* B, bool insert) {
  MergeArgs a;
  a.bytes = s->bytes.as<uint8_t>();
  a.used = s->used.as<uint32_t>();
  a.head = s->head.as<uint64_t>();
  a.ovf = s->ovf.as<uint64_t>();
  a.arena = s->arena.as<uint8_t>();
  a.arena_cap = s->arena.cap;
  a.stage = s->stage.as<uint64_t>();
  a.stage_cap = s->stage.cap / sizeof(uint64_t);
  a.B = B;
  a.seg_leaf = s->seg_leaf.as<uint32_t>();
  a.seg_begin = s->seg_begin.as<uint32_t>();
  a.seg_desc = s->seg_desc.as<uint4>();
  a.heavy_list = s->heavy.as<uint32_t>();
  a.spill_list = s->spill.as<uint32_t>();
  a.wide_list = s->wide.as<uint32_t>();
  a.ctr = s->dctr;
  a.S = s->S;
  a.is_insert = insert ? 1 : 0;
  a.kv = s->kv() ? 1u : 0u;
  a.clen = s->clen.as<uint32_t>();
  a.Bv = insert ? s->batch_vals : nullptr;
  a.vstage = s->vstage.as<uint64_t>();
  a.part = s->parts.as<unsigned long long>();
  return a;
}

// Whether a small batch's path check runs as one block that also folds the
// merge's totals and writes the counters to the host (at most 8192 (level,
// segment) pairs: each of its threads takes one chunk of eight).
bool finish_in_path_check(const cpma* s, uint64_t k) {
  if (!s->pyr_valid) return false;
  const Pyramid P = pyramid_layout(s->L);
  return std::min<uint64_t>(k, s->L) * (uint64_t)(P.H + 1) <= 8ull * kPathThreads;
}

uint64_t apply_batch(cpma* s, const uint64_t* B, uint64_t kbound, bool insert, hipStream_t st, bool small = false,
                     bool rebuild_all = false) {
  const bool segments_ready = small;
  s->fin_parts = nullptr;
  reserve_batch(s, kbound, insert);
  PhaseMark pl = phase_begin(s, CPMA_PHASE_LOCATE, st);
  const uint64_t L = s->L;
  if (segments_ready) {
    // nothing to do: the segments come with the batch
  } else if (kbound >= L) {
    // per leaf: one search of head[f] in the batch
    hipLaunchKernelGGL(k_leaf_slices, dim3(grid_for(L + 1, 256, 1u << 16)), dim3(256), 0, st, B,
                       (const unsigned long long*)&s->dctr->kprime, (const uint64_t*)s->head.as<uint64_t>(), L,
                       s->leafid.as<uint32_t>());
    HIPCHK(hipGetLastError());
    scan<uint32_t>(s, s->segpos.as<uint32_t>(), L, st, SliceFlag{s->leafid.as<uint32_t>()});
    hipLaunchKernelGGL(k_segments_by_leaf, dim3(grid_for(L + 1, 256, 1u << 16)), dim3(256), 0, st,
                       (const uint32_t*)s->leafid.as<uint32_t>(), (const unsigned long long*)&s->dctr->kprime,
                       (const uint32_t*)s->segpos.as<uint32_t>(), L, s->seg_leaf.as<uint32_t>(),
                       s->seg_begin.as<uint32_t>(), s->seg_desc.as<uint4>(), (const uint32_t*)s->used.as<uint32_t>(),
                       (const uint64_t*)s->head.as<uint64_t>(), B, s->dctr);
  } else {
    // per key: one search of the key in the heads
    hipLaunchKernelGGL(k_locate, dim3(grid_for(kbound, 256, 1u << 16)), dim3(256), 0, st, B,
                       (const unsigned long long*)&s->dctr->kprime, (const uint64_t*)s->head.as<uint64_t>(), L,
                       s->leafid.as<uint32_t>());
    HIPCHK(hipGetLastError());
    scan<uint32_t>(s, s->segpos.as<uint32_t>(), kbound, st,
                   SegFlag{s->leafid.as<uint32_t>(), (const unsigned long long*)&s->dctr->kprime});
    hipLaunchKernelGGL(k_segments, dim3(grid_for(kbound, 256, 1u << 16)), dim3(256), 0, st,
                       (const uint32_t*)s->leafid.as<uint32_t>(), (const unsigned long long*)&s->dctr->kprime,
                       (const uint32_t*)s->segpos.as<uint32_t>(), kbound, s->seg_leaf.as<uint32_t>(),
                       s->seg_begin.as<uint32_t>(), s->seg_desc.as<uint4>(), (const uint32_t*)s->used.as<uint32_t>(),
                       (const uint64_t*)s->head.as<uint64_t>(), L, B, s->dctr);
  }
  HIPCHK(hipGetLastError());
  if (s->S <= kWaveMaxS && !small && !s->cfg.uncompressed && !s->kv()) {
    // route segments: narrow (32-bit wave merge), wide (64-bit), long insert slices
    // (spill list: heavy merge)
    const uint64_t nseg = std::min<uint64_t>(kbound, L);
    hipLaunchKernelGGL(k_classify, dim3(grid_for(nseg, 256, (uint32_t)s->num_cus * 8)), dim3(256), 0, st,
                       s->seg_desc.as<uint4>(), (const uint32_t*)s->seg_begin.as<uint32_t>(), kWaveSlice,
                       insert ? 1 : 0, s->wide.as<uint32_t>(), s->spill.as<uint32_t>(), s->dctr, nseg);
    HIPCHK(hipGetLastError());
  }
  phase_end(s, pl, st, 24ull * kbound);
  MergeArgs a = merge_args(s, B, insert);
  const MergeGrids mg = merge_grids(s, kbound);
  const uint32_t lgrid = mg.lgrid, wgrid = mg.wgrid, lwaves = mg.lwaves, hgrid_spill = mg.hgrid_spill;
  // per-wave totals: each launch owns a run of slot pairs, main-merge launches
  // first, follow-up launches after them
  unsigned long long* parts = s->parts.as<unsigned long long>();
  uint32_t n_narrow = 0, n_wide = 0;
  auto slots = [&](uint32_t waves, bool narrow) {
    unsigned long long* p = parts + 2ull * (n_narrow + n_wide);
    (narrow ? n_narrow : n_wide) += waves;
    return p;
  };

  // MERGE times exactly the main merge kernel; HEAVY the follow-up kernels for
  // wide, long and heavy slices.  From here on the structure is written.
  s->mutating = true;
  PhaseMark pmg = phase_begin(s, CPMA_PHASE_MERGE, st);
  if (s->cfg.uncompressed) {
    // uncompressed leaves: one wave per touched leaf, any slice length
    a.part = slots(wgrid, true);
    hipLaunchKernelGGL(k_pma_merge, dim3(wgrid), dim3(kWave), 0, st, a);
    HIPCHK(hipGetLastError());
    phase_end(s, pmg, st);
  } else if (s->kv()) {
    // key-value leaves: one wave per touched leaf, any slice length
    a.part = slots(wgrid, true);
    hipLaunchKernelGGL(k_kv_merge, dim3(wgrid), dim3(kWave), KvLayout(s->S).total, st, a);
    HIPCHK(hipGetLastError());
    phase_end(s, pmg, st);
  } else if (small && s->S <= kWaveMaxS) {
    // every segment in one 64-bit wave pass; long insert slices in the heavy merge
    a.part = slots(wgrid, false);
    hipLaunchKernelGGL(k_merge_wave<uint64_t>, dim3(wgrid), dim3(kWave), 0, st, a, 1);
    if (insert && kbound > kWaveSlice) {
      // a slice of more than kWaveSlice keys spills to the heavy merge
      a.part = slots(hgrid_spill, false);
      hipLaunchKernelGGL(k_merge_heavy, dim3(hgrid_spill), dim3(kWave), heavy_smem(s->S, kHeavyLds), st, a,
                         kHeavyLds, 1);
    }
    HIPCHK(hipGetLastError());
    phase_end(s, pmg, st);
  } else if (s->S <= kWaveMaxS) {
    a.part = slots(wgrid, true);
    hipLaunchKernelGGL(k_merge_wave<uint32_t>, dim3(wgrid), dim3(kWave), 0, st, a);
    HIPCHK(hipGetLastError());
    phase_end(s, pmg, st);
    PhaseMark ph = phase_begin(s, CPMA_PHASE_HEAVY, st);
    a.part = slots(wgrid, false);
    hipLaunchKernelGGL(k_merge_wave<uint64_t>, dim3(wgrid), dim3(kWave), 0, st, a);
    if (insert) {  // long insert slices, one wave each
      a.part = slots(hgrid_spill, false);
      hipLaunchKernelGGL(k_merge_heavy, dim3(hgrid_spill), dim3(kWave), heavy_smem(s->S, kHeavyLds), st, a,
                         kHeavyLds, 1);
    }
    HIPCHK(hipGetLastError());
    phase_end(s, ph, st);
  } else {
    a.part = slots(lwaves, true);
    hipLaunchKernelGGL(k_merge_lane, dim3(std::max(1u, lgrid)), dim3(256), 0, st, a);
    HIPCHK(hipGetLastError());
    phase_end(s, pmg, st);
    if (insert) {
      const uint32_t hgrid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, kbound / kLaneHeavy), 1024);
      PhaseMark ph = phase_begin(s, CPMA_PHASE_HEAVY, st);
      a.part = slots(hgrid, false);
      hipLaunchKernelGGL(k_merge_heavy, dim3(hgrid), dim3(kWave), heavy_smem(s->S, 0), st, a, 0u, 0);
      HIPCHK(hipGetLastError());
      phase_end(s, ph, st);
    }
  }
  if (!rebuild_all && small && finish_in_path_check(s, kbound)) {
    s->fin_parts = parts;  // folded by the path check, which also returns the counters
    s->fin_nn = n_narrow;
    s->fin_nw = n_wide;
  } else {
    hipLaunchKernelGGL(k_fold_parts, dim3(grid_for(n_narrow + n_wide, 1024, 32)), dim3(1024), 0, st,
                       (const unsigned long long*)parts, n_narrow, n_wide, s->dctr);
  }
  HIPCHK(hipGetLastError());
  if (rebuild_all) return rebuild(s, st, insert ? 1 : 0);
  return rebalance(s, st, insert ? 1 : 0, small ? kbound : 0);
}

// Whether a batch of k keys rebuilds the whole structure.
bool wants_rebuild(const cpma* s, uint64_t k) {
  return s->n > 0 && (double)k >= s->cfg.rebuild_frac * (double)s->n;
}

// Batch of k <= kSmallBatch keys at device address src (any order, repeats
// allowed): one launch zeroes the counters and prepares it (sort, repeats,
// leaves, segments), then the merge and rebalance phases run.
// Host keys (src null) come in `ak`, at most kArgKeys of them.
uint64_t apply_small(cpma* s, const uint64_t* src, uint64_t k, bool insert, hipStream_t st,
                     const ArgKeys* ak = nullptr) {
  reserve_batch(s, k, insert);
  static const ArgKeys kNoArgKeys{};
  if (k <= kWaveSlice && s->S <= kWaveMaxS && !s->cfg.uncompressed && !s->kv() && !s->stats_on &&
      finish_in_path_check(s, k)) {
    // the whole update in one launch; a violated bound on a touched path falls
    // back to the full count
    MergeArgs a = merge_args(s, s->kdedup.as<uint64_t>(), insert);
    Pyramid P = pyramid_layout(s->L);
    P.base = s->pyr.as<uint64_t>();
    s->mutating = true;
    hipLaunchKernelGGL(k_small_update, dim3(1), dim3(kSmallThreads), 0, st, src, ak ? *ak : kNoArgKeys,
                       (uint32_t)k, (const uint64_t*)s->head.as<uint64_t>(), s->L, s->kdedup.as<uint64_t>(),
                       insert ? 1 : 0, a, s->bounds(s->L), P, s->hctr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    if (s->hctr->error) throw Fail{CPMA_ERR_DEVICE};
    const Counters c = *s->hctr;
    const uint64_t delta = take_merge(s, c, insert ? 1 : 0);
    if (c.path_unsafe) {
      s->pyr_valid = false;
      rebalance(s, st);
    }
    return delta;
  }
  PhaseMark pm = phase_begin(s, CPMA_PHASE_SORT, st);
  hipLaunchKernelGGL(k_small_prep, dim3(1), dim3(kSmallThreads), 0, st, src, ak ? *ak : kNoArgKeys, (uint32_t)k,
                     (const uint64_t*)s->head.as<uint64_t>(), s->L, (const uint32_t*)s->used.as<uint32_t>(),
                     s->kdedup.as<uint64_t>(), s->seg_leaf.as<uint32_t>(), s->seg_begin.as<uint32_t>(),
                     s->seg_desc.as<uint4>(), insert ? 1 : 0,
                     (s->S <= kWaveMaxS && !s->cfg.uncompressed) ? kWaveSlice : 0xffffffffu,
                     s->spill.as<uint32_t>(), s->dctr);
  HIPCHK(hipGetLastError());
  phase_end(s, pm, st, 16ull * k);
  return apply_batch(s, s->kdedup.as<uint64_t>(), k, insert, st, true);
}

// Sorted repeat-free batch of k keys at device address B.  Zeroes the counters.
uint64_t apply_sorted(cpma* s, const uint64_t* B, uint64_t k, bool insert, hipStream_t st) {
  if (k <= kSmallBatch && !s->kv()) return apply_small(s, B, k, insert, st);
  zero_counters(s, st);
  hipLaunchKernelGGL((k_fill<unsigned long long>), dim3(1), dim3(64), 0, st, &s->dctr->kprime, (uint64_t)1,
                     (unsigned long long)k);
  HIPCHK(hipGetLastError());
  return apply_batch(s, B, k, insert, st, false, wants_rebuild(s, k));
}

cpma_status check_config(const cpma_config& c) {
  if (c.leaf_bytes < 64 || c.leaf_bytes > 4096 || (c.leaf_bytes & (c.leaf_bytes - 1))) return CPMA_ERR_INVALID;
  if (c.range_chunk < 1 || c.range_chunk > 64 || (c.range_chunk & (c.range_chunk - 1))) return CPMA_ERR_INVALID;
  if (!c.alloc != !c.free) return CPMA_ERR_INVALID;  // both hooks or neither
  if (!(c.grow > 1.0 && c.grow <= 4.0)) return CPMA_ERR_INVALID;
  if (!(c.lo_leaf > 0 && c.lo_leaf <= c.lo_root && c.lo_root < c.up_root && c.up_root <= c.up_leaf &&
        c.up_leaf < 1.0))
    return CPMA_ERR_INVALID;
  if (!(c.lo_root * c.grow < c.up_root)) return CPMA_ERR_INVALID;
  if (!(c.build_density > c.lo_root && c.build_density < c.up_root)) return CPMA_ERR_INVALID;
  if (!(c.rebuild_frac > 0)) return CPMA_ERR_INVALID;
  if (c.uncompressed != 0 && c.uncompressed != 1) return CPMA_ERR_INVALID;
  if (c.values != 0 && c.values != 1) return CPMA_ERR_INVALID;
  if (c.values && c.uncompressed) return CPMA_ERR_INVALID;  // key-value leaves are compressed ones
  return CPMA_OK;
}

// Runs one entry point's work.  An update takes every allocation it can need
// before it writes the structure (reserve_batch), so CPMA_ERR_NOMEM leaves the
// set unchanged; a device error, or an allocation that failed after the first
// write, leaves the handle unusable.
template <class F>
cpma_status guarded(cpma* s, F&& f) {
  if (s) s->mutating = false;
  try {
    f();
    return CPMA_OK;
  } catch (const Fail& e) {
    if (s && e.st == CPMA_ERR_NOMEM && s->mutating) {
      s->broken = true;
      return CPMA_ERR_DEVICE;
    }
    if (s && e.st == CPMA_ERR_DEVICE) s->broken = true;
    return e.st;
  }
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

cpma_status cpma_config_default(cpma_config* cfg) {
  if (!cfg) return CPMA_ERR_INVALID;
  cfg->leaf_bytes = 1024;
  cfg->grow = 1.2;
  cfg->up_leaf = 0.90;
  cfg->up_root = 0.70;
  cfg->lo_leaf = 0.10;
  cfg->lo_root = 0.30;
  cfg->build_density = cfg->up_root / cfg->grow;
  cfg->range_chunk = 2;
  cfg->rebuild_frac = 1.0;
  cfg->uncompressed = 0;
  cfg->values = 0;
  cfg->alloc = nullptr;
  cfg->free = nullptr;
  cfg->ctx = nullptr;
  return CPMA_OK;
}

const char* cpma_status_str(cpma_status s) {
  switch (s) {
    case CPMA_OK: return "ok";
    case CPMA_ERR_INVALID: return "invalid argument";
    case CPMA_ERR_NOMEM: return "device allocation failed";
    case CPMA_ERR_DEVICE: return "device error";
    case CPMA_ERR_RESERVED_KEY: return "reserved key (UINT64_MAX)";
  }
  return "unknown status";
}

static cpma_status build_impl(const uint64_t* keys, const uint64_t* vals, uint64_t n, cpma_mem mem,
                              const cpma_config* cfg_in, void* stream, cpma** out, bool with_values) {
  if (!out) return CPMA_ERR_INVALID;
  *out = nullptr;
  if (n > 0 && (!keys || (with_values && !vals))) return CPMA_ERR_INVALID;
  cpma_config cfg;
  cpma_config_default(&cfg);
  if (cfg_in) {
    if (cfg_in->leaf_bytes) cfg.leaf_bytes = cfg_in->leaf_bytes;
    if (cfg_in->grow > 0) cfg.grow = cfg_in->grow;
    if (cfg_in->up_leaf > 0) cfg.up_leaf = cfg_in->up_leaf;
    if (cfg_in->up_root > 0) cfg.up_root = cfg_in->up_root;
    if (cfg_in->lo_leaf > 0) cfg.lo_leaf = cfg_in->lo_leaf;
    if (cfg_in->lo_root > 0) cfg.lo_root = cfg_in->lo_root;
    cfg.build_density = cfg_in->build_density > 0 ? cfg_in->build_density : cfg.up_root / cfg.grow;
    if (cfg_in->range_chunk) cfg.range_chunk = cfg_in->range_chunk;
    if (cfg_in->rebuild_frac > 0) cfg.rebuild_frac = cfg_in->rebuild_frac;
    cfg.uncompressed = cfg_in->uncompressed;
    cfg.values = cfg_in->values;
    cfg.alloc = cfg_in->alloc;
    cfg.free = cfg_in->free;
    cfg.ctx = cfg_in->ctx;
  }
  if (with_values) cfg.values = 1;
  cpma_status cs = check_config(cfg);
  if (cs != CPMA_OK) return cs;
  cpma* s = new cpma();
  s->cfg = cfg;
  for (DevBuf* b : s->bufs()) b->al = &s->cfg;
  s->S = cfg.leaf_bytes;
  s->q_up_leaf = llround(cfg.up_leaf * (double)kQ);
  s->q_up_root = llround(cfg.up_root * (double)kQ);
  s->q_lo_leaf = llround(cfg.lo_leaf * (double)kQ);
  s->q_lo_root = llround(cfg.lo_root * (double)kQ);
  hipStream_t st = (hipStream_t)stream;
  cpma_status r = guarded(s, [&] {
    HIPCHK(hipGetDevice(&s->device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, s->device));
    s->num_cus = prop.multiProcessorCount;
    // the interior range scan runs one generation of blocks: every block
    // resident at once, so no block starts after the others have finished
    for (int plain = 0; plain < 2; plain++) {
      int per = 0;
      HIPCHK(plain ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_rm_interior<true>, 256, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_rm_interior<false>, 256, 0));
      s->rm_blocks[plain] = (uint32_t)std::max(1, per) * (uint32_t)s->num_cus;
    }
    ensure(s->ctr_buf, sizeof(Counters), 0.0);
    s->dctr = s->ctr_buf.as<Counters>();
    HIPCHK(hipHostMalloc(&s->hctr, sizeof(Counters), hipHostMallocDefault));
    ensure(s->info_buf, sizeof(BatchInfo), 0.0);
    s->dinfo = s->info_buf.as<BatchInfo>();
    HIPCHK(hipHostMalloc(&s->hinfo, sizeof(BatchInfo), hipHostMallocDefault));
    zero_counters(s, st);
    uint64_t K = 0;
    if (n > 0) {
      const uint64_t* B = s->kv() ? kv_prepare(s, keys, vals, n, mem, st) : prepare_batch(s, keys, n, mem, st);
      read_counters(s, st);
      K = s->hctr->kprime;
      ensure(s->stage, std::max<uint64_t>(K, 1) * sizeof(uint64_t));
      HIPCHK(hipMemcpyAsync(s->stage.p, B, K * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
      if (s->kv()) {
        ensure(s->vstage, std::max<uint64_t>(K, 1) * sizeof(uint64_t));
        HIPCHK(hipMemcpyAsync(s->vstage.p, s->kvdedup.p, K * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
      }
    }
    s->n = K;
    uint64_t Lt = 1;
    if (K > 0) {
      // Total bytes of the keys as one delta chain: the head plus every delta
      // code (8 bytes per key for uncompressed leaves).
      ensure(s->ccost, K);
      if (cfg.uncompressed)
        hipLaunchKernelGGL((k_fill<uint8_t>), dim3(grid_for(K, 256, 4096)), dim3(256), 0, st, s->ccost.as<uint8_t>(),
                           K, (uint8_t)8);
      else
        hipLaunchKernelGGL(k_chain_costs, dim3(grid_for(K, 256, 1u << 16)), dim3(256), 0, st,
                           (const uint64_t*)s->stage.as<uint64_t>(), K, s->ccost.as<uint8_t>(),
                           s->kv() ? 8u : 0u);
      HIPCHK(hipGetLastError());
      ensure(s->P, (K + 1) * sizeof(uint64_t));
      scan<uint64_t>(s, s->P.as<uint64_t>(), K, st, U8Fn{s->ccost.as<uint8_t>()});
      HIPCHK(hipMemcpyAsync(&s->hctr->root_sum, s->P.as<uint64_t>() + K, 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const uint64_t tot = s->hctr->root_sum;
      Lt = std::max<uint64_t>(1, (uint64_t)std::ceil((double)tot / (cfg.build_density * (double)s->S)));
    }
    spread_fresh(s, K, Lt, st, K > 0);
    rebalance(s, st);
    reserve_growth(s);
  });
  if (r != CPMA_OK) {
    cpma_destroy(s);
    return r;
  }
  *out = s;
  return CPMA_OK;
}

cpma_status cpma_build(const uint64_t* keys, uint64_t n, cpma_mem mem, const cpma_config* cfg, void* stream,
                       cpma** out) {
  return build_impl(keys, nullptr, n, mem, cfg, stream, out, false);
}

cpma_status cpma_build_kv(const uint64_t* keys, const uint64_t* values, uint64_t n, cpma_mem mem,
                          const cpma_config* cfg, void* stream, cpma** out) {
  if (out) *out = nullptr;
  if (cfg && cfg->uncompressed) return CPMA_ERR_INVALID;
  return build_impl(keys, values, n, mem, cfg, stream, out, true);
}

static cpma_status update(cpma* s, const uint64_t* keys, uint64_t k, cpma_mem mem, int sorted, void* stream,
                          uint64_t* delta_out, bool insert) {
  (void)sorted;  // sortedness is checked on the device either way
  if (delta_out) *delta_out = 0;
  if (!s) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  if (k == 0) return CPMA_OK;
  if (!keys) return CPMA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  uint64_t delta = 0;
  cpma_status r = guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    if (k <= kSmallBatch && !s->kv()) {
      const uint64_t* src = keys;
      if (mem == CPMA_MEM_HOST && k <= kArgKeys) {
        ArgKeys ak;
        std::memcpy(ak.k, keys, k * sizeof(uint64_t));
        delta = apply_small(s, nullptr, k, insert, st, &ak);
      } else {
        if (mem == CPMA_MEM_HOST) {
          ensure(s->kin, k * sizeof(uint64_t));
          HIPCHK(hipMemcpyAsync(s->kin.p, keys, k * sizeof(uint64_t), hipMemcpyHostToDevice, st));
          src = s->kin.as<uint64_t>();
        }
        delta = apply_small(s, src, k, insert, st);
      }
    } else {
      const uint64_t* B = prepare_batch(s, keys, k, mem, st, true);
      delta = apply_batch(s, B, k, insert, st, false, wants_rebuild(s, k));
    }
    resolve_phases(s);
  });
  if (r == CPMA_OK && delta_out) *delta_out = delta;
  return r;
}

cpma_status cpma_insert_batch(cpma* s, const uint64_t* keys, uint64_t k, cpma_mem mem, int sorted, void* stream,
                              uint64_t* n_added) {
  return update(s, keys, k, mem, sorted, stream, n_added, true);
}

cpma_status cpma_delete_batch(cpma* s, const uint64_t* keys, uint64_t k, cpma_mem mem, int sorted, void* stream,
                              uint64_t* n_removed) {
  return update(s, keys, k, mem, sorted, stream, n_removed, false);
}

cpma_status cpma_insert_kv(cpma* s, const uint64_t* keys, const uint64_t* values, uint64_t k, cpma_mem mem,
                           void* stream, uint64_t* n_added) {
  if (n_added) *n_added = 0;
  if (!s || !s->kv()) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  if (k == 0) return CPMA_OK;
  if (!keys || !values || k >= (1ull << 31)) return CPMA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  uint64_t delta = 0;
  cpma_status r = guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    zero_counters(s, st);
    const uint64_t* B = kv_prepare(s, keys, values, k, mem, st);
    s->batch_vals = s->kvdedup.as<uint64_t>();
    try {
      delta = apply_batch(s, B, k, true, st, false, wants_rebuild(s, k));
    } catch (...) {
      s->batch_vals = nullptr;
      throw;
    }
    s->batch_vals = nullptr;
    resolve_phases(s);
  });
  if (r == CPMA_OK && n_added) *n_added = delta;
  return r;
}

cpma_status cpma_export_code_bytes(const cpma* cs, uint32_t* clen, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !clen || !s->kv()) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(hipMemcpyAsync(clen, s->clen.p, s->L * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

static QueryArgs query_args(const cpma* s);

cpma_status cpma_apply_updates(cpma* s, uint32_t nreq, const int32_t* kind, const uint64_t* const* keys,
                               const uint64_t* n, cpma_mem mem, uint64_t* result, void* stream) {
  if (!s || (nreq && (!kind || !keys || !n || !result)) || s->cfg.uncompressed || s->kv()) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  uint64_t m = 0;
  for (uint32_t r = 0; r < nreq; r++) {
    if (kind[r] != CPMA_REQ_INSERT && kind[r] != CPMA_REQ_DELETE) return CPMA_ERR_INVALID;
    if (n[r] && !keys[r]) return CPMA_ERR_INVALID;
    m += n[r];
    if (m >= (1ull << 31)) return CPMA_ERR_INVALID;
  }
  for (uint32_t r = 0; r < nreq; r++) result[r] = 0;
  if (m == 0) return CPMA_OK;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    // pinned staging: request table (off: nreq + 1 words, then a delete flag
    // per request), the counts read back, then either the gather table
    // (device requests) or the small host requests packed back to back
    const size_t meta = 8ull * (nreq + 1) + nreq;
    const size_t res_at = (meta + 63) & ~size_t(63);
    const size_t tab_at = (res_at + 8ull * (nreq + 3) + 63) & ~size_t(63);
    constexpr uint64_t kDirect = 1u << 15;  // host requests of at least this many keys copy directly
    uint64_t small = 0;
    if (mem == CPMA_MEM_HOST) {
      for (uint32_t r = 0; r < nreq; r++)
        if (n[r] < kDirect) small += n[r];
    }
    const size_t tab_bytes = mem == CPMA_MEM_HOST ? 8 * small : sizeof(GatherReq) * (size_t)nreq;
    uint8_t* hp = (uint8_t*)host_pin(s, tab_at + tab_bytes + 64);
    uint64_t* hoff = reinterpret_cast<uint64_t*>(hp);
    hoff[0] = 0;
    for (uint32_t r = 0; r < nreq; r++) {
      hoff[r + 1] = hoff[r] + n[r];
      hp[8ull * (nreq + 1) + r] = kind[r] == CPMA_REQ_DELETE ? 1 : 0;
    }
    ensure(s->fz_meta, meta);
    HIPCHK(hipMemcpyAsync(s->fz_meta.p, hp, meta, hipMemcpyHostToDevice, st));
    ensure(s->kin, m * sizeof(uint64_t));
    uint64_t* dkeys = s->kin.as<uint64_t>();
    if (mem == CPMA_MEM_HOST) {
      // large requests straight from their buffers; runs of small ones packed
      // in the staging buffer, one copy per run
      uint64_t* stage = reinterpret_cast<uint64_t*>(hp + tab_at);
      uint64_t sp = 0, run_sp = 0, run_dst = 0, run_n = 0;
      for (uint32_t r = 0; r <= nreq; r++) {
        const bool direct = r < nreq && n[r] >= kDirect;
        if ((r == nreq || direct) && run_n) {
          HIPCHK(hipMemcpyAsync(dkeys + run_dst, stage + run_sp, 8 * run_n, hipMemcpyHostToDevice, st));
          run_n = 0;
        }
        if (r == nreq) break;
        if (direct) {
          HIPCHK(hipMemcpyAsync(dkeys + hoff[r], keys[r], 8 * n[r], hipMemcpyHostToDevice, st));
        } else if (n[r]) {
          if (!run_n) {
            run_sp = sp;
            run_dst = hoff[r];
          }
          std::memcpy(stage + sp, keys[r], 8 * n[r]);
          sp += n[r];
          run_n += n[r];
        }
      }
    } else {
      GatherReq* tab = reinterpret_cast<GatherReq*>(hp + tab_at);
      for (uint32_t r = 0; r < nreq; r++) tab[r] = GatherReq{keys[r], hoff[r], n[r]};
      ensure(s->fz_res, std::max<size_t>(8ull * nreq, sizeof(GatherReq) * (size_t)nreq));
      HIPCHK(hipMemcpyAsync(s->fz_res.p, tab, sizeof(GatherReq) * nreq, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_fuse_gather, dim3(std::min<uint32_t>(nreq, 65535u)), dim3(256), 0, st,
                         (const GatherReq*)s->fz_res.as<GatherReq>(), nreq, dkeys);
      HIPCHK(hipGetLastError());
    }
    const uint64_t* doff = s->fz_meta.as<uint64_t>();
    const uint8_t* drdel = s->fz_meta.as<uint8_t>() + 8ull * (nreq + 1);
    const uint64_t* src = dkeys;
    // validation before anything changes
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(s->dinfo),
                       (uint64_t)(sizeof(BatchInfo) / 4), 0u);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(m, 256, 4096)), dim3(256), 0, st, src, m, s->dinfo);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(s->hinfo, s->dinfo, sizeof(BatchInfo), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (s->hinfo->has_reserved) throw Fail{CPMA_ERR_RESERVED_KEY};

    // stable key-value sort; values carry position and kind
    ensure(s->fz_byte, m);
    hipLaunchKernelGGL(k_fuse_kinds, dim3(std::min<uint32_t>(nreq, 65535u)), dim3(256), 0, st, doff, drdel, nreq,
                       s->fz_byte.as<uint8_t>());
    HIPCHK(hipGetLastError());
    const int bits = 64 - __builtin_clzll(s->hinfo->or_all | 1);
    const int passes = (bits + 7) / 8;
    ensure(s->kb0, (m + 1) * sizeof(uint64_t));
    ensure(s->kb1, m * sizeof(uint64_t));
    ensure(s->fz_v0, m * sizeof(uint32_t));
    ensure(s->fz_v1, m * sizeof(uint32_t));
    const uint32_t nblk = (uint32_t)((m + kSortTile - 1) / kSortTile);
    ensure(s->cnt, ((uint64_t)nblk * 256 + 1) * sizeof(uint32_t));
    ensure(s->koff, ((uint64_t)nblk * 256 + 1) * sizeof(uint32_t));
    const uint64_t* kin = src;
    const uint32_t* vin = nullptr;
    for (int p = 0; p < passes; p++) {
      uint64_t* kout = (p & 1) ? s->kb1.as<uint64_t>() : s->kb0.as<uint64_t>();
      uint32_t* vout = (p & 1) ? s->fz_v1.as<uint32_t>() : s->fz_v0.as<uint32_t>();
      hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, st, kin, (uint32_t)m, 8 * p,
                         s->cnt.as<uint32_t>());
      HIPCHK(hipGetLastError());
      scan<uint32_t>(s, s->koff.as<uint32_t>(), (uint64_t)nblk * 256, st, LoadFn<uint32_t>{s->cnt.as<uint32_t>()});
      hipLaunchKernelGGL(k_radix_scatter_kv, dim3(nblk), dim3(kSortThreads), 0, st, kin, kout, (uint32_t)m, 8 * p,
                         (const uint32_t*)s->koff.as<uint32_t>(), vin, (const uint8_t*)s->fz_byte.as<uint8_t>(),
                         vout);
      HIPCHK(hipGetLastError());
      kin = kout;
      vin = vout;
    }
    const uint64_t* skeys = kin;
    const uint32_t* svals = vin;

    // distinct keys, their membership, per-item credits and net changes
    ensure(s->segpos, (m + 1) * sizeof(uint32_t));
    ensure(s->kdedup, m * sizeof(uint64_t));
    ensure(s->fz_ctr, 64);
    ensure(s->fz_member, m);
    ensure(s->fz_code, m);
    unsigned long long* fctr = s->fz_ctr.as<unsigned long long>();
    scan<uint32_t>(s, s->segpos.as<uint32_t>(), m, st, FirstFlag{skeys});
    hipLaunchKernelGGL(k_compact_unique, dim3(grid_for(m, 256)), dim3(256), 0, st, skeys, m,
                       (const uint32_t*)s->segpos.as<uint32_t>(), s->kdedup.as<uint64_t>(), fctr);
    QueryArgs qa = query_args(s);
    if (m >= s->L / 8) {
      // most leaves hold batch keys: decode each such leaf once
      ensure(s->leafid, (s->L + 1) * sizeof(uint32_t));
      hipLaunchKernelGGL(k_leaf_slices, dim3(grid_for(s->L + 1, 256, 1u << 16)), dim3(256), 0, st,
                         (const uint64_t*)s->kdedup.as<uint64_t>(), (const unsigned long long*)fctr,
                         (const uint64_t*)s->head.as<uint64_t>(), s->L, s->leafid.as<uint32_t>());
      hipLaunchKernelGGL(k_fuse_member_leaf, dim3((uint32_t)std::min<uint64_t>(s->L, (uint64_t)s->num_cus * 32)),
                         dim3(kWave), 8ull * s->S, st, qa, (const uint64_t*)s->kdedup.as<uint64_t>(),
                         (const uint32_t*)s->leafid.as<uint32_t>(), s->fz_member.as<uint8_t>());
    } else {
      hipLaunchKernelGGL(k_fuse_member, dim3(grid_for(m, 256, (uint32_t)s->num_cus * 16)), dim3(256), 0, st, qa,
                         (const uint64_t*)s->kdedup.as<uint64_t>(), (const unsigned long long*)fctr,
                         s->fz_member.as<uint8_t>());
    }
    hipLaunchKernelGGL(k_fuse_credit, dim3(grid_for(m, 256)), dim3(256), 0, st, skeys, svals, m,
                       (const uint32_t*)s->segpos.as<uint32_t>(), (const uint8_t*)s->fz_member.as<uint8_t>(),
                       s->fz_byte.as<uint8_t>(), s->fz_code.as<uint8_t>());
    HIPCHK(hipGetLastError());
    // net batches: inserts into kb1, deletes into kin (both free once sorted);
    // packed positions in kb0
    ensure(s->kin, m * sizeof(uint64_t));
    uint64_t* dpos = s->kb0.as<uint64_t>();
    uint64_t* dins = s->kb1.as<uint64_t>();
    uint64_t* ddel = s->kin.as<uint64_t>();
    scan<uint64_t>(s, dpos, m, st, FuseSplitFn{s->fz_code.as<uint8_t>(), fctr});
    hipLaunchKernelGGL(k_fuse_split, dim3(grid_for(m, 256)), dim3(256), 0, st,
                       (const uint64_t*)s->kdedup.as<uint64_t>(), (const uint8_t*)s->fz_code.as<uint8_t>(),
                       (const uint64_t*)dpos, dins, ddel, fctr);
    // per-request counts
    ensure(s->fz_res, 8ull * nreq);
    unsigned long long* dres = s->fz_res.as<unsigned long long>();
    hipLaunchKernelGGL((k_fill<unsigned long long>), dim3(grid_for(nreq, 256)), dim3(256), 0, st, dres,
                       (uint64_t)nreq, 0ull);
    hipLaunchKernelGGL(k_fuse_reduce, dim3(grid_for((m + 1023) / 1024, 4, (uint32_t)s->num_cus * 16)), dim3(256),
                       0, st, (const uint8_t*)s->fz_byte.as<uint8_t>(), m, doff, nreq, dres);
    HIPCHK(hipGetLastError());
    uint64_t* hres = reinterpret_cast<uint64_t*>(hp + res_at);
    HIPCHK(hipMemcpyAsync(hres, dres, 8ull * nreq, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hres + nreq, fctr, 24, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const uint64_t nins = hres[nreq + 1], ndel = hres[nreq + 2];
    std::vector<uint64_t> counts(hres, hres + nreq);  // the pinned staging may move below
    uint64_t net = 0;
    for (uint32_t r = 0; r < nreq; r++) net += kind[r] == CPMA_REQ_INSERT ? counts[r] : (0 - counts[r]);
    if (net != nins - ndel) throw Fail{CPMA_ERR_DEVICE};  // credits disagree with the net batches
    // deletes first (they only free room), then inserts; the insert batch's
    // memory is taken before the deletes write anything
    if (nins) reserve_batch(s, nins, true);
    if (ndel && apply_sorted(s, ddel, ndel, false, st) != ndel) throw Fail{CPMA_ERR_DEVICE};
    if (nins && apply_sorted(s, dins, nins, true, st) != nins) throw Fail{CPMA_ERR_DEVICE};
    std::copy(counts.begin(), counts.end(), result);
    resolve_phases(s);
  });
}

// The interior scan of range_map: the plain-CPMA instance for compressed sets
// without values, the general one otherwise.
static uint32_t interior_blocks(const cpma* s, const QueryArgs& a) {
  return s->rm_blocks[a.zero_fill && !a.raw && !a.vals ? 1 : 0];
}
static void launch_interior(const QueryArgs& a, uint32_t blocks, hipStream_t st, const uint64_t* voff,
                            const uint64_t* first, uint32_t chunk, unsigned long long* dsum, unsigned long long* dcount,
                            unsigned long long* alg) {
  if (a.zero_fill && !a.raw && !a.vals)
    hipLaunchKernelGGL(k_rm_interior<true>, dim3(blocks), dim3(256), 0, st, a, voff, first, chunk, dsum, dcount, alg);
  else
    hipLaunchKernelGGL(k_rm_interior<false>, dim3(blocks), dim3(256), 0, st, a, voff, first, chunk, dsum, dcount, alg);
}

static QueryArgs query_args(const cpma* s) {
  QueryArgs a;
  a.head = (const uint64_t*)s->head.p;
  a.bytes = (const uint8_t*)s->bytes.p;
  a.used = s->code_bytes();
  a.L = s->L;
  a.S = s->S;
  a.raw = s->cfg.uncompressed ? 1u : 0u;
  a.fill = (const uint32_t*)s->used.p;
  a.vals = 0;
  a.zero_fill = s->cfg.values ? 0u : 1u;
  return a;
}

// values: sum the values of key-value leaves instead of the keys.
static cpma_status range_map_impl(const cpma* cs, const uint64_t* lo, const uint64_t* hi, uint64_t q, cpma_mem mem,
                                  uint64_t* sum, uint64_t* count, void* stream, bool values) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s) return CPMA_ERR_INVALID;
  if (values && !s->kv()) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  if (q == 0) return CPMA_OK;
  if (!lo || !hi || !sum || !count) return CPMA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    QueryArgs a = query_args(s);
    a.q = q;
    a.vals = values ? 1u : 0u;
    unsigned long long* dsum = (unsigned long long*)sum;
    unsigned long long* dcount = (unsigned long long*)count;
    if (mem == CPMA_MEM_HOST) {
      ensure(s->qa, q * 8);
      ensure(s->qb, q * 8);
      HIPCHK(hipMemcpyAsync(s->qa.p, lo, q * 8, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(s->qb.p, hi, q * 8, hipMemcpyHostToDevice, st));
      a.lo = s->qa.as<uint64_t>();
      a.hi = s->qb.as<uint64_t>();
      ensure(s->qsum, q * 8);
      ensure(s->qcount, q * 8);
      dsum = s->qsum.as<unsigned long long>();
      dcount = s->qcount.as<unsigned long long>();
    } else {
      a.lo = lo;
      a.hi = hi;
    }
    ensure(s->qfirst, q * 8);
    ensure(s->qnvis, q * 8);
    ensure(s->qvoff, (q + 1) * 8);
    PhaseMark pq = phase_begin(s, CPMA_PHASE_QUERY, st);
    // statistics: one byte-count slot per wave of the end and interior kernels
    // few queries: a wave per query (key sums only)
    const bool wave_ends = q <= (uint64_t)s->num_cus * 64 && !values;
    const uint32_t egrid = wave_ends ? grid_for(q, 1, (uint32_t)s->num_cus * 64)
                                     : grid_for(q, 256, (uint32_t)s->num_cus * 16);
    const uint64_t ewaves = wave_ends ? egrid : 4ull * egrid;
    const uint32_t blocks = interior_blocks(s, a);
    const uint64_t nslots = ewaves + 4ull * blocks;
    unsigned long long* qalg = nullptr;
    if (s->stats_on && ((s->stats_mask >> CPMA_PHASE_RANGE_SCAN) & 1u)) {
      ensure(s->qparts, 8 * nslots);
      qalg = s->qparts.as<unsigned long long>();
    }
    if (wave_ends)
      hipLaunchKernelGGL(k_rm_ends_wave, dim3(egrid), dim3(kWave), 0, st, a, s->qfirst.as<uint64_t>(),
                         s->qnvis.as<uint64_t>(), dsum, dcount, qalg);
    else
      hipLaunchKernelGGL(k_rm_ends, dim3(egrid), dim3(256), 0, st, a, s->qfirst.as<uint64_t>(),
                         s->qnvis.as<uint64_t>(), dsum, dcount, qalg);
    HIPCHK(hipGetLastError());
    scan<uint64_t>(s, s->qvoff.as<uint64_t>(), q, st, LoadFn<uint64_t>{s->qnvis.as<uint64_t>()});
    PhaseMark ps = phase_begin(s, CPMA_PHASE_RANGE_SCAN, st);
    launch_interior(a, blocks, st, s->qvoff.as<uint64_t>(), s->qfirst.as<uint64_t>(), s->cfg.range_chunk, dsum,
                    dcount, qalg ? qalg + ewaves : qalg);
    HIPCHK(hipGetLastError());
    phase_end(s, ps, st, 32ull * q);
    phase_end(s, pq, st);
    if (qalg) {
      hipLaunchKernelGGL(k_fold_sum, dim3(1), dim3(1024), 0, st, (const unsigned long long*)qalg, nslots, s->dqalg);
      HIPCHK(hipGetLastError());
    }
    if (mem == CPMA_MEM_HOST) {
      HIPCHK(hipMemcpyAsync(sum, dsum, q * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(count, dcount, q * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      resolve_phases(s);
    }
  });
}

cpma_status cpma_range_map(const cpma* cs, const uint64_t* lo, const uint64_t* hi, uint64_t q, cpma_mem mem,
                           uint64_t* sum, uint64_t* count, void* stream) {
  return range_map_impl(cs, lo, hi, q, mem, sum, count, stream, false);
}

cpma_status cpma_range_map_values(const cpma* cs, const uint64_t* lo, const uint64_t* hi, uint64_t q, cpma_mem mem,
                                  uint64_t* vsum, uint64_t* count, void* stream) {
  return range_map_impl(cs, lo, hi, q, mem, vsum, count, stream, true);
}

cpma_status cpma_get(const cpma* cs, const uint64_t* keys, uint64_t q, cpma_mem mem, uint64_t* values,
                     uint8_t* found, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !s->kv()) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  if (q == 0) return CPMA_OK;
  if (!keys || !values || !found) return CPMA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    QueryArgs a = query_args(s);
    a.q = q;
    const uint64_t* dk = keys;
    uint64_t* dv = values;
    uint8_t* df = found;
    if (mem == CPMA_MEM_HOST) {
      ensure(s->qa, q * 8);
      ensure(s->qsum, q * 8);
      ensure(s->qout, q);
      HIPCHK(hipMemcpyAsync(s->qa.p, keys, q * 8, hipMemcpyHostToDevice, st));
      dk = s->qa.as<uint64_t>();
      dv = s->qsum.as<uint64_t>();
      df = s->qout.as<uint8_t>();
    }
    hipLaunchKernelGGL(k_kv_get, dim3(grid_for(q, 256, (uint32_t)s->num_cus * 16)), dim3(256), 0, st, a, dk, dv,
                       df);
    HIPCHK(hipGetLastError());
    if (mem == CPMA_MEM_HOST) {
      HIPCHK(hipMemcpyAsync(values, dv, q * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(found, df, q, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  });
}

}  // extern "C"

// ---- range_map without allocation ---------------------------------------------
// Per-query scratch of cpma_range_map_noalloc: first interior leaf, interior
// leaf count and their prefix sums (q, q and q + 1 words), then the prefix
// sum's block totals.  Each GPU holds one copy for the life of the process.
namespace {
constexpr uint64_t kNoAllocScratchWords = 3ull * CPMA_NOALLOC_MAX_QUERIES + 1024;
}  // namespace
static __device__ __align__(256) uint64_t scratch[kNoAllocScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
uint64_t* g_noalloc_ptr[kMaxDevices];  // device address of `scratch` on each GPU, once looked up

// The device address of the scratch array on `dev` (current), looked up once.
uint64_t* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Fail{CPMA_ERR_DEVICE};
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      hipGetLastError();
      throw Fail{CPMA_ERR_DEVICE};
    }
    g_noalloc_ptr[dev] = reinterpret_cast<uint64_t*>(p);
  }
  return g_noalloc_ptr[dev];
}
}  // namespace

extern "C" {

cpma_status cpma_range_map_noalloc(const cpma* cs, const uint64_t* lo, const uint64_t* hi, uint64_t q,
                                   uint64_t* sum, uint64_t* count, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  if (q > CPMA_NOALLOC_MAX_QUERIES) return CPMA_ERR_INVALID;
  if (q == 0) return CPMA_OK;
  if (!lo || !hi || !sum || !count) return CPMA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    if (3 * q + 1 + scan_scratch_elems(q) > kNoAllocScratchWords) throw Fail{CPMA_ERR_DEVICE};
    uint64_t* w = noalloc_scratch(s->device);
    uint64_t* first = w;
    uint64_t* nvis = w + q;
    uint64_t* voff = w + 2 * q;          // q + 1 words
    uint64_t* tmp = w + 3 * q + 1;       // the prefix sum's block totals
    QueryArgs a = query_args(s);
    a.q = q;
    a.lo = lo;
    a.hi = hi;
    unsigned long long* dsum = (unsigned long long*)sum;
    unsigned long long* dcount = (unsigned long long*)count;
    // the same kernels as cpma_range_map, without statistics
    const bool wave_ends = q <= (uint64_t)s->num_cus * 64;
    const uint32_t egrid = wave_ends ? grid_for(q, 1, (uint32_t)s->num_cus * 64)
                                     : grid_for(q, 256, (uint32_t)s->num_cus * 16);
    if (wave_ends)
      hipLaunchKernelGGL(k_rm_ends_wave, dim3(egrid), dim3(kWave), 0, st, a, first, nvis, dsum, dcount,
                         (unsigned long long*)nullptr);
    else
      hipLaunchKernelGGL(k_rm_ends, dim3(egrid), dim3(256), 0, st, a, first, nvis, dsum, dcount,
                         (unsigned long long*)nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(scan_exclusive<uint64_t>(LoadFn<uint64_t>{nvis}, q, voff, tmp, st));
    launch_interior(a, interior_blocks(s, a), st, voff, first, s->cfg.range_chunk, dsum, dcount, nullptr);
    HIPCHK(hipGetLastError());
  });
}

cpma_status cpma_contains(const cpma* cs, const uint64_t* keys, uint64_t q, cpma_mem mem, uint8_t* out,
                          void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  if (q == 0) return CPMA_OK;
  if (!keys || !out) return CPMA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    QueryArgs a = query_args(s);
    a.q = q;
    const uint64_t* dk = keys;
    uint8_t* dout = out;
    if (mem == CPMA_MEM_HOST) {
      ensure(s->qa, q * 8);
      ensure(s->qout, q);
      HIPCHK(hipMemcpyAsync(s->qa.p, keys, q * 8, hipMemcpyHostToDevice, st));
      dk = s->qa.as<uint64_t>();
      dout = s->qout.as<uint8_t>();
    }
    PhaseMark pq = phase_begin(s, CPMA_PHASE_QUERY, st);
    hipLaunchKernelGGL(k_contains, dim3(grid_for(q, 256, (uint32_t)s->num_cus * 16)), dim3(256), 0, st, a, dk,
                       dout);
    HIPCHK(hipGetLastError());
    phase_end(s, pq, st);
    if (mem == CPMA_MEM_HOST) {
      HIPCHK(hipMemcpyAsync(out, dout, q, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  });
}

static FgArgs fg_args(const cpma* s, uint32_t nv) {
  FgArgs g;
  g.bytes = (const uint8_t*)s->bytes.p;
  g.used = s->code_bytes();
  g.head = (const uint64_t*)s->head.p;
  g.L = s->L;
  g.S = s->S;
  g.nv = nv;
  return g;
}

static uint32_t fg_grid(const cpma* s) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((s->L + 3) / 4, (uint64_t)s->num_cus * 16));
}

}  // extern "C"

namespace {

// Level-synchronous BFS from `source` into lv (nv entries, device); returns the
// number of levels.  front / seen bitmaps and the per-block counts live in
// s->fg_c; on return `front` holds the last level's bitmap.
uint32_t bfs_levels(cpma* s, uint32_t nv, uint32_t source, bool symmetric, uint32_t* lv, hipStream_t st,
                    BfsBits* bits_out = nullptr, unsigned long long** cpart_out = nullptr,
                    uint32_t* cgrid_out = nullptr) {
  hipLaunchKernelGGL((k_fill<uint32_t>), dim3(grid_for(nv, 256, 4096)), dim3(256), 0, st, lv, (uint64_t)nv,
                     0xffffffffu);
  hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, lv + source, (uint64_t)1, 0u);
  HIPCHK(hipGetLastError());
  const FgArgs g = fg_args(s, nv);
  // bitmaps of the current level and of the visited vertices, rebuilt after
  // every level together with the level sizes (one slot pair per block,
  // summed into the last pair)
  const uint32_t nw = (nv + 31) / 32;
  const uint32_t cgrid = grid_for(nw, 256, (uint32_t)s->num_cus * 8);
  const uint64_t bits_words = 2ull * ((nw + 1) & ~1u);  // keeps the slots 8-byte aligned
  ensure(s->fg_c, 4 * bits_words + 16ull * (cgrid + 1));
  uint32_t* front = s->fg_c.as<uint32_t>();
  uint32_t* seen = front + (bits_words / 2);
  unsigned long long* cpart = reinterpret_cast<unsigned long long*>(front + bits_words);
  const BfsBits bb{front, seen};
  uint64_t* hc = reinterpret_cast<uint64_t*>(host_pin(s, 16));
  hipLaunchKernelGGL(k_fg_level_bits, dim3(cgrid), dim3(256), 0, st, (const uint32_t*)lv, nv, 0u, front, seen,
                     cpart);
  HIPCHK(hipGetLastError());
  // the step runs bottom-up once the level is large against the unvisited
  // set (its vertices have the most edges, so top-down gets dear early)
  uint64_t frontier = 1, unvisited = nv - 1;
  uint32_t cur = 0;
  for (; frontier > 0 && cur < nv; cur++) {
    if (!symmetric || 4 * frontier <= unvisited)
      hipLaunchKernelGGL(k_fg_bfs_step<false>, dim3(fg_grid(s)), dim3(256), 0, st, g, bb, lv, cur);
    else
      hipLaunchKernelGGL(k_fg_bfs_step<true>, dim3(fg_grid(s)), dim3(256), 0, st, g, bb, lv, cur);
    hipLaunchKernelGGL(k_fg_level_bits, dim3(cgrid), dim3(256), 0, st, (const uint32_t*)lv, nv, cur + 1, front,
                       seen, cpart);
    hipLaunchKernelGGL(k_fg_fold_counts, dim3(1), dim3(1024), 0, st, (const unsigned long long*)cpart, cgrid,
                       cpart + 2ull * cgrid);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hc, cpart + 2ull * cgrid, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    frontier = hc[0];
    unvisited = hc[1];
  }
  if (bits_out) *bits_out = bb;
  if (cpart_out) *cpart_out = cpart;
  if (cgrid_out) *cgrid_out = cgrid;
  return cur;  // levels 0 .. cur - 1 are non-empty
}

}  // namespace

extern "C" {

cpma_status cpma_fgraph_bfs(const cpma* cs, uint32_t nv, uint32_t source, int symmetric, cpma_mem mem,
                            uint32_t* level, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !level || nv == 0 || source >= nv) return CPMA_ERR_INVALID;
  if (s->S > kWaveMaxS || s->cfg.uncompressed) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    uint32_t* lv = level;
    if (mem == CPMA_MEM_HOST) {
      ensure(s->fg_level, (uint64_t)nv * 4);
      lv = s->fg_level.as<uint32_t>();
    }
    bfs_levels(s, nv, source, symmetric != 0, lv, st);
    if (mem == CPMA_MEM_HOST) {
      HIPCHK(hipMemcpyAsync(level, lv, (uint64_t)nv * 4, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
  });
}

cpma_status cpma_fgraph_offsets(const cpma* cs, uint32_t nv, cpma_mem mem, uint64_t* off, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !off || nv == 0) return CPMA_ERR_INVALID;
  if (s->S > kWaveMaxS || s->cfg.uncompressed) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    uint64_t* dof = off;
    if (mem == CPMA_MEM_HOST) {
      ensure(s->fg_acc, ((uint64_t)nv + 1) * 8);
      dof = s->fg_acc.as<uint64_t>();
    }
    ensure(s->fg_deg, (uint64_t)nv * 4);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(grid_for(nv, 256, 8192)), dim3(256), 0, st, s->fg_deg.as<uint32_t>(),
                       (uint64_t)nv, 0u);
    const FgArgs g = fg_args(s, nv);
    hipLaunchKernelGGL(k_fg_degree, dim3(fg_grid(s)), dim3(256), 0, st, g, s->fg_deg.as<uint32_t>());
    HIPCHK(hipGetLastError());
    scan<uint64_t>(s, dof, nv, st, U32AsU64Fn{s->fg_deg.as<uint32_t>()});
    if (mem == CPMA_MEM_HOST)
      HIPCHK(hipMemcpyAsync(off, dof, ((uint64_t)nv + 1) * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

cpma_status cpma_fgraph_cc(const cpma* cs, uint32_t nv, cpma_mem mem, uint32_t* label, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !label || nv == 0) return CPMA_ERR_INVALID;
  if (s->S > kWaveMaxS || s->cfg.uncompressed) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    uint32_t* lab = label;
    if (mem == CPMA_MEM_HOST) {
      ensure(s->fg_level, (uint64_t)nv * 4);
      lab = s->fg_level.as<uint32_t>();
    }
    ensure(s->fg_c, 16);
    uint32_t* changed = s->fg_c.as<uint32_t>();
    uint32_t* hc = reinterpret_cast<uint32_t*>(host_pin(s, 16));
    const uint32_t vg = grid_for(nv, 256, 8192);
    hipLaunchKernelGGL(k_fg_iota, dim3(vg), dim3(256), 0, st, lab, nv);
    const FgArgs g = fg_args(s, nv);
    for (uint32_t it = 0; it <= nv; it++) {
      hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, changed, (uint64_t)1, 0u);
      hipLaunchKernelGGL(k_fg_cc_prop, dim3(fg_grid(s)), dim3(256), 0, st, g, lab, changed);
      hipLaunchKernelGGL(k_fg_cc_jump, dim3(vg), dim3(256), 0, st, lab, nv);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hc, changed, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (!hc[0]) break;
    }
    if (mem == CPMA_MEM_HOST) HIPCHK(hipMemcpyAsync(label, lab, (uint64_t)nv * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

cpma_status cpma_fgraph_bc(const cpma* cs, uint32_t nv, uint32_t source, cpma_mem mem, double* sigma,
                           double* delta, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !delta || nv == 0 || source >= nv) return CPMA_ERR_INVALID;
  if (s->S > kWaveMaxS || s->cfg.uncompressed) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    ensure(s->fg_level, (uint64_t)nv * 4);
    uint32_t* lv = s->fg_level.as<uint32_t>();
    double* sg = (mem == CPMA_MEM_DEVICE && sigma) ? sigma : nullptr;
    double* dl = mem == CPMA_MEM_DEVICE ? delta : nullptr;
    if (!sg) {
      ensure(s->fg_p, (uint64_t)nv * 8);
      sg = s->fg_p.as<double>();
    }
    if (!dl) {
      ensure(s->fg_acc, (uint64_t)nv * 8);
      dl = s->fg_acc.as<double>();
    }
    BfsBits bb;
    unsigned long long* cpart = nullptr;
    uint32_t cgrid = 0;
    const uint32_t nlev = bfs_levels(s, nv, source, true, lv, st, &bb, &cpart, &cgrid);
    const uint32_t vg = grid_for(nv, 256, 8192);
    hipLaunchKernelGGL((k_fill<double>), dim3(vg), dim3(256), 0, st, sg, (uint64_t)nv, 0.0);
    hipLaunchKernelGGL((k_fill<double>), dim3(vg), dim3(256), 0, st, dl, (uint64_t)nv, 0.0);
    hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(64), 0, st, sg + source, (uint64_t)1, 1.0);
    const FgArgs g = fg_args(s, nv);
    uint32_t* front = const_cast<uint32_t*>(bb.front);
    uint32_t* seen = const_cast<uint32_t*>(bb.seen);
    // path counts, level by level outwards, then dependencies inwards
    for (uint32_t l = 1; l < nlev; l++) {
      hipLaunchKernelGGL(k_fg_level_bits, dim3(cgrid), dim3(256), 0, st, (const uint32_t*)lv, nv, l, front, seen,
                         cpart);
      hipLaunchKernelGGL(k_fg_bc_level<false>, dim3(fg_grid(s)), dim3(256), 0, st, g, bb, (const uint32_t*)lv, l,
                         (const double*)sg, (const double*)dl, sg);
    }
    for (uint32_t l = nlev; l-- > 0;) {
      if (l + 1 >= nlev) continue;  // the last level depends on nothing
      hipLaunchKernelGGL(k_fg_level_bits, dim3(cgrid), dim3(256), 0, st, (const uint32_t*)lv, nv, l, front, seen,
                         cpart);
      hipLaunchKernelGGL(k_fg_bc_level<true>, dim3(fg_grid(s)), dim3(256), 0, st, g, bb, (const uint32_t*)lv, l,
                         (const double*)sg, (const double*)dl, dl);
    }
    HIPCHK(hipGetLastError());
    if (mem == CPMA_MEM_HOST) {
      HIPCHK(hipMemcpyAsync(delta, dl, (uint64_t)nv * 8, hipMemcpyDeviceToHost, st));
      if (sigma) HIPCHK(hipMemcpyAsync(sigma, sg, (uint64_t)nv * 8, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
  });
}

cpma_status cpma_fgraph_pagerank(const cpma* cs, uint32_t nv, int iters, double damping, cpma_mem mem, float* p,
                                 void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !p || nv == 0 || iters < 0 || !(damping >= 0.0 && damping <= 1.0)) return CPMA_ERR_INVALID;
  if (s->S > kWaveMaxS || s->cfg.uncompressed) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    float* pv = p;
    if (mem == CPMA_MEM_HOST) {
      ensure(s->fg_p, (uint64_t)nv * 4);
      pv = s->fg_p.as<float>();
    }
    ensure(s->fg_deg, (uint64_t)nv * 4);
    ensure(s->fg_c, (uint64_t)nv * 4);
    ensure(s->fg_acc, (uint64_t)nv * 4);
    const uint32_t vg = grid_for(nv, 256, 8192);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(vg), dim3(256), 0, st, s->fg_deg.as<uint32_t>(), (uint64_t)nv, 0u);
    hipLaunchKernelGGL((k_fill<float>), dim3(vg), dim3(256), 0, st, pv, (uint64_t)nv, 1.0f / (float)nv);
    const FgArgs g = fg_args(s, nv);
    PhaseMark pq = phase_begin(s, CPMA_PHASE_QUERY, st);
    hipLaunchKernelGGL(k_fg_degree, dim3(fg_grid(s)), dim3(256), 0, st, g, s->fg_deg.as<uint32_t>());
    const float base = (float)((1.0 - damping) / (double)nv);
    for (int it = 0; it < iters; it++) {
      hipLaunchKernelGGL(k_pr_contrib, dim3(vg), dim3(256), 0, st, (const float*)pv,
                         (const uint32_t*)s->fg_deg.as<uint32_t>(), nv, s->fg_c.as<float>(), s->fg_acc.as<float>());
      hipLaunchKernelGGL(k_fg_pull, dim3(fg_grid(s)), dim3(256), 0, st, g, (const float*)s->fg_c.as<float>(),
                         s->fg_acc.as<float>());
      hipLaunchKernelGGL(k_pr_update, dim3(vg), dim3(256), 0, st, (const float*)s->fg_acc.as<float>(), nv, base,
                         (float)damping, pv);
    }
    HIPCHK(hipGetLastError());
    phase_end(s, pq, st);
    if (mem == CPMA_MEM_HOST) HIPCHK(hipMemcpyAsync(p, pv, (uint64_t)nv * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    resolve_phases(s);
  });
}

uint64_t cpma_size(const cpma* s) { return s ? s->n : 0; }

uint64_t cpma_bytes(const cpma* s) { return s ? s->L * ((uint64_t)s->S + 8 + 4 + (s->kv() ? 4 : 0)) : 0; }

uint64_t cpma_bytes_held(const cpma* cs) {
  if (!cs) return 0;
  cpma* s = const_cast<cpma*>(cs);
  uint64_t total = 0;
  for (DevBuf* b : s->bufs()) total += b->cap;
  return total;
}

cpma_status cpma_trim(cpma* s, void* stream) {
  if (!s) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  if (hipSetDevice(s->device) != hipSuccess || hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
    hipGetLastError();
    return CPMA_ERR_DEVICE;
  }
  // the structure and the small counters the handle's pointers refer to stay
  const DevBuf* keep[] = {&s->bytes, &s->used, &s->head, &s->clen, &s->ctr_buf, &s->info_buf, &s->qalg_buf};
  for (DevBuf* b : s->bufs()) {
    if (std::find(std::begin(keep), std::end(keep), b) != std::end(keep)) continue;
    release(*b);
  }
  // the leaf arrays keep the room of the growth that made them: copy each to
  // a fitting allocation (an array stays as it is if that allocation fails)
  const size_t fit[4] = {(size_t)(s->L * (uint64_t)s->S), (size_t)(s->L * 4), (size_t)(s->L * 8),
                         (size_t)(s->L * 4)};
  DevBuf* arr[4] = {&s->bytes, &s->used, &s->head, &s->clen};
  for (int i = 0; i < (s->kv() ? 4 : 3); i++) {
    const size_t want = fit[i] + 256;
    if (arr[i]->cap <= want) continue;
    void* p = nullptr;
    try {
      p = dev_alloc(arr[i]->al, want);
    } catch (const Fail&) {
      p = nullptr;
    }
    if (!p) continue;
    if (hipMemcpyAsync(p, arr[i]->p, fit[i], hipMemcpyDeviceToDevice, (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
      hipGetLastError();
      dev_free(arr[i]->al, p);
      return CPMA_ERR_DEVICE;
    }
    dev_free(arr[i]->al, arr[i]->p);
    arr[i]->p = p;
    arr[i]->cap = want;
  }
  s->pyr_valid = false;
  s->wol_L = 0;
  return CPMA_OK;
}

cpma_status cpma_geometry(const cpma* s, uint64_t* num_leaves, uint32_t* leaf_bytes) {
  if (!s) return CPMA_ERR_INVALID;
  if (num_leaves) *num_leaves = s->L;
  if (leaf_bytes) *leaf_bytes = s->S;
  return CPMA_OK;
}

cpma_status cpma_export(const cpma* cs, uint8_t* bytes, uint32_t* used, uint64_t* head, void* stream) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s) return CPMA_ERR_INVALID;
  if (s->broken) return CPMA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    if (bytes) HIPCHK(hipMemcpyAsync(bytes, s->bytes.p, s->L * (uint64_t)s->S, hipMemcpyDeviceToHost, st));
    if (used) HIPCHK(hipMemcpyAsync(used, s->used.p, s->L * 4, hipMemcpyDeviceToHost, st));
    if (head) HIPCHK(hipMemcpyAsync(head, s->head.p, s->L * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

cpma_status cpma_stats_select(cpma* s, uint32_t phase_mask) {
  if (!s || (phase_mask >> CPMA_PHASE_NUM) != 0) return CPMA_ERR_INVALID;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(hipDeviceSynchronize());
    resolve_phases(s);
    if (phase_mask) {
      ensure(s->qalg_buf, sizeof(unsigned long long), 0.0);
      s->dqalg = s->qalg_buf.as<unsigned long long>();
      HIPCHK(hipMemset(s->dqalg, 0, sizeof(unsigned long long)));
      HIPCHK(hipDeviceSynchronize());
      memset(s->stats, 0, sizeof(s->stats));
    }
    s->stats_on = phase_mask != 0;
    s->stats_mask = phase_mask;
  });
}

cpma_status cpma_stats_enable(cpma* s, int on) {
  return cpma_stats_select(s, on ? (1u << CPMA_PHASE_NUM) - 1u : 0u);
}

cpma_status cpma_stats_get(const cpma* cs, cpma_phase_stat* out, int n) {
  cpma* s = const_cast<cpma*>(cs);
  if (!s || !out || n < 0) return CPMA_ERR_INVALID;
  return guarded(s, [&] {
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(hipDeviceSynchronize());
    resolve_phases(s);
    cpma_phase_stat tmp[CPMA_PHASE_NUM];
    memcpy(tmp, s->stats, sizeof(tmp));
    if (s->dqalg) {
      unsigned long long q = 0;
      HIPCHK(hipMemcpy(&q, s->dqalg, sizeof(q), hipMemcpyDeviceToHost));
      tmp[CPMA_PHASE_RANGE_SCAN].alg_bytes += q;
    }
    for (int i = 0; i < n && i < CPMA_PHASE_NUM; i++) out[i] = tmp[i];
  });
}

void cpma_destroy(cpma* s) {
  if (!s) return;
  hipDeviceSynchronize();
  for (const auto& p : s->pending) {
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  for (hipEvent_t e : s->evpool) hipEventDestroy(e);
  for (DevBuf* b : s->bufs()) release(*b);
  if (s->hctr) hipHostFree(s->hctr);
  if (s->hinfo) hipHostFree(s->hinfo);
  if (s->hpin) hipHostFree(s->hpin);
  delete s;
}

}  // extern "C"

// ---- autotuner ------------------------------------------------------------------
namespace {

struct DevScratch {
  std::vector<void*> ptrs;
  ~DevScratch() {
    for (void* p : ptrs) hipFree(p);
  }
  template <typename T>
  T* get(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess) {
      hipGetLastError();
      throw Fail{CPMA_ERR_NOMEM};
    }
    ptrs.push_back(p);
    return reinterpret_cast<T*>(p);
  }
};

struct Handle {
  cpma* h = nullptr;
  ~Handle() { cpma_destroy(h); }
};

// Least device time of `reps` runs of f() after one warm-up, in ms (events on st).
template <class F>
double time_min(hipStream_t st, int reps, F&& f) {
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  double best = 1e30;
  for (int r = 0; r <= reps; r++) {
    HIPCHK(hipEventRecord(a, st));
    f(r);
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    if (r > 0) best = std::min(best, (double)ms);
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return best;
}

void st_check(cpma_status r) {
  if (r != CPMA_OK) throw Fail{r};
}

}  // namespace

extern "C" cpma_status cpma_autotune(const uint64_t* keys, uint64_t n, cpma_mem mem, const cpma_tune_hint* hint_in,
                                     const cpma_config* base, void* stream, cpma_config* out,
                                     cpma_tune_report* report) {
  if (!out || n == 0 || !keys) return CPMA_ERR_INVALID;
  cpma_config cfg;
  cpma_config_default(&cfg);
  if (base) {
    if (base->leaf_bytes) cfg.leaf_bytes = base->leaf_bytes;
    if (base->grow > 0) cfg.grow = base->grow;
    if (base->up_leaf > 0) cfg.up_leaf = base->up_leaf;
    if (base->up_root > 0) cfg.up_root = base->up_root;
    if (base->lo_leaf > 0) cfg.lo_leaf = base->lo_leaf;
    if (base->lo_root > 0) cfg.lo_root = base->lo_root;
    cfg.build_density = base->build_density > 0 ? base->build_density : cfg.up_root / cfg.grow;
    if (base->range_chunk) cfg.range_chunk = base->range_chunk;
    if (base->rebuild_frac > 0) cfg.rebuild_frac = base->rebuild_frac;
    if (base->uncompressed || base->values) return CPMA_ERR_INVALID;  // the tuner times key-only CPMA leaves
  }
  cpma_status cs = check_config(cfg);
  if (cs != CPMA_OK) return cs;
  cpma_tune_hint hint{};
  if (hint_in) hint = *hint_in;
  if (!hint.batch) hint.batch = std::max<uint64_t>(1, n / 10);
  if (!hint.range_keys) hint.range_keys = 1000;
  if (!hint.queries) hint.queries = 100000;
  if (!hint.sample_keys) hint.sample_keys = 1ull << 22;
  if (hint.insert_weight < 0) hint.insert_weight = 0.5;
  if (hint.insert_weight > 1) return CPMA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  cpma_tune_report rep{};
  try {
    DevScratch sc;
    const uint64_t* dk = keys;
    if (mem == CPMA_MEM_HOST) {
      uint64_t* d = sc.get<uint64_t>(n);
      HIPCHK(hipMemcpyAsync(d, keys, n * 8, hipMemcpyHostToDevice, st));
      dk = d;
    }
    BatchInfo* di = sc.get<BatchInfo>(1);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(di),
                       (uint64_t)(sizeof(BatchInfo) / 4), 0u);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, dk, n, di);
    HIPCHK(hipGetLastError());
    BatchInfo bi;
    HIPCHK(hipMemcpyAsync(&bi, di, sizeof(bi), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bi.has_reserved) return CPMA_ERR_RESERVED_KEY;
    const int bits = 64 - __builtin_clzll(bi.or_all | 1);
    const long double space = std::ldexp(1.0L, bits);  // keys lie in [0, 2^bits)
    // density-preserving sample: the keys below T
    const uint64_t* sample = dk;
    uint64_t ns = n;
    long double Tl = space;
    if (n > hint.sample_keys) {
      const uint64_t cap = std::min<uint64_t>(n, 4 * hint.sample_keys);
      uint64_t* buf = sc.get<uint64_t>(cap);
      unsigned long long* cnt = sc.get<unsigned long long>(1);
      Tl = space * (long double)hint.sample_keys / (long double)n;
      for (int tries = 0;; tries++) {
        const uint64_t T = (uint64_t)std::min<long double>(Tl, 18446744073709551615.0L);
        hipLaunchKernelGGL((k_fill<uint64_t>), dim3(1), dim3(64), 0, st, (uint64_t*)cnt, (uint64_t)1, 0ull);
        hipLaunchKernelGGL(k_sample_below, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, dk, n, T, buf, cap, cnt);
        HIPCHK(hipGetLastError());
        unsigned long long c = 0;
        HIPCHK(hipMemcpyAsync(&c, cnt, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (c <= cap && (c >= hint.sample_keys / 4 || tries >= 8)) {
          ns = c;
          break;
        }
        if (tries >= 16) throw Fail{CPMA_ERR_DEVICE};
        Tl = (c > cap) ? Tl / 2 : Tl * 2;
      }
      sample = buf;
    }
    if (ns == 0) {
      ns = std::min<uint64_t>(n, hint.sample_keys);
      sample = dk;
      Tl = space;
    }
    const uint64_t T = (uint64_t)std::min<long double>(Tl, 18446744073709551615.0L);
    rep.sample_n = ns;
    const uint64_t kk = std::max<uint64_t>(
        1, (uint64_t)((long double)hint.batch * (long double)ns / (long double)n));
    const uint64_t q = hint.queries;
    const uint64_t width = std::max<uint64_t>(
        1, (uint64_t)((long double)hint.range_keys * (long double)T / (long double)ns));
    uint64_t* ins = sc.get<uint64_t>(kk);
    uint64_t* qlo = sc.get<uint64_t>(q);
    uint64_t* qhi = sc.get<uint64_t>(q);
    uint64_t* qs = sc.get<uint64_t>(q);
    uint64_t* qc = sc.get<uint64_t>(q);
    hipLaunchKernelGGL(k_gen_ranges, dim3(grid_for(q, 256, 4096)), dim3(256), 0, st, qlo, qhi, q, T, width,
                       0x7475ull);
    HIPCHK(hipGetLastError());
    const uint32_t sizes[5] = {256, 512, 1024, 2048, 4096};
    double best_score = 1e300;
    uint32_t bestS = cfg.leaf_bytes;
    for (int c = 0; c < 5; c++) {
      cpma_config tc = cfg;
      tc.leaf_bytes = sizes[c];
      Handle h;
      st_check(cpma_build(sample, ns, CPMA_MEM_DEVICE, &tc, st, &h.h));
      const double ims = time_min(st, 3, [&](int r) {
        hipLaunchKernelGGL(k_gen_uniform, dim3(grid_for(kk, 256, 4096)), dim3(256), 0, st, ins, kk, T,
                           0x1000ull + (uint64_t)r);
        st_check(cpma_insert_batch(h.h, ins, kk, CPMA_MEM_DEVICE, 0, st, nullptr));
      });
      const double rms = time_min(st, 3, [&](int) {
        st_check(cpma_range_map(h.h, qlo, qhi, q, CPMA_MEM_DEVICE, qs, qc, st));
      });
      rep.leaf_bytes[c] = sizes[c];
      rep.insert_ms[c] = ims;
      rep.range_ms[c] = rms;
      const double score = hint.insert_weight * ims + (1.0 - hint.insert_weight) * rms;
      if (score < best_score) {
        best_score = score;
        bestS = sizes[c];
      }
    }
    cfg.leaf_bytes = bestS;
    const uint32_t chunks[6] = {1, 2, 4, 8, 16, 32};
    uint32_t bestC = cfg.range_chunk;
    {
      Handle h;
      st_check(cpma_build(sample, ns, CPMA_MEM_DEVICE, &cfg, st, &h.h));
      double best = 1e300;
      for (int c = 0; c < 6; c++) {
        h.h->cfg.range_chunk = chunks[c];
        const double ms = time_min(st, 3, [&](int) {
          st_check(cpma_range_map(h.h, qlo, qhi, q, CPMA_MEM_DEVICE, qs, qc, st));
        });
        rep.chunk[c] = chunks[c];
        rep.chunk_ms[c] = ms;
        if (ms < best) {
          best = ms;
          bestC = chunks[c];
        }
      }
    }
    cfg.range_chunk = bestC;
    rep.best_leaf_bytes = bestS;
    rep.best_chunk = bestC;
    // rebuild cut-over: the insert batch (and a delete of it) with the full
    // rebuild forced and with the counted path, at the winning leaf size
    {
      const double r = (double)kk / (double)ns;
      double ms2[2];
      for (int v = 0; v < 2; v++) {
        cpma_config tc = cfg;
        tc.rebuild_frac = v == 0 ? std::max(1e-9, 0.5 * r) : 1e30;
        Handle h;
        st_check(cpma_build(sample, ns, CPMA_MEM_DEVICE, &tc, st, &h.h));
        ms2[v] = time_min(st, 3, [&](int rr) {
          hipLaunchKernelGGL(k_gen_uniform, dim3(grid_for(kk, 256, 4096)), dim3(256), 0, st, ins, kk, T,
                             0x2000ull + (uint64_t)rr);
          st_check(cpma_insert_batch(h.h, ins, kk, CPMA_MEM_DEVICE, 0, st, nullptr));
          st_check(cpma_delete_batch(h.h, ins, kk, CPMA_MEM_DEVICE, 0, st, nullptr));
        });
      }
      rep.rebuild_ms = ms2[0];
      rep.batch_path_ms = ms2[1];
      // batches of this relative size rebuild only where that was faster
      cfg.rebuild_frac = ms2[0] < ms2[1] ? std::min(cfg.rebuild_frac, r) : std::max(cfg.rebuild_frac, 2.0 * r);
      rep.best_rebuild_frac = cfg.rebuild_frac;
    }
  } catch (const Fail& e) {
    return e.st;
  }
  *out = cfg;
  if (report) *report = rep;
  return CPMA_OK;
}
