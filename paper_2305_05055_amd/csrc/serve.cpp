// Serving loop over one CPMA (declarations in include/cpma.h).
//
// Continuous batching with two threads and two staging slots:
//  - the stager admits queued requests in arrival order while the in-flight
//    HBM footprint and the number of requests in flight allow, and uploads
//    each admitted request's data into the open slot on its own stream (the
//    next step is filled while the current one runs on the device);
//  - the executor, the set's single writer, takes the open slot as soon as it
//    is free, runs all of the step's range requests as one batched range_map
//    (they see the state left by earlier steps) and then the step's inserts
//    and deletes in arrival order as one fused update call, and finishes each
//    request, which returns its footprint and slot to the admission budget.
// Updates and queries are thereby phased per step as in the paper's F-Graph (a
// single writer, no locks on the structure), and a request that arrives while
// a step is on the GPU is admitted and uploaded at once instead of waiting for
// that step to end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "cpma.h"

namespace {

// Device memory kept across steps; grows, keeping its first `keep` bytes.
struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
};

bool grow(DBuf& b, size_t need, size_t keep, hipStream_t st) {
  if (b.cap >= need) return true;
  const size_t want = std::max(need, 2 * b.cap) + 4096;
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    hipGetLastError();
    return false;
  }
  if (keep && (hipMemcpyAsync(p, b.p, keep, hipMemcpyDeviceToDevice, st) != hipSuccess ||
               hipStreamSynchronize(st) != hipSuccess)) {
    hipFree(p);
    return false;
  }
  if (b.p) hipFree(b.p);
  b.p = p;
  b.cap = want;
  return true;
}

void drop(DBuf& b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

// One step's staged inputs: range bounds and update keys, in device memory.
struct Slot {
  std::vector<cpma_request*> reqs;
  std::vector<uint64_t> off;  // per request: first word of its ranges (lo / hi) or of its keys
  uint64_t nranges = 0, nkeys = 0;
  DBuf dlo, dhi, dkeys;
  hipEvent_t ev = nullptr;  // recorded after the slot's last upload
  int state = 0;            // 0 free, 1 being filled, 2 taken by the executor
  bool uploading = false;
  cpma_status staged = CPMA_OK;  // an upload that failed: the step's requests finish with it
};

}  // namespace

struct cpma_server {
  cpma* set = nullptr;
  uint64_t budget = 0;
  uint32_t slots_cap = 0;
  int device = 0;
  std::mutex m;
  std::condition_variable cv;
  std::deque<cpma_request*> q;
  bool stopping = false;
  uint64_t steps = 0;
  uint64_t inflight_bytes = 0;
  uint32_t inflight_reqs = 0;
  Slot slot[2];
  int filling = -1;  // the slot the stager fills, -1 if none is open
  hipStream_t copy_st = nullptr, exec_st = nullptr;
  std::thread stager, executor;
  // executor scratch
  DBuf dsum, dcnt;
  std::vector<uint64_t> hsum, hcnt;
  std::vector<const uint64_t*> ukeys;
  std::vector<uint64_t> un, ures;
  std::vector<int32_t> ukind;
};

extern "C" uint64_t cpma_clock_ns(void) {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

namespace {

// Device bytes a request occupies while in flight: its inputs and outputs plus
// the per-key scratch of the fused update (key copies, sort buffers with
// positions, per-key flags, leaf segments, overflow room).
uint64_t footprint(const cpma_request* r) {
  return r->kind == CPMA_REQ_RANGE ? 48ull * r->n + 64 : 128ull * r->n + 64;
}

// Keys one fused update call takes (positions are 31-bit).
constexpr uint64_t kMaxStepUpdateKeys = (1ull << 31) - 1;

void finish(cpma_request* r, cpma_status st, uint64_t step) {
  r->status = (int32_t)st;
  r->step = step;
  r->t_done_ns = cpma_clock_ns();
  __atomic_store_n(&r->done, 1, __ATOMIC_RELEASE);
}

// Returns finished requests' footprint and slots to the admission budget.
void release(cpma_server* s, const std::vector<cpma_request*>& rs) {
  uint64_t b = 0;
  for (cpma_request* r : rs) b += footprint(r);
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->inflight_bytes -= b;
    s->inflight_reqs -= (uint32_t)rs.size();
  }
  s->cv.notify_all();
}

// Uploads one admitted request into slot sl (stager thread, outside the lock).
cpma_status upload(cpma_server* s, Slot& sl, cpma_request* r) {
  const size_t n8 = r->n * 8;
  if (r->kind == CPMA_REQ_RANGE) {
    const size_t used = sl.nranges * 8;
    if (!grow(sl.dlo, used + n8, used, s->copy_st) || !grow(sl.dhi, used + n8, used, s->copy_st))
      return CPMA_ERR_NOMEM;
    if (n8 && (hipMemcpyAsync((uint8_t*)sl.dlo.p + used, r->keys, n8, hipMemcpyHostToDevice, s->copy_st) !=
                   hipSuccess ||
               hipMemcpyAsync((uint8_t*)sl.dhi.p + used, r->hi, n8, hipMemcpyHostToDevice, s->copy_st) !=
                   hipSuccess))
      return CPMA_ERR_DEVICE;
    sl.off.push_back(sl.nranges);
    sl.nranges += r->n;
  } else {
    const size_t used = sl.nkeys * 8;
    if (!grow(sl.dkeys, used + n8, used, s->copy_st)) return CPMA_ERR_NOMEM;
    if (n8 && hipMemcpyAsync((uint8_t*)sl.dkeys.p + used, r->keys, n8, hipMemcpyHostToDevice, s->copy_st) !=
                  hipSuccess)
      return CPMA_ERR_DEVICE;
    sl.off.push_back(sl.nkeys);
    sl.nkeys += r->n;
  }
  sl.reqs.push_back(r);
  return CPMA_OK;
}

void stage_loop(cpma_server* s) {
  hipSetDevice(s->device);
  for (;;) {
    std::vector<cpma_request*> adm;
    Slot* sl = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->m);
      auto free_slot = [&] { return s->slot[0].state == 0 ? 0 : (s->slot[1].state == 0 ? 1 : -1); };
      auto admissible = [&] {
        if (s->q.empty()) return false;
        if (s->inflight_reqs == 0) return true;
        return s->inflight_reqs < s->slots_cap && s->inflight_bytes + footprint(s->q.front()) <= s->budget;
      };
      s->cv.wait(lk, [&] {
        return (s->stopping && s->q.empty()) || (admissible() && (s->filling >= 0 || free_slot() >= 0));
      });
      if (s->stopping && s->q.empty()) return;
      if (s->filling < 0) {
        const int f = free_slot();
        Slot& x = s->slot[f];
        x.reqs.clear();
        x.off.clear();
        x.nranges = x.nkeys = 0;
        x.staged = CPMA_OK;
        x.state = 1;
        s->filling = f;
      }
      sl = &s->slot[s->filling];
      while (admissible()) {
        cpma_request* r = s->q.front();
        if (r->kind != CPMA_REQ_RANGE && sl->nkeys + r->n > kMaxStepUpdateKeys && !sl->reqs.empty()) break;
        s->inflight_bytes += footprint(r);
        s->inflight_reqs += 1;
        s->q.pop_front();
        adm.push_back(r);
      }
      sl->uploading = true;
    }
    const uint64_t t = cpma_clock_ns();
    for (cpma_request* r : adm) {
      r->t_admit_ns = t;
      const cpma_status st = upload(s, *sl, r);
      if (st != CPMA_OK && sl->staged == CPMA_OK) sl->staged = st;
      if (st != CPMA_OK) {
        sl->reqs.push_back(r);
        sl->off.push_back(0);
      }
    }
    hipEventRecord(sl->ev, s->copy_st);
    {
      std::lock_guard<std::mutex> lk(s->m);
      sl->uploading = false;
    }
    s->cv.notify_all();
  }
}

void run_step(cpma_server* s, Slot& sl, uint64_t id) {
  hipStreamWaitEvent(s->exec_st, sl.ev, 0);
  if (sl.staged != CPMA_OK) {
    for (cpma_request* r : sl.reqs) finish(r, sl.staged, id);
    release(s, sl.reqs);
    return;
  }
  // 1. every range request of the step in one launch
  std::vector<cpma_request*> done;
  if (sl.nranges) {
    cpma_status st = CPMA_OK;
    if (!grow(s->dsum, sl.nranges * 8, 0, s->exec_st) || !grow(s->dcnt, sl.nranges * 8, 0, s->exec_st))
      st = CPMA_ERR_NOMEM;
    s->hsum.resize(sl.nranges);
    s->hcnt.resize(sl.nranges);
    if (st == CPMA_OK)
      st = cpma_range_map(s->set, (const uint64_t*)sl.dlo.p, (const uint64_t*)sl.dhi.p, sl.nranges,
                          CPMA_MEM_DEVICE, (uint64_t*)s->dsum.p, (uint64_t*)s->dcnt.p, s->exec_st);
    if (st == CPMA_OK &&
        (hipMemcpyAsync(s->hsum.data(), s->dsum.p, sl.nranges * 8, hipMemcpyDeviceToHost, s->exec_st) !=
             hipSuccess ||
         hipMemcpyAsync(s->hcnt.data(), s->dcnt.p, sl.nranges * 8, hipMemcpyDeviceToHost, s->exec_st) !=
             hipSuccess ||
         hipStreamSynchronize(s->exec_st) != hipSuccess))
      st = CPMA_ERR_DEVICE;
    for (size_t i = 0; i < sl.reqs.size(); i++) {
      cpma_request* r = sl.reqs[i];
      if (r->kind != CPMA_REQ_RANGE) continue;
      if (st == CPMA_OK)
        for (uint64_t j = 0; j < r->n; j++) {
          r->sum[j] = s->hsum[sl.off[i] + j];
          r->count[j] = s->hcnt[sl.off[i] + j];
        }
      finish(r, st, id);
      done.push_back(r);
    }
  } else {
    for (cpma_request* r : sl.reqs)
      if (r->kind == CPMA_REQ_RANGE) {
        finish(r, CPMA_OK, id);
        done.push_back(r);
      }
  }
  release(s, done);
  // 2. updates in arrival order, as one fused call
  s->ukeys.clear();
  s->un.clear();
  s->ukind.clear();
  std::vector<cpma_request*> ups;
  for (size_t i = 0; i < sl.reqs.size(); i++) {
    cpma_request* r = sl.reqs[i];
    if (r->kind == CPMA_REQ_RANGE) continue;
    ups.push_back(r);
    s->ukeys.push_back((const uint64_t*)sl.dkeys.p + sl.off[i]);
    s->un.push_back(r->n);
    s->ukind.push_back(r->kind);
  }
  if (ups.empty()) return;
  s->ures.assign(ups.size(), 0);
  const cpma_status st = cpma_apply_updates(s->set, (uint32_t)ups.size(), s->ukind.data(), s->ukeys.data(),
                                            s->un.data(), CPMA_MEM_DEVICE, s->ures.data(), s->exec_st);
  for (size_t i = 0; i < ups.size(); i++) {
    ups[i]->result = st == CPMA_OK ? s->ures[i] : 0;
    finish(ups[i], st, id);
  }
  release(s, ups);
}

void exec_loop(cpma_server* s) {
  hipSetDevice(s->device);
  for (;;) {
    int si;
    {
      std::unique_lock<std::mutex> lk(s->m);
      auto ready = [&] {
        return s->filling >= 0 && !s->slot[s->filling].reqs.empty() && !s->slot[s->filling].uploading;
      };
      s->cv.wait(lk, [&] {
        return ready() || (s->stopping && s->q.empty() &&
                           (s->filling < 0 || (s->slot[s->filling].reqs.empty() && !s->slot[s->filling].uploading)));
      });
      if (!ready()) return;  // stopping and drained
      si = s->filling;
      s->filling = -1;
      s->slot[si].state = 2;
    }
    s->cv.notify_all();  // the stager may open the other slot
    run_step(s, s->slot[si], s->steps++);
    {
      std::lock_guard<std::mutex> lk(s->m);
      s->slot[si].state = 0;
    }
    s->cv.notify_all();
  }
}

}  // namespace

extern "C" {

cpma_status cpma_server_start(cpma* set, const cpma_server_config* cfg, cpma_server** out) {
  if (!set || !out) return CPMA_ERR_INVALID;
  cpma_server* s = new cpma_server();
  s->set = set;
  s->budget = (cfg && cfg->hbm_budget) ? cfg->hbm_budget : (16ull << 30);
  s->slots_cap = (cfg && cfg->max_slots) ? cfg->max_slots : 4096u;
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->copy_st, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->exec_st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->slot[0].ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->slot[1].ev, hipEventDisableTiming) != hipSuccess) {
    hipGetLastError();
    if (s->copy_st) hipStreamDestroy(s->copy_st);
    if (s->exec_st) hipStreamDestroy(s->exec_st);
    for (Slot& x : s->slot)
      if (x.ev) hipEventDestroy(x.ev);
    delete s;
    return CPMA_ERR_DEVICE;
  }
  s->executor = std::thread(exec_loop, s);
  s->stager = std::thread(stage_loop, s);
  *out = s;
  return CPMA_OK;
}

cpma_status cpma_server_submit(cpma_server* s, cpma_request* r) {
  if (!s || !r) return CPMA_ERR_INVALID;
  if (r->kind < CPMA_REQ_RANGE || r->kind > CPMA_REQ_DELETE) return CPMA_ERR_INVALID;
  if (r->n && (!r->keys || (r->kind == CPMA_REQ_RANGE && (!r->hi || !r->sum || !r->count))))
    return CPMA_ERR_INVALID;
  r->done = 0;
  r->status = CPMA_OK;
  r->result = 0;
  r->t_admit_ns = 0;
  {
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stopping) return CPMA_ERR_INVALID;
    s->q.push_back(r);
  }
  s->cv.notify_all();
  return CPMA_OK;
}

cpma_status cpma_server_stop(cpma_server* s, uint64_t* steps_run) {
  if (!s) return CPMA_ERR_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stopping = true;
  }
  s->cv.notify_all();
  s->stager.join();
  {
    std::lock_guard<std::mutex> lk(s->m);  // wakes the executor once the stager is gone
  }
  s->cv.notify_all();
  s->executor.join();
  if (steps_run) *steps_run = s->steps;
  hipStreamSynchronize(s->copy_st);
  hipStreamSynchronize(s->exec_st);
  for (Slot& x : s->slot) {
    drop(x.dlo);
    drop(x.dhi);
    drop(x.dkeys);
    hipEventDestroy(x.ev);
  }
  drop(s->dsum);
  drop(s->dcnt);
  hipStreamDestroy(s->copy_st);
  hipStreamDestroy(s->exec_st);
  delete s;
  return CPMA_OK;
}

}  // extern "C"
