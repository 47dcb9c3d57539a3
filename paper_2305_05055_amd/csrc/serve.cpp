// Serving loop over one CPMA (declarations in include/cpma.h).
//
// A worker thread owns the set as its single writer.  Requests queue in arrival
// order; each step admits the longest prefix of the queue that fits the slot
// cap and the in-flight HBM budget, runs all admitted range requests as one
// batched range_map launch (they see the state left by earlier steps), then
// applies the admitted inserts and deletes in arrival order with one fused
// call (one sort of all their keys, net delete and insert batches).  Updates and
// queries are thereby phased as in the paper's F-Graph (a single writer, no
// locks on the structure).
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "cpma.h"

struct cpma_server {
  cpma* set = nullptr;
  uint64_t budget = 0;
  uint32_t slots = 0;
  std::mutex m;
  std::condition_variable cv;
  std::deque<cpma_request*> q;
  bool stopping = false;
  uint64_t steps = 0;
  std::thread worker;
  std::vector<uint64_t> lo, hi, sum, cnt;  // fused range batch (host)
  std::vector<const uint64_t*> ukeys;  // fused update batch (host)
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

void run_step(cpma_server* s, const std::vector<cpma_request*>& step) {
  const uint64_t id = s->steps++;
  // 1. every range request of the step in one launch
  uint64_t total = 0;
  for (cpma_request* r : step)
    if (r->kind == CPMA_REQ_RANGE) total += r->n;
  if (total) {
    s->lo.resize(total);
    s->hi.resize(total);
    s->sum.resize(total);
    s->cnt.resize(total);
    uint64_t o = 0;
    for (cpma_request* r : step) {
      if (r->kind != CPMA_REQ_RANGE) continue;
      for (uint64_t i = 0; i < r->n; i++) {
        s->lo[o + i] = r->keys[i];
        s->hi[o + i] = r->hi[i];
      }
      o += r->n;
    }
    const cpma_status st = cpma_range_map(s->set, s->lo.data(), s->hi.data(), total, CPMA_MEM_HOST,
                                          s->sum.data(), s->cnt.data(), nullptr);
    o = 0;
    for (cpma_request* r : step) {
      if (r->kind != CPMA_REQ_RANGE) continue;
      for (uint64_t i = 0; i < r->n; i++) {
        r->sum[i] = s->sum[o + i];
        r->count[i] = s->cnt[o + i];
      }
      o += r->n;
      finish(r, st, id);
    }
  } else {
    for (cpma_request* r : step)
      if (r->kind == CPMA_REQ_RANGE) finish(r, CPMA_OK, id);
  }
  // 2. updates in arrival order, as one fused call
  s->ukeys.clear();
  s->un.clear();
  s->ukind.clear();
  std::vector<cpma_request*> ups;
  for (cpma_request* r : step) {
    if (r->kind == CPMA_REQ_RANGE) continue;
    ups.push_back(r);
    s->ukeys.push_back(r->keys);
    s->un.push_back(r->n);
    s->ukind.push_back(r->kind);
  }
  if (ups.empty()) return;
  s->ures.assign(ups.size(), 0);
  const cpma_status st = cpma_apply_updates(s->set, (uint32_t)ups.size(), s->ukind.data(), s->ukeys.data(),
                                            s->un.data(), CPMA_MEM_HOST, s->ures.data(), nullptr);
  for (size_t i = 0; i < ups.size(); i++) {
    ups[i]->result = st == CPMA_OK ? s->ures[i] : 0;
    finish(ups[i], st, id);
  }
}

void work(cpma_server* s) {
  for (;;) {
    std::vector<cpma_request*> step;
    {
      std::unique_lock<std::mutex> lk(s->m);
      s->cv.wait(lk, [&] { return s->stopping || !s->q.empty(); });
      if (s->q.empty()) return;  // stopping and drained
      uint64_t bytes = 0, ukeys = 0;
      while (!s->q.empty() && step.size() < s->slots) {
        cpma_request* r = s->q.front();
        const uint64_t f = footprint(r);
        const uint64_t u = r->kind == CPMA_REQ_RANGE ? 0 : r->n;
        if (!step.empty() && (bytes + f > s->budget || ukeys + u > kMaxStepUpdateKeys)) break;
        bytes += f;
        ukeys += u;
        step.push_back(r);
        s->q.pop_front();
      }
    }
    run_step(s, step);
  }
}

}  // namespace

extern "C" {

cpma_status cpma_server_start(cpma* set, const cpma_server_config* cfg, cpma_server** out) {
  if (!set || !out) return CPMA_ERR_INVALID;
  cpma_server* s = new cpma_server();
  s->set = set;
  s->budget = (cfg && cfg->hbm_budget) ? cfg->hbm_budget : (16ull << 30);
  s->slots = (cfg && cfg->max_slots) ? cfg->max_slots : 4096u;
  s->worker = std::thread(work, s);
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
  {
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stopping) return CPMA_ERR_INVALID;
    s->q.push_back(r);
  }
  s->cv.notify_one();
  return CPMA_OK;
}

cpma_status cpma_server_stop(cpma_server* s, uint64_t* steps_run) {
  if (!s) return CPMA_ERR_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stopping = true;
  }
  s->cv.notify_one();
  s->worker.join();
  if (steps_run) *steps_run = s->steps;
  delete s;
  return CPMA_OK;
}

}  // extern "C"
