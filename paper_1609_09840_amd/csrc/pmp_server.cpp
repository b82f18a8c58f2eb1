// Serving loop of libpmp: continuous batching of hash requests.
//
// Requests (each a ragged batch of strings of one variant) arrive on any
// thread through pmp_server_submit. One dispatcher thread owns a few
// in-flight positions ("lanes"), each a HIP stream with its own plan and
// device arena. Whenever a lane is free it takes as many queued requests as
// its arena, the in-flight byte budget and the batch limits admit and hashes
// all of them in ONE launch (pmp::run_batches over one descriptor per
// request); while that batch runs on the device, new arrivals queue and go
// out on the next free lane, so batches overlap on the device. Requests
// whose data already sits on the device are hashed in place; host requests
// are staged through the lane's pinned buffer (payload and offsets in,
// hashes out). A completed request's latency (submit to results visible
// where the caller asked for them) is recorded for the p50/p99 report.
//
// Latency: while any lane is busy or any request is queued the dispatcher
// polls the lanes' completion events without sleeping, and when idle it
// keeps polling the queue for a configurable time before it sleeps on a
// condition variable, so a request that arrives at a steady rate meets an
// awake dispatcher and a finished batch is seen within a poll.
//
// Errors found on the device: each launch is followed, on the lane's
// stream, by a copy of the plan's status word into pinned host memory. When
// a batch flagged bad offsets, the lane's status word and node accumulators
// are cleared and every request of the batch is hashed again on its own,
// so that only the requests whose offsets are bad fail (PMP_E_OFFSETS from
// pmp_server_wait) and the others complete with correct outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pmp.h"
#include "pmp_batch.h"
#include "pmp_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_us() {
  return std::chrono::duration<double, std::micro>(Clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket = 0;
  pmp_request r{};
  uint64_t span = 0;         // payload bytes of the request (host requests), for the statistics
  uint64_t stage_bytes = 0;  // arena bytes for payload + offsets (host requests)
  uint64_t out_bytes = 0;
  uint64_t budget_bytes = 0;  // bytes charged against the in-flight budget (device requests)
  double t_submit = 0, t_done = 0;
  int status = 1;  // 1 pending, 0 done, < 0 error
};

uint64_t up16(uint64_t x) { return (x + 15) & ~uint64_t(15); }

struct Lane {
  hipStream_t stream = nullptr;
  pmp_plan* plan = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* d_arena = nullptr;
  uint8_t* h_stage = nullptr;  // pinned, same layout as d_arena
  volatile int32_t* h_status = nullptr;  // pinned copy of the plan's status word after the batch
  uint64_t arena = 0;
  uint64_t inflight = 0;  // device-request bytes of the batch, charged against the budget
  std::vector<Req*> reqs;
  std::vector<pmp_batch> batches;  // descriptors of the launch (kept for an error re-run)
  std::vector<uint64_t> out_at;    // per request: output offset in the arena (host requests)
  std::vector<int> req_status;     // per request: result of the error re-run
  bool busy = false;
};

int fail(int code, const char* msg) { return pmp::set_error(code, msg); }

}  // namespace

struct pmp_server {
  pmp_server_config cfg{};
  std::vector<Lane> lanes;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::atomic<int64_t> queued{0};  // queue length, read without the lock while spinning
  std::atomic<bool> stop{false};
  bool sleeping = false;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  uint64_t inflight = 0;  // device-request bytes in flight over all lanes
  // statistics
  std::vector<double> lat_us;
  uint64_t done_n = 0, rejected = 0, failed = 0, batches = 0, bytes = 0;
  double first_submit = -1, last_done = 0;
};

namespace {

inline void cpu_relax() { __builtin_ia32_pause(); }

// Launch one lane's batch. Called by the dispatcher with the lock released.
int launch_lane(pmp_server* S, Lane& L) {
  const size_t n = L.reqs.size();
  L.batches.assign(n, pmp_batch{});
  std::vector<const pmp_batch*> bp(n);
  uint64_t front = 0, out_lo = L.arena, out_hi = L.arena;
  bool host_any = false;
  L.out_at.assign(n, 0);
  for (size_t k = 0; k < n; ++k) {
    const pmp_request& r = L.reqs[k]->r;
    pmp_batch& x = L.batches[k];
    x.count = r.count;
    x.flags = r.flags;
    x.wide = r.wide;
    x.keys = r.wide ? (const void*)S->cfg.d_keys64 : (const void*)S->cfg.d_keys32;
    x.buf_bytes = r.buf_bytes;
    if (r.device_resident) {
      x.buf = r.buf;
      x.offsets = r.offsets;
      x.out = r.out;
    } else {
      host_any = true;
      // payload, then offsets, from the front; outputs from the back
      std::memcpy(L.h_stage + front, r.buf, r.buf_bytes);
      x.buf = L.d_arena + front;
      front += up16(r.buf_bytes);
      std::memcpy(L.h_stage + front, r.offsets, (size_t)(r.count + 1) * 8);
      x.offsets = (const int64_t*)(L.d_arena + front);
      front += up16((uint64_t)(r.count + 1) * 8);
      out_lo -= up16(L.reqs[k]->out_bytes);
      L.out_at[k] = out_lo;
      x.out = L.d_arena + out_lo;
    }
    bp[k] = &x;
  }
  hipError_t e = hipSuccess;
  if (host_any && front) e = hipMemcpyAsync(L.d_arena, L.h_stage, front, hipMemcpyHostToDevice, L.stream);
  if (e != hipSuccess) return PMP_E_HIP;
  int rc = pmp::run_batches(L.plan, bp.data(), (int)n, L.stream);
  if (rc) return rc;
  e = hipMemcpyAsync((void*)L.h_status, pmp::plan_status_word(L.plan), sizeof(int32_t), hipMemcpyDeviceToHost, L.stream);
  if (e == hipSuccess && host_any && out_hi > out_lo)
    e = hipMemcpyAsync(L.h_stage + out_lo, L.d_arena + out_lo, out_hi - out_lo, hipMemcpyDeviceToHost, L.stream);
  if (e == hipSuccess) e = hipEventRecord(L.done, L.stream);
  return e == hipSuccess ? PMP_OK : PMP_E_HIP;
}

// After a batch that flagged bad offsets: clear the lane's status word and
// node accumulators, then hash each request of the batch on its own and
// keep its own status. Synchronous on the lane's stream; called with the
// lock released. Host requests re-use the payload already in the arena and
// their outputs are copied back afterwards.
void rerun_alone(Lane& L) {
  const size_t n = L.reqs.size();
  L.req_status.assign(n, PMP_OK);
  if (pmp::plan_clear_async(L.plan, L.stream) != PMP_OK) {
    L.req_status.assign(n, PMP_E_HIP);
    *L.h_status = 0;
    return;
  }
  for (size_t k = 0; k < n; ++k) {
    const pmp_batch* one = &L.batches[k];
    int rc = pmp::run_batches(L.plan, &one, 1, L.stream);
    hipError_t e = hipSuccess;
    if (rc == PMP_OK)
      e = hipMemcpyAsync((void*)L.h_status, pmp::plan_status_word(L.plan), sizeof(int32_t), hipMemcpyDeviceToHost,
                         L.stream);
    if (rc == PMP_OK && e == hipSuccess) e = hipStreamSynchronize(L.stream);
    if (rc == PMP_OK && e != hipSuccess) rc = PMP_E_HIP;
    if (rc == PMP_OK && *L.h_status) {
      rc = (*L.h_status & pmp::STATUS_OFFSETS) ? PMP_E_OFFSETS : PMP_E_INTERNAL;
      if (pmp::plan_clear_async(L.plan, L.stream) != PMP_OK) rc = PMP_E_HIP;
    }
    L.req_status[k] = rc;
  }
  uint64_t lo = L.arena;
  for (size_t k = 0; k < n; ++k)
    if (!L.reqs[k]->r.device_resident) lo = std::min(lo, L.out_at[k]);
  hipError_t e = hipSuccess;
  if (lo < L.arena) e = hipMemcpyAsync(L.h_stage + lo, L.d_arena + lo, L.arena - lo, hipMemcpyDeviceToHost, L.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L.stream);
  *L.h_status = 0;
  if (e != hipSuccess)
    for (int& s : L.req_status)
      if (s == PMP_OK) s = PMP_E_HIP;
}

// Finish a lane whose event has completed: copy host outputs, time stamps,
// per-request status (rc for all, or the per-request results of a re-run).
void finish_lane(pmp_server* S, Lane& L, int rc, bool per_request) {
  const double t = now_us();
  for (size_t k = 0; k < L.reqs.size(); ++k) {
    Req* q = L.reqs[k];
    const int st = per_request ? L.req_status[k] : rc;
    if (st == PMP_OK && !q->r.device_resident) std::memcpy(q->r.out, L.h_stage + L.out_at[k], q->out_bytes);
    q->t_done = t;
    q->status = st;
    if (st == PMP_OK) {
      S->lat_us.push_back(t - q->t_submit);
      S->done_n++;
      S->bytes += q->r.device_resident ? q->r.buf_bytes : q->span;
      S->last_done = t;
    } else {
      S->failed++;
    }
  }
  S->inflight -= L.inflight;
  L.inflight = 0;
  L.reqs.clear();
  L.busy = false;
}

// Take queued requests into lane L while they fit. Returns how many.
size_t admit(pmp_server* S, Lane& L) {
  uint64_t used = 0, dev_bytes = 0;
  int64_t strings = 0;
  while (!S->queue.empty() && (int)L.reqs.size() < S->cfg.max_requests_per_batch) {
    Req* q = S->queue.front();
    if (!q->r.device_resident && used + q->stage_bytes + up16(q->out_bytes) > L.arena) break;
    if (S->cfg.max_inflight_bytes && S->inflight + dev_bytes + q->budget_bytes > S->cfg.max_inflight_bytes) break;
    if (!L.reqs.empty() && S->cfg.max_batch_strings > 0 && strings + q->r.count > S->cfg.max_batch_strings) break;
    if (!q->r.device_resident) used += q->stage_bytes + up16(q->out_bytes);
    dev_bytes += q->budget_bytes;
    strings += q->r.count;
    L.reqs.push_back(q);
    S->queue.pop_front();
    S->queued.fetch_sub(1, std::memory_order_relaxed);
  }
  L.inflight = dev_bytes;
  S->inflight += dev_bytes;
  return L.reqs.size();
}

void dispatcher(pmp_server* S) {
  (void)hipSetDevice(S->cfg.device);
  const double spin_us = S->cfg.idle_spin_us;
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    // 1. retire lanes whose batch is complete
    bool any_busy = false, retired = false;
    for (Lane& L : S->lanes) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      retired = true;
      if (q != hipSuccess) {
        finish_lane(S, L, PMP_E_HIP, false);
      } else if (*L.h_status != 0) {
        lk.unlock();
        rerun_alone(L);
        lk.lock();
        finish_lane(S, L, PMP_OK, true);
      } else {
        finish_lane(S, L, PMP_OK, false);
      }
    }
    if (retired) S->cv_done.notify_all();
    if (S->stop.load() && S->queue.empty() && !any_busy) break;
    // 2. admit queued requests into a free lane
    Lane* free_lane = nullptr;
    for (Lane& L : S->lanes)
      if (!L.busy) {
        free_lane = &L;
        break;
      }
    if (free_lane && !S->queue.empty() && admit(S, *free_lane)) {
      Lane& L = *free_lane;
      L.busy = true;
      S->batches++;
      lk.unlock();
      const int rc = launch_lane(S, L);
      lk.lock();
      if (rc != PMP_OK) {
        finish_lane(S, L, rc, false);
        S->cv_done.notify_all();
      }
      continue;
    }
    // 3. work outstanding: poll again without sleeping
    if (any_busy || !S->queue.empty()) {
      lk.unlock();
      for (int i = 0; i < 32; ++i) cpu_relax();
      lk.lock();
      continue;
    }
    // 4. idle: watch the queue for a while, then sleep until work arrives
    if (spin_us > 0) {
      lk.unlock();
      const double t0 = now_us();
      while (S->queued.load(std::memory_order_relaxed) == 0 && !S->stop.load() && now_us() - t0 < spin_us)
        for (int i = 0; i < 32; ++i) cpu_relax();
      lk.lock();
      if (!S->queue.empty() || S->stop.load()) continue;
    }
    S->sleeping = true;
    S->cv_work.wait(lk, [&] { return S->stop.load() || !S->queue.empty(); });
    S->sleeping = false;
  }
}

void release(pmp_server* S) {
  for (Lane& L : S->lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.d_arena) (void)hipFree(L.d_arena);
    if (L.h_stage) (void)hipHostFree(L.h_stage);
    if (L.h_status) (void)hipHostFree((void*)L.h_status);
    if (L.plan) (void)pmp_plan_destroy(L.plan);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
}

// Host offsets must be in order and inside the payload (device-resident
// offsets are checked by the kernel).
bool host_offsets_ok(const pmp_request* r) {
  if (r->count <= 0) return true;
  const int64_t* o = r->offsets;
  if (o[0] < 0) return false;
  for (int64_t i = 0; i < r->count; ++i)
    if (o[i + 1] < o[i]) return false;
  return (uint64_t)o[r->count] <= r->buf_bytes;
}

}  // namespace

extern "C" {

int pmp_server_create(const pmp_server_config* cfg, pmp_server** out) {
  if (!cfg || !out || cfg->lanes < 1 || cfg->lanes > 16 || !cfg->d_keys32 || !cfg->d_keys64 ||
      cfg->max_requests_per_batch < 1 || cfg->idle_spin_us < 0 || cfg->idle_spin_us > 1000000)
    return fail(PMP_E_INVALID_ARG, "bad server configuration");
  hipError_t e = hipSetDevice(cfg->device);
  if (e != hipSuccess) return fail(PMP_E_HIP, "hipSetDevice");
  pmp_server* S = new pmp_server();
  S->cfg = *cfg;
  S->lanes.resize(cfg->lanes);
  // each lane's plan is sized once for the most a lane can hold, so that no
  // launch of the loop allocates
  uint64_t reserve = cfg->reserve_bytes;
  if (cfg->max_inflight_bytes) reserve = std::max(reserve, cfg->max_inflight_bytes);
  if (cfg->lane_bytes) reserve = std::max(reserve, cfg->lane_bytes);
  for (Lane& L : S->lanes) {
    L.arena = cfg->lane_bytes;
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess ||
        pmp_plan_create(cfg->device, &L.plan) != PMP_OK ||
        hipHostMalloc((void**)&L.h_status, sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        (L.arena && hipMalloc(&L.d_arena, L.arena) != hipSuccess) ||
        (L.arena && hipHostMalloc((void**)&L.h_stage, L.arena, hipHostMallocDefault) != hipSuccess)) {
      release(S);
      return fail(PMP_E_NOMEM, "server lane allocation failed");
    }
    *L.h_status = 0;
    // each request of a launch rounds its workspace up by at most 3 slots of 512 bytes
    if (reserve) (void)pmp_plan_reserve(L.plan, reserve + 1536 * (uint64_t)cfg->max_requests_per_batch, 0);
  }
  S->th = std::thread(dispatcher, S);
  *out = S;
  return PMP_OK;
}

int pmp_server_submit(pmp_server* S, const pmp_request* r, uint64_t* ticket) {
  if (!S || !r || !ticket || r->count < 0 || r->wide > 1 || (r->flags & ~(PMP_NO_MIX | PMP_OUT_FIELD)))
    return fail(PMP_E_INVALID_ARG, "bad request");
  if (r->count > 0 && (!r->offsets || !r->out || (!r->buf && r->buf_bytes)))
    return fail(PMP_E_INVALID_ARG, "request pointers missing");
  if (!r->device_resident && !host_offsets_ok(r))
    return fail(PMP_E_OFFSETS, "request offsets out of order or past buf_bytes");
  Req* q = new Req();
  q->r = *r;
  const uint64_t osz = (r->flags & PMP_OUT_FIELD) ? (r->wide ? 16 : 8) : (r->wide ? 8 : 4);
  q->out_bytes = osz * (uint64_t)r->count;
  const char* refuse = nullptr;
  if (!r->device_resident) {
    if (r->count > 0) q->span = (uint64_t)(r->offsets[r->count] - r->offsets[0]);
    q->stage_bytes = up16(r->buf_bytes) + up16((uint64_t)(r->count + 1) * 8);
    if (q->stage_bytes + up16(q->out_bytes) > S->cfg.lane_bytes) refuse = "request larger than a lane's arena";
  } else {
    q->budget_bytes = r->buf_bytes;
    if (S->cfg.max_inflight_bytes && q->budget_bytes > S->cfg.max_inflight_bytes)
      refuse = "request larger than the in-flight byte budget";
  }
  if (refuse) {  // can never be admitted
    delete q;
    std::lock_guard<std::mutex> lk(S->mu);
    S->rejected++;
    return fail(PMP_E_NOMEM, refuse);
  }
  q->t_submit = now_us();
  bool wake = false;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop.load()) {
      delete q;
      return fail(PMP_E_INVALID_ARG, "server is stopping");
    }
    q->ticket = S->next_ticket++;
    if (S->first_submit < 0) S->first_submit = q->t_submit;
    S->reqs[q->ticket] = q;
    S->queue.push_back(q);
    S->queued.fetch_add(1, std::memory_order_relaxed);
    *ticket = q->ticket;
    wake = S->sleeping;
  }
  if (wake) S->cv_work.notify_one();
  return PMP_OK;
}

int pmp_server_wait(pmp_server* S, uint64_t ticket, int64_t timeout_us) {
  if (!S) return fail(PMP_E_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(PMP_E_INVALID_ARG, "unknown ticket");
  Req* q = it->second;
  auto ready = [&] { return q->status != 1; };
  if (timeout_us < 0) S->cv_done.wait(lk, ready);
  else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return 1;
  const int st = q->status;
  S->reqs.erase(it);
  delete q;
  if (st == PMP_E_OFFSETS) return fail(PMP_E_OFFSETS, "request offsets out of order or past buf_bytes");
  return st;
}

int pmp_server_stats(pmp_server* S, pmp_server_report* st) {
  if (!S || !st) return fail(PMP_E_INVALID_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(st, 0, sizeof *st);
  st->completed = S->done_n;
  st->rejected = S->rejected;
  st->batches = S->batches;
  st->bytes = S->bytes;
  st->failed = S->failed;
  if (!S->lat_us.empty()) {
    std::vector<double> v = S->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[(size_t)std::min<double>(v.size() - 1, p * (v.size() - 1) + 0.5)]; };
    st->p50_us = pct(0.50);
    st->p99_us = pct(0.99);
    st->max_us = v.back();
    double s = 0;
    for (double x : v) s += x;
    st->mean_us = s / v.size();
    st->span_us = S->last_done - S->first_submit;
  }
  return PMP_OK;
}

int pmp_server_reset_stats(pmp_server* S) {
  if (!S) return fail(PMP_E_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  S->lat_us.clear();
  S->done_n = S->batches = S->bytes = S->rejected = S->failed = 0;
  S->first_submit = -1;
  S->last_done = 0;
  return PMP_OK;
}

int pmp_server_replay(pmp_server* S, const pmp_request* reqs, int64_t n, const double* arrival_us,
                      double* latency_us) {
  if (!S || n < 0 || (n > 0 && (!reqs || !arrival_us))) return fail(PMP_E_INVALID_ARG, "bad arguments");
  std::vector<uint64_t> tickets(n);
  const double t0 = now_us();
  for (int64_t k = 0; k < n; ++k) {
    // sleep through long gaps, spin the last stretch for an exact arrival
    const double gap = arrival_us[k] - (now_us() - t0);
    if (gap > 200) std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(gap - 100)));
    while (now_us() - t0 < arrival_us[k]) {
    }
    const int rc = pmp_server_submit(S, reqs + k, &tickets[k]);
    if (rc) return rc;
  }
  int worst = PMP_OK;
  for (int64_t k = 0; k < n; ++k) {
    double lat = -1;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      auto it = S->reqs.find(tickets[k]);
      if (it != S->reqs.end()) {
        Req* q = it->second;
        S->cv_done.wait(lk, [&] { return q->status != 1; });
        lat = q->t_done - q->t_submit;
      }
    }
    const int rc = pmp_server_wait(S, tickets[k], -1);
    if (rc < 0) worst = rc;
    if (latency_us) latency_us[k] = lat;
  }
  return worst;
}

int pmp_server_status(pmp_server* S) {
  if (!S) return fail(PMP_E_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] {
    if (!S->queue.empty()) return false;
    for (const Lane& L : S->lanes)
      if (L.busy) return false;
    return true;
  });
  int worst = PMP_OK;
  for (Lane& L : S->lanes) {
    const int rc = pmp_plan_status(L.plan, (pmp_stream_t)L.stream);
    if (rc != PMP_OK && worst == PMP_OK) worst = rc;
  }
  return worst;
}

int pmp_server_destroy(pmp_server* S) {
  if (!S) return PMP_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop.store(true);
  }
  S->cv_work.notify_all();
  if (S->th.joinable()) S->th.join();
  release(S);
  return PMP_OK;
}

}  // extern "C"
