// Continuous-batching request server.
//
// A worker thread owns `slots` HIP streams. Submitted requests wait in a FIFO;
// the head is admitted while the bytes it needs (its data plus, for
// multi-pass sizes, an equal scratch region) fit the HBM budget next to the
// resident tables. Whenever a stream is free, every admitted request not yet
// launched is generated on the device from (seed, request id) and
// transformed in ONE persistent batch launch (uneven sizes and mixed kinds)
// on that stream; completion is observed through an event. Requests that
// arrive while batches run are admitted as memory frees up and launched on
// the next free stream, so their work overlaps with the running batches.
// Results are bit-identical to a lone transform: every job's arithmetic is
// independent of what shares its launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "frntt_internal.hpp"

namespace frntt {

int batch_impl_ws(frntt_ctx* ctx, const frntt_job* jobs, void* const* scratch, const JobPlan* plans, int n_jobs,
                  hipStream_t stream);

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id;
  int kind;
  int log_n;
  uint64_t seed;
  Clock::time_point t_submit;
  Clock::time_point t_done;
  JobPlan jp;           // algorithm and plan, fixed at submission
  size_t need = 0;      // data bytes, plus scratch bytes if the plan has several passes
  void* buf = nullptr;  // data, then scratch
  size_t bytes = 0;
  int state = 0;        // 0 queued, 1 admitted, 2 launched, 3 done, 4 released, 5 cancelled
};

struct InFlight {
  int slot;
  hipEvent_t event;
  std::vector<uint64_t> ids;
};

// Device bytes of a request: its data, and an equal scratch region when its
// plan has more than one pass (passes alternate between the two).
size_t request_bytes(int log_n, const Plan& plan) {
  return ((size_t)32 << log_n) + scratch_bytes_for(log_n, 1, plan.n_pass);
}

}  // namespace

}  // namespace frntt

struct frntt_server {
  frntt_ctx* ctx = nullptr;
  size_t budget = 0;
  size_t in_use = 0;       // bytes held by admitted, unreleased requests
  size_t pool_bytes = 0;   // bytes allocated in the pool (used or free)
  size_t peak = 0;
  int n_slots = 0;
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  std::mutex mu;
  std::condition_variable cv;        // wakes the worker
  std::condition_variable cv_done;   // wakes drain()
  std::deque<uint64_t> queue;        // submitted, not admitted
  std::deque<uint64_t> admitted;     // admitted, not launched
  std::unordered_map<uint64_t, frntt::Request> reqs;
  std::map<size_t, std::vector<void*>> free_bufs;  // pool by buffer size
  std::vector<frntt::InFlight> inflight;
  uint64_t next_id = 1;
  uint64_t completed = 0, batches = 0;
  uint64_t inflight_requests = 0;    // launched, not yet complete
  uint64_t peak_inflight_batches = 0, peak_inflight_requests = 0;
  uint64_t outstanding = 0;          // submitted and not done
  bool release_on_done = false;      // recycle buffers as soon as a request completes
  bool stalled = false;              // queue head cannot be admitted and nothing runs
  bool stop = false;
  int error = 0;
  std::thread worker;
};

namespace frntt {

namespace {

// Take a buffer for `log_n` from the pool (allocating if needed) while the
// budget allows; called with the lock held.
bool take_buffer(frntt_server* s, Request& r) {
  const size_t need = r.need;
  if (s->in_use + need + s->ctx->table_bytes > s->budget) return false;
  auto& fl = s->free_bufs[need];
  void* p = nullptr;
  if (!fl.empty()) {
    p = fl.back();
    fl.pop_back();
  } else {
    // drop cached buffers of other sizes if the pool itself would exceed the budget
    while (s->pool_bytes + need + s->ctx->table_bytes > s->budget) {
      bool freed = false;
      for (auto& kv : s->free_bufs)
        if (!kv.second.empty()) {
          hipFree(kv.second.back());
          kv.second.pop_back();
          s->pool_bytes -= kv.first;
          freed = true;
          break;
        }
      if (!freed) break;
    }
    if (hipMalloc(&p, need) != hipSuccess) return false;
    s->pool_bytes += need;
  }
  r.buf = p;
  r.bytes = need;
  s->in_use += need;
  if (s->in_use > s->peak) s->peak = s->in_use;
  return true;
}

void give_back(frntt_server* s, Request& r) {
  if (!r.buf) return;
  s->free_bufs[r.bytes].push_back(r.buf);
  s->in_use -= r.bytes;
  r.buf = nullptr;
  r.bytes = 0;
}

void worker_main(frntt_server* s) {
  hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // 1. admission in arrival order
    while (!s->queue.empty()) {
      Request& r = s->reqs[s->queue.front()];
      if (!take_buffer(s, r)) break;
      r.state = 1;
      s->admitted.push_back(r.id);
      s->queue.pop_front();
    }
    // 2. launch everything admitted on a free stream
    int slot = -1;
    for (int i = 0; i < s->n_slots; ++i)
      if (!s->slot_busy[(size_t)i]) {
        slot = i;
        break;
      }
    if (slot >= 0 && !s->admitted.empty()) {
      std::vector<frntt_job> jobs;
      std::vector<void*> scratch;
      std::vector<JobPlan> plans;
      std::vector<uint64_t> ids;
      hipStream_t st = s->streams[(size_t)slot];
      while (!s->admitted.empty()) {
        Request& r = s->reqs[s->admitted.front()];
        s->admitted.pop_front();
        const uint64_t n = 1ull << r.log_n;
        frntt_generate(s->ctx, r.buf, r.seed, r.id, 0, n, st);
        jobs.push_back({r.buf, r.log_n, r.kind});
        const size_t data = (size_t)32 << r.log_n;
        scratch.push_back(r.need > data ? (uint8_t*)r.buf + data : nullptr);
        plans.push_back(r.jp);
        ids.push_back(r.id);
        r.state = 2;
      }
      lk.unlock();
      int rc = batch_impl_ws(s->ctx, jobs.data(), scratch.data(), plans.data(), (int)jobs.size(), st);
      hipEvent_t ev = nullptr;
      if (rc == FRNTT_OK && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) rc = FRNTT_EHIP;
      if (rc == FRNTT_OK && hipEventRecord(ev, st) != hipSuccess) rc = FRNTT_EHIP;
      lk.lock();
      if (rc != FRNTT_OK) {
        s->error = rc;
        if (ev) hipEventDestroy(ev);
        for (uint64_t id : ids) {  // fail them as done so waiters return
          Request& r = s->reqs[id];
          r.state = 3;
          r.t_done = Clock::now();
          --s->outstanding;
        }
        s->cv_done.notify_all();
      } else {
        s->slot_busy[(size_t)slot] = true;
        s->inflight.push_back({slot, ev, ids});
        ++s->batches;
        s->inflight_requests += ids.size();
        s->peak_inflight_batches = std::max<uint64_t>(s->peak_inflight_batches, s->inflight.size());
        s->peak_inflight_requests = std::max(s->peak_inflight_requests, s->inflight_requests);
      }
      continue;
    }
    // 3. completions
    bool any = false;
    for (size_t i = 0; i < s->inflight.size();) {
      InFlight& f = s->inflight[i];
      if (hipEventQuery(f.event) == hipSuccess) {
        const auto now = Clock::now();
        for (uint64_t id : f.ids) {
          Request& r = s->reqs[id];
          r.state = 3;
          r.t_done = now;
          ++s->completed;
          --s->outstanding;
          if (s->release_on_done) give_back(s, r);
        }
        hipEventDestroy(f.event);
        s->inflight_requests -= f.ids.size();
        s->slot_busy[(size_t)f.slot] = false;
        s->inflight.erase(s->inflight.begin() + (long)i);
        any = true;
      } else {
        ++i;
      }
    }
    if (any) {
      s->cv_done.notify_all();
      continue;
    }
    if (s->stop) {
      // requests never admitted are cancelled; running ones finish first
      while (!s->queue.empty()) {
        Request& r = s->reqs[s->queue.front()];
        r.state = 5;
        --s->outstanding;
        s->queue.pop_front();
      }
      if (s->inflight.empty() && s->admitted.empty()) break;
    }
    // nothing runs, nothing is ready, and the queue head does not fit: only
    // the client releasing finished results can make progress
    const bool st = !s->queue.empty() && s->inflight.empty() && s->admitted.empty();
    if (st != s->stalled) {
      s->stalled = st;
      if (st) s->cv_done.notify_all();
    }
    if (!s->inflight.empty()) {
      // poll the device at a fine grain while work is in flight
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      s->cv.wait_for(lk, std::chrono::milliseconds(50));
    }
  }
}

}  // namespace

}  // namespace frntt

using namespace frntt;

extern "C" {

int frntt_server_create(frntt_server** out, frntt_ctx* ctx, size_t hbm_budget_bytes, int slots) {
  if (!out || !ctx || slots < 1 || slots > 16) return FRNTT_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes <= ctx->table_bytes) return FRNTT_EINVAL;
  frntt_server* s = new (std::nothrow) frntt_server();
  if (!s) return FRNTT_ENOMEM;
  s->ctx = ctx;
  s->budget = hbm_budget_bytes;
  s->n_slots = slots;
  hipSetDevice(ctx->device);
  for (int i = 0; i < slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) hipStreamDestroy(x);
      delete s;
      return FRNTT_EHIP;
    }
    s->streams.push_back(st);
    s->slot_busy.push_back(false);
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return FRNTT_OK;
}

int frntt_server_submit(frntt_server* s, int kind, int log_n, uint64_t data_seed, uint64_t* ticket) {
  if (!s || !ticket || kind < FRNTT_FWD || kind > FRNTT_COSET_INV) return FRNTT_EINVAL;
  if (log_n < 1 || log_n > s->ctx->max_log_n) return FRNTT_ERANGE;
  // the algorithm and plan are fixed now; the buffer is sized for them
  frntt::JobPlan jp;
  frntt::resolve_plan(s->ctx, FRNTT_ALGO_AUTO, log_n, &jp.algo, &jp.plan);
  const size_t need = request_bytes(log_n, jp.plan);
  {
    // the pass-twiddle tables this request will use count against the
    // budget from the start: a request that could never fit is refused
    // before anything is built; otherwise they are built now (once per size
    // and direction)
    const size_t extra = frntt::pending_pass_table_bytes(s->ctx, jp.plan, kind);
    if (need + s->ctx->table_bytes + extra > s->budget) return FRNTT_EBUSY;
    std::vector<frntt::PassParams> tmp;
    const int rc = frntt::build_passes(s->ctx, jp.plan, log_n, 1, kind, nullptr, nullptr, &tmp, jp.algo);
    if (rc != FRNTT_OK) return rc;
  }
  if (need + s->ctx->table_bytes > s->budget) return FRNTT_EBUSY;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return FRNTT_ESTATE;
  Request r;
  r.id = s->next_id++;
  r.kind = kind;
  r.log_n = log_n;
  r.jp = jp;
  r.need = need;
  r.seed = data_seed;
  r.t_submit = Clock::now();
  s->reqs[r.id] = r;
  s->queue.push_back(r.id);
  ++s->outstanding;
  *ticket = r.id;
  s->cv.notify_one();
  return FRNTT_OK;
}

int frntt_server_poll(frntt_server* s, uint64_t ticket, int* done, double* latency_ms) {
  if (!s || !done) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.state >= 4) return FRNTT_ESTATE;
  *done = it->second.state == 3 ? 1 : 0;
  if (latency_ms)
    *latency_ms = *done ? std::chrono::duration<double, std::milli>(it->second.t_done - it->second.t_submit).count()
                        : 0.0;
  return s->error && *done ? s->error : FRNTT_OK;
}

int frntt_server_result(frntt_server* s, uint64_t ticket, void* host_out) {
  if (!s || !host_out) return FRNTT_EINVAL;
  void* buf = nullptr;
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.state != 3 || !it->second.buf) return FRNTT_ESTATE;
    buf = it->second.buf;
    bytes = (size_t)32 << it->second.log_n;
  }
  hipSetDevice(s->ctx->device);
  hipError_t e = hipMemcpy(host_out, buf, bytes, hipMemcpyDeviceToHost);
  std::lock_guard<std::mutex> lk(s->mu);
  Request& r = s->reqs[ticket];
  give_back(s, r);
  r.state = 4;
  s->cv.notify_one();
  return e == hipSuccess ? FRNTT_OK : set_hip_error(s->ctx, e);
}

int frntt_server_release(frntt_server* s, uint64_t ticket) {
  if (!s) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.state != 3) return FRNTT_ESTATE;
  give_back(s, it->second);  // no-op if already recycled on completion
  it->second.state = 4;
  s->cv.notify_one();
  return FRNTT_OK;
}

int frntt_server_drain(frntt_server* s, double timeout_s) {
  if (!s) return FRNTT_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const auto until = Clock::now() + std::chrono::duration<double>(timeout_s);
  while (s->outstanding > 0) {
    if (s->stalled) return FRNTT_EBUSY;  // finished results hold the budget
    if (s->cv_done.wait_until(lk, until) == std::cv_status::timeout && s->outstanding > 0) return FRNTT_EBUSY;
  }
  return s->error ? s->error : FRNTT_OK;
}

int frntt_server_set_release_on_done(frntt_server* s, int on) {
  if (!s) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->release_on_done = on != 0;
  return FRNTT_OK;
}

int frntt_server_stats(frntt_server* s, uint64_t* completed, uint64_t* batches, uint64_t* peak_bytes) {
  if (!s) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (batches) *batches = s->batches;
  if (peak_bytes) *peak_bytes = s->peak + s->ctx->table_bytes;
  return FRNTT_OK;
}

int frntt_server_peak_inflight(frntt_server* s, uint64_t* batches, uint64_t* requests) {
  if (!s) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (batches) *batches = s->peak_inflight_batches;
  if (requests) *requests = s->peak_inflight_requests;
  return FRNTT_OK;
}

int frntt_server_destroy(frntt_server* s) {
  if (!s) return FRNTT_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_one();
  }
  if (s->worker.joinable()) s->worker.join();
  hipSetDevice(s->ctx->device);
  for (hipStream_t st : s->streams) {
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  for (auto& kv : s->reqs)
    if (kv.second.buf) hipFree(kv.second.buf);
  for (auto& kv : s->free_bufs)
    for (void* p : kv.second) hipFree(p);
  delete s;
  return FRNTT_OK;
}

}  // extern "C"
