// Continuous-batching server for normalize requests (C ABI in include/nrm.h).
//
// A request is one normalize of n elements whose input already lives in
// device memory. The scheduling core (nrm_sched.h: queue, HBM-budget
// admission, output arena, slots, completions) is driven here by one
// scheduler thread, which in each pass
//   1. polls the slots: a slot whose batch has finished (its event) releases
//      its requests' output blocks and budget and reports them complete;
//   2. admits waiting requests in arrival order while the HBM budget (input +
//      output bytes of every admitted request) and a free slot allow;
//   3. launches the admitted requests as one ragged batch (row-table form)
//      on the free slot's stream (a group of one request may take the plain
//      path instead), or, in per-request mode, one plain normalize call per
//      request. With spreading, waiting requests are shared out over the
//      free slots, so they run alone and concurrently while slots are free
//      and are grouped only when the queue outgrows the slots.
// Requests that arrive while batches are in flight join the next batch as
// soon as a slot and memory free up; several slots run concurrently.
// A replay thread can submit a whole trace at its scheduled arrival times
// (open loop); latency is measured from the scheduled arrival.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "nrm_ctx.h"
#include "nrm_sched.h"

using nrm::DeviceGuard;
using nrm::fail;
using nrm::hip_fail;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// The GPU side of the scheduler: per slot a context, a stream and an event.
class HipExecutor : public nrm::Executor {
 public:
  struct SlotRes {
    nrm_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
  };
  std::vector<SlotRes> slots;
  char* arena_base = nullptr;
  int accum = NRM_ACC_F32;
  std::string msg;

  int launch(int k, const nrm_row* rows_in, int64_t count, bool batched) override {
    SlotRes& s = slots[(size_t)k];
    std::vector<nrm_row> rows(rows_in, rows_in + count);
    for (nrm_row& r : rows) r.out = arena_base + reinterpret_cast<int64_t>(r.out);
    int st = NRM_OK;
    if (batched) {
      st = nrm_normalize_rows(s.ctx, rows.data(), count, accum, s.stream);
    } else {
      for (const nrm_row& r : rows) {
        st = nrm_normalize_ex(s.ctx, r.out, r.out_dtype, r.in, r.in_dtype, r.n, accum, s.stream);
        if (st != NRM_OK) break;
      }
    }
    if (st == NRM_OK) {
      hipError_t e = hipEventRecord(s.done, s.stream);
      if (e != hipSuccess) st = hip_fail(e, "hipEventRecord");
    }
    if (st != NRM_OK) {
      // rows already enqueued before a failing call may still run: let them
      // finish before their memory is handed out again
      msg = nrm_last_error();
      (void)hipStreamSynchronize(s.stream);
    }
    return st;
  }

  int query(int k) override {
    hipError_t e = hipEventQuery(slots[(size_t)k].done);
    if (e == hipErrorNotReady) return 0;
    if (e == hipSuccess) return 1;
    msg = std::string("hipEventQuery: ") + hipGetErrorString(e);
    return NRM_EHIP;
  }

  std::string message() override { return msg; }
};

bool valid_dtype(int dt) { return dt == NRM_F32 || dt == NRM_BF16 || dt == NRM_F16; }

int check_request(const nrm_request& r) {
  if (r.n < 0) return fail(NRM_EINVAL, "request with n < 0");
  if (!valid_dtype(r.in_dtype) || !valid_dtype(r.out_dtype)) return fail(NRM_EINVAL, "request with unknown dtype");
  if (r.n > 0 && !r.in) return fail(NRM_EINVAL, "request with NULL input");
  return NRM_OK;
}

}  // namespace

struct nrm_server {
  nrm_server_config cfg{};
  int device = 0;
  HipExecutor ex;
  nrm::Scheduler* core = nullptr;
  std::mutex wake_mu;                 // with cv: wakes the scheduler thread
  std::condition_variable cv;
  std::atomic<bool> stop{false};
  std::thread scheduler;
  std::thread replayer;
  std::atomic<int> replay_running{0};

  void run();
};

void nrm_server::run() {
  DeviceGuard g(device);
  int64_t last_activity = now_ns();
  while (true) {
    const bool progressed = core->step(now_ns());
    if (stop.load() && !progressed && core->idle()) break;
    if (progressed) {
      last_activity = now_ns();
    } else if (core->any_busy() || now_ns() - last_activity < (int64_t)cfg.idle_spin_us * 1000) {
      // poll the slots' events (and the queue) again without sleeping: an
      // arrival is then picked up without a thread wake-up
      std::this_thread::yield();
    } else {
      std::unique_lock<std::mutex> lk(wake_mu);
      cv.wait_for(lk, std::chrono::microseconds(200));
    }
  }
}

extern "C" {

int nrm_server_default_config(nrm_server_config* cfg) {
  if (!cfg) return fail(NRM_EINVAL, "NULL argument");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->slots = 4;
  cfg->budget_bytes = int64_t(64) << 30;
  cfg->arena_bytes = 0;
  cfg->max_batch_rows = 256;
  cfg->max_batch_elems = int64_t(1) << 27;
  cfg->batching = 1;
  cfg->graph = 1;
  cfg->accum = NRM_ACC_F32;
  cfg->single_plain = 1;
  cfg->spread = 1;
  cfg->idle_spin_us = 1000;
  cfg->min_batch_rows = 4;  // the best balance of p50 and p99 over 20k-200k requests/s on MI355X
  return NRM_OK;
}

int nrm_server_create(nrm_server** out, int device, const nrm_server_config* cfg) {
  if (!out || !cfg) return fail(NRM_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 64) return fail(NRM_EINVAL, "slots must be 1..64");
  if (cfg->budget_bytes < 1) return fail(NRM_EINVAL, "budget_bytes must be positive");
  if (cfg->max_batch_rows < 1 || cfg->max_batch_rows > (int64_t(1) << 20)) return fail(NRM_EINVAL, "max_batch_rows must be 1..2^20");
  if (cfg->max_batch_elems < 1) return fail(NRM_EINVAL, "max_batch_elems must be positive");
  if (cfg->batching != 0 && cfg->batching != 1) return fail(NRM_EINVAL, "batching must be 0 or 1");
  if (cfg->graph != 0 && cfg->graph != 1) return fail(NRM_EINVAL, "graph must be 0 or 1");
  if (cfg->accum != NRM_ACC_F32 && cfg->accum != NRM_ACC_KAHAN) return fail(NRM_EINVAL, "unknown accumulation mode");
  if (cfg->hold_outputs != 0 && cfg->hold_outputs != 1) return fail(NRM_EINVAL, "hold_outputs must be 0 or 1");
  if (cfg->use_batch_params != 0 && cfg->use_batch_params != 1) return fail(NRM_EINVAL, "use_batch_params must be 0 or 1");
  if (cfg->single_plain != 0 && cfg->single_plain != 1) return fail(NRM_EINVAL, "single_plain must be 0 or 1");
  if (cfg->spread != 0 && cfg->spread != 1) return fail(NRM_EINVAL, "spread must be 0 or 1");
  if (cfg->idle_spin_us < 0 || cfg->idle_spin_us > 1000000) return fail(NRM_EINVAL, "idle_spin_us must be 0..10^6");
  if (cfg->min_batch_rows < 1 || cfg->min_batch_rows > (1 << 20)) return fail(NRM_EINVAL, "min_batch_rows must be 1..2^20");
  if (device < 0) {
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  }
  DeviceGuard g(device);
  nrm_server* s = new nrm_server();
  s->cfg = *cfg;
  s->device = device;
  // outputs live in the arena; a request's output is at most two thirds of
  // its budget (FP32 out of a 2-byte input), which sizes the default arena
  const int64_t arena = cfg->arena_bytes > 0 ? cfg->arena_bytes : cfg->budget_bytes * 2 / 3 + (int64_t(1) << 20);
  hipError_t e = hipMalloc(&s->ex.arena_base, (size_t)arena);
  if (e != hipSuccess) {
    delete s;
    return fail(NRM_ENOMEM, std::string("server arena hipMalloc: ") + hipGetErrorString(e));
  }
  s->ex.accum = cfg->accum;
  s->ex.slots.resize(cfg->slots);
  nrm::SchedConfig sc;
  sc.slots = cfg->slots;
  sc.batching = cfg->batching != 0;
  sc.single_plain = cfg->single_plain != 0;
  sc.spread = cfg->spread != 0;
  sc.hold_outputs = cfg->hold_outputs != 0;
  sc.min_batch_rows = cfg->min_batch_rows;
  sc.max_batch_rows = cfg->max_batch_rows;
  sc.max_batch_elems = cfg->max_batch_elems;
  sc.budget_bytes = cfg->budget_bytes;
  s->core = new nrm::Scheduler(sc, arena, &s->ex);
  for (HipExecutor::SlotRes& sl : s->ex.slots) {
    int st = nrm_create(&sl.ctx, device);
    if (st == NRM_OK) {
      nrm_batch_params bp;
      nrm_get_batch_params(sl.ctx, &bp);
      bp.graph = cfg->graph;
      if (cfg->use_batch_params) bp = cfg->batch_params;
      st = nrm_set_batch_params(sl.ctx, &bp);
    }
    if (st == NRM_OK) st = nrm_batch_reserve(sl.ctx, cfg->max_batch_rows, cfg->max_batch_elems);
    if (st == NRM_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
      st = fail(NRM_EHIP, "hipStreamCreate");
    if (st == NRM_OK && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
      st = fail(NRM_EHIP, "hipEventCreate");
    if (st != NRM_OK) {
      nrm_server_destroy(s);
      return st;
    }
  }
  s->scheduler = std::thread([s] { s->run(); });
  *out = s;
  return NRM_OK;
}

int nrm_server_submit(nrm_server* s, const nrm_request* reqs, int64_t count) {
  if (!s || (count > 0 && !reqs) || count < 0) return fail(NRM_EINVAL, "bad arguments");
  for (int64_t i = 0; i < count; ++i) {
    int st = check_request(reqs[i]);
    if (st != NRM_OK) return st;
    if (nrm::Scheduler::need_of(reqs[i]) > s->cfg.budget_bytes)
      return fail(NRM_EINVAL, "request larger than the server's budget");
  }
  const int64_t t = now_ns();
  std::vector<int64_t> arrival((size_t)count);
  for (int64_t i = 0; i < count; ++i) arrival[(size_t)i] = reqs[i].t_arrival_ns > 0 ? reqs[i].t_arrival_ns : t;
  s->core->submit(reqs, arrival.data(), count);
  s->cv.notify_one();
  return NRM_OK;
}

int nrm_server_replay(nrm_server* s, const nrm_request* reqs, int64_t count, int64_t* t0_ns) {
  if (!s || count < 0 || (count > 0 && !reqs)) return fail(NRM_EINVAL, "bad arguments");
  if (s->replay_running.load()) return fail(NRM_EINVAL, "a replay is already running");
  for (int64_t i = 0; i < count; ++i) {
    int st = check_request(reqs[i]);
    if (st != NRM_OK) return st;
    if (i > 0 && reqs[i].t_arrival_ns < reqs[i - 1].t_arrival_ns) return fail(NRM_EINVAL, "arrivals out of order");
  }
  if (s->replayer.joinable()) s->replayer.join();
  std::vector<nrm_request> trace(reqs, reqs + count);
  const int64_t origin = now_ns() + 2000000;  // start 2 ms from now
  if (t0_ns) *t0_ns = origin;
  s->replay_running.store(1);
  s->replayer = std::thread([s, trace, origin] {
    size_t i = 0;
    while (i < trace.size() && !s->stop.load()) {
      const int64_t due = origin + trace[i].t_arrival_ns;
      int64_t t = now_ns();
      if (t < due) {
        if (due - t > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(due - t - 100000));
        continue;
      }
      // submit every request that is due, stamped with its scheduled arrival
      size_t j = i;
      std::vector<int64_t> arrival;
      while (j < trace.size() && origin + trace[j].t_arrival_ns <= t) {
        arrival.push_back(origin + trace[j].t_arrival_ns);
        ++j;
      }
      s->core->submit(&trace[i], arrival.data(), (int64_t)(j - i));
      s->cv.notify_one();
      i = j;
    }
    s->replay_running.store(0);
  });
  return NRM_OK;
}

int nrm_server_poll(nrm_server* s, nrm_completion* out, int64_t max, int64_t* count) {
  if (!s || !count || max < 0 || (max > 0 && !out)) return fail(NRM_EINVAL, "bad arguments");
  *count = s->core->take_done(out, max, reinterpret_cast<int64_t>(s->ex.arena_base));
  return NRM_OK;
}

int nrm_server_release(nrm_server* s, int64_t id) {
  if (!s) return fail(NRM_EINVAL, "NULL server");
  if (!s->core->release(id)) return fail(NRM_EINVAL, "no held output with this id");
  s->cv.notify_one();
  return NRM_OK;
}

int nrm_server_stats(nrm_server* s, nrm_server_counters* st) {
  if (!s || !st) return fail(NRM_EINVAL, "NULL argument");
  s->core->stats(st);
  st->replaying = s->replay_running.load();
  return NRM_OK;
}

int nrm_server_last_failure(nrm_server* s) {
  if (!s) return fail(NRM_EINVAL, "NULL server");
  std::string msg;
  const int st = s->core->first_error(&msg);
  if (st != NRM_OK) return fail(st, msg);
  return NRM_OK;
}

int nrm_server_destroy(nrm_server* s) {
  if (!s) return NRM_OK;
  s->stop.store(true);
  s->cv.notify_all();
  if (s->replayer.joinable()) s->replayer.join();
  if (s->scheduler.joinable()) s->scheduler.join();
  DeviceGuard g(s->device);
  for (HipExecutor::SlotRes& sl : s->ex.slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);  // teardown: errors were reported per request
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ctx) nrm_destroy(sl.ctx);
  }
  if (s->ex.arena_base) (void)hipFree(s->ex.arena_base);
  delete s->core;
  delete s;
  return NRM_OK;
}

}  // extern "C"
