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
//
// With the device queue (device_queue = 1) nothing is launched per request:
// a slot holds one request, which the executor publishes into a ring in
// pinned host memory; one persistent kernel (nrm_dq.h) picks it up, runs it,
// and writes the slot's completion word into that memory, which query()
// reads. The kernel ends after dq_idle_us without new requests and is
// started again by the next one (or, should it have ended just as a request
// was published, by the next query that finds it gone with work pending).
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
#include "nrm_dq.h"
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

// The device queue's side of the scheduler: slot k's request lives in ring
// entry k of the pinned block until it completes. A request longer than
// plain_above runs instead as the plain call on slot k's own stream (plain).
class DqExecutor : public nrm::Executor {
 public:
  HipExecutor plain;                // per slot: context, stream, event for the long requests
  int64_t plain_above = int64_t(1) << 20;
  std::vector<char> on_plain;       // per slot: its request runs as a plain call
  std::vector<hipStream_t> set_aside;  // streams found to share the kernel's hardware queue
  nrm::DqHost* host = nullptr;      // pinned, coherent (host address)
  nrm::DqHost* host_dev = nullptr;  // the same memory's device address
  nrm::DqDev* dev = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ended = nullptr;       // recorded after each launch of the kernel
  bool launched = false;
  uint64_t epoch = 0;               // launches so far
  uint64_t seq = 0;                 // requests published so far
  int64_t last_check_ns = 0;        // last time query() looked at the kernel
  // The first failure to start or observe the kernel, kept: a request stays
  // published in the ring, so once its slot has completed with an error (and
  // its output memory gone back to the arena) no kernel may run again.
  int broken = NRM_OK;
  std::string broken_msg;
  int accum = NRM_ACC_F32;
  int64_t blocks = 0;
  unsigned long long idle_ticks = 0;
  unsigned long long slice_ticks = 0;
  char* arena_base = nullptr;
  std::vector<uint64_t> tag;        // per slot: the completion word its request will write
  std::vector<char> empty;          // per slot: an n == 0 request, complete at once
  std::string msg;

  int allocate(int device, int slots, int64_t nblocks, int64_t idle_us, int64_t slice_us) {
    int rate_khz = 0;
    hipError_t e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute (wall clock rate)");
    idle_ticks = (unsigned long long)idle_us * (unsigned long long)(rate_khz > 0 ? rate_khz : 100000) / 1000ull;
    slice_ticks = (unsigned long long)slice_us * (unsigned long long)(rate_khz > 0 ? rate_khz : 100000) / 1000ull;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute (compute units)");
    // one block per compute unit leaves room for the plain calls' blocks;
    // with every request in the kernel, two
    blocks = nblocks > 0 ? nblocks : (plain_above < nrm::DQ_MAX_N ? 1 : 2) * (int64_t)cus;
    if (blocks < nrm::RES_MAX_SEGMENTS) return fail(NRM_EINVAL, "dq_blocks must be at least 64");
    e = hipHostMalloc(reinterpret_cast<void**>(&host), sizeof(nrm::DqHost), hipHostMallocCoherent | hipHostMallocMapped);
    if (e != hipSuccess) return fail(NRM_ENOMEM, std::string("device queue hipHostMalloc: ") + hipGetErrorString(e));
    std::memset(host, 0, sizeof(nrm::DqHost));
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&host_dev), host, 0);
    if (e != hipSuccess) return hip_fail(e, "hipHostGetDevicePointer");
    e = hipMalloc(reinterpret_cast<void**>(&dev), sizeof(nrm::DqDev));
    if (e != hipSuccess) return fail(NRM_ENOMEM, std::string("device queue hipMalloc: ") + hipGetErrorString(e));
    e = hipMemset(dev, 0, sizeof(nrm::DqDev));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ended, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "device queue setup");
    tag.assign((size_t)slots, 0);
    empty.assign((size_t)slots, 0);
    on_plain.assign((size_t)slots, 0);
    plain.arena_base = arena_base;
    plain.accum = accum;
    plain.slots.resize((size_t)(plain_above < nrm::DQ_MAX_N ? slots : 0));
    for (HipExecutor::SlotRes& sl : plain.slots) {
      int st = nrm_create(&sl.ctx, device);
      if (st == NRM_OK) st = separate_stream(rate_khz, &sl.stream);
      if (st == NRM_OK && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
        st = fail(NRM_EHIP, "hipEventCreate");
      if (st != NRM_OK) return st;
    }
    return NRM_OK;
  }

  // A new stream whose hardware queue is not the kernel's. Streams share the
  // runtime's few hardware queues, and a kernel queued behind the persistent
  // one on a shared queue waits until it ends (up to dq_idle_us), so each
  // candidate is tried while a bounded one-thread kernel holds the kernel's
  // stream: a candidate whose empty kernel does not finish within 5 ms shares
  // the queue and is set aside (kept, so that it keeps its queue).
  int separate_stream(int rate_khz, hipStream_t* out) {
    *out = nullptr;
    const unsigned long long hold_ticks = 20000ull * (unsigned long long)(rate_khz > 0 ? rate_khz : 100000) / 1000ull;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return fail(NRM_EHIP, "hipEventCreate");
    int st = NRM_OK;
    for (int attempt = 0; attempt < 16 && !*out && st == NRM_OK; ++attempt) {
      hipStream_t cand = nullptr;
      if (hipStreamCreateWithFlags(&cand, hipStreamNonBlocking) != hipSuccess) {
        st = fail(NRM_EHIP, "hipStreamCreate");
        break;
      }
      __atomic_store_n(&host->hold, 0, __ATOMIC_RELEASE);
      hipError_t e = nrm::launch_dq_hold(host_dev, hold_ticks, stream);
      if (e == hipSuccess) e = nrm::launch_dq_touch(cand);
      if (e == hipSuccess) e = hipEventRecord(ev, cand);
      bool alone = false;
      const int64_t t0 = now_ns();
      while (e == hipSuccess && now_ns() - t0 < 5000000) {
        e = hipEventQuery(ev);
        if (e == hipSuccess) {
          alone = true;
          break;
        }
        if (e == hipErrorNotReady) e = hipSuccess;
      }
      __atomic_store_n(&host->hold, 1, __ATOMIC_RELEASE);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e == hipSuccess) e = hipStreamSynchronize(cand);
      if (e != hipSuccess) {
        (void)hipStreamDestroy(cand);
        st = hip_fail(e, "device queue stream probe");
        break;
      }
      if (alone) *out = cand;
      else set_aside.push_back(cand);
    }
    (void)hipEventDestroy(ev);
    if (st == NRM_OK && !*out) st = fail(NRM_EHIP, "device queue: no stream apart from the kernel's hardware queue");
    return st;
  }

  // Start the kernel unless it is running.
  int ensure_running() {
    if (broken != NRM_OK) return fail(broken, broken_msg);
    hipError_t e = hipSuccess;
    if (launched) {
      e = hipEventQuery(ended);
      if (e == hipErrorNotReady) return NRM_OK;
    }
    if (e == hipSuccess) {
      epoch += 1;
      const nrm::DqArgs a{host_dev, dev, epoch, idle_ticks, slice_ticks};
      e = nrm::launch_dq(a, accum, blocks, stream);
      if (e == hipSuccess) e = hipEventRecord(ended, stream);
      if (e == hipSuccess) {
        launched = true;
        return NRM_OK;
      }
    }
    broken = hip_fail(e, "device queue launch");
    broken_msg = nrm_last_error();
    return broken;
  }

  int launch(int k, const nrm_row* rows, int64_t count, bool) override {
    for (int64_t i = 0; i < count; ++i) {  // the scheduler gives this executor one row per slot
      const nrm_row& r = rows[i];
      if (r.n == 0) {
        empty[(size_t)k] = 1;
        continue;
      }
      if (r.n > plain_above) {
        const int st = plain.launch(k, &r, 1, false);
        if (st != NRM_OK) {
          msg = plain.message();
          return st;
        }
        on_plain[(size_t)k] = 1;
        return NRM_OK;
      }
      if (broken != NRM_OK) {  // nothing more is published once the kernel failed
        msg = broken_msg;
        return fail(broken, broken_msg);
      }
      // four words, each with the request's tag above bit 48 (addresses and
      // n are checked to fit below it when the request is submitted)
      const uint64_t t = nrm::dq_pub_tag(seq) << nrm::DQ_TAG_SHIFT;
      uint64_t* w = host->pub[seq % nrm::DQ_PUB].w;
      const uint64_t words[4] = {reinterpret_cast<uint64_t>(r.in) | t,
                                 reinterpret_cast<uint64_t>(arena_base + reinterpret_cast<int64_t>(r.out)) | t,
                                 (uint64_t)r.n | t,
                                 ((uint64_t)r.in_dtype | (uint64_t)r.out_dtype << 8 | (uint64_t)k << 16) | t};
      for (int j = 0; j < 4; ++j) __atomic_store_n(w + j, words[j], __ATOMIC_RELEASE);
      tag[(size_t)k] = nrm::dq_tag(seq);
      seq += 1;
    }
    const int st = ensure_running();
    if (st != NRM_OK) msg = nrm_last_error();
    return st;
  }

  int query(int k) override {
    if (empty[(size_t)k]) {
      empty[(size_t)k] = 0;
      return 1;
    }
    if (on_plain[(size_t)k]) {
      const int q = plain.query(k);
      if (q != 0) on_plain[(size_t)k] = 0;
      if (q < 0) msg = plain.message();
      return q;
    }
    const uint64_t v = __atomic_load_n(&host->done[k], __ATOMIC_ACQUIRE);
    if (v == tag[(size_t)k]) {
      tag[(size_t)k] = 0;
      if (__atomic_load_n(&host->stalled[k], __ATOMIC_ACQUIRE) == v) {
        msg = "device queue: a wait for a request's partial sums gave up (its output is not valid)";
        return NRM_EDEVICE;
      }
      return 1;
    }
    // A kernel that ended (its idle limit or its slice) just as a request
    // was published has not seen it: look (at most every 20 us) and start it
    // again.
    const int64_t t = now_ns();
    if (t - last_check_ns > 20000) {
      last_check_ns = t;
      const int st = ensure_running();
      if (st != NRM_OK) {
        msg = nrm_last_error();
        return st;
      }
    }
    return 0;
  }

  std::string message() override { return msg; }

  // End the kernel (it stops once nothing new is published) and free.
  void shutdown() {
    if (host) __atomic_store_n(&host->stop, 1, __ATOMIC_RELEASE);
    if (stream) (void)hipStreamSynchronize(stream);  // teardown: the kernel's end is all that is awaited
    for (HipExecutor::SlotRes& sl : plain.slots) {
      if (sl.stream) (void)hipStreamSynchronize(sl.stream);  // teardown: errors were reported per request
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.ctx) nrm_destroy(sl.ctx);
    }
    plain.slots.clear();
    for (hipStream_t st : set_aside) (void)hipStreamDestroy(st);
    set_aside.clear();
    if (ended) (void)hipEventDestroy(ended);
    if (stream) (void)hipStreamDestroy(stream);
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    ended = nullptr;
    stream = nullptr;
    dev = nullptr;
    host = nullptr;
  }
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
  DqExecutor dq;
  char* arena_base = nullptr;
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
  cfg->device_queue = 0;
  cfg->dq_blocks = 0;
  cfg->dq_idle_us = 100000;
  cfg->dq_plain_above = int64_t(1) << 20;
  cfg->dq_slice_us = 10000;
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
  if (cfg->device_queue != 0 && cfg->device_queue != 1) return fail(NRM_EINVAL, "device_queue must be 0 or 1");
  if (cfg->device_queue) {
    if (cfg->slots > nrm::DQ_RING) return fail(NRM_EINVAL, "device queue: slots must be 1..64");
    if (cfg->dq_blocks != 0 && (cfg->dq_blocks < nrm::RES_MAX_SEGMENTS || cfg->dq_blocks > (1 << 16)))
      return fail(NRM_EINVAL, "dq_blocks must be 0 or 64..65536");
    if (cfg->dq_idle_us < 1 || cfg->dq_idle_us > 10000000) return fail(NRM_EINVAL, "dq_idle_us must be 1..10^7");
    if (cfg->dq_plain_above < 1 || cfg->dq_plain_above > nrm::DQ_MAX_N)
      return fail(NRM_EINVAL, "dq_plain_above must be 1..2^25");
    if (cfg->dq_slice_us < 0 || cfg->dq_slice_us > 10000000) return fail(NRM_EINVAL, "dq_slice_us must be 0..10^7");
  }
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
  hipError_t e = hipMalloc(&s->arena_base, (size_t)arena);
  if (e != hipSuccess) {
    delete s;
    return fail(NRM_ENOMEM, std::string("server arena hipMalloc: ") + hipGetErrorString(e));
  }
  s->ex.arena_base = s->arena_base;
  s->ex.accum = cfg->accum;
  s->dq.arena_base = s->arena_base;
  if (cfg->device_queue && ((reinterpret_cast<uint64_t>(s->arena_base) + (uint64_t)arena) >> nrm::DQ_TAG_SHIFT) != 0) {
    (void)hipFree(s->arena_base);
    delete s;
    return fail(NRM_EUNSUPPORTED, "device queue: output arena above 2^48");
  }
  s->dq.accum = cfg->accum;
  s->dq.plain_above = cfg->dq_plain_above;
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
  if (cfg->device_queue) {
    // one request per slot, published to the kernel as soon as admitted
    sc.batching = false;
    sc.max_batch_rows = 1;
    s->core = new nrm::Scheduler(sc, arena, &s->dq);
    const int st = s->dq.allocate(device, cfg->slots, cfg->dq_blocks, cfg->dq_idle_us, cfg->dq_slice_us);
    if (st != NRM_OK) {
      nrm_server_destroy(s);
      return st;
    }
    s->scheduler = std::thread([s] { s->run(); });
    *out = s;
    return NRM_OK;
  }
  s->ex.slots.resize(cfg->slots);
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
    if (s->cfg.device_queue && reqs[i].n > nrm::DQ_MAX_N)
      return fail(NRM_EINVAL, "device queue: request larger than 2^25 elements");
    if (s->cfg.device_queue && (reinterpret_cast<uint64_t>(reqs[i].in) >> nrm::DQ_TAG_SHIFT) != 0)
      return fail(NRM_EINVAL, "device queue: input address above 2^48");
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
    if (nrm::Scheduler::need_of(reqs[i]) > s->cfg.budget_bytes)
      return fail(NRM_EINVAL, "request larger than the server's budget");
    if (s->cfg.device_queue && reqs[i].n > nrm::DQ_MAX_N)
      return fail(NRM_EINVAL, "device queue: request larger than 2^25 elements");
    if (s->cfg.device_queue && (reinterpret_cast<uint64_t>(reqs[i].in) >> nrm::DQ_TAG_SHIFT) != 0)
      return fail(NRM_EINVAL, "device queue: input address above 2^48");
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
  *count = s->core->take_done(out, max, reinterpret_cast<int64_t>(s->arena_base));
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
  s->dq.shutdown();
  for (HipExecutor::SlotRes& sl : s->ex.slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);  // teardown: errors were reported per request
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ctx) nrm_destroy(sl.ctx);
  }
  if (s->arena_base) (void)hipFree(s->arena_base);
  delete s->core;
  delete s;
  return NRM_OK;
}

}  // extern "C"
