// CPU tests of the serving core (paper_2207_00257_amd/csrc/nrm_sched.h) with
// a fake executor in place of the GPU: admission order, HBM-budget
// back-pressure, arena coalescing, slot reuse, spreading and grouping,
// latency accounting on a fake clock, launch and execution failures, held
// outputs, and a two-thread run (for the thread sanitizer). Built and run by
// tests/test_sched_cpu.py, plain and under AddressSanitizer +
// UndefinedBehaviorSanitizer and ThreadSanitizer. Exit status 0: all passed.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <string>
#include <thread>
#include <vector>

#include "nrm_sched.h"

using nrm::Arena;
using nrm::SchedConfig;
using nrm::Scheduler;

static int g_failures = 0;
#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #cond); \
      ++g_failures;                                                          \
    }                                                                        \
  } while (0)

// A launch finishes `delay` fake nanoseconds after it starts; launches and
// executions can be made to fail.
struct FakeExecutor : nrm::Executor {
  struct Launch {
    int slot;
    std::vector<nrm_row> rows;
    bool batched;
    int64_t start;
  };
  int64_t* clock;
  int64_t delay = 100;
  std::vector<int64_t> finish;      // per slot
  std::vector<int> exec_status;     // per slot: what query reports when done
  std::vector<Launch> launches;
  int fail_launch_at = -1;          // index of the launch that fails to start
  int fail_exec_at = -1;            // index of the launch whose work fails
  std::atomic<int64_t> queries{0};

  FakeExecutor(int slots, int64_t* c) : clock(c), finish((size_t)slots, -1), exec_status((size_t)slots, 1) {}

  int launch(int slot, const nrm_row* rows, int64_t count, bool batched) override {
    const int idx = (int)launches.size();
    launches.push_back(Launch{slot, std::vector<nrm_row>(rows, rows + count), batched, *clock});
    if (idx == fail_launch_at) return NRM_EHIP;
    finish[(size_t)slot] = *clock + delay;
    exec_status[(size_t)slot] = idx == fail_exec_at ? NRM_EHIP : 1;
    return NRM_OK;
  }
  int query(int slot) override {
    queries++;
    if (*clock < finish[(size_t)slot]) return 0;
    return exec_status[(size_t)slot];
  }
  std::string message() override { return "fake failure"; }
};

static nrm_request req(int64_t id, int64_t n, int in_dt = NRM_F32, int out_dt = NRM_F32) {
  nrm_request r{};
  r.id = id;
  r.in = reinterpret_cast<const void*>(0x1000 + 64 * id);
  r.n = n;
  r.in_dtype = in_dt;
  r.out_dtype = out_dt;
  return r;
}

static std::vector<nrm_completion> drain(Scheduler& s) {
  std::vector<nrm_completion> out(4096);
  const int64_t k = s.take_done(out.data(), (int64_t)out.size(), 0);
  out.resize((size_t)k);
  return out;
}

static void test_arena_coalescing() {
  Arena a(1 << 20);
  std::vector<int64_t> offs;
  for (int i = 0; i < 16; ++i) offs.push_back(a.alloc(1000 * (i + 1)));
  for (int64_t o : offs) CHECK(o >= 0);
  for (size_t i = 0; i < offs.size(); ++i)
    for (size_t j = i + 1; j < offs.size(); ++j) CHECK(offs[i] != offs[j]);
  for (int64_t o : offs) CHECK(o % 256 == 0);
  // free every other block, then the rest: everything merges back into one
  for (size_t i = 0; i < offs.size(); i += 2) CHECK(a.release(offs[i]));
  CHECK(a.free_blocks() > 1);
  for (size_t i = 1; i < offs.size(); i += 2) CHECK(a.release(offs[i]));
  CHECK(a.free_blocks() == 1);
  CHECK(a.used_blocks() == 0);
  CHECK(a.largest_free() == (1 << 20));
  CHECK(!a.release(12345));  // not a block
  CHECK(a.alloc(1 << 21) == -1);  // larger than the arena
  // first fit reuses the lowest hole that fits
  int64_t x = a.alloc(4096), y = a.alloc(4096), z = a.alloc(4096);
  CHECK(a.release(y));
  CHECK(a.alloc(1024) == y);
  (void)x;
  (void)z;
}

static void test_fifo_admission_and_slot_reuse() {
  int64_t clock = 0;
  SchedConfig cfg;
  cfg.slots = 1;
  cfg.max_batch_rows = 2;
  cfg.min_batch_rows = 1;
  cfg.single_plain = false;
  FakeExecutor ex(1, &clock);
  Scheduler s(cfg, 1 << 24, &ex);
  std::vector<nrm_request> rs;
  std::vector<int64_t> t;
  for (int i = 0; i < 6; ++i) {
    rs.push_back(req(i, 100));
    t.push_back(0);
  }
  s.submit(rs.data(), t.data(), (int64_t)rs.size());
  int64_t expect_next = 0;
  CHECK(s.step(clock));  // the first two launch; later pairs launch in the step that completes a pair
  for (int round = 0; round < 3; ++round) {
    CHECK((int)ex.launches.size() == round + 1);
    const auto& l = ex.launches.back();
    CHECK(l.slot == 0);
    CHECK(l.batched);
    CHECK(l.rows.size() == 2);
    for (const nrm_row& r : l.rows) CHECK(r.in == reinterpret_cast<const void*>(0x1000 + 64 * expect_next++));
    CHECK(!s.step(clock));  // the slot is busy: nothing to do
    clock += ex.delay;
    // the slot finishes and is reused by the next two requests in the same step
    CHECK(s.step(clock));
    auto d = drain(s);
    CHECK(d.size() == 2);
    for (const auto& c : d) CHECK(c.status == NRM_OK && c.t_done_ns == clock && c.t_arrival_ns == 0);
  }
  CHECK(s.idle());
  nrm_server_counters c{};
  s.stats(&c);
  CHECK(c.in_flight == 0 && c.queued == 0 && c.budget_used == 0 && c.batches == 3 && c.launches == 3);
}

static void test_budget_back_pressure() {
  int64_t clock = 0;
  SchedConfig cfg;
  cfg.slots = 4;
  cfg.budget_bytes = 8 * 1000 * 3;  // three FP32 requests of 1000 elements (8 bytes each)
  cfg.spread = true;
  FakeExecutor ex(4, &clock);
  Scheduler s(cfg, 1 << 24, &ex);
  std::vector<nrm_request> rs;
  std::vector<int64_t> t;
  for (int i = 0; i < 7; ++i) {
    rs.push_back(req(i, 1000));
    t.push_back(0);
  }
  s.submit(rs.data(), t.data(), 7);
  s.step(clock);
  nrm_server_counters c{};
  s.stats(&c);
  CHECK(c.budget_used == 3 * 8000);  // admission stops at the budget
  CHECK(c.queued == 4);
  CHECK(c.budget_used <= cfg.budget_bytes);
  int64_t admitted = 0;
  for (const auto& l : ex.launches) admitted += (int64_t)l.rows.size();
  CHECK(admitted == 3);
  // nothing more until memory is released
  clock += 10;
  s.step(clock);
  s.stats(&c);
  CHECK(c.queued == 4);
  clock += ex.delay;
  s.step(clock);  // three complete, three more admitted
  s.stats(&c);
  CHECK(c.queued == 1 && c.budget_used == 3 * 8000);
  // a request larger than the remaining budget waits; arrival order is kept
  for (int k = 0; k < 4; ++k) {
    clock += ex.delay;
    s.step(clock);
  }
  CHECK(s.idle());
  auto d = drain(s);
  CHECK(d.size() == 7);
  // launches happened in id order
  int64_t next = 0;
  for (const auto& l : ex.launches)
    for (const nrm_row& r : l.rows) CHECK(r.in == reinterpret_cast<const void*>(0x1000 + 64 * next++));
}

static void test_spread_and_grouping() {
  int64_t clock = 0;
  SchedConfig cfg;
  cfg.slots = 4;
  cfg.min_batch_rows = 2;
  FakeExecutor ex(4, &clock);
  Scheduler s(cfg, 1 << 24, &ex);
  std::vector<nrm_request> rs;
  std::vector<int64_t> t;
  for (int i = 0; i < 8; ++i) {
    rs.push_back(req(i, 64));
    t.push_back(0);
  }
  s.submit(rs.data(), t.data(), 8);
  s.step(clock);
  CHECK(ex.launches.size() == 4);
  for (const auto& l : ex.launches) {
    CHECK(l.rows.size() == 2);  // spread: each free slot takes its share
    CHECK(l.batched);           // two rows reach min_batch_rows
  }
  clock += ex.delay;
  s.step(clock);
  // one request: below min_batch_rows, and single_plain: runs as plain calls
  nrm_request one = req(100, 64);
  int64_t t0 = clock;
  s.submit(&one, &t0, 1);
  s.step(clock);
  CHECK(ex.launches.size() == 5 && !ex.launches.back().batched);
  // without spreading the first free slot takes all waiting requests
  int64_t clock2 = 0;
  cfg.spread = false;
  FakeExecutor ex2(4, &clock2);
  Scheduler s2(cfg, 1 << 24, &ex2);
  s2.submit(rs.data(), t.data(), 8);
  s2.step(clock2);
  CHECK(ex2.launches.size() == 1 && ex2.launches[0].rows.size() == 8);
}

static void test_latency_accounting() {
  int64_t clock = 1000;
  SchedConfig cfg;
  cfg.slots = 1;
  cfg.max_batch_rows = 1;
  FakeExecutor ex(1, &clock);
  ex.delay = 50;
  Scheduler s(cfg, 1 << 24, &ex);
  nrm_request a = req(1, 10), b = req(2, 10);
  int64_t ta = 900, tb = 950;
  s.submit(&a, &ta, 1);
  s.submit(&b, &tb, 1);
  s.step(clock);  // a launches at 1000
  clock = 1050;
  s.step(clock);  // a done at 1050, b launches at 1050
  clock = 1100;
  s.step(clock);
  auto d = drain(s);
  CHECK(d.size() == 2);
  CHECK(d[0].id == 1 && d[0].t_arrival_ns == 900 && d[0].t_launch_ns == 1000 && d[0].t_done_ns == 1050);
  CHECK(d[1].id == 2 && d[1].t_arrival_ns == 950 && d[1].t_launch_ns == 1050 && d[1].t_done_ns == 1100);
}

static void test_launch_failure_completes_at_once() {
  int64_t clock = 0;
  SchedConfig cfg;
  cfg.slots = 2;
  cfg.min_batch_rows = 1;
  cfg.single_plain = false;
  FakeExecutor ex(2, &clock);
  ex.fail_launch_at = 0;
  Scheduler s(cfg, 1 << 24, &ex);
  std::vector<nrm_request> rs = {req(0, 100), req(1, 100), req(2, 100)};
  std::vector<int64_t> t = {0, 0, 0};
  s.submit(rs.data(), t.data(), 3);
  s.step(clock);
  // the failed launch's requests complete now with the error, their memory
  // is free again, and its slot stays free for later work
  auto d = drain(s);
  CHECK(!d.empty());
  for (const auto& c : d) CHECK(c.status == NRM_EHIP && c.t_done_ns == clock);
  nrm_server_counters c{};
  s.stats(&c);
  CHECK(c.failed == (int64_t)d.size());
  std::string msg;
  CHECK(s.first_error(&msg) == NRM_EHIP && msg == "fake failure");
  for (int k = 0; k < 4; ++k) {
    clock += ex.delay;
    s.step(clock);
  }
  auto d2 = drain(s);
  CHECK(d.size() + d2.size() == 3);
  for (const auto& c2 : d2) CHECK(c2.status == NRM_OK);
  CHECK(s.idle());
  s.stats(&c);
  CHECK(c.budget_used == 0 && c.in_flight == 0);
  CHECK(s.arena().used_blocks() == 0);
}

static void test_execution_failure_and_held_outputs() {
  int64_t clock = 0;
  SchedConfig cfg;
  cfg.slots = 1;
  cfg.max_batch_rows = 1;
  cfg.hold_outputs = true;
  FakeExecutor ex(1, &clock);
  ex.fail_exec_at = 1;
  Scheduler s(cfg, 1 << 24, &ex);
  std::vector<nrm_request> rs = {req(0, 1000), req(1, 1000), req(2, 1000)};
  std::vector<int64_t> t = {0, 0, 0};
  s.submit(rs.data(), t.data(), 3);
  for (int k = 0; k < 4; ++k) {
    s.step(clock);
    clock += ex.delay;
  }
  auto d = drain(s);
  CHECK(d.size() == 3);
  CHECK(d[0].status == NRM_OK && d[1].status == NRM_EHIP && d[2].status == NRM_OK);
  nrm_server_counters c{};
  s.stats(&c);
  CHECK(c.held == 2);                    // the failed request holds nothing
  CHECK(c.budget_used == 2 * 8000);
  CHECK(s.release(0) && s.release(2));
  CHECK(!s.release(1) && !s.release(0));  // released or never held
  s.stats(&c);
  CHECK(c.held == 0 && c.budget_used == 0);
  CHECK(s.arena().used_blocks() == 0);
}

static void test_arena_exhaustion_waits() {
  int64_t clock = 0;
  SchedConfig cfg;
  cfg.slots = 2;
  cfg.min_batch_rows = 1;
  FakeExecutor ex(2, &clock);
  Scheduler s(cfg, 4096, &ex);  // room for one 1024-element FP32 output at a time
  std::vector<nrm_request> rs = {req(0, 1024), req(1, 1024)};
  std::vector<int64_t> t = {0, 0};
  s.submit(rs.data(), t.data(), 2);
  s.step(clock);
  nrm_server_counters c{};
  s.stats(&c);
  CHECK(c.queued == 1);
  clock += ex.delay;
  s.step(clock);
  clock += ex.delay;
  s.step(clock);
  CHECK(s.idle());
  CHECK(drain(s).size() == 2);
}

// One thread drives step() on a real clock while another submits, polls and
// reads the counters: the core's locking under the thread sanitizer.
static void test_two_threads() {
  std::atomic<int64_t> clock_ns{0};
  int64_t clock = 0;
  SchedConfig cfg;
  cfg.slots = 3;
  FakeExecutor ex(3, &clock);
  ex.delay = 0;
  Scheduler s(cfg, 1 << 26, &ex);
  std::atomic<bool> stop{false};
  std::thread driver([&] {
    while (!stop.load()) {
      s.step(clock);  // clock is only touched by this thread
      std::this_thread::yield();
    }
    while (!s.idle()) s.step(clock);
  });
  int64_t got = 0;
  const int total = 2000;
  for (int i = 0; i < total; ++i) {
    nrm_request r = req(i, 1 + i % 977, i % 3 == 0 ? NRM_BF16 : NRM_F32, i % 3 == 0 ? NRM_BF16 : NRM_F32);
    int64_t ta = clock_ns.fetch_add(1);
    s.submit(&r, &ta, 1);
    if (i % 50 == 0) {
      nrm_server_counters c{};
      s.stats(&c);
      CHECK(c.in_flight >= 0 && c.budget_used >= 0);
      got += (int64_t)drain(s).size();
    }
  }
  stop.store(true);
  driver.join();
  got += (int64_t)drain(s).size();
  CHECK(got == total);
  nrm_server_counters c{};
  s.stats(&c);
  CHECK(c.in_flight == 0 && c.budget_used == 0);
}

int main() {
  test_arena_coalescing();
  test_fifo_admission_and_slot_reuse();
  test_budget_back_pressure();
  test_spread_and_grouping();
  test_latency_accounting();
  test_launch_failure_completes_at_once();
  test_execution_failure_and_held_outputs();
  test_arena_exhaustion_waits();
  test_two_threads();
  if (g_failures) {
    fprintf(stderr, "%d check(s) failed\n", g_failures);
    return 1;
  }
  printf("sched_test: all passed\n");
  return 0;
}
