// The continuous-batching core of the normalize server, free of any GPU
// call: request queue, HBM-budget admission, the output arena, slots, and
// completion accounting. The device work goes through an Executor, so the
// same core runs on the GPU (nrm_server.cpp) and, in the CPU tests, on a fake
// executor that finishes work after chosen delays or fails on purpose.
//
// One thread drives step(); submit(), take_done(), release() and stats() may
// be called from other threads (they lock the core's mutex).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nrm.h"

namespace nrm {

inline int64_t sched_dtype_size(int dt) { return dt == NRM_F32 ? 4 : 2; }

// First-fit allocator over [0, size) in 256-byte units, coalescing free
// neighbours on release.
class Arena {
 public:
  explicit Arena(int64_t size) : size_(size) {
    if (size > 0) free_[0] = size;
  }
  // Offset of a block of at least `bytes` bytes (rounded up to 256), or -1.
  int64_t alloc(int64_t bytes) {
    bytes = std::max<int64_t>(256, (bytes + 255) / 256 * 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        return off;
      }
    }
    return -1;
  }
  // Returns false if `off` is not an allocated block.
  bool release(int64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    int64_t len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + len) {
      len += next->second;
      free_.erase(next);
    }
    auto prev = free_.lower_bound(off);
    if (prev != free_.begin()) {
      --prev;
      if (prev->first + prev->second == off) {
        prev->second += len;
        return true;
      }
    }
    free_[off] = len;
    return true;
  }
  int64_t size() const { return size_; }
  int64_t free_blocks() const { return (int64_t)free_.size(); }
  int64_t used_blocks() const { return (int64_t)used_.size(); }
  int64_t largest_free() const {
    int64_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }

 private:
  int64_t size_;
  std::map<int64_t, int64_t> free_;  // offset -> length
  std::map<int64_t, int64_t> used_;
};

// Where a slot's work runs. launch() starts `count` rows on the slot (one
// batched call, or one plain call per row; a row's `out` is its offset in
// the output arena); query() reports whether the slot's last launch has
// finished: 1 done, 0 running, or a negative nrm status when that work
// failed. message() describes the last failure.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual int launch(int slot, const nrm_row* rows, int64_t count, bool batched) = 0;
  virtual int query(int slot) = 0;
  virtual std::string message() = 0;
};

struct SchedConfig {
  int slots = 4;
  bool batching = true;
  bool single_plain = true;
  bool spread = true;
  bool hold_outputs = false;
  int64_t min_batch_rows = 4;
  int64_t max_batch_rows = 256;
  int64_t max_batch_elems = int64_t(1) << 27;
  int64_t budget_bytes = int64_t(64) << 30;
};

class Scheduler {
 public:
  struct Pending {
    nrm_request req{};
    int64_t t_arrival = 0;  // scheduled arrival, the latency origin
    int64_t out_off = -1;
    int64_t budget = 0;
    int64_t t_launch = 0;
  };

  Scheduler(const SchedConfig& cfg, int64_t arena_bytes, Executor* ex)
      : cfg_(cfg), arena_(arena_bytes), ex_(ex), slots_((size_t)cfg.slots) {}

  // Bytes a request holds while admitted: its input and its output.
  static int64_t need_of(const nrm_request& r) {
    return r.n * (sched_dtype_size(r.in_dtype) + sched_dtype_size(r.out_dtype));
  }

  // Queue requests that arrived at t_arrival[i] (the latency origin).
  void submit(const nrm_request* reqs, const int64_t* t_arrival, int64_t count) {
    std::lock_guard<std::mutex> lk(mu_);
    for (int64_t i = 0; i < count; ++i) {
      Pending p;
      p.req = reqs[i];
      p.t_arrival = t_arrival[i];
      queue_.push_back(p);
      in_flight_ += 1;
    }
  }

  // One pass at time `now`: report finished slots, then admit waiting
  // requests into free slots and launch them. Returns whether anything
  // happened.
  bool step(int64_t now) {
    bool progressed = false;
    for (size_t k = 0; k < slots_.size(); ++k) {
      SlotState& s = slots_[k];
      if (!s.busy) continue;
      const int q = ex_->query((int)k);
      if (q == 0) continue;
      std::lock_guard<std::mutex> lk(mu_);
      complete_locked(s.reqs, now, q == 1 ? NRM_OK : q);
      s.reqs.clear();
      s.busy = false;
      progressed = true;
    }
    int64_t free_slots = 0;
    for (const SlotState& s : slots_) free_slots += s.busy ? 0 : 1;
    for (size_t k = 0; k < slots_.size(); ++k) {
      SlotState& s = slots_[k];
      if (s.busy) continue;
      std::vector<Pending> batch;
      {
        std::lock_guard<std::mutex> lk(mu_);
        int64_t share = cfg_.max_batch_rows;
        if (cfg_.spread) share = std::min<int64_t>(share, ((int64_t)queue_.size() + free_slots - 1) / free_slots);
        free_slots -= 1;
        int64_t elems = 0;
        while (!queue_.empty() && (int64_t)batch.size() < share) {
          Pending& p = queue_.front();
          const int64_t need = need_of(p.req);
          if (!batch.empty() && elems + p.req.n > cfg_.max_batch_elems) break;
          if (budget_used_ + need > cfg_.budget_bytes) break;  // wait for memory
          const int64_t off = arena_.alloc(std::max<int64_t>(p.req.n * sched_dtype_size(p.req.out_dtype), 1));
          if (off < 0) break;  // wait for the arena
          p.out_off = off;
          p.budget = need;
          budget_used_ += need;
          elems += p.req.n;
          batch.push_back(p);
          queue_.pop_front();
        }
      }
      if (batch.empty()) break;
      launch_on((int)k, batch, now);
      progressed = true;
    }
    return progressed;
  }

  // The two below read the slots: call them from the thread that drives step().
  bool idle() {
    std::lock_guard<std::mutex> lk(mu_);
    for (const SlotState& s : slots_)
      if (s.busy) return false;
    return queue_.empty();
  }
  bool any_busy() const {
    for (const SlotState& s : slots_)
      if (s.busy) return true;
    return false;
  }

  // Move up to `max` completions out.
  int64_t take_done(nrm_completion* out, int64_t max, int64_t out_base) {
    std::lock_guard<std::mutex> lk(mu_);
    const int64_t k = std::min<int64_t>(max, (int64_t)done_.size());
    for (int64_t i = 0; i < k; ++i) {
      out[i] = done_[(size_t)i];
      out[i].out = reinterpret_cast<void*>(out_base + reinterpret_cast<int64_t>(out[i].out));
    }
    done_.erase(done_.begin(), done_.begin() + k);
    return k;
  }

  // Release a held output; false if there is none with this id.
  bool release(int64_t id) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = held_.find(id);
    if (it == held_.end()) return false;
    arena_.release(it->second.out_off);
    budget_used_ -= it->second.budget;
    held_.erase(it);
    return true;
  }

  void stats(nrm_server_counters* c) {
    std::lock_guard<std::mutex> lk(mu_);
    c->in_flight = in_flight_;
    c->queued = (int64_t)queue_.size();
    c->held = (int64_t)held_.size();
    c->budget_used = budget_used_;
    c->batches = batches_;
    c->launches = launches_;
    c->failed = failed_;
  }
  // The first failure's status and message (NRM_OK if none).
  int first_error(std::string* msg) {
    std::lock_guard<std::mutex> lk(mu_);
    if (msg) *msg = error_msg_;
    return error_;
  }
  Arena& arena() { return arena_; }

 private:
  struct SlotState {
    bool busy = false;
    std::vector<Pending> reqs;
  };

  void launch_on(int k, std::vector<Pending>& batch, int64_t now) {
    std::vector<nrm_row> rows(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
      Pending& p = batch[i];
      p.t_launch = now;
      rows[i].in = p.req.in;
      rows[i].out = reinterpret_cast<void*>(p.out_off);  // offset into the arena; the executor adds its base
      rows[i].n = p.req.n;
      rows[i].in_dtype = p.req.in_dtype;
      rows[i].out_dtype = p.req.out_dtype;
    }
    const bool small_group =
        (int64_t)rows.size() < cfg_.min_batch_rows || (cfg_.single_plain && rows.size() == 1);
    const bool batched = cfg_.batching && !small_group;
    const int st = ex_->launch(k, rows.data(), (int64_t)rows.size(), batched);
    std::lock_guard<std::mutex> lk(mu_);
    batches_ += 1;
    launches_ += batched ? 1 : (int64_t)rows.size();
    if (st != NRM_OK) {
      // nothing runs for these requests: they complete now with the error,
      // and their memory goes back at once; the slot stays free
      complete_locked(batch, now, st);
      return;
    }
    slots_[(size_t)k].reqs.swap(batch);
    slots_[(size_t)k].busy = true;
  }

  void complete_locked(std::vector<Pending>& reqs, int64_t now, int status) {
    for (Pending& p : reqs) {
      if (cfg_.hold_outputs && status == NRM_OK) {
        held_[p.req.id] = p;
      } else {
        arena_.release(p.out_off);
        budget_used_ -= p.budget;
      }
      nrm_completion c;
      c.id = p.req.id;
      c.out = reinterpret_cast<void*>(p.out_off);
      c.t_arrival_ns = p.t_arrival;
      c.t_launch_ns = p.t_launch;
      c.t_done_ns = now;
      c.status = status;
      c.pad = 0;
      done_.push_back(c);
      in_flight_ -= 1;
      if (status != NRM_OK) {
        failed_ += 1;
        if (error_ == NRM_OK) {
          error_ = status;
          error_msg_ = ex_->message();
        }
      }
    }
  }

  SchedConfig cfg_;
  Arena arena_;
  Executor* ex_;
  std::vector<SlotState> slots_;  // driven by the step() thread only
  std::mutex mu_;                 // guards everything below
  std::deque<Pending> queue_;
  std::vector<nrm_completion> done_;
  std::map<int64_t, Pending> held_;
  int64_t budget_used_ = 0;
  int64_t in_flight_ = 0;
  int64_t batches_ = 0;
  int64_t launches_ = 0;
  int64_t failed_ = 0;
  int error_ = NRM_OK;
  std::string error_msg_;
};

}  // namespace nrm
