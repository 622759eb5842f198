// The context object behind nrm_ctx* and host-side helpers shared by the
// C ABI's translation units. Private to libnrm.so.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "nrm_batch.h"
#include "nrm_internal.h"

namespace nrm {

std::string& last_error();

inline int fail(int status, const std::string& what) {
  last_error() = what;
  return status;
}

inline int hip_fail(hipError_t e, const char* where) {
  return fail(NRM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

constexpr int kTimingRing = 1024;
// Pinned staging buffers of the batched path, used in turn: a call waits only
// for the call this many before it to have finished with its buffer.
constexpr int kStagingRing = 4;

// Makes `dev` current for the guard's lifetime. The device was validated
// when the context was created; should switching still fail, the next HIP
// call reports the error and every caller checks that call.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) : dev_(dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = dev;  // nothing to restore
    if (prev_ != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev_ != dev_) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = 0, dev_ = 0;
};


// Device workspace and host staging of the batched path.
struct BatchWorkspace {
  int64_t cap_rows = 0;
  int64_t cap_items = 0;
  int64_t cap_chunks = 0;
  void* dev = nullptr;         // one allocation, carved into the pointers below
  BatchHeader* hdr[kStagingRing] = {};  // device views of the staging buffers' headers
  RowDesc* table[kStagingRing] = {};    // device views of their row tables
  RowDesc* rows = nullptr;
  Item* items = nullptr;
  int64_t* lrow_first = nullptr;
  RowDesc* lrows = nullptr;
  int64_t* lstart = nullptr;
  RowRes* lsum = nullptr;
  int32_t* chunk_lrow = nullptr;
  int64_t* round_agg = nullptr;
  BatchHeader* hdr_dev = nullptr;
  int64_t* cnt = nullptr;
  int* error = nullptr;
  void* partials = nullptr;
  unsigned long long* tagged = nullptr;  // resident rows' tagged partials
  unsigned long long* rowtot = nullptr;  // resident rows' tagged totals
  unsigned* arrivals = nullptr;          // resident rows' arrival counts
  void* host = nullptr;        // pinned staging (host view): kStagingRing buffers of `staging` bytes,
                               // each a header, then a row table
  size_t staging = 0;
  int next = 0;                // the buffer the next call uses
  hipEvent_t staged[kStagingRing] = {};  // recorded after the call that used the buffer
  bool staged_pending[kStagingRing] = {};
  // captured launch sequences: per reduction kind (plain, compensated,
  // softmax) and staging buffer (the planner reads its buffer's header)
  hipGraphExec_t graph[3][kStagingRing] = {};
  hipStream_t capture_stream = nullptr;
  // timing ring of (before, after) event pairs
  std::vector<hipEvent_t> events;
  int64_t timed_calls = 0;
};

}  // namespace nrm

struct nrm_ctx {
  // held by every entry point for its host-side work on the context (the
  // tuned-parameter map, workspace growth, the staging ring, the timing
  // ring), so that host threads sharing a context, the default one included,
  // do not race on them; recursive for entry points that call others
  mutable std::recursive_mutex mu;
  nrm_batch_params bparams{};
  nrm::BatchWorkspace batch;
  int device = 0;
  nrm_params params{};
  // tuned parameters (nrm_tune.cpp): used per call while params_set is false
  bool params_set = false;
  std::string arch;
  std::map<int64_t, std::pair<bool, nrm_params>> tuned;  // call key -> (has an entry, parameters)
  // plain-path workspace
  void* partials = nullptr;
  int64_t partials_cap = 0;  // entries (each up to 8 bytes)
  unsigned* ticket = nullptr;
  int* dev_error = nullptr;  // device error word of the non-batched kernels (NLL targets)
  float* sum = nullptr;      // 2 floats
  nrm::PlainResidentWs res{};  // the single-launch mid-size form's exchange
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> events;  // 3 per recorded call
  int64_t timed_calls = 0;
};

namespace nrm {
// The process-wide default context of the current device (created on first use).
int default_ctx(nrm_ctx** out);
// The library's launch parameters for `device` (grids sized by its CU count).
nrm_params device_params(int device);
// Host validation of a plain call (no HIP call): NRM_OK, or the error status
// with nrm_last_error() set. n == 0 is valid.
int check_plain_args(const void* out, int out_dtype, const void* in, int in_dtype, int64_t n, int accum);
// Resolve a plain call's launch plan from parameters q (host only).
int plan_plain(const nrm_params& q, void* out, int out_dt, const void* in, int in_dt, int64_t n, int acc,
               PlainPlan* p);
// Release the batched workspace of a context (waits for the device).
void batch_free(nrm_ctx* c);
// The device's architecture name (gfx950), or "" (nrm_tune.cpp).
std::string device_arch(int device);
// Overlay the tuning cache's entry for this call's key on *p; false if none.
bool tuned_plain(const std::string& arch, int in_dt, int out_dt, int acc, int64_t n, nrm_params* p);
// The context's lock for the rest of an entry point.
using CtxLock = std::lock_guard<std::recursive_mutex>;

}  // namespace nrm
