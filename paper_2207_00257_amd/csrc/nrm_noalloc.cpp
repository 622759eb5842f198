// nrm_normalize_noalloc: the plain normalize without a context and without
// any device allocation, for callers that cannot call hipMalloc (code under
// stream capture, tight serving loops, harnesses that forbid allocation).
//
// The plain path's workspace (one partial per reduce block, the combine
// ticket, the hoisted sum) lives in `scratch`, a fixed array in this code
// object. Each device holds its own copy at its own address, which host code
// must obtain with hipGetSymbolAddress while that device is current: the
// array's name in host code is only a stand-in for the symbol. That address
// is looked up once per device, on the device's first call, and kept; every
// launch takes it as a plain kernel argument, like a context's workspace.
//
// The kernels are the plain path's own (launch_small, launch_reduce,
// launch_map), with the device's default launch parameters, so a call gives
// the same bits as nrm_normalize_ex on the default context.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "nrm_ctx.h"

using nrm::fail;
using nrm::hip_fail;

namespace {

// Reduce blocks whose partials fit the scratch array (8 bytes each: a
// compensated pair). With the default parameters the plain-accumulation
// height bound asks for more than 512 blocks only above 2^30 elements; 16384
// blocks cover n <= 2^34 for either input size (compensated accumulation has
// no height bound and keeps 512 blocks).
constexpr int64_t kScratchPartials = 16384;
constexpr size_t kSumOffset = kScratchPartials * 8;  // two floats: the sum (compensated: hi, lo)
constexpr size_t kTicketOffset = kSumOffset + 128;   // the last-block combine's ticket, 0 between calls
// the mid-size single-launch form: call number (0), arrival count (8, 0
// between calls), stall marker (16), error word (24), merged total (32), then
// its segments' tagged partials
constexpr size_t kResOffset = kTicketOffset + 128;
constexpr size_t kResSlotsOffset = kResOffset + 256;
constexpr size_t kScratchBytes = kResSlotsOffset + 256 * 16;
static_assert(kScratchBytes == NRM_NOALLOC_SCRATCH_BYTES, "scratch size must match the header");

// Zero-initialized when the code object is loaded on a device; the ticket is
// also cleared once per device before the first use (below) and every reduce
// leaves it at 0.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

__global__ void clear_ticket_kernel(unsigned* ticket) { *ticket = 0u; }

constexpr int kMaxDevices = 64;

struct DeviceScratch {
  char* ptr = nullptr;  // device address of this device's copy of `scratch`
  nrm_params params{};  // the device's default launch parameters
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];
std::atomic<bool> g_ready[kMaxDevices];

// The current device's scratch address and parameters; on its first call the
// address is looked up (with that device current) and the ticket cleared on
// `s`, ahead of the call's own kernels.
int scratch_of(int dev, hipStream_t s, const DeviceScratch** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(NRM_EUNSUPPORTED, "device index beyond the library's 64");
  if (!g_ready[dev].load(std::memory_order_acquire)) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ready[dev].load(std::memory_order_relaxed)) {
      void* p = nullptr;
      hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
      if (!p) return fail(NRM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
      char* base = static_cast<char*>(p);
      hipLaunchKernelGGL(clear_ticket_kernel, dim3(1), dim3(1), 0, s, reinterpret_cast<unsigned*>(base + kTicketOffset));
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "scratch ticket clear launch");
      g_dev[dev].ptr = base;
      g_dev[dev].params = nrm::device_params(dev);
      g_ready[dev].store(true, std::memory_order_release);
    }
  }
  *out = &g_dev[dev];
  return NRM_OK;
}

}  // namespace

extern "C" int nrm_normalize_noalloc(void* out, int out_dtype, const void* in, int in_dtype, int64_t n, int accum,
                                     void* stream) {
  int st = nrm::check_plain_args(out, out_dtype, in, in_dtype, n, accum);
  if (st != NRM_OK || n == 0) return st;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceScratch* d = nullptr;
  st = scratch_of(dev, s, &d);
  if (st != NRM_OK) return st;
  float* sum = reinterpret_cast<float*>(d->ptr + kSumOffset);
  if (n <= d->params.small_n && n <= nrm::small_capacity(in_dtype)) {
    e = nrm::launch_small(in, in_dtype, out, out_dtype, n, accum, sum, s);
    if (e != hipSuccess) return hip_fail(e, "small normalize kernel launch");
    return NRM_OK;
  }
  if (n <= d->params.resident_n && n <= nrm::plain_resident_capacity()) {
    char* r = d->ptr + kResOffset;
    const nrm::PlainResidentWs w{reinterpret_cast<unsigned long long*>(d->ptr + kResSlotsOffset),
                                 reinterpret_cast<unsigned long long*>(r + 32), reinterpret_cast<unsigned*>(r + 8),
                                 reinterpret_cast<unsigned long long*>(r), reinterpret_cast<unsigned long long*>(r + 16),
                                 reinterpret_cast<int*>(r + 24), sum};
    e = nrm::launch_plain_resident(in, in_dtype, out, out_dtype, n, accum, w, s);
    if (e != hipSuccess) return hip_fail(e, "mid-size normalize kernel launch");
    return NRM_OK;
  }
  nrm::PlainPlan plan;
  st = nrm::plan_plain(d->params, out, out_dtype, in, in_dtype, n, accum, &plan);
  if (st != NRM_OK) return st;
  if (plan.grid > kScratchPartials)
    return fail(NRM_EINVAL, "n too large for the allocation-free call: it needs more than 16384 reduce blocks "
                            "(with the default parameters, above 2^34 elements in plain accumulation)");
  nrm::PlainWorkspace ws{d->ptr, reinterpret_cast<unsigned*>(d->ptr + kTicketOffset), sum};
  e = nrm::launch_reduce(plan, ws, s);
  if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  e = nrm::launch_map(plan, ws, s);
  if (e != hipSuccess) return hip_fail(e, "map kernel launch");
  return NRM_OK;
}
