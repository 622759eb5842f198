// C ABI of libnrm.so (declared in include/nrm.h): argument validation,
// launch planning, contexts with their device workspace, and kernel timing.
// All compute runs in the HIP kernels of nrm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nrm_ctx.h"

using nrm::fail;
using nrm::hip_fail;
using nrm::kTimingRing;
using nrm::DeviceGuard;

namespace nrm {
std::string& last_error() {
  thread_local std::string msg;
  return msg;
}
}  // namespace nrm


namespace {

// Defaults: the best shape found by the tuner (paper_2207_00257_amd/tune.py)
// on MI355X for n = 2^28 FP32. The reduce gives each of two blocks per CU one
// contiguous chunk, reads all but the input's last 256 MiB with a
// non-temporal hint and that tail with a temporal one (it stays in the
// last-level cache, where the map finds it), and ends without a grid-wide
// ticket: every map block merges the reduce's partials itself. The map runs
// 64 blocks per CU over tiles of 2^12 elements (block b takes tiles b,
// b + grid, ...), two 16-byte vectors per thread per iteration.
nrm_params default_params() {
  nrm_params p;
  std::memset(&p, 0, sizeof(p));
  p.block = 512;  // 16 wavefronts per CU: 256 threads ran 7 % slower from n = 2^29 on (equal at 2^28)
  p.unroll = 2;
  p.grid = 512;
  p.layout = NRM_LAYOUT_CHUNK;
  p.reduce_nt = 1;
  p.max_height = 36;
  p.map_block = 512;
  p.map_unroll = 2;
  p.map_grid = 16384;
  p.map_layout = NRM_LAYOUT_TILE;
  p.map_nt = 1;
  p.reverse_map = 0;
  // the last 256 MiB read with a temporal hint stay in the 256 MB last-level
  // cache, where the map finds them (measured: 256 saves ~35 us of the map at
  // 2^28 FP32; 288 overflows the cache and saves nothing)
  p.reduce_keep_mib = 256;
  p.tile_log2 = 12;
  p.fused_combine = 1;
  // n <= 2^18 in one launch of a block per 4096 elements (one read, one
  // write); above, the two kernels. Measured per call on MI355X (device time
  // of a synchronized call): 8.6-12.6 us up to 2^18 against 12.1-13.2 us for
  // two kernels; beyond 64 segments the exchange costs more than the kernel
  // boundary (2^20: 17.5 against 13.3 us). The one-block form (small_n) lost
  // to it from 2^14 on (2^16: 17.5 us).
  p.small_n = 0;
  p.resident_n = 1 << 18;
  return p;
}

int check_params(const nrm_params& p) {
  auto ok_b = [](int b) { return b >= 64 && b <= 1024 && b % 64 == 0; };
  auto ok_u = [](int u) { return u == 1 || u == 2 || u == 4 || u == 8; };
  auto ok_l = [](int l) { return l == NRM_LAYOUT_CHUNK || l == NRM_LAYOUT_STRIDE || l == NRM_LAYOUT_TILE; };
  auto ok_f = [](int f) { return f == 0 || f == 1; };
  if (!ok_b(p.block) || !ok_b(p.map_block)) return fail(NRM_EINVAL, "block sizes must be 64..1024, multiples of 64");
  if (!ok_u(p.unroll) || !ok_u(p.map_unroll)) return fail(NRM_EINVAL, "unroll and map_unroll must be 1, 2, 4 or 8");
  if (p.grid < 1 || p.map_grid < 1) return fail(NRM_EINVAL, "grid and map_grid must be positive");
  if (!ok_l(p.layout) || !ok_l(p.map_layout)) return fail(NRM_EINVAL, "unknown layout");
  // h <= max_height + 26 levels: gamma_h + u stays below 4e-6 up to max_height 40 (h = 66)
  if (p.max_height < 24 || p.max_height > 40) return fail(NRM_EINVAL, "max_height must be 24..40");
  if (!ok_f(p.reduce_nt) || !ok_f(p.map_nt) || !ok_f(p.reverse_map))
    return fail(NRM_EINVAL, "reduce_nt, map_nt and reverse_map must be 0 or 1");
  if (p.reduce_keep_mib < 0 || p.reduce_keep_mib > 4096) return fail(NRM_EINVAL, "reduce_keep_mib must be 0..4096");
  if (p.tile_log2 < 10 || p.tile_log2 > 22) return fail(NRM_EINVAL, "tile_log2 must be 10..22");
  if (!ok_f(p.fused_combine)) return fail(NRM_EINVAL, "fused_combine must be 0 or 1");
  if (p.small_n < 0 || p.small_n > (1 << 16)) return fail(NRM_EINVAL, "small_n must be 0..2^16");
  if (p.resident_n < 0 || p.resident_n > (1 << 20)) return fail(NRM_EINVAL, "resident_n must be 0..2^20");
  return NRM_OK;
}

// The context's small workspace: the ticket (0), the sum (128), the device
// error word (192), the mid-size single-launch form's call number (256),
// arrival count (264), stall marker (272) and merged total (288), and from
// 512 its segments' tagged partials (256 x 16 bytes).
constexpr size_t kSmallWs = 512 + 256 * 16;

std::mutex g_default_mu;
std::map<int, nrm_ctx*> g_default;

}  // namespace

namespace nrm {
int default_ctx(nrm_ctx** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_default_mu);
  auto it = g_default.find(dev);
  if (it != g_default.end()) {
    *out = it->second;
    return NRM_OK;
  }
  nrm_ctx* c = nullptr;
  int st = nrm_create(&c, dev);
  if (st != NRM_OK) return st;
  g_default[dev] = c;
  *out = c;
  return NRM_OK;
}
}  // namespace nrm

namespace {


// Reduce blocks of the NLL loss: enough loads in flight for the gathers,
// few enough partials for the one-block combine.
constexpr int64_t kNllMaxGrid = 1024;  // 1024 partials: the one-wavefront merge (2048 blocks ran 4 % slower)

int ensure_partials(nrm_ctx* c, int64_t entries) {
  if (entries <= c->partials_cap) return NRM_OK;
  int64_t cap = std::max<int64_t>(entries, 16384);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, (size_t)cap * 8);
  if (e != hipSuccess) return fail(NRM_ENOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
  if (c->partials) {
    hipError_t e2 = hipDeviceSynchronize();  // the old buffer may still be in use
    (void)hipFree(c->partials);  // freed whatever the sync reported
    if (e2 != hipSuccess) return hip_fail(e2, "hipDeviceSynchronize");
  }
  c->partials = p;
  c->partials_cap = cap;
  return NRM_OK;
}


bool valid_dtype(int dt) { return dt == NRM_F32 || dt == NRM_BF16 || dt == NRM_F16; }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Blocks and per-block chunk for `nvec` vectors in steps of `step` vectors,
// at most `max_blocks` blocks unless `max_iters` per block forces more.
void split(int64_t nvec, int64_t step, int64_t max_blocks, int64_t max_iters, int64_t* blocks,
           int64_t* chunk) {
  int64_t iters = ceil_div(nvec, step);
  if (iters == 0) {
    *blocks = 1;
    *chunk = step;
    return;
  }
  int64_t b = std::min(max_blocks, iters);
  if (max_iters > 0) b = std::max(b, ceil_div(iters, max_iters));
  int64_t per = ceil_div(iters, b);
  *blocks = ceil_div(iters, per);
  *chunk = per * step;
}

}  // namespace

namespace nrm {

int plan_plain(const nrm_params& q, void* out, int out_dt, const void* in, int in_dt, int64_t n, int acc,
               PlainPlan* p) {
  const int si = nrm::dtype_size(in_dt), so = nrm::dtype_size(out_dt);
  const uintptr_t ai = reinterpret_cast<uintptr_t>(in), ao = reinterpret_cast<uintptr_t>(out);
  if (ai % si) return fail(NRM_EINVAL, "in is not aligned to its element size");
  if (ao % so) return fail(NRM_EINVAL, "out is not aligned to its element size");
  const int vec = nrm::dtype_vec(in_dt);
  p->in = in;
  p->out = out;
  p->n = n;
  p->in_dt = in_dt;
  p->out_dt = out_dt;
  p->acc = acc;
  // The vector body starts on a 128-byte line so that every wavefront's
  // accesses cover whole lines (partial lines at both ends of each access
  // cost about a tenth of the bandwidth with non-temporal stores); the head
  // before it (at most 63 elements) is handled by block 0, one per thread.
  int64_t mis = (int64_t)(ai & 127);
  p->head = std::min<int64_t>(mis ? (128 - mis) / si : 0, n);
  p->nvec = (n - p->head) / vec;
  p->tail_begin = p->head + p->nvec * vec;
  const int64_t out_align = std::min(16, vec * so);
  p->vector_map = ((ao + (uintptr_t)(p->head * so)) % (uintptr_t)out_align) == 0;
  p->block = q.block;
  p->unroll = q.unroll;
  p->layout = q.layout;
  p->reduce_nt = q.reduce_nt;
  p->map_block = q.map_block;
  p->map_unroll = q.map_unroll;
  p->map_layout = q.map_layout;
  p->map_nt = q.map_nt;
  p->reverse_map = q.reverse_map;
  p->keep_from = std::max<int64_t>(0, p->nvec - ((int64_t)q.reduce_keep_mib << 20) / 16);
  // Iterations per reduce block are bounded so that the height of a thread's
  // summation tree stays within max_height (plain mode); compensated chains
  // have no such bound (their error does not grow with the chain).
  int64_t max_iters = 0;
  if (acc == NRM_ACC_F32) {
    max_iters = 1;
    while (nrm::thread_tree_height(in_dt, acc, q.unroll, max_iters + 1) <= q.max_height) ++max_iters;
  }
  const int64_t step = (int64_t)q.block * q.unroll;
  split(p->nvec, step, q.grid, max_iters, &p->grid, &p->chunk);
  p->tile = 0;
  if (q.layout == NRM_LAYOUT_TILE) {
    // whole block-iterations per tile; a block's tiles together stay within
    // max_iters iterations
    int64_t per_tile = std::max<int64_t>(1, ceil_div((int64_t(1) << q.tile_log2) / vec, step));
    if (max_iters > 0) per_tile = std::min(per_tile, max_iters);
    p->tile = per_tile * step;
    const int64_t ntiles = std::max<int64_t>(1, ceil_div(p->nvec, p->tile));
    int64_t g = std::min<int64_t>(q.grid, ntiles);
    if (max_iters > 0) g = std::max(g, ceil_div(ntiles, max_iters / per_tile));
    p->grid = g;
  }
  p->map_units = (si == 2 && so == 4) ? 2 * p->nvec : p->nvec;
  const int64_t map_step = (int64_t)q.map_block * q.map_unroll;
  split(p->map_units, map_step, q.map_grid, 0, &p->map_grid, &p->map_chunk);
  p->map_tile = 0;
  if (q.map_layout == NRM_LAYOUT_TILE) {
    const int unit_elems = (si == 2 && so == 4) ? 4 : vec;
    p->map_tile = std::max<int64_t>(1, ceil_div((int64_t(1) << q.tile_log2) / unit_elems, map_step)) * map_step;
    p->map_grid = std::min<int64_t>(q.map_grid, std::max<int64_t>(1, ceil_div(p->map_units, p->map_tile)));
  }
  p->fused = q.fused_combine && p->vector_map && p->grid <= 1024;
  if (p->grid > 65536) return fail(NRM_EINVAL, "n too large for these launch parameters (over 65536 reduce blocks)");
  if (p->map_grid > INT32_MAX) return fail(NRM_EINVAL, "n too large for one launch");
  return NRM_OK;
}

nrm_params device_params(int device) {
  nrm_params p = default_params();
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0) {
    p.grid = 2 * cus;       // reduce: 2 blocks per CU
    p.map_grid = 64 * cus;  // map: 64 blocks per CU
  }
  return p;
}

}  // namespace nrm

namespace {

bool ranges_partially_overlap(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
  uintptr_t a0 = (uintptr_t)a, a1 = a0 + (uintptr_t)abytes;
  uintptr_t b0 = (uintptr_t)b, b1 = b0 + (uintptr_t)bbytes;
  bool overlap = a0 < b1 && b0 < a1;
  bool identical = a0 == b0 && abytes == bbytes;
  return overlap && !identical;
}

}  // namespace

extern "C" {

namespace {
bool overlaps(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
  if (!a || !b || abytes <= 0 || bbytes <= 0) return false;
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + (uintptr_t)abytes, b0 = (uintptr_t)b, b1 = b0 + (uintptr_t)bbytes;
  return a0 < b1 && b0 < a1;
}
}  // namespace

int nrm_nll_loss(nrm_ctx* c, float* out, float* total_weight, const float* logp, const int64_t* target,
                 const float* weight, int64_t n, int64_t classes, int64_t ignore_index, int reduction, int accum,
                 void* stream) {
  if (n < 0) return fail(NRM_EINVAL, "n < 0");
  if (classes < 1) return fail(NRM_EINVAL, "classes < 1");
  if (reduction != NRM_NLL_NONE && reduction != NRM_NLL_SUM && reduction != NRM_NLL_MEAN)
    return fail(NRM_EINVAL, "unknown reduction");
  if (accum != NRM_ACC_F32 && accum != NRM_ACC_KAHAN) return fail(NRM_EINVAL, "unknown accumulation mode");
  if (n > 0 && classes > INT64_MAX / 4 / n) return fail(NRM_EINVAL, "n * classes too large");
  if (n == 0 && reduction == NRM_NLL_NONE) return NRM_OK;
  if (!out || (n > 0 && (!logp || !target))) return fail(NRM_EINVAL, "NULL pointer");
  auto misaligned = [](const void* p, size_t a) { return p && reinterpret_cast<uintptr_t>(p) % a; };
  if (misaligned(out, 4) || misaligned(total_weight, 4) || misaligned(logp, 4) || misaligned(weight, 4) ||
      misaligned(target, 8))
    return fail(NRM_EINVAL, "pointer not aligned to its element size");
  const int64_t out_bytes = 4 * (reduction == NRM_NLL_NONE ? n : 1);
  const int64_t logp_bytes = 4 * n * classes, target_bytes = 8 * n, weight_bytes = weight ? 4 * classes : 0;
  for (const auto& o : {std::make_pair((const void*)out, out_bytes), std::make_pair((const void*)total_weight,
                                                                                     (int64_t)(total_weight ? 4 : 0))})
    if (overlaps(o.first, o.second, logp, logp_bytes) || overlaps(o.first, o.second, target, target_bytes) ||
        overlaps(o.first, o.second, weight, weight_bytes))
      return fail(NRM_EOVERLAP, "an output overlaps an input");
  if (overlaps(out, out_bytes, total_weight, total_weight ? 4 : 0))
    return fail(NRM_EOVERLAP, "out and total_weight overlap");
  if (!c) {
    int st = nrm::default_ctx(&c);
    if (st != NRM_OK) return st;
  }
  nrm::CtxLock lk(c->mu);
  DeviceGuard g(c->device);
  nrm::NllPlan p;
  p.logp = logp;
  p.target = target;
  p.weight = weight;
  p.n = n;
  p.c = classes;
  p.ignore = ignore_index;
  p.reduction = reduction;
  p.acc = accum;
  p.out = out;
  p.total_weight = total_weight;
  p.grid = nrm::nll_grid(n, kNllMaxGrid);
  int st = ensure_partials(c, 2 * p.grid);
  if (st != NRM_OK) return st;
  hipError_t e = nrm::launch_nll(p, c->partials, c->dev_error, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "NLL kernel launch");
  return NRM_OK;
}

int nrm_layerforward(int form, float* hidden, const float* input, float* output, int64_t rows, void* stream) {
  if (form != NRM_LF_ALL_BARRIERS && form != NRM_LF_ELIMINATED && form != NRM_LF_PROMOTED && form != NRM_LF_REGISTERS)
    return fail(NRM_EINVAL, "unknown form");
  if (rows < 0 || rows % 16) return fail(NRM_EINVAL, "rows must be a non-negative multiple of 16");
  if (rows / 16 > INT32_MAX) return fail(NRM_EINVAL, "too many rows for one launch");
  if (rows == 0) return NRM_OK;
  if (!hidden || !input || !output) return fail(NRM_EINVAL, "NULL pointer");
  auto misaligned = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 4 != 0; };
  if (misaligned(hidden) || misaligned(input) || misaligned(output))
    return fail(NRM_EINVAL, "pointer not aligned to 4 bytes");
  if (overlaps(hidden, 64 * rows, input, 4 * rows) || overlaps(hidden, 64 * rows, output, 4 * rows) ||
      overlaps(input, 4 * rows, output, 4 * rows))
    return fail(NRM_EOVERLAP, "hidden, input and output must not overlap");
  hipError_t e = nrm::launch_layerforward(form, hidden, input, output, rows, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "layerforward kernel launch");
  return NRM_OK;
}

}  // extern "C"

namespace nrm {
int check_plain_args(const void* out, int out_dtype, const void* in, int in_dtype, int64_t n, int accum) {
  if (n < 0) return fail(NRM_EINVAL, "n < 0");
  if (!valid_dtype(in_dtype) || !valid_dtype(out_dtype)) return fail(NRM_EINVAL, "unknown dtype");
  if (accum != NRM_ACC_F32 && accum != NRM_ACC_KAHAN) return fail(NRM_EINVAL, "unknown accumulation mode");
  if (n == 0) return NRM_OK;
  if (!in || !out) return fail(NRM_EINVAL, "NULL data pointer with n > 0");
  const int64_t si = dtype_size(in_dtype), so = dtype_size(out_dtype);
  if (n > INT64_MAX / 8) return fail(NRM_EINVAL, "n too large");
  if (ranges_partially_overlap(in, n * si, out, n * so))
    return fail(NRM_EOVERLAP, "in and out overlap without being the same array");
  if (reinterpret_cast<uintptr_t>(in) % si) return fail(NRM_EINVAL, "in is not aligned to its element size");
  if (reinterpret_cast<uintptr_t>(out) % so) return fail(NRM_EINVAL, "out is not aligned to its element size");
  return NRM_OK;
}
}  // namespace nrm

extern "C" {

const char* nrm_status_string(int status) {
  switch (status) {
    case NRM_OK: return "ok";
    case NRM_EINVAL: return "invalid argument";
    case NRM_EOVERLAP: return "input and output overlap without being the same array";
    case NRM_ENOMEM: return "workspace allocation failed";
    case NRM_EHIP: return "HIP runtime error";
    case NRM_EUNSUPPORTED: return "unsupported dtype or mode";
    case NRM_EDEVICE: return "the device reported invalid data";
    default: return "unknown status";
  }
}

const char* nrm_last_error(void) { return nrm::last_error().c_str(); }

int nrm_create(nrm_ctx** ctx, int device) {
  if (!ctx) return fail(NRM_EINVAL, "ctx is NULL");
  *ctx = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0) {
    e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  }
  if (device >= count) return fail(NRM_EINVAL, "no such device");
  DeviceGuard g(device);
  nrm_ctx* c = new nrm_ctx();
  c->device = device;
  c->params = nrm::device_params(device);
  c->arch = nrm::device_arch(device);
  nrm_default_batch_params(&c->bparams);
  void* small = nullptr;
  e = hipMalloc(&small, kSmallWs);
  if (e != hipSuccess) {
    delete c;
    return fail(NRM_ENOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
  }
  e = hipMemset(small, 0, kSmallWs);
  if (e != hipSuccess) {
    (void)hipFree(small);  // already failing
    delete c;
    return hip_fail(e, "hipMemset");
  }
  char* sm = static_cast<char*>(small);
  c->ticket = reinterpret_cast<unsigned*>(sm);
  c->sum = reinterpret_cast<float*>(sm + 128);
  c->dev_error = reinterpret_cast<int*>(sm + 192);
  c->res = nrm::PlainResidentWs{reinterpret_cast<unsigned long long*>(sm + 512),
                                reinterpret_cast<unsigned long long*>(sm + 288), reinterpret_cast<unsigned*>(sm + 264),
                                reinterpret_cast<unsigned long long*>(sm + 256),
                                reinterpret_cast<unsigned long long*>(sm + 272), c->dev_error, c->sum};
  int st = ensure_partials(c, 16384);
  if (st != NRM_OK) {
    (void)hipFree(small);
    delete c;
    return st;
  }
  *ctx = c;
  return NRM_OK;
}

int nrm_destroy(nrm_ctx* c) {
  if (!c) return NRM_OK;
  {
    std::lock_guard<std::mutex> lk(g_default_mu);
    for (auto it = g_default.begin(); it != g_default.end(); ++it)
      if (it->second == c) return fail(NRM_EINVAL, "the default context cannot be destroyed");
  }
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();  // teardown: errors were reported by the calls themselves
  for (hipEvent_t ev : c->events) (void)hipEventDestroy(ev);
  nrm::batch_free(c);
  if (c->partials) (void)hipFree(c->partials);
  if (c->ticket) (void)hipFree(c->ticket);
  delete c;
  return NRM_OK;
}

int nrm_default_params(nrm_params* params) {
  if (!params) return fail(NRM_EINVAL, "NULL argument");
  *params = default_params();
  return NRM_OK;
}

int nrm_set_params(nrm_ctx* c, const nrm_params* params) {
  if (!c || !params) return fail(NRM_EINVAL, "NULL argument");
  nrm::CtxLock lk(c->mu);
  int st = check_params(*params);
  if (st != NRM_OK) return st;
  c->params = *params;
  c->params_set = true;  // explicit parameters replace the tuning cache's
  return NRM_OK;
}

int nrm_get_params(const nrm_ctx* c, nrm_params* params) {
  if (!c || !params) return fail(NRM_EINVAL, "NULL argument");
  nrm::CtxLock lk(c->mu);
  *params = c->params;
  return NRM_OK;
}

int nrm_set_timing(nrm_ctx* c, int enable) {
  if (!c) return fail(NRM_EINVAL, "ctx is NULL");
  nrm::CtxLock lk(c->mu);
  if (enable && c->events.empty()) {
    DeviceGuard g(c->device);
    c->events.resize(3 * kTimingRing);
    for (auto& ev : c->events) {
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    c->batch.events.resize(2 * kTimingRing);
    for (auto& ev : c->batch.events) {
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
  }
  c->timing = enable != 0;
  c->timed_calls = 0;
  c->batch.timed_calls = 0;
  return NRM_OK;
}

int nrm_kernel_times(nrm_ctx* c, double* reduce_ms, double* map_ms, int64_t* calls) {
  if (!c) return fail(NRM_EINVAL, "ctx is NULL");
  nrm::CtxLock lk(c->mu);
  double r = 0, m = 0;
  int64_t k = std::min<int64_t>(c->timed_calls, kTimingRing);
  for (int64_t i = 0; i < k; ++i) {
    hipEvent_t* ev = &c->events[3 * i];
    hipError_t e = hipEventSynchronize(ev[2]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float a = 0, b = 0;
    e = hipEventElapsedTime(&a, ev[0], ev[1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    e = hipEventElapsedTime(&b, ev[1], ev[2]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    r += a;
    m += b;
  }
  if (reduce_ms) *reduce_ms = r;
  if (map_ms) *map_ms = m;
  if (calls) *calls = k;
  return NRM_OK;
}

namespace {
// The parameters of one call: the context's explicit ones, or the tuning
// cache's entry for the call's key over the context's defaults (looked up
// once per key and context).
const nrm_params& call_params(nrm_ctx* c, int in_dt, int out_dt, int acc, int64_t n) {
  if (c->params_set) return c->params;
  int k = 0;
  while ((int64_t(1) << (k + 1)) <= n && k < 62) ++k;
  const int64_t key = ((int64_t)(in_dt * 3 + out_dt) * 2 + acc) * 64 + k;
  auto it = c->tuned.find(key);
  if (it == c->tuned.end()) {
    nrm_params q = c->params;
    bool has = nrm::tuned_plain(c->arch, in_dt, out_dt, acc, n, &q);
    if (has && check_params(q) != NRM_OK) has = false;  // an entry this build would reject
    it = c->tuned.emplace(key, std::make_pair(has, q)).first;
  }
  return it->second.first ? it->second.second : c->params;
}
}  // namespace

int nrm_normalize_ex(nrm_ctx* c, void* out, int out_dtype, const void* in, int in_dtype, int64_t n,
                     int accum, void* stream) {
  int st0 = nrm::check_plain_args(out, out_dtype, in, in_dtype, n, accum);
  if (st0 != NRM_OK || n == 0) return st0;
  if (!c) {
    int st = nrm::default_ctx(&c);
    if (st != NRM_OK) return st;
  }
  nrm::CtxLock lk(c->mu);
  const nrm_params& q = call_params(c, in_dtype, out_dtype, accum, n);
  if (n <= q.small_n && n <= nrm::small_capacity(in_dtype)) {
    // one block, the input held in registers: one read, one write, one launch
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t* ev = nullptr;
    if (c->timing) {
      ev = &c->events[3 * (c->timed_calls % kTimingRing)];
      c->timed_calls++;
      (void)hipEventRecord(ev[0], s);
    }
    hipError_t e = nrm::launch_small(in, in_dtype, out, out_dtype, n, accum, c->sum, s);
    if (e != hipSuccess) return hip_fail(e, "small normalize kernel launch");
    if (ev) {
      (void)hipEventRecord(ev[1], s);
      (void)hipEventRecord(ev[2], s);
    }
    return NRM_OK;
  }
  if (n <= q.resident_n && n <= nrm::plain_resident_capacity()) {
    // one block per segment, held in registers across the exchange of sums
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t* ev = nullptr;
    if (c->timing) {
      ev = &c->events[3 * (c->timed_calls % kTimingRing)];
      c->timed_calls++;
      (void)hipEventRecord(ev[0], s);
    }
    hipError_t e = nrm::launch_plain_resident(in, in_dtype, out, out_dtype, n, accum, c->res, s);
    if (e != hipSuccess) return hip_fail(e, "mid-size normalize kernel launch");
    if (ev) {
      (void)hipEventRecord(ev[1], s);
      (void)hipEventRecord(ev[2], s);
    }
    return NRM_OK;
  }
  nrm::PlainPlan plan;
  int st = nrm::plan_plain(q, out, out_dtype, in, in_dtype, n, accum, &plan);
  if (st != NRM_OK) return st;
  DeviceGuard g(c->device);
  st = ensure_partials(c, plan.grid);
  if (st != NRM_OK) return st;
  nrm::PlainWorkspace ws{c->partials, c->ticket, c->sum};
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t* ev = nullptr;
  if (c->timing) {
    ev = &c->events[3 * (c->timed_calls % kTimingRing)];
    c->timed_calls++;
    (void)hipEventRecord(ev[0], s);
  }
  hipError_t e = nrm::launch_reduce(plan, ws, s);
  if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  if (ev) (void)hipEventRecord(ev[1], s);
  e = nrm::launch_map(plan, ws, s);
  if (e != hipSuccess) return hip_fail(e, "map kernel launch");
  if (ev) (void)hipEventRecord(ev[2], s);
  return NRM_OK;
}

int nrm_get_last_sum(nrm_ctx* c, void* stream, float* sum) {
  if (!sum) return fail(NRM_EINVAL, "sum is NULL");
  if (!c) {
    int st = nrm::default_ctx(&c);
    if (st != NRM_OK) return st;
  }
  nrm::CtxLock lk(c->mu);
  DeviceGuard g(c->device);
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = hipMemcpy(sum, c->sum, sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "reading the last sum");
  return NRM_OK;
}

int nrm_normalize_form(int form, float* out, const float* in, int64_t n, int block, void* stream) {
  if (form != NRM_FORM_NAIVE && form != NRM_FORM_PERBLOCK) return fail(NRM_EINVAL, "unknown form");
  if (n < 1 || n > (int64_t(1) << 20)) return fail(NRM_EINVAL, "n must be 1..2^20");
  if (block < 64 || block > 1024 || block % 64) return fail(NRM_EINVAL, "block must be 64..1024, a multiple of 64");
  if (!in || !out) return fail(NRM_EINVAL, "NULL data pointer");
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) % 4)
    return fail(NRM_EINVAL, "pointers must be 4-byte aligned");
  if (ranges_partially_overlap(in, n * 4, out, n * 4) || in == out)
    return fail(NRM_EOVERLAP, "the un-hoisted forms read the input while others write: in and out must not overlap");
  hipError_t e = nrm::launch_form(form, out, in, n, block, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "form kernel launch");
  return NRM_OK;
}

int nrm_ceiling(int kind, void* dst, const void* src, int64_t bytes, int64_t grid, void* stream) {
  if (kind != NRM_CEILING_COPY && kind != NRM_CEILING_READ) return fail(NRM_EINVAL, "unknown ceiling kind");
  if (bytes < 0 || bytes % 16) return fail(NRM_EINVAL, "bytes must be a non-negative multiple of 16");
  if (grid < 1 || grid > (1 << 20)) return fail(NRM_EINVAL, "grid must be 1..2^20");
  if (bytes == 0) return NRM_OK;
  if (!dst || !src) return fail(NRM_EINVAL, "NULL pointer");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return fail(NRM_EINVAL, "pointers must be 16-byte aligned");
  const int64_t dst_bytes = kind == NRM_CEILING_COPY ? bytes : 4 * grid;
  if (overlaps(dst, dst_bytes, src, bytes)) return fail(NRM_EOVERLAP, "dst overlaps src");
  hipError_t e = nrm::launch_ceiling(kind, dst, src, bytes, grid, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "ceiling kernel launch");
  return NRM_OK;
}

int normalize(float* out, const float* in, int64_t n) {
  return nrm_normalize_ex(nullptr, out, NRM_F32, in, NRM_F32, n, NRM_ACC_F32, nullptr);
}

}  // extern "C"
