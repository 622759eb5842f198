// C ABI of the ragged batched path (include/nrm.h): workspace and pinned
// staging management, host validation, the launch sequence (planner, the
// resident rows, phase 1, row sums, phase 2) and its optional capture in a
// hipGraph. The per-call header and row table are written to pinned,
// coherent host memory that the planner reads in place, so a captured graph
// replays new batches unchanged; a ring of such buffers (one graph each) lets
// a call be enqueued while the previous ones still run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "nrm_ctx.h"

using nrm::BatchArgs;
using nrm::BatchHeader;
using nrm::BatchPlan;
using nrm::BatchWorkspace;
using nrm::DeviceGuard;
using nrm::RowDesc;
using nrm::fail;
using nrm::hip_fail;

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Staging layout: the header, then the row table from this offset.
constexpr size_t kTableOffset = 256;
// The planner's counters, then the device error word, in one small region.
constexpr size_t kErrorOffset = sizeof(int64_t) * nrm::CNT_COUNT;
constexpr size_t kSmallBytes = 128;
static_assert(kErrorOffset + sizeof(int) <= kSmallBytes, "counters and error word must fit");
static_assert(sizeof(BatchHeader) <= kTableOffset, "header must fit before the table");
int64_t align_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

nrm_batch_params default_batch_params() {
  nrm_batch_params p;
  std::memset(&p, 0, sizeof(p));
  // On MI355X: within a few percent of the tuner's best for the 4096-row
  // ragged workload, and with persistent grids small enough that small
  // batches (serving) do not pay for dispatching idle blocks.
  p.block = 256;
  p.unroll = 8;
  p.map_unroll = 4;
  p.grid = 2048;
  p.tile_log2 = 15;
  p.short_regs = 4;
  p.graph = 1;  // replay captured graphs (one per staging buffer and reduction kind)
  p.map_block = 1024;
  p.map_grid = 1024;
  p.keep_mib = 256;
  // rows up to 64 segments of 2^14 elements (2^20) are held on chip between
  // their read and their write; two 512-thread blocks per CU
  p.resident_segments = 64;
  p.resident_grid = 512;
  // rows of up to 2048 elements one per wavefront, 16 wavefronts per CU
  p.wave_max = 2048;
  p.wave_grid = 1024;
  return p;
}

int check_batch_params(const nrm_batch_params& p) {
  auto ok_u = [](int u) { return u == 1 || u == 2 || u == 4 || u == 8; };
  if (p.block < 64 || p.block > 1024 || p.block % 64 || p.map_block < 64 || p.map_block > 1024 || p.map_block % 64)
    return fail(NRM_EINVAL, "block and map_block must be 64..1024, multiples of 64");
  if (p.map_grid < 1 || p.map_grid > (1 << 20)) return fail(NRM_EINVAL, "map_grid must be 1..2^20");
  if (!ok_u(p.unroll) || !ok_u(p.map_unroll) || !ok_u(p.short_regs))
    return fail(NRM_EINVAL, "unroll, map_unroll and short_regs must be 1, 2, 4 or 8");
  if (p.grid < 1 || p.grid > (1 << 20)) return fail(NRM_EINVAL, "grid must be 1..2^20");
  if (p.tile_log2 < 10 || p.tile_log2 > 22) return fail(NRM_EINVAL, "tile_log2 must be 10..22");
  if (p.graph != 0 && p.graph != 1) return fail(NRM_EINVAL, "graph must be 0 or 1");
  if (p.keep_mib < 0 || p.keep_mib > 4096) return fail(NRM_EINVAL, "keep_mib must be 0..4096");
  if (p.resident_segments < 0 || p.resident_segments > nrm::RES_MAX_SEGMENTS)
    return fail(NRM_EINVAL, "resident_segments must be 0..64");
  if (p.resident_grid < 1 || p.resident_grid > (1 << 20)) return fail(NRM_EINVAL, "resident_grid must be 1..2^20");
  // the blocks of one resident row wait for each other: the kernel must be
  // able to hold a whole row's segments in running blocks at once
  if (p.resident_grid < p.resident_segments)
    return fail(NRM_EINVAL, "resident_grid must be at least resident_segments");
  if (p.wave_max < 0 || p.wave_max > nrm::WAVE_MAX_ELEMS) return fail(NRM_EINVAL, "wave_max must be 0..2048");
  if (p.wave_grid < 1 || p.wave_grid > (1 << 20)) return fail(NRM_EINVAL, "wave_grid must be 1..2^20");
  // a tile's per-thread summation tree must stay within the plain path's
  // height bound (36) for every input dtype: 4-byte elements give the most
  // iterations, 2-byte elements the most additions per iteration
  const int64_t tile = int64_t(1) << p.tile_log2;
  for (int dt : {NRM_F32, NRM_BF16}) {
    int64_t iters = ceil_div(tile, (int64_t)p.block * p.unroll * nrm::dtype_vec(dt));
    if (nrm::thread_tree_height(dt, NRM_ACC_F32, p.unroll, iters) > 36)
      return fail(NRM_EINVAL, "tile too long for block * unroll: a thread's summation tree would exceed height 36");
  }
  return NRM_OK;
}

// Rows of at most this many elements are not long: single-pass rows, or
// resident rows when those are on.
int64_t short_max_of(const nrm_batch_params& p) {
  return p.resident_segments > 0 ? (int64_t)p.resident_segments << nrm::RES_LOG2 : (int64_t)p.block * p.short_regs * 4;
}

bool any_graph(const BatchWorkspace& w) {
  for (const auto& per_kind : w.graph)
    for (hipGraphExec_t g : per_kind)
      if (g) return true;
  return false;
}

void destroy_graph(BatchWorkspace& w) {
  for (auto& per_kind : w.graph)
    for (hipGraphExec_t& g : per_kind) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Layout of the single device allocation.
struct Layout {
  size_t rows, items, lrow_first, lrows, lstart, lsum, chunk_lrow, round_agg, hdr_dev, small, partials, tagged, rowtot,
      arrivals, total;
};

// Phase-2 chunks a workspace holds beyond one per item: the planner sizes the
// chunks to a multiple of the phase-2 grid when this allows it.
constexpr int64_t kExtraChunks = 2048;

Layout layout_for(int64_t cap_rows, int64_t cap_items, int64_t cap_chunks) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = (size_t)align_up((int64_t)(off + bytes), 256);
    return at;
  };
  L.rows = take(sizeof(RowDesc) * cap_rows);
  L.items = take(sizeof(nrm::Item) * cap_items);
  L.lrow_first = take(sizeof(int64_t) * cap_rows);
  L.lrows = take(sizeof(RowDesc) * cap_rows);
  L.lstart = take(sizeof(int64_t) * cap_rows);
  L.lsum = take(sizeof(nrm::RowRes) * cap_rows);
  L.chunk_lrow = take(sizeof(int32_t) * cap_chunks);
  L.round_agg = take(sizeof(int64_t) * 4 * (size_t)ceil_div(cap_rows, nrm::PLAN_ROUND_ROWS));
  L.hdr_dev = take(sizeof(BatchHeader));
  L.small = take(kSmallBytes);  // the planner's counters, then the error word
  L.partials = take(8 * cap_items);
  L.tagged = take(16 * cap_items);
  L.rowtot = take(16 * cap_items);
  L.arrivals = take(4 * cap_items);
  L.total = off;
  return L;
}

int reserve(nrm_ctx* c, int64_t rows, int64_t items) {
  BatchWorkspace& w = c->batch;
  if (rows <= w.cap_rows && items <= w.cap_items && w.dev) return NRM_OK;
  int64_t cap_rows = std::max<int64_t>({rows, w.cap_rows, 64});
  int64_t cap_items = std::max<int64_t>({items, w.cap_items, 1024});
  const int64_t cap_chunks = cap_items + kExtraChunks;
  Layout L = layout_for(cap_rows, cap_items, cap_chunks);
  // the old buffers may still be in use by enqueued work
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  destroy_graph(w);
  void* dev = nullptr;
  e = hipMalloc(&dev, L.total);
  if (e != hipSuccess) return fail(NRM_ENOMEM, std::string("batched workspace hipMalloc: ") + hipGetErrorString(e));
  // Per-call header and row table: pinned, coherent host memory that the
  // planner reads directly (no copy, no DMA latency per call).
  void* host = nullptr;
  const size_t staging = (size_t)align_up((int64_t)(kTableOffset + sizeof(RowDesc) * (size_t)cap_rows), 256);
  e = hipHostMalloc(&host, staging * nrm::kStagingRing, hipHostMallocCoherent | hipHostMallocMapped);
  if (e != hipSuccess) {
    (void)hipFree(dev);  // already failing
    return fail(NRM_ENOMEM, std::string("pinned staging hipHostMalloc: ") + hipGetErrorString(e));
  }
  void* host_dev = nullptr;
  e = hipHostGetDevicePointer(&host_dev, host, 0);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    (void)hipHostFree(host);
    return hip_fail(e, "hipHostGetDevicePointer");
  }
  int err_word = 0;
  if (w.dev) {
    // keep a pending device error of the old workspace
    e = hipMemcpy(&err_word, w.error, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {  // the old workspace stays as it was
      (void)hipFree(dev);
      (void)hipHostFree(host);
      return hip_fail(e, "hipMemcpy (device error word)");
    }
    (void)hipFree(w.dev);
  }
  if (w.host) (void)hipHostFree(w.host);
  char* d = static_cast<char*>(dev);
  w.dev = dev;
  w.host = host;
  w.staging = staging;
  w.next = 0;
  for (int b = 0; b < nrm::kStagingRing; ++b) {
    char* base = static_cast<char*>(host_dev) + staging * b;
    w.hdr[b] = reinterpret_cast<BatchHeader*>(base);
    w.table[b] = reinterpret_cast<RowDesc*>(base + kTableOffset);
  }
  w.rows = reinterpret_cast<RowDesc*>(d + L.rows);
  w.items = reinterpret_cast<nrm::Item*>(d + L.items);
  w.lrow_first = reinterpret_cast<int64_t*>(d + L.lrow_first);
  w.lrows = reinterpret_cast<RowDesc*>(d + L.lrows);
  w.lstart = reinterpret_cast<int64_t*>(d + L.lstart);
  w.lsum = reinterpret_cast<nrm::RowRes*>(d + L.lsum);
  w.chunk_lrow = reinterpret_cast<int32_t*>(d + L.chunk_lrow);
  w.round_agg = reinterpret_cast<int64_t*>(d + L.round_agg);
  w.hdr_dev = reinterpret_cast<BatchHeader*>(d + L.hdr_dev);
  w.cnt = reinterpret_cast<int64_t*>(d + L.small);
  w.error = reinterpret_cast<int*>(d + L.small + kErrorOffset);
  w.partials = d + L.partials;
  w.tagged = reinterpret_cast<unsigned long long*>(d + L.tagged);
  w.rowtot = reinterpret_cast<unsigned long long*>(d + L.rowtot);
  w.arrivals = reinterpret_cast<unsigned*>(d + L.arrivals);
  w.cap_rows = cap_rows;
  w.cap_items = cap_items;
  w.cap_chunks = cap_chunks;
  for (bool& p : w.staged_pending) p = false;
  // the counters (the call number starts at 0) and the resident rows' tags
  e = hipMemset(d + L.small, 0, kSmallBytes);
  // tags, totals and arrival counts: contiguous, all start at 0
  if (e == hipSuccess) e = hipMemset(d + L.tagged, 0, L.total - L.tagged);
  if (e == hipSuccess && err_word) e = hipMemcpy(w.error, &err_word, sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemset");
  for (hipEvent_t& ev : w.staged)
    if (!ev) {
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
  return NRM_OK;
}

// Items a batch of `rows` rows and at most `elems` elements can need.
int64_t items_bound(const nrm_batch_params& p, int64_t rows, int64_t elems) {
  // a long row has ceil(n / tile) items, a resident row ceil(n / 2^RES_LOG2)
  const int lg = p.resident_segments > 0 ? std::min(p.tile_log2, nrm::RES_LOG2) : p.tile_log2;
  return rows + ceil_div(std::max<int64_t>(elems, 0), int64_t(1) << lg);
}

BatchArgs args_of(const nrm_ctx* c, int buf) {
  const BatchWorkspace& w = c->batch;
  BatchArgs a;
  a.hdr = w.hdr[buf];
  a.rows = w.rows;
  a.items = w.items;
  a.lrow_first = w.lrow_first;
  a.lrows = w.lrows;
  a.lstart = w.lstart;
  a.lsum = w.lsum;
  a.chunk_lrow = w.chunk_lrow;
  a.cnt = w.cnt;
  a.error = w.error;
  a.partials = w.partials;
  a.cap_rows = w.cap_rows;
  a.cap_items = w.cap_items;
  a.cap_chunks = w.cap_chunks;
  a.tile = int64_t(1) << c->bparams.tile_log2;
  a.tile_log2 = c->bparams.tile_log2;
  a.short_max = short_max_of(c->bparams);
  a.map_grid = c->bparams.map_grid;
  a.min_chunk = (int64_t)c->bparams.map_block * c->bparams.map_unroll * 4;
  // tiles counted at 4 bytes per element: at most keep_mib MiB for any dtype
  a.keep_tiles = ((int64_t)c->bparams.keep_mib << 20) / (a.tile * 4);
  a.res_on = c->bparams.resident_segments > 0;
  a.tagged = w.tagged;
  a.rowtot = w.rowtot;
  a.arrivals = w.arrivals;
  a.wave_max = c->bparams.wave_max;
  a.split_plan = w.cap_rows > nrm::PLAN_SPLIT_ROWS;
  a.round_agg = w.round_agg;
  a.hdr_dev = w.hdr_dev;
  return a;
}

BatchPlan plan_of(const nrm_ctx* c, int acc) {
  BatchPlan p;
  p.acc = acc;
  p.block = c->bparams.block;
  p.unroll = c->bparams.unroll;
  p.map_unroll = c->bparams.map_unroll;
  p.short_regs = c->bparams.short_regs;
  p.grid = c->bparams.grid;
  p.map_block = c->bparams.map_block;
  p.map_grid = c->bparams.map_grid;
  p.res_grid = c->bparams.resident_segments > 0 ? c->bparams.resident_grid : 0;
  p.wave_grid = c->bparams.wave_max > 0 ? c->bparams.wave_grid : 0;
  return p;
}

int capture_graph(nrm_ctx* c, int acc, int buf) {
  BatchWorkspace& w = c->batch;
  hipGraphExec_t& g = w.graph[acc][buf];
  if (g) (void)hipGraphExecDestroy(g);
  g = nullptr;
  hipError_t e;
  if (!w.capture_stream) {
    e = hipStreamCreateWithFlags(&w.capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  }
  e = hipStreamBeginCapture(w.capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t e2 = nrm::launch_batch(plan_of(c, acc), args_of(c, buf), w.capture_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(w.capture_stream, &graph);
  if (e2 != hipSuccess) return hip_fail(e2, "batched launch (capture)");
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  return NRM_OK;
}

// Stage the header (and table) in the next ring buffer, then run the launch
// sequence on `s`.
int run_batch(nrm_ctx* c, const BatchHeader& h, const nrm_row* table, int64_t nrows, int acc,
              hipStream_t s) {
  BatchWorkspace& w = c->batch;
  hipError_t e;
  const int buf = w.next;
  if (w.staged_pending[buf]) {  // the call that used this buffer before must be done with it
    e = hipEventSynchronize(w.staged[buf]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    w.staged_pending[buf] = false;
  }
  BatchHeader hd = h;
  hd.table = w.table[buf];
  char* host = static_cast<char*>(w.host) + w.staging * buf;
  std::memcpy(host, &hd, sizeof(hd));
  if (table) std::memcpy(host + kTableOffset, table, sizeof(RowDesc) * (size_t)nrows);
  hipEvent_t* ev = nullptr;
  if (c->timing) {
    ev = &w.events[2 * (w.timed_calls % nrm::kTimingRing)];
    w.timed_calls++;
    (void)hipEventRecord(ev[0], s);  // timing only
  }
  if (c->bparams.graph) {
    if (!w.graph[acc][buf]) {
      int st = capture_graph(c, acc, buf);
      if (st != NRM_OK) return st;
    }
    e = hipGraphLaunch(w.graph[acc][buf], s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  } else {
    e = nrm::launch_batch(plan_of(c, acc), args_of(c, buf), s);
    if (e != hipSuccess) return hip_fail(e, "batched kernel launch");
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  e = hipEventRecord(w.staged[buf], s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  w.staged_pending[buf] = true;
  w.next = (buf + 1) % nrm::kStagingRing;
  return NRM_OK;
}

bool valid_dtype(int dt) { return dt == NRM_F32 || dt == NRM_BF16 || dt == NRM_F16; }

}  // namespace

namespace nrm {
void batch_free(nrm_ctx* c) {
  BatchWorkspace& w = c->batch;
  destroy_graph(w);
  if (w.capture_stream) (void)hipStreamDestroy(w.capture_stream);
  for (hipEvent_t ev : w.staged)
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : w.events) (void)hipEventDestroy(ev);
  if (w.dev) (void)hipFree(w.dev);
  if (w.host) (void)hipHostFree(w.host);
  w = BatchWorkspace();
}
}  // namespace nrm

extern "C" {

int nrm_default_batch_params(nrm_batch_params* params) {
  if (!params) return fail(NRM_EINVAL, "NULL argument");
  *params = default_batch_params();
  return NRM_OK;
}

int nrm_set_batch_params(nrm_ctx* c, const nrm_batch_params* params) {
  if (!c || !params) return fail(NRM_EINVAL, "NULL argument");
  nrm::CtxLock lk(c->mu);
  int st = check_batch_params(*params);
  if (st != NRM_OK) return st;
  if (std::memcmp(params, &c->bparams, sizeof(*params)) != 0) {
    DeviceGuard g(c->device);
    if (any_graph(c->batch)) {
      hipError_t e = hipDeviceSynchronize();  // a replay may still be running
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      destroy_graph(c->batch);
    }
    c->bparams = *params;
  }
  return NRM_OK;
}

int nrm_get_batch_params(const nrm_ctx* c, nrm_batch_params* params) {
  if (!c || !params) return fail(NRM_EINVAL, "NULL argument");
  nrm::CtxLock lk(c->mu);
  *params = c->bparams;
  return NRM_OK;
}

int nrm_batch_reserve(nrm_ctx* c, int64_t max_rows, int64_t max_elems) {
  if (!c) return fail(NRM_EINVAL, "ctx is NULL");
  nrm::CtxLock lk(c->mu);
  if (max_rows < 0 || max_elems < 0) return fail(NRM_EINVAL, "negative reservation");
  if (max_rows > INT32_MAX) return fail(NRM_EINVAL, "more than 2^31 - 1 rows");
  DeviceGuard g(c->device);
  return reserve(c, max_rows, items_bound(c->bparams, max_rows, max_elems));
}

namespace {
int check_csr_buffers(const void* out, int out_dtype, const void* in, int in_dtype, int64_t capacity) {
  const int64_t si = nrm::dtype_size(in_dtype), so = nrm::dtype_size(out_dtype);
  if (!in || !out) return fail(NRM_EINVAL, "NULL data pointer");
  if (capacity > INT64_MAX / 8) return fail(NRM_EINVAL, "capacity too large");
  if ((reinterpret_cast<uintptr_t>(in) % si) || (reinterpret_cast<uintptr_t>(out) % so))
    return fail(NRM_EINVAL, "in or out is not aligned to its element size");
  uintptr_t a0 = (uintptr_t)in, a1 = a0 + (uintptr_t)(capacity * si);
  uintptr_t b0 = (uintptr_t)out, b1 = b0 + (uintptr_t)(capacity * so);
  if (a0 < b1 && b0 < a1 && !(a0 == b0 && si == so))
    return fail(NRM_EOVERLAP, "in and out overlap without being the same array");
  return NRM_OK;
}
}  // namespace

namespace {
// lse[rows] must not overlap in or out (capacity elements each).
int check_lse(const void* out, int out_dtype, const void* in, int in_dtype, int64_t capacity, const float* lse,
              int64_t rows) {
  const int64_t si = nrm::dtype_size(in_dtype), so = nrm::dtype_size(out_dtype);
  const uintptr_t l0 = (uintptr_t)lse, l1 = l0 + (uintptr_t)(rows * (int64_t)sizeof(float));
  const uintptr_t a0 = (uintptr_t)in, a1 = a0 + (uintptr_t)(capacity * si);
  const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (uintptr_t)(capacity * so);
  if ((l0 < a1 && a0 < l1) || (l0 < b1 && b0 < l1)) return fail(NRM_EOVERLAP, "lse overlaps in or out");
  return NRM_OK;
}

// The CSR form of both operations: validation before any HIP call, the
// capacity read from offsets[rows] when not given, then one batched run of
// the reduction kind `acc` (with lse written for softmax when non-NULL).
int run_csr(nrm_ctx* c, void* out, int out_dtype, const void* in, int in_dtype, const int64_t* offsets,
            int64_t rows, int64_t capacity, int acc, float* lse, void* stream) {
  if (rows < 0) return fail(NRM_EINVAL, "rows < 0");
  if (!valid_dtype(in_dtype) || !valid_dtype(out_dtype)) return fail(NRM_EINVAL, "unknown dtype");
  if (rows == 0) return NRM_OK;
  if (rows > INT32_MAX) return fail(NRM_EINVAL, "more than 2^31 - 1 rows");
  if (!offsets) return fail(NRM_EINVAL, "offsets is NULL");
  if (lse && (reinterpret_cast<uintptr_t>(lse) % sizeof(float)))
    return fail(NRM_EINVAL, "lse is not aligned to 4 bytes");
  if (capacity == 0 && !lse) return NRM_OK;  // every row is empty (or invalid)
  if (capacity > 0) {
    int st = check_csr_buffers(out, out_dtype, in, in_dtype, capacity);
    if (st == NRM_OK && lse) st = check_lse(out, out_dtype, in, in_dtype, capacity, lse, rows);
    if (st != NRM_OK) return st;
  }
  if (!c) {
    int st = nrm::default_ctx(&c);
    if (st != NRM_OK) return st;
  }
  nrm::CtxLock lk(c->mu);
  DeviceGuard g(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (capacity < 0) {
    int64_t last = 0;
    hipError_t e = hipMemcpyAsync(&last, offsets + rows, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading offsets[rows]");
    if (last <= 0 && !lse) return NRM_OK;
    capacity = last > 0 ? last : 0;
    if (capacity > 0) {
      int st = check_csr_buffers(out, out_dtype, in, in_dtype, capacity);
      if (st != NRM_OK) return st;
    }
  }
  if (lse && capacity > 0) {
    int st = check_lse(out, out_dtype, in, in_dtype, capacity, lse, rows);
    if (st != NRM_OK) return st;
  }
  int st = reserve(c, rows, items_bound(c->bparams, rows, capacity));
  if (st != NRM_OK) return st;
  BatchHeader h;
  std::memset(&h, 0, sizeof(h));
  h.nrows = rows;
  h.mode = nrm::BATCH_CSR;
  h.csr_in_dt = in_dtype;
  h.csr_out_dt = out_dtype;
  h.offsets = offsets;
  h.csr_in = static_cast<const char*>(in);
  h.csr_out = static_cast<char*>(out);
  h.capacity = capacity;
  h.lse = lse;
  return run_batch(c, h, nullptr, rows, acc, s);
}
}  // namespace

int nrm_normalize_batched_ex(nrm_ctx* c, void* out, int out_dtype, const void* in, int in_dtype,
                             const int64_t* offsets, int64_t rows, int64_t capacity, int accum,
                             void* stream) {
  if (accum != NRM_ACC_F32 && accum != NRM_ACC_KAHAN) return fail(NRM_EINVAL, "unknown accumulation mode");
  return run_csr(c, out, out_dtype, in, in_dtype, offsets, rows, capacity, accum, nullptr, stream);
}

int nrm_softmax_batched(nrm_ctx* c, float* out, const float* in, const int64_t* offsets, int64_t rows,
                        int64_t capacity, float* lse, void* stream) {
  return run_csr(c, out, NRM_F32, in, NRM_F32, offsets, rows, capacity, nrm::ACC_SOFTMAX, lse, stream);
}

int normalize_batched(float* out, const float* in, const int64_t* offsets, int64_t rows) {
  return nrm_normalize_batched_ex(nullptr, out, NRM_F32, in, NRM_F32, offsets, rows, -1, NRM_ACC_F32, nullptr);
}

int nrm_normalize_rows(nrm_ctx* c, const nrm_row* rows, int64_t nrows, int accum, void* stream) {
  if (nrows < 0) return fail(NRM_EINVAL, "nrows < 0");
  if (accum != NRM_ACC_F32 && accum != NRM_ACC_KAHAN) return fail(NRM_EINVAL, "unknown accumulation mode");
  if (nrows == 0) return NRM_OK;
  if (nrows > INT32_MAX) return fail(NRM_EINVAL, "more than 2^31 - 1 rows");
  if (!rows) return fail(NRM_EINVAL, "rows is NULL");
  int64_t total = 0, longest = 0;
  for (int64_t r = 0; r < nrows; ++r) {
    const nrm_row& d = rows[r];
    if (d.n < 0) return fail(NRM_EINVAL, "row with n < 0");
    if (!valid_dtype(d.in_dtype) || !valid_dtype(d.out_dtype)) return fail(NRM_EINVAL, "row with unknown dtype");
    if (d.n == 0) continue;
    if (!d.in || !d.out) return fail(NRM_EINVAL, "row with NULL data pointer");
    const int64_t si = nrm::dtype_size(d.in_dtype), so = nrm::dtype_size(d.out_dtype);
    if ((reinterpret_cast<uintptr_t>(d.in) % si) || (reinterpret_cast<uintptr_t>(d.out) % so))
      return fail(NRM_EINVAL, "row pointer not aligned to its element size");
    uintptr_t a0 = (uintptr_t)d.in, a1 = a0 + (uintptr_t)(d.n * si);
    uintptr_t b0 = (uintptr_t)d.out, b1 = b0 + (uintptr_t)(d.n * so);
    if (a0 < b1 && b0 < a1 && !(a0 == b0 && si == so))
      return fail(NRM_EOVERLAP, "a row's in and out overlap without being the same array");
    total += d.n;
    longest = std::max(longest, d.n);
  }
  if (!c) {
    int st = nrm::default_ctx(&c);
    if (st != NRM_OK) return st;
  }
  nrm::CtxLock lk(c->mu);
  if (longest > (int64_t(1) << c->bparams.tile_log2) * nrm::MAX_ROW_TILES)
    return fail(NRM_EINVAL, "row too long for the batched path's tile size");
  DeviceGuard g(c->device);
  int st = reserve(c, nrows, items_bound(c->bparams, nrows, total));
  if (st != NRM_OK) return st;
  BatchHeader h;
  std::memset(&h, 0, sizeof(h));
  h.nrows = nrows;
  h.mode = nrm::BATCH_TABLE;
  return run_batch(c, h, rows, nrows, accum, static_cast<hipStream_t>(stream));
}

int nrm_get_device_error(nrm_ctx* c, void* stream) {
  if (!c) {
    int st = nrm::default_ctx(&c);
    if (st != NRM_OK) return st;
  }
  nrm::CtxLock lk(c->mu);
  DeviceGuard g(c->device);
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  // the batched workspace's word and the context's word of the other kernels
  int word = 0;
  for (int* p : {c->batch.dev ? c->batch.error : nullptr, c->dev_error}) {
    if (!p) continue;
    int w = 0;
    e = hipMemcpy(&w, p, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the device error flag");
    if (w) {
      e = hipMemset(p, 0, sizeof(int));
      if (e != hipSuccess) return hip_fail(e, "clearing the device error flag");
    }
    word |= w;
  }
  if (!word) return NRM_OK;
  if (word & nrm::NRM_DEVERR_STALL) {
    // a wait that gave up may have left arrival counts behind: start them over
    if (c->batch.dev) e = hipMemset(c->batch.arrivals, 0, sizeof(unsigned) * (size_t)c->batch.cap_items);
    if (e == hipSuccess) e = hipMemset(c->res.arrivals, 0, sizeof(unsigned));
    if (e != hipSuccess) return hip_fail(e, "clearing the arrival counts");
  }
  std::string why;
  if (word & nrm::NRM_DEVERR_OFFSETS) why += "CSR offsets negative, decreasing or past capacity; ";
  if (word & nrm::NRM_DEVERR_ROW) why += "invalid table row or row with too many tiles; ";
  if (word & nrm::NRM_DEVERR_CAPACITY) why += "batch larger than the workspace; ";
  if (word & nrm::NRM_DEVERR_TARGET) why += "NLL target outside [0, classes); ";
  if (word & nrm::NRM_DEVERR_STALL) why += "a resident row's segment sums did not all arrive within the spin limit; ";
  return fail(NRM_EDEVICE, why + "those rows or samples were skipped");
}

int nrm_batch_times(nrm_ctx* c, double* total_ms, int64_t* calls) {
  if (!c) return fail(NRM_EINVAL, "ctx is NULL");
  nrm::CtxLock lk(c->mu);
  BatchWorkspace& w = c->batch;
  double t = 0;
  int64_t k = std::min<int64_t>(w.timed_calls, nrm::kTimingRing);
  for (int64_t i = 0; i < k; ++i) {
    hipError_t e = hipEventSynchronize(w.events[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0;
    e = hipEventElapsedTime(&ms, w.events[2 * i], w.events[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    t += ms;
  }
  if (total_ms) *total_ms = t;
  if (calls) *calls = k;
  return NRM_OK;
}

}  // extern "C"
