// Ragged batched normalize on gfx950: every row of a batch is normalized on
// its own, out_r[i] = in_r[i] / sum(in_r), with the per-row sum hoisted out
// of the element-wise divide exactly as in the plain path (arXiv 2207.00257,
// Fig. 1 and Sec. IV-C), in one persistent launch sequence for the batch.
//
//   batch_plan_kernel    one block: resolves the row table (from CSR offsets
//                        or a descriptor table), validates it, classifies
//                        rows, and writes the work-item table by exclusive
//                        scans: first the tiles of every long row
//                        (ceil(n / tile) each, consecutive per row), then one
//                        item per short row (n <= short_max).
//   batch_phase1_kernel  persistent blocks walk the items. A single-pass item
//                        keeps its row in registers: one read, block sum,
//                        divide, one write. A tile item writes its partial.
//   batch_phase2_kernel  persistent blocks walk the tile items: each merges
//                        its row's partials in a fixed order (the kernel
//                        boundary is the barrier that makes them visible;
//                        every tile of a row computes the same sum) and
//                        divides its tile by it.
// Each block walks items blockIdx.x, blockIdx.x + gridDim.x, ... and fetches
// the next item's descriptor while it processes the current one.
//
// All per-call inputs are read through fixed pointers (a header and the row
// table in pinned host memory, read once by the planner), so the three
// launches can be captured once in a hipGraph and replayed for any batch
// that fits the workspace. A row's summation order
// depends only on its length, its start alignment modulo 16 bytes, its
// dtypes, the accumulation mode and the launch parameters: never on the
// other rows or its position in the batch.
#include "nrm_batch.h"
#include "nrm_device.h"

namespace nrm {
namespace {

using namespace dev;

// ---- geometry of one contiguous segment --------------------------------------

struct Geom {
  int64_t head;        // elements before the first 16-byte aligned vector
  int64_t nvec;        // whole 16-byte vectors after the head
  int64_t tail_begin;  // first element after the vectors
};

template <int DT>
__device__ __forceinline__ Geom geometry(const char* p, int64_t n) {
  constexpr int SI = Elem<DT>::SIZE, VEC = Elem<DT>::VEC;
  Geom g;
  const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(p) & 15);
  g.head = mis ? (16 - mis) / SI : 0;
  if (g.head > n) g.head = n;
  g.nvec = (n - g.head) / VEC;
  g.tail_begin = g.head + g.nvec * VEC;
  return g;
}

// Output vectors can be stored whole when the output segment has the same
// alignment as the input's vector body.
template <int DTI, int DTO>
__device__ __forceinline__ bool out_vector_ok(const char* out_seg, int64_t head) {
  constexpr int SO = Elem<DTO>::SIZE, VEC = Elem<DTI>::VEC;
  constexpr int A = VEC * SO < 16 ? VEC * SO : 16;
  return (reinterpret_cast<uintptr_t>(out_seg + head * SO) % A) == 0;
}

template <int DTI, int DTO>
__device__ __forceinline__ void store_quotients(char* out_seg, int64_t head, int64_t v, bool vec_ok,
                                                const float (&q)[Elem<DTI>::VEC]) {
  constexpr int VEC = Elem<DTI>::VEC;
  if (vec_ok) {
    store_vec<DTO, VEC>(out_seg + head * Elem<DTO>::SIZE, v, q);
  } else {
#pragma unroll
    for (int c = 0; c < VEC; ++c) store_one<DTO>(out_seg, head + v * VEC + c, q[c]);
  }
}

// ---- planner ---------------------------------------------------------------------

constexpr int PLAN_THREADS = 1024;

__device__ __forceinline__ bool valid_dt(int dt) { return dt == NRM_F32 || dt == NRM_BF16 || dt == NRM_F16; }

__device__ __forceinline__ int64_t long_tiles(int64_t n, int64_t short_max, int64_t tile) {
  return n <= short_max ? 0 : (n + tile - 1) / tile;
}

__global__ void __launch_bounds__(PLAN_THREADS) batch_plan_kernel(BatchArgs a) {
  __shared__ int64_t scan_long[PLAN_THREADS];
  __shared__ int64_t scan_short[PLAN_THREADS];
  __shared__ BatchHeader hs;
  const int t = threadIdx.x;
  if (t == 0) hs = *a.hdr;  // one read of the header (pinned host memory)
  __syncthreads();
  const BatchHeader* h = &hs;
  const int64_t nrows = h->nrows;
  if (nrows < 0 || nrows > a.cap_rows) {
    if (t == 0) {
      atomicOr(a.error, NRM_DEVERR_CAPACITY);
      a.n_items[0] = 0;
      a.n_items[1] = 0;
    }
    return;
  }
  const int64_t per = (nrows + PLAN_THREADS - 1) / PLAN_THREADS;
  const int64_t r0 = t * per < nrows ? t * per : nrows;
  const int64_t r1 = r0 + per < nrows ? r0 + per : nrows;
  int err = 0;
  int64_t nl = 0, ns = 0;
  for (int64_t r = r0; r < r1; ++r) {
    RowDesc d;
    if (h->mode == BATCH_CSR) {
      const int64_t b = h->offsets[r], e = h->offsets[r + 1];
      const int si = h->csr_in_dt == NRM_F32 ? 4 : 2, so = h->csr_out_dt == NRM_F32 ? 4 : 2;
      d.in = h->csr_in + b * si;
      d.out = h->csr_out + b * so;
      d.n = e - b;
      d.in_dt = h->csr_in_dt;
      d.out_dt = h->csr_out_dt;
      if (b < 0 || e < b || e > h->capacity) {
        err |= NRM_DEVERR_OFFSETS;
        d.n = 0;
      }
    } else {
      d = h->table[r];
      if (d.n < 0 || !valid_dt(d.in_dt) || !valid_dt(d.out_dt) || (d.n > 0 && (!d.in || !d.out))) {
        err |= NRM_DEVERR_ROW;
        d.n = 0;
      }
    }
    if (long_tiles(d.n, a.short_max, a.tile) > MAX_ROW_TILES) {
      err |= NRM_DEVERR_ROW;
      d.n = 0;
    }
    a.rows[r] = d;
    nl += long_tiles(d.n, a.short_max, a.tile);
    ns += (d.n > 0 && d.n <= a.short_max) ? 1 : 0;
  }
  scan_long[t] = nl;
  scan_short[t] = ns;
  __syncthreads();
  for (int off = 1; off < PLAN_THREADS; off <<= 1) {
    int64_t vl = t >= off ? scan_long[t - off] : 0;
    int64_t vs = t >= off ? scan_short[t - off] : 0;
    __syncthreads();
    scan_long[t] += vl;
    scan_short[t] += vs;
    __syncthreads();
  }
  const int64_t total_long = scan_long[PLAN_THREADS - 1];
  const int64_t total = total_long + scan_short[PLAN_THREADS - 1];
  if (total <= a.cap_items) {
    int64_t sl = scan_long[t] - nl;                // this thread's first long-tile item
    int64_t ss = total_long + scan_short[t] - ns;  // and first short-row item
    for (int64_t r = r0; r < r1; ++r) {
      const int64_t n = a.rows[r].n;
      const int64_t k = long_tiles(n, a.short_max, a.tile);
      for (int64_t j = 0; j < k; ++j) a.items[sl + j] = Item{(int32_t)r, (int32_t)j};
      sl += k;
      if (n > 0 && n <= a.short_max) a.items[ss++] = Item{(int32_t)r, 0};
    }
  }
  if (err) atomicOr(a.error, err);
  if (t == PLAN_THREADS - 1) {
    if (total > a.cap_items) {
      atomicOr(a.error, NRM_DEVERR_CAPACITY);
      a.n_items[0] = 0;
      a.n_items[1] = 0;
    } else {
      a.n_items[0] = total;
      a.n_items[1] = total_long;
    }
  }
}

// ---- single-pass rows (held in registers) --------------------------------------------

template <int DTI, int DTO, int ACC, int KB>
__device__ __forceinline__ void single_pass(const RowDesc& d, Acc<ACC>* slots, float* s_bcast) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int NA = accumulators(DTI, ACC, KB);
  const int B = blockDim.x, t = threadIdx.x;
  const Geom g = geometry<DTI>(d.in, d.n);
  const u4* body = reinterpret_cast<const u4*>(d.in + g.head * Elem<DTI>::SIZE);
  u4 r[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int64_t v = t + (int64_t)k * B;
    if (v < g.nvec) r[k] = load_vec<false>(body + v);
  }
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    if (t + (int64_t)k * B < g.nvec) {
      float x[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[(k * VEC + c) % NA].add(x[c]);
    }
  }
  if (t < g.head) acc[0].add(load_one<DTI>(d.in, t));
  if (t < d.n - g.tail_begin) acc[0].add(load_one<DTI>(d.in, g.tail_begin + t));
  merge_chains<ACC, NA>(acc);
  Acc<ACC> tot = block_reduce<ACC>(acc[0], slots);
  if (t == 0) *s_bcast = tot.value();
  __syncthreads();
  const float S = *s_bcast;
  const bool vec_ok = out_vector_ok<DTI, DTO>(d.out, g.head);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int64_t v = t + (int64_t)k * B;
    if (v < g.nvec) {
      float x[VEC], q[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int c = 0; c < VEC; ++c) q[c] = x[c] / S;
      store_quotients<DTI, DTO>(d.out, g.head, v, vec_ok, q);
    }
  }
  if (t < g.head) store_one<DTO>(d.out, t, load_one<DTI>(d.in, t) / S);
  if (t < d.n - g.tail_begin) {
    const int64_t i = g.tail_begin + t;
    store_one<DTO>(d.out, i, load_one<DTI>(d.in, i) / S);
  }
}

// ---- tiles of long rows ------------------------------------------------------------

// Sum of elements [b, e) of a row; valid in thread 0.
template <int DTI, int ACC, int U>
__device__ __forceinline__ Acc<ACC> tile_reduce(const char* in_row, int64_t b, int64_t e,
                                                Acc<ACC>* slots) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int NA = accumulators(DTI, ACC, U);
  constexpr int FLUSH = CHAIN_ADDS / adds_per_iteration(DTI, ACC, U);
  const char* seg = in_row + b * Elem<DTI>::SIZE;
  const int64_t n = e - b;
  const Geom g = geometry<DTI>(seg, n);
  const u4* p = reinterpret_cast<const u4*>(seg + g.head * Elem<DTI>::SIZE) + threadIdx.x;
  const int64_t B = blockDim.x, step = B * U;
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  Acc<ACC> run;
  run.zero();
  int since_flush = 0;
  for (int64_t base = 0; base < g.nvec; base += step) {
    if (base + step <= g.nvec) {
      u4 r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load_vec<true>(p + base + u * B);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float x[VEC];
        widen<DTI>(r[u], x);
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[(u * VEC + c) % NA].add(x[c]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (base + u * B + (int64_t)threadIdx.x < g.nvec) {
          float x[VEC];
          widen<DTI>(load_vec<true>(p + base + u * B), x);
#pragma unroll
          for (int c = 0; c < VEC; ++c) acc[(u * VEC + c) % NA].add(x[c]);
        }
      }
    }
    if constexpr (ACC == NRM_ACC_F32) {
      if (++since_flush == FLUSH) {
        since_flush = 0;
        merge_chains<ACC, NA>(acc);
        run.merge(acc[0]);
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k].zero();
      }
    }
  }
  if ((int64_t)threadIdx.x < g.head) acc[0].add(load_one<DTI>(seg, threadIdx.x));
  if ((int64_t)threadIdx.x < n - g.tail_begin) acc[0].add(load_one<DTI>(seg, g.tail_begin + threadIdx.x));
  merge_chains<ACC, NA>(acc);
  run.merge(acc[0]);
  return block_reduce<ACC>(run, slots);
}

// out[i] = in[i] / S for elements [b, e) of a row.
template <int DTI, int DTO, int U>
__device__ __forceinline__ void tile_map(const RowDesc& d, int64_t b, int64_t e, float S) {
  constexpr int VEC = Elem<DTI>::VEC;
  const char* in_seg = d.in + b * Elem<DTI>::SIZE;
  char* out_seg = d.out + b * Elem<DTO>::SIZE;
  const int64_t n = e - b;
  const Geom g = geometry<DTI>(in_seg, n);
  const u4* body = reinterpret_cast<const u4*>(in_seg + g.head * Elem<DTI>::SIZE);
  const bool vec_ok = out_vector_ok<DTI, DTO>(out_seg, g.head);
  const int64_t B = blockDim.x, step = B * U;
  for (int64_t base = 0; base < g.nvec; base += step) {
    const int64_t v0 = base + threadIdx.x;
    if (base + step <= g.nvec) {
      u4 r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load_vec<true>(body + v0 + u * B);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float x[VEC], q[VEC];
        widen<DTI>(r[u], x);
#pragma unroll
        for (int c = 0; c < VEC; ++c) q[c] = x[c] / S;
        store_quotients<DTI, DTO>(out_seg, g.head, v0 + u * B, vec_ok, q);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (v0 + u * B < g.nvec) {
          float x[VEC], q[VEC];
          widen<DTI>(load_vec<true>(body + v0 + u * B), x);
#pragma unroll
          for (int c = 0; c < VEC; ++c) q[c] = x[c] / S;
          store_quotients<DTI, DTO>(out_seg, g.head, v0 + u * B, vec_ok, q);
        }
      }
    }
  }
  if ((int64_t)threadIdx.x < g.head)
    store_one<DTO>(out_seg, threadIdx.x, load_one<DTI>(in_seg, threadIdx.x) / S);
  const int64_t i = g.tail_begin + threadIdx.x;
  if (i < n) store_one<DTO>(out_seg, i, load_one<DTI>(in_seg, i) / S);
}

// ---- dtype dispatch of one item --------------------------------------------------------

template <int ACC, int KB>
__device__ __forceinline__ void dispatch_single(const RowDesc& d, Acc<ACC>* slots, float* s_bcast) {
#define NRM_SP(I, O) single_pass<I, O, ACC, KB>(d, slots, s_bcast)
  switch (d.in_dt * 3 + d.out_dt) {
    case NRM_F32 * 3 + NRM_F32: NRM_SP(NRM_F32, NRM_F32); break;
    case NRM_F32 * 3 + NRM_BF16: NRM_SP(NRM_F32, NRM_BF16); break;
    case NRM_F32 * 3 + NRM_F16: NRM_SP(NRM_F32, NRM_F16); break;
    case NRM_BF16 * 3 + NRM_F32: NRM_SP(NRM_BF16, NRM_F32); break;
    case NRM_BF16 * 3 + NRM_BF16: NRM_SP(NRM_BF16, NRM_BF16); break;
    case NRM_BF16 * 3 + NRM_F16: NRM_SP(NRM_BF16, NRM_F16); break;
    case NRM_F16 * 3 + NRM_F32: NRM_SP(NRM_F16, NRM_F32); break;
    case NRM_F16 * 3 + NRM_BF16: NRM_SP(NRM_F16, NRM_BF16); break;
    default: NRM_SP(NRM_F16, NRM_F16); break;
  }
#undef NRM_SP
}

template <int ACC, int U>
__device__ __forceinline__ Acc<ACC> dispatch_tile_reduce(const RowDesc& d, int64_t b, int64_t e,
                                                         Acc<ACC>* slots) {
  switch (d.in_dt) {
    case NRM_F32: return tile_reduce<NRM_F32, ACC, U>(d.in, b, e, slots);
    case NRM_BF16: return tile_reduce<NRM_BF16, ACC, U>(d.in, b, e, slots);
    default: return tile_reduce<NRM_F16, ACC, U>(d.in, b, e, slots);
  }
}

template <int U>
__device__ __forceinline__ void dispatch_tile_map(const RowDesc& d, int64_t b, int64_t e, float S) {
#define NRM_TM(I, O) tile_map<I, O, U>(d, b, e, S)
  switch (d.in_dt * 3 + d.out_dt) {
    case NRM_F32 * 3 + NRM_F32: NRM_TM(NRM_F32, NRM_F32); break;
    case NRM_F32 * 3 + NRM_BF16: NRM_TM(NRM_F32, NRM_BF16); break;
    case NRM_F32 * 3 + NRM_F16: NRM_TM(NRM_F32, NRM_F16); break;
    case NRM_BF16 * 3 + NRM_F32: NRM_TM(NRM_BF16, NRM_F32); break;
    case NRM_BF16 * 3 + NRM_BF16: NRM_TM(NRM_BF16, NRM_BF16); break;
    case NRM_BF16 * 3 + NRM_F16: NRM_TM(NRM_BF16, NRM_F16); break;
    case NRM_F16 * 3 + NRM_F32: NRM_TM(NRM_F16, NRM_F32); break;
    case NRM_F16 * 3 + NRM_BF16: NRM_TM(NRM_F16, NRM_BF16); break;
    default: NRM_TM(NRM_F16, NRM_F16); break;
  }
#undef NRM_TM
}

// ---- the two persistent phases ------------------------------------------------------------

template <int ACC, int U, int KB>
__global__ void __launch_bounds__(1024) batch_phase1_kernel(BatchArgs a) {
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ float s_bcast;
  const int64_t n_items = a.n_items[0];
  const int64_t n_long = a.n_items[1];
  Acc<ACC>* part = reinterpret_cast<Acc<ACC>*>(a.partials);
  int64_t item = blockIdx.x;
  if (item >= n_items) return;
  Item it = a.items[item];
  RowDesc d = a.rows[it.row];
  while (true) {
    // the next item's descriptor is fetched while this one is processed
    const int64_t next = item + gridDim.x;
    Item it_next = it;
    if (next < n_items) it_next = a.items[next];
    if (item >= n_long) {
      dispatch_single<ACC, KB>(d, slots, &s_bcast);
    } else {
      const int64_t b = (int64_t)it.tile * a.tile;
      const int64_t e = b + a.tile < d.n ? b + a.tile : d.n;
      Acc<ACC> p = dispatch_tile_reduce<ACC, U>(d, b, e, slots);
      if (threadIdx.x == 0) part[item] = p;  // read after the kernel boundary
    }
    if (next >= n_items) break;
    it = it_next;
    d = a.rows[it.row];
    item = next;
    __syncthreads();  // the block's LDS is reused by the next item
  }
}

// The row's sum from its `count` tile partials, in a fixed order that
// depends only on count: up to 64 partials one per lane of wavefront 0,
// merged by the DPP tree; more through the LDS halving tree. Valid in
// every thread on return.
template <int ACC>
__device__ __forceinline__ float row_sum(const Acc<ACC>* part, int64_t count, Acc<ACC>* tree,
                                         Acc<ACC>* tiles, float* s_bcast) {
  if (count <= 64) {
    if (threadIdx.x < 64) {
      Acc<ACC> v;
      v.zero();
      if ((int64_t)threadIdx.x < count) v = part[threadIdx.x];
      v = wave_reduce<ACC>(v);
      if (threadIdx.x == 0) *s_bcast = v.value();
    }
  } else {
    Acc<ACC> tot = combine_partials<ACC>(part, count, tree, tiles);
    if (threadIdx.x == 0) *s_bcast = tot.value();
  }
  __syncthreads();
  return *s_bcast;
}

template <int ACC, int U>
__global__ void __launch_bounds__(1024) batch_phase2_kernel(BatchArgs a) {
  __shared__ Acc<ACC> tree[COMBINE_TILE];
  __shared__ Acc<ACC> tiles[MAX_COMBINE_TILES];
  __shared__ float s_bcast;
  const int64_t n_long = a.n_items[1];
  const Acc<ACC>* part = reinterpret_cast<const Acc<ACC>*>(a.partials);
  int64_t item = blockIdx.x;
  if (item >= n_long) return;
  Item it = a.items[item];
  RowDesc d = a.rows[it.row];
  while (true) {
    const int64_t next = item + gridDim.x;
    Item it_next = it;
    if (next < n_long) it_next = a.items[next];
    const int64_t count = (d.n + a.tile - 1) / a.tile;
    const float S = row_sum<ACC>(part + (item - it.tile), count, tree, tiles, &s_bcast);
    const int64_t b = (int64_t)it.tile * a.tile;
    const int64_t e = b + a.tile < d.n ? b + a.tile : d.n;
    dispatch_tile_map<U>(d, b, e, S);
    if (next >= n_long) break;
    it = it_next;
    d = a.rows[it.row];
    item = next;
    __syncthreads();  // s_bcast and the trees are reused by the next item
  }
}

template <int ACC, int U>
hipError_t phase1_kb(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  switch (p.short_regs) {
    case 1: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 1>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    case 2: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 2>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    case 4: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 4>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    default: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 8>), dim3(p.grid), dim3(p.block), 0, s, a); break;
  }
  return hipGetLastError();
}

template <int ACC>
hipError_t phase1_u(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  switch (p.unroll) {
    case 1: return phase1_kb<ACC, 1>(p, a, s);
    case 2: return phase1_kb<ACC, 2>(p, a, s);
    case 4: return phase1_kb<ACC, 4>(p, a, s);
    default: return phase1_kb<ACC, 8>(p, a, s);
  }
}

template <int ACC>
hipError_t phase2_u(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  switch (p.map_unroll) {
    case 1: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 1>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    case 2: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 2>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    case 4: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 4>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    default: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 8>), dim3(p.grid), dim3(p.block), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(PLAN_THREADS), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = p.acc == NRM_ACC_KAHAN ? phase1_u<NRM_ACC_KAHAN>(p, a, s) : phase1_u<NRM_ACC_F32>(p, a, s);
  if (e != hipSuccess) return e;
  return p.acc == NRM_ACC_KAHAN ? phase2_u<NRM_ACC_KAHAN>(p, a, s) : phase2_u<NRM_ACC_F32>(p, a, s);
}

}  // namespace nrm
