// HIP kernels of the plain normalize path for gfx950 (MI355X).
//
// normalize (arXiv 2207.00257, Fig. 1) divides every element by the sum of
// all elements. The sum is invariant across the kernel's threads, so it is
// computed once (Sec. IV-C, parallel loop-invariant code motion; the O(N)
// form of the Fig. 1 caption) and the kernel is split at a grid-wide barrier
// into two phases (the splitting of a parallel loop at a barrier, Sec. III-B):
//
//   reduce_kernel  every block sums a share of the input into one partial:
//                  16-byte vector loads feed U*VEC independent binary32
//                  chains per thread; the chains are combined pairwise; a
//                  wavefront reduces with DPP lane moves (no LDS, no barrier);
//                  the wavefronts of a block meet in one LDS slot each behind
//                  one block barrier (the block barrier of Fig. 1's shared-
//                  memory variant). Fused combine (the default): the block
//                  stores its partial and ends. Otherwise the last block to
//                  finish (an agent-scope ticket; partials travel by
//                  agent-scope atomic stores and loads, coherent across the
//                  XCDs' separate L2 caches) combines all partials in a fixed
//                  tree in LDS (the halving loop of Fig. 7) and writes the sum.
//                  Loads are non-temporal except the input's last
//                  reduce_keep_mib MiB, which stay in the last-level cache
//                  for the map.
//   map_kernel     (fused) every block first merges the reduce's partials with
//                  one wavefront in the same fixed order, so all blocks divide
//                  by the same bits; then out[i] = in[i] / sum with a
//                  correctly rounded binary32 division, 16-byte vector loads,
//                  non-temporal vector stores.
//
// The kernel boundary between the two is the grid-wide barrier. No float
// atomics are used: for given sizes, alignment and launch parameters every
// addition happens in the same order on every run.
#include <type_traits>

#include "nrm_device.h"

namespace nrm {
namespace {

using namespace dev;

// ---- phase 1: block partials and the grid combine ------------------------------

struct ReduceArgs {
  const char* in;      // the input (element 0)
  const u4* body;      // first 16-byte aligned vector of the input
  int64_t head;        // elements before body
  int64_t nvec;        // vectors in the body
  int64_t tail_begin;  // first element after the body
  int64_t n;
  int64_t chunk;       // vectors per block (layout CHUNK), multiple of blockDim * U
  int64_t tile;        // vectors per tile (layout TILE), multiple of blockDim * U
  int layout;
  int fused;           // 1: publish the partial and end; the map blocks combine
  int64_t keep_from;   // vectors from here on: temporal loads even when NT
  void* partials;      // Acc<ACC>[gridDim.x]
  unsigned* ticket;    // 0 on entry, left 0 on exit
  float* sum;          // out: the hoisted invariant
};

template <int DT, int ACC, int U, bool NT>
__global__ void __launch_bounds__(1024) reduce_kernel(ReduceArgs a) {
  constexpr int VEC = Elem<DT>::VEC;
  constexpr int NA = accumulators(DT, ACC, U);
  // Plain binary32: every FLUSH iterations (16 additions per chain) the
  // chains are summed pairwise into a running total and restarted, so the
  // height of the thread's summation tree grows by one per FLUSH iterations
  // instead of one per iteration. Compensated chains need no flush.
  constexpr int FLUSH = CHAIN_ADDS / adds_per_iteration(DT, ACC, U);
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ int is_last;

  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  Acc<ACC> run;
  run.zero();
  int since_flush = 0;

  const int64_t B = blockDim.x;
  const int64_t step = B * U;
  int64_t begin, end, stride;
  if (a.layout == NRM_LAYOUT_CHUNK) {
    begin = (int64_t)blockIdx.x * a.chunk;
    end = begin + a.chunk < a.nvec ? begin + a.chunk : a.nvec;
    stride = step;
  } else {
    begin = (int64_t)blockIdx.x * step;
    end = a.nvec;
    stride = (int64_t)gridDim.x * step;
  }
  const u4* p = a.body + threadIdx.x;
  // Full iterations only in the steady-state loops (non-temporal loads, then
  // temporal ones from keep_from on); at most one partial iteration remains.
  auto full = [&](int64_t base, auto nt) {
    u4 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = load_vec<decltype(nt)::value>(p + base + u * B);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float x[VEC];
      widen<DT>(r[u], x);
#pragma unroll
      for (int k = 0; k < VEC; ++k) acc[(u * VEC + k) % NA].add(x[k]);
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
  };
  // the one partial iteration a block can have: vectors [base, end)
  auto partial = [&](int64_t base, int64_t end) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * B + (int64_t)threadIdx.x < end) {
        float x[VEC];
        widen<DT>(load_vec<NT>(p + base + u * B), x);
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc[(u * VEC + k) % NA].add(x[k]);
      }
    }
  };
  if (a.layout == NRM_LAYOUT_TILE) {
    // tiles blockIdx.x, blockIdx.x + gridDim.x, ...; only the input's last
    // tile can end in a partial iteration, and it is its block's last
    const int64_t tile_stride = (int64_t)gridDim.x * a.tile;
    for (int64_t tb = (int64_t)blockIdx.x * a.tile; tb < a.nvec; tb += tile_stride) {
      const int64_t te = tb + a.tile < a.nvec ? tb + a.tile : a.nvec;
      int64_t base = tb;
      for (; base + step <= te; base += step) {
        if (NT && base < a.keep_from) full(base, std::integral_constant<bool, NT>());
        else full(base, std::integral_constant<bool, false>());
      }
      if (base < te) partial(base, te);
    }
  } else {
    const int64_t last_full = end - step;  // a base <= last_full starts a full iteration
    int64_t base = begin;
    if (NT) {
      const int64_t nt_end = a.keep_from < last_full + 1 ? a.keep_from : last_full + 1;
      for (; base < nt_end; base += stride) full(base, std::integral_constant<bool, NT>());
    }
    for (; base <= last_full; base += stride) full(base, std::integral_constant<bool, false>());
    if (base < end) partial(base, end);
  }
  // unaligned head and the tail shorter than a vector: block 0
  if (blockIdx.x == 0) {
    if ((int64_t)threadIdx.x < a.head) acc[0].add(load_one<DT>(a.in, threadIdx.x));
    if ((int64_t)threadIdx.x < a.n - a.tail_begin) acc[0].add(load_one<DT>(a.in, a.tail_begin + threadIdx.x));
  }
  merge_chains<ACC, NA>(acc);
  run.merge(acc[0]);

  Acc<ACC> blk = block_reduce<ACC>(run, slots);

  // publish the partial; the last block to arrive combines all of them, or,
  // fused, every block of the map kernel does (after the kernel boundary, so
  // no fence and no ticket here)
  Acc<ACC>* part = reinterpret_cast<Acc<ACC>*>(a.partials);
  if (a.fused) {
    if (threadIdx.x == 0) publish(part, blockIdx.x, blk);
    return;
  }
  if (threadIdx.x == 0) {
    publish(part, blockIdx.x, blk);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    unsigned prev = __hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = prev == gridDim.x - 1;
  }
  lds_barrier();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

  __shared__ Acc<ACC> tree[COMBINE_TILE];
  __shared__ Acc<ACC> tiles[MAX_COMBINE_TILES];
  Acc<ACC> total = combine_partials<ACC>(part, gridDim.x, tree, tiles);
  if (threadIdx.x == 0) {
    a.sum[0] = total.value();
    // ready for the next call on this workspace (stream-ordered)
    __hip_atomic_store(a.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- phase 2: the divide map ---------------------------------------------------------

struct MapArgs {
  const char* in;
  char* out;
  const u4* body;      // first aligned input vector
  char* out_body;      // output element `head`
  int64_t head, nvec, tail_begin, n;
  int64_t chunk;       // units per block (layout CHUNK), multiple of blockDim * U
  int64_t tile;        // units per tile (layout TILE), multiple of blockDim * U
  int layout;
  int reverse;
  const float* sum;    // the sum (not fused)
  // fused combine: every block merges the reduce's partials itself
  int fused;
  int acc;             // nrm_accum of the partials
  const void* partials;
  int64_t nparts;      // at most 1024
  float* sum_out;      // block 0 stores the merged sum here
};

// Units of the map: a 16-byte input vector, or, for a 2-byte input with
// binary32 output, 8 bytes (4 elements), so that every lane stores exactly
// one 16-byte output vector and each store instruction is fully coalesced.
template <int DTI, int DTO>
struct MapUnit {
  static constexpr bool HALF = Elem<DTI>::SIZE == 2 && DTO == NRM_F32;
  static constexpr int ELEMS = HALF ? 4 : Elem<DTI>::VEC;
  using T = typename std::conditional<HALF, u2, u4>::type;
};

// The divisor of the map: the reduce's sum, or (fused) the merge of its
// partials by wavefront 0 of this block, in the same fixed order in every
// block (bitwise the same value everywhere).
__device__ __forceinline__ float map_divisor(const MapArgs& a) {
  if (!a.fused) return a.sum[0];
  __shared__ float s_sum;
  if (threadIdx.x < 64) {
    float v;
    if (a.acc == NRM_ACC_KAHAN)
      v = combine_wave<NRM_ACC_KAHAN, false>(static_cast<const Acc<NRM_ACC_KAHAN>*>(a.partials), a.nparts).value();
    else
      v = combine_wave<NRM_ACC_F32, false>(static_cast<const Acc<NRM_ACC_F32>*>(a.partials), a.nparts).value();
    if (threadIdx.x == 0) {
      s_sum = v;
      if (blockIdx.x == 0) a.sum_out[0] = v;
    }
  }
  lds_barrier();
  return s_sum;
}

template <int DTI, int DTO, int U, bool NT>
__global__ void __launch_bounds__(1024) map_kernel(MapArgs a) {
  using MU = MapUnit<DTI, DTO>;
  using T = typename MU::T;
  constexpr int VEC = MU::ELEMS;
  const T* body = reinterpret_cast<const T*>(a.body);
  const float S = map_divisor(a);
  const int64_t B = blockDim.x;
  const int64_t step = B * U;
  auto widen_unit = [](T r, float (&x)[VEC]) {
    if constexpr (MU::HALF) widen_half<DTI>(r, x);
    else widen<DTI>(r, x);
  };
  // one block-iteration over units [base, base + step) clipped to end
  auto iteration = [&](int64_t base, int64_t end) {
    const int64_t v0 = base + threadIdx.x;
    if (base + step <= end) {
      T r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load_vec<NT>(body + v0 + u * B);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float x[VEC], q[VEC];
        widen_unit(r[u], x);
#pragma unroll
        for (int k = 0; k < VEC; ++k) q[k] = x[k] / S;
        store_vec<DTO, VEC>(a.out_body, v0 + u * B, q);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (v0 + u * B < end) {
          float x[VEC], q[VEC];
          widen_unit(load_vec<NT>(body + v0 + u * B), x);
#pragma unroll
          for (int k = 0; k < VEC; ++k) q[k] = x[k] / S;
          store_vec<DTO, VEC>(a.out_body, v0 + u * B, q);
        }
      }
    }
  };
  if (a.layout == NRM_LAYOUT_TILE) {
    const int64_t tile_stride = (int64_t)gridDim.x * a.tile;
    for (int64_t tb = (int64_t)blockIdx.x * a.tile; tb < a.nvec; tb += tile_stride) {
      const int64_t te = tb + a.tile < a.nvec ? tb + a.tile : a.nvec;
      for (int64_t base = tb; base < te; base += step) iteration(base, te);
    }
  } else {
    int64_t begin, end, stride;
    if (a.layout == NRM_LAYOUT_CHUNK) {
      begin = (int64_t)blockIdx.x * a.chunk;
      end = begin + a.chunk < a.nvec ? begin + a.chunk : a.nvec;
      stride = step;
    } else {
      begin = (int64_t)blockIdx.x * step;
      end = a.nvec;
      stride = (int64_t)gridDim.x * step;
    }
    const int64_t iters = end > begin ? (end - begin + stride - 1) / stride : 0;
    for (int64_t it = 0; it < iters; ++it) iteration(begin + (a.reverse ? iters - 1 - it : it) * stride, end);
  }
  if (blockIdx.x == 0) {
    if ((int64_t)threadIdx.x < a.head)
      store_one<DTO>(a.out, threadIdx.x, load_one<DTI>(a.in, threadIdx.x) / S);
    const int64_t t = a.tail_begin + threadIdx.x;
    if (t < a.n) store_one<DTO>(a.out, t, load_one<DTI>(a.in, t) / S);
  }
}

// Element-wise map for outputs whose alignment differs from the input's.
template <int DTI, int DTO>
__global__ void __launch_bounds__(256) map_scalar_kernel(const char* in, char* out, int64_t n,
                                                         const float* sum) {
  const float S = sum[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    store_one<DTO>(out, i, load_one<DTI>(in, i) / S);
}

// ---- dispatch ---------------------------------------------------------------------

template <int DT, int ACC, int U>
hipError_t reduce_u(const PlainPlan& p, const ReduceArgs& a, hipStream_t s) {
  if (p.reduce_nt)
    hipLaunchKernelGGL((reduce_kernel<DT, ACC, U, true>), dim3(p.grid), dim3(p.block), 0, s, a);
  else
    hipLaunchKernelGGL((reduce_kernel<DT, ACC, U, false>), dim3(p.grid), dim3(p.block), 0, s, a);
  return hipGetLastError();
}

template <int DT, int ACC>
hipError_t reduce_acc(const PlainPlan& p, const ReduceArgs& a, hipStream_t s) {
  switch (p.unroll) {
    case 1: return reduce_u<DT, ACC, 1>(p, a, s);
    case 2: return reduce_u<DT, ACC, 2>(p, a, s);
    case 4: return reduce_u<DT, ACC, 4>(p, a, s);
    default: return reduce_u<DT, ACC, 8>(p, a, s);
  }
}

template <int DT>
hipError_t reduce_dt(const PlainPlan& p, const ReduceArgs& a, hipStream_t s) {
  return p.acc == NRM_ACC_KAHAN ? reduce_acc<DT, NRM_ACC_KAHAN>(p, a, s)
                                : reduce_acc<DT, NRM_ACC_F32>(p, a, s);
}

template <int DTI, int DTO, int U>
hipError_t map_u(const PlainPlan& p, const MapArgs& a, hipStream_t s) {
  if (p.map_nt)
    hipLaunchKernelGGL((map_kernel<DTI, DTO, U, true>), dim3(p.map_grid), dim3(p.map_block), 0, s, a);
  else
    hipLaunchKernelGGL((map_kernel<DTI, DTO, U, false>), dim3(p.map_grid), dim3(p.map_block), 0, s, a);
  return hipGetLastError();
}

template <int DTI, int DTO>
hipError_t map_pair(const PlainPlan& p, const MapArgs& a, hipStream_t s) {
  if (!p.vector_map) {
    int64_t blocks = (p.n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((map_scalar_kernel<DTI, DTO>), dim3(blocks), dim3(256), 0, s, a.in, a.out,
                       p.n, a.sum);
    return hipGetLastError();
  }
  switch (p.map_unroll) {
    case 1: return map_u<DTI, DTO, 1>(p, a, s);
    case 2: return map_u<DTI, DTO, 2>(p, a, s);
    case 4: return map_u<DTI, DTO, 4>(p, a, s);
    default: return map_u<DTI, DTO, 8>(p, a, s);
  }
}

template <int DTI>
hipError_t map_in(const PlainPlan& p, const MapArgs& a, hipStream_t s) {
  switch (p.out_dt) {
    case NRM_F32: return map_pair<DTI, NRM_F32>(p, a, s);
    case NRM_BF16: return map_pair<DTI, NRM_BF16>(p, a, s);
    default: return map_pair<DTI, NRM_F16>(p, a, s);
  }
}

}  // namespace

hipError_t launch_reduce(const PlainPlan& p, const PlainWorkspace& ws, hipStream_t s) {
  ReduceArgs a;
  a.in = static_cast<const char*>(p.in);
  a.body = reinterpret_cast<const u4*>(a.in + p.head * dtype_size(p.in_dt));
  a.head = p.head;
  a.nvec = p.nvec;
  a.tail_begin = p.tail_begin;
  a.n = p.n;
  a.chunk = p.chunk;
  a.tile = p.tile;
  a.layout = p.layout;
  a.fused = p.fused;
  a.keep_from = p.keep_from;
  a.partials = ws.partials;
  a.ticket = ws.ticket;
  a.sum = ws.sum;
  switch (p.in_dt) {
    case NRM_F32: return reduce_dt<NRM_F32>(p, a, s);
    case NRM_BF16: return reduce_dt<NRM_BF16>(p, a, s);
    default: return reduce_dt<NRM_F16>(p, a, s);
  }
}

hipError_t launch_map(const PlainPlan& p, const PlainWorkspace& ws, hipStream_t s) {
  MapArgs a;
  a.in = static_cast<const char*>(p.in);
  a.out = static_cast<char*>(p.out);
  a.body = reinterpret_cast<const u4*>(a.in + p.head * dtype_size(p.in_dt));
  a.out_body = a.out + p.head * dtype_size(p.out_dt);
  a.head = p.head;
  a.nvec = p.map_units;
  a.tail_begin = p.tail_begin;
  a.n = p.n;
  a.chunk = p.map_chunk;
  a.tile = p.map_tile;
  a.layout = p.map_layout;
  a.reverse = p.reverse_map;
  a.sum = ws.sum;
  a.fused = p.fused;
  a.acc = p.acc;
  a.partials = ws.partials;
  a.nparts = p.grid;
  a.sum_out = ws.sum;
  switch (p.in_dt) {
    case NRM_F32: return map_in<NRM_F32>(p, a, s);
    case NRM_BF16: return map_in<NRM_BF16>(p, a, s);
    default: return map_in<NRM_F16>(p, a, s);
  }
}

}  // namespace nrm
