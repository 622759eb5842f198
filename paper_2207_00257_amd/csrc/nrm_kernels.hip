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
//                  one __syncthreads (the block barrier of Fig. 1's shared-
//                  memory variant). The last block to finish (an agent-scope
//                  ticket; partials travel by agent-scope atomic stores and
//                  loads, coherent across the XCDs' separate L2 caches)
//                  combines all partials in a fixed tree in LDS (the halving
//                  loop of Fig. 7) and writes the sum.
//   map_kernel     out[i] = in[i] / sum with a correctly rounded binary32
//                  division, 16-byte vector loads, non-temporal vector stores.
//
// The kernel boundary between the two is the grid-wide barrier. No float
// atomics are used: for given sizes, alignment and launch parameters every
// addition happens in the same order on every run.
#include "nrm_internal.h"

namespace nrm {
namespace {

typedef unsigned int u32;
typedef u32 u4 __attribute__((ext_vector_type(4)));
typedef u32 u2 __attribute__((ext_vector_type(2)));

// ---- bit reinterpretation ------------------------------------------------------
// Always through a by-value parameter: this compiler reads element 0 when
// __builtin_bit_cast is applied directly to an element of an ext_vector_type.
__device__ __forceinline__ float f32_bits(u32 w) { return __builtin_bit_cast(float, w); }
__device__ __forceinline__ u32 bits_f32(float v) { return __builtin_bit_cast(u32, v); }
__device__ __forceinline__ int ibits_f32(float v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ float f32_ibits(int w) { return __builtin_bit_cast(float, w); }
__device__ __forceinline__ float f32_of_f16_bits(unsigned short h) {
  return (float)__builtin_bit_cast(_Float16, h);
}
__device__ __forceinline__ u32 bits_bf16(__bf16 v) { return __builtin_bit_cast(unsigned short, v); }
__device__ __forceinline__ u32 bits_f16(_Float16 v) { return __builtin_bit_cast(unsigned short, v); }

// ---- storage types ---------------------------------------------------------

template <int DT>
struct Elem {
  static constexpr int SIZE = DT == NRM_F32 ? 4 : 2;
  static constexpr int VEC = 16 / SIZE;  // elements per 16-byte vector
};

// Widen one 16-byte vector to VEC binary32 values (exact for all three types).
template <int DT>
__device__ __forceinline__ void widen(u4 r, float (&x)[Elem<DT>::VEC]) {
  if constexpr (DT == NRM_F32) {
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = f32_bits(r[k]);
  } else if constexpr (DT == NRM_BF16) {
    // bfloat16 is the upper half of a binary32
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[2 * k] = f32_bits(r[k] << 16);
      x[2 * k + 1] = f32_bits(r[k] & 0xFFFF0000u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[2 * k] = f32_of_f16_bits((unsigned short)(r[k] & 0xFFFFu));
      x[2 * k + 1] = f32_of_f16_bits((unsigned short)(r[k] >> 16));
    }
  }
}

template <int DT>
__device__ __forceinline__ float load_one(const char* base, int64_t i) {
  if constexpr (DT == NRM_F32) {
    return reinterpret_cast<const float*>(base)[i];
  } else if constexpr (DT == NRM_BF16) {
    u32 h = reinterpret_cast<const unsigned short*>(base)[i];
    return f32_bits(h << 16);
  } else {
    return (float)reinterpret_cast<const _Float16*>(base)[i];
  }
}

// binary32 -> storage type, round to nearest even (gfx950 converts BF16 in hardware).
template <int DT>
__device__ __forceinline__ void store_one(char* base, int64_t i, float q) {
  if constexpr (DT == NRM_F32) {
    reinterpret_cast<float*>(base)[i] = q;
  } else if constexpr (DT == NRM_BF16) {
    reinterpret_cast<__bf16*>(base)[i] = (__bf16)q;
  } else {
    reinterpret_cast<_Float16*>(base)[i] = (_Float16)q;
  }
}

template <int DT>
__device__ __forceinline__ u32 pack2(float a, float b) {
  if constexpr (DT == NRM_BF16) {
    return bits_bf16((__bf16)a) | (bits_bf16((__bf16)b) << 16);
  } else {
    return bits_f16((_Float16)a) | (bits_f16((_Float16)b) << 16);
  }
}

// Store VEC quotients as element group `vi` of the output (VEC * size bytes).
template <int DTO, int VEC>
__device__ __forceinline__ void store_vec(char* out, int64_t vi, const float (&q)[VEC]) {
  if constexpr (DTO == NRM_F32) {
    u4* p = reinterpret_cast<u4*>(out) + vi * (VEC / 4);
#pragma unroll
    for (int h = 0; h < VEC / 4; ++h) {
      u4 v = {bits_f32(q[4 * h]), bits_f32(q[4 * h + 1]), bits_f32(q[4 * h + 2]),
              bits_f32(q[4 * h + 3])};
      __builtin_nontemporal_store(v, p + h);
    }
  } else if constexpr (VEC == 8) {
    u4 v = {pack2<DTO>(q[0], q[1]), pack2<DTO>(q[2], q[3]), pack2<DTO>(q[4], q[5]),
            pack2<DTO>(q[6], q[7])};
    __builtin_nontemporal_store(v, reinterpret_cast<u4*>(out) + vi);
  } else {
    u2 v = {pack2<DTO>(q[0], q[1]), pack2<DTO>(q[2], q[3])};
    __builtin_nontemporal_store(v, reinterpret_cast<u2*>(out) + vi);
  }
}

template <bool NT>
__device__ __forceinline__ u4 load_vec(const u4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// ---- accumulators ------------------------------------------------------------

template <int ACC>
struct Acc;

// Plain binary32 chain.
template <>
struct Acc<NRM_ACC_F32> {
  float s;
  __device__ __forceinline__ void zero() { s = 0.0f; }
  __device__ __forceinline__ void add(float x) { s = s + x; }
  __device__ __forceinline__ void merge(const Acc& o) { s = s + o.s; }
  __device__ __forceinline__ float value() const { return s; }
};

// Compensated chain: value hi + lo. Adding an element is Kahan's update
// (Kahan 1965); merging two chains is Knuth's TwoSum of the high parts plus
// the low parts, renormalised with Dekker's FastTwoSum (the error-free
// transformations of Ogita, Rump and Oishi's Sum2).
template <>
struct Acc<NRM_ACC_KAHAN> {
  float hi, lo;
  __device__ __forceinline__ void zero() { hi = 0.0f; lo = 0.0f; }
  __device__ __forceinline__ void add(float x) {
    float y = x + lo;
    float t = hi + y;
    lo = y - (t - hi);
    hi = t;
  }
  __device__ __forceinline__ void merge(const Acc& o) {
    float s = hi + o.hi;
    float bb = s - hi;
    float e = (hi - (s - bb)) + (o.hi - bb);
    float l = e + (lo + o.lo);
    float h = s + l;
    lo = l - (h - s);
    hi = h;
  }
  __device__ __forceinline__ float value() const { return hi + lo; }
};

// ---- wavefront and block reduction ------------------------------------------

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return f32_ibits(__builtin_amdgcn_update_dpp(0, ibits_f32(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float readlane(float v, int lane) {
  return f32_ibits(__builtin_amdgcn_readlane(ibits_f32(v), lane));
}

constexpr int QP_SWAP1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int QP_SWAP2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int ROW_HALF_MIRROR = 0x141;
constexpr int ROW_MIRROR = 0x140;

// Sum over the 64 lanes of a wavefront. Within each row of 16 lanes, four DPP
// steps (pair, quad, half-row mirror, row mirror) leave the row sum in every
// lane of the row (each step adds a lane's value to its partner's, and
// addition is commutative, so partners hold identical bits). The four row
// sums are then combined as (r0 + r1) + (r2 + r3). Every lane returns it.
template <int ACC>
__device__ __forceinline__ Acc<ACC> wave_reduce(Acc<ACC> a) {
  if constexpr (ACC == NRM_ACC_F32) {
    float v = a.s;
    v = v + dpp<QP_SWAP1>(v);
    v = v + dpp<QP_SWAP2>(v);
    v = v + dpp<ROW_HALF_MIRROR>(v);
    v = v + dpp<ROW_MIRROR>(v);
    Acc<ACC> r;
    r.s = (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
    return r;
  } else {
    // TwoSum-based merge is symmetric in its operands (both the sum and the
    // exact error term are), so partner lanes again hold identical bits.
    Acc<ACC> o;
    o.hi = dpp<QP_SWAP1>(a.hi); o.lo = dpp<QP_SWAP1>(a.lo); a.merge(o);
    o.hi = dpp<QP_SWAP2>(a.hi); o.lo = dpp<QP_SWAP2>(a.lo); a.merge(o);
    o.hi = dpp<ROW_HALF_MIRROR>(a.hi); o.lo = dpp<ROW_HALF_MIRROR>(a.lo); a.merge(o);
    o.hi = dpp<ROW_MIRROR>(a.hi); o.lo = dpp<ROW_MIRROR>(a.lo); a.merge(o);
    Acc<ACC> r0, r1, r2, r3;
    r0.hi = readlane(a.hi, 0); r0.lo = readlane(a.lo, 0);
    r1.hi = readlane(a.hi, 16); r1.lo = readlane(a.lo, 16);
    r2.hi = readlane(a.hi, 32); r2.lo = readlane(a.lo, 32);
    r3.hi = readlane(a.hi, 48); r3.lo = readlane(a.lo, 48);
    r0.merge(r1);
    r2.merge(r3);
    r0.merge(r2);
    return r0;
  }
}

constexpr int MAX_WAVES = 1024 / 64;

// Cross-block exchange of partials inside one kernel. The L2 is per XCD; the
// values travel with agent-scope atomic stores and loads, which are coherent
// across the XCDs' L2 caches (sc1) without relying on L2 write-back and
// invalidation, and the agent-scope fences around the ticket order them.
__device__ __forceinline__ void publish(Acc<NRM_ACC_F32>* p, int64_t i, const Acc<NRM_ACC_F32>& v) {
  __hip_atomic_store(reinterpret_cast<u32*>(p) + i, bits_f32(v.s), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish(Acc<NRM_ACC_KAHAN>* p, int64_t i, const Acc<NRM_ACC_KAHAN>& v) {
  unsigned long long w = (unsigned long long)bits_f32(v.hi) | ((unsigned long long)bits_f32(v.lo) << 32);
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p) + i, w, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fetch(const Acc<NRM_ACC_F32>* p, int64_t i, Acc<NRM_ACC_F32>& v) {
  v.s = f32_bits(__hip_atomic_load(reinterpret_cast<const u32*>(p) + i,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void fetch(const Acc<NRM_ACC_KAHAN>* p, int64_t i, Acc<NRM_ACC_KAHAN>& v) {
  unsigned long long w = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p) + i,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.hi = f32_bits((u32)w);
  v.lo = f32_bits((u32)(w >> 32));
}

// Sum over the block; the result is valid in thread 0 (zero elsewhere). One
// LDS slot per wavefront and one barrier; then thread 0 merges the wavefront
// sums in a fixed pairwise tree. A caller that reuses `slots` must put a
// barrier between two calls.
template <int ACC>
__device__ __forceinline__ Acc<ACC> block_reduce(Acc<ACC> a, Acc<ACC>* slots) {
  a = wave_reduce<ACC>(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  if (lane == 0) slots[wave] = a;
  __syncthreads();
  Acc<ACC> r;
  r.zero();
  if (threadIdx.x == 0) {
    for (int s = 1; s < waves; s <<= 1)
      for (int i = 0; i + s < waves; i += 2 * s) slots[i].merge(slots[i + s]);
    r = slots[0];
  }
  return r;
}

// ---- phase 1: block partials and the grid combine ------------------------------

struct ReduceArgs {
  const char* in;      // the input (element 0)
  const u4* body;      // first 16-byte aligned vector of the input
  int64_t head;        // elements before body
  int64_t nvec;        // vectors in the body
  int64_t tail_begin;  // first element after the body
  int64_t n;
  int64_t chunk;       // vectors per block (layout CHUNK), multiple of blockDim * U
  int layout;
  void* partials;      // Acc<ACC>[gridDim.x]
  unsigned* ticket;    // 0 on entry, left 0 on exit
  float* sum;          // out: the hoisted invariant
};

constexpr int COMBINE_TILE = 1024;     // partials merged per LDS tree pass
constexpr int MAX_COMBINE_TILES = 64;  // at most 65536 blocks in a reduce launch

// Pairwise sum of the thread's chains into acc[0] (fixed tree).
template <int ACC, int NA>
__device__ __forceinline__ void merge_chains(Acc<ACC> (&acc)[NA]) {
#pragma unroll
  for (int s = 1; s < NA; s <<= 1)
#pragma unroll
    for (int k = 0; k + s < NA; k += 2 * s) acc[k].merge(acc[k + s]);
}

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
  for (int64_t base = begin; base < end; base += stride) {
    u4 r[U];
    if (base + step <= end) {
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load_vec<NT>(p + base + u * B);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float x[VEC];
        widen<DT>(r[u], x);
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc[(u * VEC + k) % NA].add(x[k]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (base + u * B + (int64_t)threadIdx.x < end) {
          float x[VEC];
          widen<DT>(load_vec<NT>(p + base + u * B), x);
#pragma unroll
          for (int k = 0; k < VEC; ++k) acc[(u * VEC + k) % NA].add(x[k]);
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
  // unaligned head and the tail shorter than a vector: block 0
  if (blockIdx.x == 0) {
    if ((int64_t)threadIdx.x < a.head) acc[0].add(load_one<DT>(a.in, threadIdx.x));
    if ((int64_t)threadIdx.x < a.n - a.tail_begin) acc[0].add(load_one<DT>(a.in, a.tail_begin + threadIdx.x));
  }
  merge_chains<ACC, NA>(acc);
  run.merge(acc[0]);

  Acc<ACC> blk = block_reduce<ACC>(run, slots);

  // publish the partial; the last block to arrive combines all of them
  Acc<ACC>* part = reinterpret_cast<Acc<ACC>*>(a.partials);
  if (threadIdx.x == 0) {
    publish(part, blockIdx.x, blk);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    unsigned prev = __hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

  // Fixed-order combine: tiles of COMBINE_TILE partials are merged by a
  // halving tree in LDS (each level adds slot i + s into slot i, then a
  // barrier); thread 0 then merges the tile results pairwise.
  __shared__ Acc<ACC> tree[COMBINE_TILE];
  __shared__ Acc<ACC> tiles[MAX_COMBINE_TILES];
  const int64_t G = gridDim.x;
  const int ntiles = (int)((G + COMBINE_TILE - 1) / COMBINE_TILE);
  for (int t = 0; t < ntiles; ++t) {
    const int64_t t0 = (int64_t)t * COMBINE_TILE;
    for (int i = threadIdx.x; i < COMBINE_TILE; i += blockDim.x) {
      if (t0 + i < G) fetch(part, t0 + i, tree[i]);
      else tree[i].zero();
    }
    __syncthreads();
    for (int s = COMBINE_TILE / 2; s >= 1; s >>= 1) {
      for (int i = threadIdx.x; i < s; i += blockDim.x) tree[i].merge(tree[i + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) tiles[t] = tree[0];
    __syncthreads();
  }
  Acc<ACC> total;
  total.zero();
  if (threadIdx.x == 0) {
    for (int s = 1; s < ntiles; s <<= 1)
      for (int i = 0; i + s < ntiles; i += 2 * s) tiles[i].merge(tiles[i + s]);
    total = tiles[0];
  }
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
  int64_t chunk;       // vectors per block (layout CHUNK), multiple of blockDim * U
  int layout;
  int reverse;
  const float* sum;
};

template <int DTI, int DTO, int U, bool NT>
__global__ void __launch_bounds__(1024) map_kernel(MapArgs a) {
  constexpr int VEC = Elem<DTI>::VEC;
  const float S = a.sum[0];
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
  const int64_t iters = end > begin ? (end - begin + stride - 1) / stride : 0;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t base = begin + (a.reverse ? iters - 1 - it : it) * stride;
    const int64_t v0 = base + threadIdx.x;
    if (base + step <= end) {
      u4 r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load_vec<NT>(a.body + v0 + u * B);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float x[VEC], q[VEC];
        widen<DTI>(r[u], x);
#pragma unroll
        for (int k = 0; k < VEC; ++k) q[k] = x[k] / S;
        store_vec<DTO, VEC>(a.out_body, v0 + u * B, q);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (v0 + u * B < end) {
          float x[VEC], q[VEC];
          widen<DTI>(load_vec<NT>(a.body + v0 + u * B), x);
#pragma unroll
          for (int k = 0; k < VEC; ++k) q[k] = x[k] / S;
          store_vec<DTO, VEC>(a.out_body, v0 + u * B, q);
        }
      }
    }
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
  a.layout = p.layout;
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
  a.nvec = p.nvec;
  a.tail_begin = p.tail_begin;
  a.n = p.n;
  a.chunk = p.map_chunk;
  a.layout = p.map_layout;
  a.reverse = p.reverse_map;
  a.sum = ws.sum;
  switch (p.in_dt) {
    case NRM_F32: return map_in<NRM_F32>(p, a, s);
    case NRM_BF16: return map_in<NRM_BF16>(p, a, s);
    default: return map_in<NRM_F16>(p, a, s);
  }
}

}  // namespace nrm
