// normalize in one kernel for large n: the reduce and the divide map of the
// plain path (arXiv 2207.00257, Fig. 1 with the sum hoisted, Sec. IV-C) run as
// two phases of one cooperative launch, so that the first chunk each block
// reads stays in its registers until the second phase divides it, and the
// kernel boundary between the phases becomes an exchange of sums.
//
//   phase A  block b of G sums chunks b, b + G, b + 2G, ... (CHUNK_VECS
//            16-byte vectors each; binary32 chains per thread, no barrier
//            until the end), keeping chunk b in registers; the chunks from
//            keep_from on are read with a temporal hint. Then one block
//            reduce (DPP, one LDS slot per wavefront), and the block's sum
//            goes out as tagged words. The last block to arrive merges the G
//            sums in block order (a fixed tree: the bits depend on n and G
//            only) and publishes the total.
//   phase B  every block divides the chunk it holds and stores it, and takes
//            the other chunks from the last one down (phase A read those
//            last, so the last-level cache still has them).
//
// The launch is cooperative, so all G blocks are resident together and the
// blocks waiting for the total never hold a place a missing block needs;
// the waits are bounded all the same (NRM_DEVERR_STALL). The last block to
// finish resets the arrival counter and moves the call number on (every
// block read it before).
#include <type_traits>

#include "nrm_batch.h"
#include "nrm_device.h"
#include "nrm_internal.h"

namespace nrm {
namespace {

using namespace dev;

constexpr int FB = 512;     // threads per block
constexpr int GL = 8;       // loads in flight per thread while streaming past the held chunk
constexpr int HV = 16;      // vectors per thread in a chunk
constexpr int64_t CHUNK_VECS = (int64_t)FB * HV;
static_assert(HV % GL == 0 && FUSED_MAX_BLOCKS % FB == 0, "shapes");
constexpr uint32_t FSPIN = 1u << 18;
constexpr std::true_type TRUE_{};
constexpr std::false_type FALSE_{};

struct FusedArgs {
  const char* in;
  char* out;
  const u4* body;        // first 16-byte aligned input vector
  char* out_body;        // output element `head`
  int64_t head, nvec, tail_begin, n;
  int64_t nchunks;
  int64_t keep_from;     // chunks from here on are loaded with a temporal hint
  FusedWs w;
};

__device__ __forceinline__ uint32_t tag_of(unsigned long long call) { return (uint32_t)(call % 0xFFFFFFFFull) + 1u; }

template <int ACC>
__device__ __forceinline__ void put_tagged(unsigned long long* p, uint32_t ep, const Acc<ACC>& v) {
  float f[2];
  if constexpr (ACC == NRM_ACC_F32) {
    f[0] = v.s;
    f[1] = 0.0f;
  } else {
    f[0] = v.hi;
    f[1] = v.lo;
  }
  constexpr int W = ACC == NRM_ACC_F32 ? 1 : 2;
#pragma unroll
  for (int k = 0; k < W; ++k)
    __hip_atomic_store(p + k, ((unsigned long long)ep << 32) | bits_f32(f[k]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Reads a tagged value; false while its tag is not `ep`.
template <int ACC>
__device__ __forceinline__ bool get_tagged(const unsigned long long* p, uint32_t ep, Acc<ACC>& v) {
  constexpr int W = ACC == NRM_ACC_F32 ? 1 : 2;
  float f[2] = {0.0f, 0.0f};
  bool ok = true;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const unsigned long long x = __hip_atomic_load(p + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    f[k] = f32_bits((uint32_t)x);
    ok = ok && (uint32_t)(x >> 32) == ep;
  }
  if constexpr (ACC == NRM_ACC_F32) {
    v.s = f[0];
  } else {
    v.hi = f[0];
    v.lo = f[1];
  }
  return ok;
}

__device__ __forceinline__ void fused_give_up(const FusedWs& w) { atomicOr(w.error, NRM_DEVERR_STALL); }

// Chunks go through buffer resources: base = the chunk's first byte, range =
// its bytes that exist. A load past the range reads 0 (+0 in every storage
// type) and a store past it is dropped, which covers a partial last chunk.
// In a full chunk the per-load distance rides in the scalar offset; in a
// partial one it goes into the vector offset, the part the range check sees.
constexpr int kNT = 2;  // cache policy: non-temporal

__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

template <bool FULL, int AUX>
__device__ __forceinline__ u4 bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t dist) {
  if constexpr (FULL) return __builtin_amdgcn_raw_buffer_load_b128(r, voff, dist, AUX);
  else return __builtin_amdgcn_raw_buffer_load_b128(r, voff + dist, 0, AUX);
}

// VEC quotients as one output vector (VEC elements of DTO) at byte voff + dist.
template <bool FULL, int DTO, int VEC>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t dist, const float (&q)[VEC]) {
  const uint32_t vo = FULL ? voff : voff + dist, so = FULL ? dist : 0u;
  if constexpr (DTO == NRM_F32) {
#pragma unroll
    for (int h = 0; h < VEC / 4; ++h)
      __builtin_amdgcn_raw_buffer_store_b128(
          u4{bits_f32(q[4 * h]), bits_f32(q[4 * h + 1]), bits_f32(q[4 * h + 2]), bits_f32(q[4 * h + 3])}, r,
          vo + 16u * h, so, kNT);
  } else if constexpr (VEC == 8) {
    __builtin_amdgcn_raw_buffer_store_b128(
        u4{pack2<DTO>(q[0], q[1]), pack2<DTO>(q[2], q[3]), pack2<DTO>(q[4], q[5]), pack2<DTO>(q[6], q[7])}, r, vo,
        so, kNT);
  } else {
    __builtin_amdgcn_raw_buffer_store_b64(u2{pack2<DTO>(q[0], q[1]), pack2<DTO>(q[2], q[3])}, r, vo, so, kNT);
  }
}

template <int DTI, int DTO, int ACC>
__global__ void __launch_bounds__(FB) __attribute__((amdgpu_waves_per_eu(4, 4))) fused_kernel(FusedArgs a) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int NA_MAX = ACC == NRM_ACC_F32 ? 8 : 4;
  constexpr int NA = VEC < NA_MAX ? VEC : NA_MAX;
  constexpr uint32_t OUTV = VEC * Elem<DTO>::SIZE;  // bytes per output vector
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ int s_last;
  __shared__ float s_sum;
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x, G = gridDim.x;
  const FusedWs& w = a.w;
  const unsigned long long call = __hip_atomic_load(w.call, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t ep = tag_of(call);

  auto in_rsrc = [&](int64_t c) {
    const int64_t v0 = c * CHUNK_VECS, left = a.nvec - v0;
    return chunk_rsrc(a.body + v0, 16 * (left < CHUNK_VECS ? left : CHUNK_VECS));
  };
  auto out_rsrc = [&](int64_t c) {
    const int64_t v0 = c * CHUNK_VECS, left = a.nvec - v0;
    return chunk_rsrc(a.out_body + v0 * OUTV, OUTV * (left < CHUNK_VECS ? left : CHUNK_VECS));
  };
  // K vectors of this thread's share of chunk c, from its vector `first`
  // on (stride FB), temporal or not
  auto load = [&](auto temporal, int64_t c, int first, auto& dst) {
    constexpr int K = sizeof(dst) / sizeof(dst[0]);
    constexpr int AUX = decltype(temporal)::value ? 0 : kNT;
    const __amdgpu_buffer_rsrc_t r = in_rsrc(c);
    const uint32_t voff = 16u * (uint32_t)t;
    if ((c + 1) * CHUNK_VECS <= a.nvec) {
#pragma unroll
      for (int k = 0; k < K; ++k) dst[k] = bload<true, AUX>(r, voff, 16u * (uint32_t)((first + k) * FB));
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) dst[k] = bload<false, AUX>(r, voff, 16u * (uint32_t)((first + k) * FB));
    }
  };
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  auto add = [&](const u4& r) {
    float x[VEC];
    widen<DTI>(r, x);
#pragma unroll
    for (int k = 0; k < VEC; ++k) acc[k % NA].add(x[k]);
  };

  // ---- phase A -------------------------------------------------------------
  u4 held[HV];
  const bool holds = b < a.nchunks;
  if (holds) {
    load(FALSE_, b, 0, held);  // every load of the held chunk in flight at once
#pragma unroll
    for (int k = 0; k < HV; ++k) add(held[k]);
  }
  // the others stream through GL loads at a time (the held chunk takes half
  // the register budget)
#pragma unroll 1
  for (int64_t c = b + G; c < a.nchunks; c += G) {
    const bool temporal = c >= a.keep_from;
#pragma unroll 1
    for (int g = 0; g < HV / GL; ++g) {
      u4 r[GL];
      if (temporal) load(TRUE_, c, g * GL, r);
      else load(FALSE_, c, g * GL, r);
#pragma unroll
      for (int k = 0; k < GL; ++k) add(r[k]);
    }
  }
  // the unaligned head belongs to chunk 0's block, the short tail to the
  // last chunk's
  if (b == 0 && t < a.head) acc[0].add(load_one<DTI>(a.in, t));
  if (b == (a.nchunks - 1) % G && t < a.n - a.tail_begin) acc[0].add(load_one<DTI>(a.in, a.tail_begin + t));
  merge_chains<ACC, NA>(acc);
  const Acc<ACC> part = block_reduce<ACC>(acc[0], slots);
  // arrive; the last block to arrive merges the G block sums
  if (t == 0) {
    put_tagged<ACC>(w.slots + 2 * b, ep, part);
    const unsigned prev = __hip_atomic_fetch_add(w.arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev == (unsigned)(G - 1);
  }
  lds_barrier();
  if (s_last) {
    // thread t merges block sums t and t + FB, then the block tree
    Acc<ACC> v[FUSED_MAX_BLOCKS / FB];
    for (uint32_t spin = 0;; ++spin) {
      bool ok = true;
#pragma unroll
      for (int j = 0; j < FUSED_MAX_BLOCKS / FB; ++j) {
        const int64_t k = t + (int64_t)j * FB;
        v[j].zero();
        if (k < G) ok = get_tagged<ACC>(w.slots + 2 * k, ep, v[j]) && ok;
      }
      if (__syncthreads_and(ok)) break;
      if (spin >= FSPIN) {
        if (t == 0) fused_give_up(w);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int s = 1; s < FUSED_MAX_BLOCKS / FB; s <<= 1)
#pragma unroll
      for (int j = 0; j + s < FUSED_MAX_BLOCKS / FB; j += 2 * s) v[j].merge(v[j + s]);
    lds_barrier();  // slots are reused
    const Acc<ACC> total = block_reduce<ACC>(v[0], slots);
    if (t == 0) {
      put_tagged<ACC>(w.total, ep, total);
      s_sum = total.value();
      w.sum_out[0] = total.value();
    }
  } else if (t == 0) {
    Acc<ACC> total;
    uint32_t spin = 0;
    while (!get_tagged<ACC>(w.total, ep, total)) {
      if (++spin >= FSPIN) {
        fused_give_up(w);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    s_sum = total.value();
  }
  lds_barrier();
  const float S = s_sum;

  // ---- phase B -------------------------------------------------------------
  // (the host takes this form only when out is aligned like in)
  auto divide_store = [&](int64_t c, int first, const u4* r, auto kk) {
    constexpr int K = decltype(kk)::value;
    const __amdgpu_buffer_rsrc_t o = out_rsrc(c);
    const uint32_t voff = OUTV * (uint32_t)t;
    const bool full = (c + 1) * CHUNK_VECS <= a.nvec;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float x[VEC], q[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int e = 0; e < VEC; ++e) q[e] = x[e] / S;
      const uint32_t dist = OUTV * (uint32_t)((first + k) * FB);
      if (full) bstore<true, DTO, VEC>(o, voff, dist, q);
      else bstore<false, DTO, VEC>(o, voff, dist, q);
    }
  };
  auto edges = [&](int64_t c) {
    if (c == 0 && t < a.head) store_one<DTO>(a.out, t, load_one<DTI>(a.in, t) / S);
    if (c == a.nchunks - 1 && t < a.n - a.tail_begin)
      store_one<DTO>(a.out, a.tail_begin + t, load_one<DTI>(a.in, a.tail_begin + t) / S);
  };
  // chunks below min(G, nchunks) are held by their blocks; the others go
  // from the last one down, block b taking nchunks - 1 - b, then G further
  const int64_t first_b = a.nchunks - 1 - b;
  if (holds) {
    if (first_b >= G) {
      // the first streamed chunk's loads go out before the held chunk's
      // divides, so that the memory system has work meanwhile
      u4 r[GL];
      load(FALSE_, first_b, 0, r);
#pragma unroll
      for (int g = 0; g < HV / GL; ++g) divide_store(b, g * GL, held + g * GL, std::integral_constant<int, GL>());
      edges(b);
      divide_store(first_b, 0, r, std::integral_constant<int, GL>());
#pragma unroll
      for (int g = 1; g < HV / GL; ++g) {
        load(FALSE_, first_b, g * GL, r);
        divide_store(first_b, g * GL, r, std::integral_constant<int, GL>());
      }
      edges(first_b);
    } else {
#pragma unroll
      for (int g = 0; g < HV / GL; ++g) divide_store(b, g * GL, held + g * GL, std::integral_constant<int, GL>());
      edges(b);
    }
  }
#pragma unroll 1
  for (int64_t c = first_b - G; c >= G; c -= G) {
    u4 r[HV];
    load(FALSE_, c, 0, r);
#pragma unroll
    for (int g = 0; g < HV / GL; ++g) divide_store(c, g * GL, r + g * GL, std::integral_constant<int, GL>());
    edges(c);
  }
  // the last block out resets the arrivals and moves the call on
  if (t == 0) {
    const unsigned prev = __hip_atomic_fetch_add(w.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == (unsigned)(G - 1)) {
      __hip_atomic_store(w.arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(w.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(w.call, call + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int DTI, int DTO, int ACC>
hipError_t launch_one(FusedArgs a, int64_t max_grid, hipStream_t s) {
  const void* f = reinterpret_cast<const void*>(&fused_kernel<DTI, DTO, ACC>);
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, FB, 0);
  if (e != hipSuccess) return e;
  // every block resident at once (the cooperative launch checks it), at
  // most FUSED_MAX_BLOCKS of them
  int64_t grid = (int64_t)cus * per_cu;
  if (grid > FUSED_MAX_BLOCKS) grid = FUSED_MAX_BLOCKS;
  if (max_grid > 0 && grid > max_grid) grid = max_grid;
  if (grid < 1) return hipErrorInvalidConfiguration;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(f, dim3((unsigned)grid), dim3(FB), args, 0, s);
}

template <int ACC, int DTI>
hipError_t fused_in(const FusedArgs& a, int out_dt, int64_t max_grid, hipStream_t s) {
  switch (out_dt) {
    case NRM_F32: return launch_one<DTI, NRM_F32, ACC>(a, max_grid, s);
    case NRM_BF16: return launch_one<DTI, NRM_BF16, ACC>(a, max_grid, s);
    default: return launch_one<DTI, NRM_F16, ACC>(a, max_grid, s);
  }
}

template <int ACC>
hipError_t fused_acc(const FusedArgs& a, int in_dt, int out_dt, int64_t max_grid, hipStream_t s) {
  switch (in_dt) {
    case NRM_F32: return fused_in<ACC, NRM_F32>(a, out_dt, max_grid, s);
    case NRM_BF16: return fused_in<ACC, NRM_BF16>(a, out_dt, max_grid, s);
    default: return fused_in<ACC, NRM_F16>(a, out_dt, max_grid, s);
  }
}

}  // namespace

hipError_t launch_fused(const PlainPlan& p, const FusedWs& w, int64_t max_grid, hipStream_t s) {
  FusedArgs a;
  a.in = static_cast<const char*>(p.in);
  a.out = static_cast<char*>(p.out);
  a.body = reinterpret_cast<const u4*>(a.in + p.head * dtype_size(p.in_dt));
  a.out_body = a.out + p.head * dtype_size(p.out_dt);
  a.head = p.head;
  a.nvec = p.nvec;
  a.tail_begin = p.tail_begin;
  a.n = p.n;
  a.nchunks = (p.nvec + CHUNK_VECS - 1) / CHUNK_VECS;
  // the temporal tail (reduce_keep_mib of the input), in whole chunks
  a.keep_from = p.keep_from / CHUNK_VECS;
  a.w = w;
  return p.acc == NRM_ACC_KAHAN ? fused_acc<NRM_ACC_KAHAN>(a, p.in_dt, p.out_dt, max_grid, s)
                                : fused_acc<NRM_ACC_F32>(a, p.in_dt, p.out_dt, max_grid, s);
}

}  // namespace nrm
