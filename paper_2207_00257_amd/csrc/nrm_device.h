// Device-side building blocks shared by the plain and batched normalize
// kernels: storage-type conversions, accumulators, the wavefront (DPP) and
// block reductions, the cross-block exchange of partials, and the fixed-order
// combine of partials.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrm_internal.h"

namespace nrm {
namespace dev {

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

template <bool NT>
__device__ __forceinline__ u2 load_vec(const u2* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Widen 8 bytes of a 2-byte type (4 elements) to binary32.
template <int DT>
__device__ __forceinline__ void widen_half(u2 r, float (&x)[4]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if constexpr (DT == NRM_BF16) {
      x[2 * k] = f32_bits(r[k] << 16);
      x[2 * k + 1] = f32_bits(r[k] & 0xFFFF0000u);
    } else {
      x[2 * k] = f32_of_f16_bits((unsigned short)(r[k] & 0xFFFFu));
      x[2 * k + 1] = f32_of_f16_bits((unsigned short)(r[k] >> 16));
    }
  }
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

// Row softmax (an internal accumulation kind next to the two public modes):
// a base-2 exponent k (an integer held in binary32) and the sum s of
// exp2(x * log2(e) - k) over the elements seen, with k >= every x * log2(e)
// so that each term is in (0, 1]. When an element exceeds k, k moves up to
// the next integer and s is rescaled by an exact power of two; merging two
// chains rescales both to the larger k the same way. Rescaling therefore
// adds no rounding: s stays a plain sum of positive terms, with the same
// error bound as a plain binary32 sum of its summation tree's height. Then
// softmax_i = exp2(x_i log2(e) - k) / s and lse = (k + log2 s) ln 2.
constexpr float LOG2E_F = 1.44269504088896340736f;  // log2(e), rounded to binary32
constexpr float LN2_F = 0.693147180559945309417f;   // ln(2), rounded to binary32
constexpr float K_NONE = -1.0e30f;                  // k of an empty chain

// s * 2^d for an integer-valued d <= 0 (exact unless the result leaves the
// normal range); d below -256 gives 0.
__device__ __forceinline__ float scale_pow2(float s, float d) {
  return __builtin_amdgcn_ldexpf(s, (int)fmaxf(d, -256.0f));
}

template <>
struct Acc<ACC_SOFTMAX> {
  float k, s;
  __device__ __forceinline__ void zero() { k = K_NONE; s = 0.0f; }
  __device__ __forceinline__ void add(float x) {
    const float y = x * LOG2E_F;
    if (y > k) {
      const float kn = __builtin_ceilf(y);
      s = scale_pow2(s, k - kn);
      k = kn;
    }
    s += __builtin_amdgcn_exp2f(__builtin_fmaf(x, LOG2E_F, -k));  // one rounding in the argument
  }
  __device__ __forceinline__ void merge(const Acc& o) {
    const float kn = fmaxf(k, o.k);
    s = scale_pow2(s, k - kn) + scale_pow2(o.s, o.k - kn);
    k = kn;
  }
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

// Sum over each row of 16 lanes: four DPP steps (pair, quad, half-row
// mirror, row mirror) leave the row's sum in every lane of the row, with
// identical bits in all of them (each step adds a lane's value to its
// partner's, and the merges are symmetric in their operands). Lanes read
// only lanes of their own row, so a row whose 16 lanes are all active may
// run it while other rows of the wavefront are inactive.
template <int ACC>
__device__ __forceinline__ Acc<ACC> row16_reduce(Acc<ACC> a) {
  if constexpr (ACC == NRM_ACC_F32) {
    float v = a.s;
    v = v + dpp<QP_SWAP1>(v);
    v = v + dpp<QP_SWAP2>(v);
    v = v + dpp<ROW_HALF_MIRROR>(v);
    v = v + dpp<ROW_MIRROR>(v);
    a.s = v;
  } else if constexpr (ACC == ACC_SOFTMAX) {
    // the merge is symmetric in its operands (a maximum and a sum of two
    // exactly rescaled terms), so partner lanes again hold identical bits
    Acc<ACC> o;
    o.k = dpp<QP_SWAP1>(a.k); o.s = dpp<QP_SWAP1>(a.s); a.merge(o);
    o.k = dpp<QP_SWAP2>(a.k); o.s = dpp<QP_SWAP2>(a.s); a.merge(o);
    o.k = dpp<ROW_HALF_MIRROR>(a.k); o.s = dpp<ROW_HALF_MIRROR>(a.s); a.merge(o);
    o.k = dpp<ROW_MIRROR>(a.k); o.s = dpp<ROW_MIRROR>(a.s); a.merge(o);
  } else {
    // TwoSum-based merge is symmetric in its operands (both the sum and the
    // exact error term are), so partner lanes again hold identical bits.
    Acc<ACC> o;
    o.hi = dpp<QP_SWAP1>(a.hi); o.lo = dpp<QP_SWAP1>(a.lo); a.merge(o);
    o.hi = dpp<QP_SWAP2>(a.hi); o.lo = dpp<QP_SWAP2>(a.lo); a.merge(o);
    o.hi = dpp<ROW_HALF_MIRROR>(a.hi); o.lo = dpp<ROW_HALF_MIRROR>(a.lo); a.merge(o);
    o.hi = dpp<ROW_MIRROR>(a.hi); o.lo = dpp<ROW_MIRROR>(a.lo); a.merge(o);
  }
  return a;
}

// Sum over the 64 lanes of a wavefront: each row of 16 lanes by
// row16_reduce, then the four row sums combined as (r0 + r1) + (r2 + r3).
// Every lane returns it.
template <int ACC>
__device__ __forceinline__ Acc<ACC> wave_reduce(Acc<ACC> a) {
  a = row16_reduce<ACC>(a);
  if constexpr (ACC == NRM_ACC_F32) {
    const float v = a.s;
    Acc<ACC> r;
    r.s = (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
    return r;
  } else if constexpr (ACC == ACC_SOFTMAX) {
    Acc<ACC> r0, r1, r2, r3;
    r0.k = readlane(a.k, 0); r0.s = readlane(a.s, 0);
    r1.k = readlane(a.k, 16); r1.s = readlane(a.s, 16);
    r2.k = readlane(a.k, 32); r2.s = readlane(a.s, 32);
    r3.k = readlane(a.k, 48); r3.s = readlane(a.s, 48);
    r0.merge(r1);
    r2.merge(r3);
    r0.merge(r2);
    return r0;
  } else {
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
__device__ __forceinline__ void publish(Acc<ACC_SOFTMAX>* p, int64_t i, const Acc<ACC_SOFTMAX>& v) {
  unsigned long long w = (unsigned long long)bits_f32(v.k) | ((unsigned long long)bits_f32(v.s) << 32);
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
__device__ __forceinline__ void fetch(const Acc<ACC_SOFTMAX>* p, int64_t i, Acc<ACC_SOFTMAX>& v) {
  unsigned long long w = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p) + i,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.k = f32_bits((u32)w);
  v.s = f32_bits((u32)(w >> 32));
}

// Block barrier for LDS traffic only: workgroup-scope fences on the local
// address space around s_barrier, which is all the block's threads exchange
// where it is used. (On gfx950 a block's wavefronts share one CU, and the
// compiler lowers even __syncthreads()'s fences to waits on LDS operations:
// neither barrier waits for global stores; code that needs them complete
// waits for them itself.)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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
  lds_barrier();
  Acc<ACC> r;
  r.zero();
  if (threadIdx.x == 0) {
    for (int s = 1; s < waves; s <<= 1)
      for (int i = 0; i + s < waves; i += 2 * s) slots[i].merge(slots[i + s]);
    r = slots[0];
  }
  return r;
}

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

// Up to 1024 partials merged by wavefront 0 alone, no LDS and no barrier:
// lane l holds partials l, l + 64, ... (up to 16), merges them pairwise, then
// the DPP wavefront tree; height 4 + 6. Call from all 64 lanes of wavefront
// 0; the result is valid in lane 0. ATOMIC: read with agent-scope atomic
// loads (partials published inside the same kernel); otherwise plain loads
// (partials written by an earlier kernel).
template <int ACC, bool ATOMIC>
__device__ __forceinline__ Acc<ACC> combine_wave(const Acc<ACC>* part, int64_t count) {
  Acc<ACC> v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k].zero();
    const int64_t i = threadIdx.x + 64 * k;
    if (i < count) {
      if constexpr (ATOMIC) fetch(part, i, v[k]);
      else v[k] = part[i];
    }
  }
#pragma unroll
  for (int s = 1; s < 16; s <<= 1)
#pragma unroll
    for (int k = 0; k + s < 16; k += 2 * s) v[k].merge(v[k + s]);
  return wave_reduce<ACC>(v[0]);
}

// Merge `count` partials (published with `publish`) into one value in a
// fixed order that depends only on count: up to 1024 partials in wavefront 0
// (registers and DPP); more in tiles of COMBINE_TILE partials merged by a
// halving tree in LDS (each level adds slot i + s into slot i, then a
// barrier: the shared-memory reduction pattern of Fig. 7), after which thread
// 0 merges the tile results pairwise. Every thread of the block must call it;
// the result is valid in thread 0. count <= COMBINE_TILE * MAX_COMBINE_TILES.
template <int ACC>
__device__ __forceinline__ Acc<ACC> combine_partials(const Acc<ACC>* part, int64_t count,
                                                     Acc<ACC>* tree, Acc<ACC>* tiles) {
  if (count <= 64 * 16) {
    // wavefront 0 alone; the same height as the LDS tree below
    Acc<ACC> total;
    total.zero();
    if (threadIdx.x < 64) total = combine_wave<ACC, true>(part, count);
    return total;
  }
  const int ntiles = (int)((count + COMBINE_TILE - 1) / COMBINE_TILE);
  for (int t = 0; t < ntiles; ++t) {
    const int64_t t0 = (int64_t)t * COMBINE_TILE;
    for (int i = threadIdx.x; i < COMBINE_TILE; i += blockDim.x) {
      if (t0 + i < count) fetch(part, t0 + i, tree[i]);
      else tree[i].zero();
    }
    lds_barrier();
    for (int s = COMBINE_TILE / 2; s >= 1; s >>= 1) {
      for (int i = threadIdx.x; i < s; i += blockDim.x) tree[i].merge(tree[i + s]);
      lds_barrier();
    }
    if (threadIdx.x == 0) tiles[t] = tree[0];
    lds_barrier();
  }
  Acc<ACC> total;
  total.zero();
  if (threadIdx.x == 0) {
    for (int s = 1; s < ntiles; s <<= 1)
      for (int i = 0; i + s < ntiles; i += 2 * s) tiles[i].merge(tiles[i + s]);
    if (ntiles > 0) total = tiles[0];
  }
  return total;
}

}  // namespace dev
}  // namespace nrm
