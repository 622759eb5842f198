// Row-level device code shared by the ragged batched kernels
// (nrm_batched.hip) and the serving device queue (nrm_dq.hip): the geometry
// of one contiguous segment, the element-wise map of a row, the softmax
// chains' shared-exponent helpers, and the resident rows' exchange (a
// segment held in one block's registers from its read to its write while the
// row's blocks exchange tagged partial sums). Included by each of those
// files into its own anonymous namespace.
#pragma once

#include "nrm_batch.h"
#include "nrm_device.h"

namespace nrm {
namespace {

using namespace dev;

// ---- geometry of one contiguous segment --------------------------------------

// A segment's vector body starts on a 128-byte boundary (one cache line), so
// every wavefront's 1 KiB access covers whole lines: a body that is only
// 16-byte aligned straddles a line at each end of every access, and with
// non-temporal stores those partial lines cost about a tenth of the map's
// bandwidth. The head before the boundary (at most 31 binary32 or 63 2-byte
// elements, fewer than the 64 threads of the smallest block) and the tail
// after the last whole vector are handled one element per thread.
constexpr int BODY_ALIGN = 128;

struct Geom {
  int64_t head;        // elements before the body's 128-byte boundary
  int64_t nvec;        // whole 16-byte vectors in the body
  int64_t tail_begin;  // first element after the vectors
};

template <int DT>
__device__ __forceinline__ Geom geometry(const char* p, int64_t n) {
  constexpr int SI = Elem<DT>::SIZE, VEC = Elem<DT>::VEC;
  Geom g;
  const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(p) & (BODY_ALIGN - 1));
  g.head = mis ? (BODY_ALIGN - mis) / SI : 0;
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

// ---- the element-wise map of a row ---------------------------------------------------

// normalize: x / S with the row's sum, a correctly rounded binary32 division.
// softmax: exp2(x log2(e) - k) times 1/s (the correctly rounded reciprocal of
// the row's scaled sum, formed once per block) with the row's exponent k; the
// exponent argument is one fused multiply-add (one rounding), the same
// expression as in the softmax chains' terms.
template <int ACC>
struct RowMap {
  float S;
  __device__ __forceinline__ static RowMap of(const Acc<ACC>& acc) { return RowMap{acc.value()}; }
  __device__ __forceinline__ static RowMap of(const RowRes& r) { return RowMap{r.a}; }
  __device__ __forceinline__ RowRes result() const { return RowRes{S, 0.0f}; }
  __device__ __forceinline__ float operator()(float x) const { return x / S; }
};

template <>
struct RowMap<ACC_SOFTMAX> {
  float k, s, rs;
  __device__ __forceinline__ static RowMap make(float k, float s) { return RowMap{k, s, 1.0f / s}; }
  __device__ __forceinline__ static RowMap of(const Acc<ACC_SOFTMAX>& acc) { return make(acc.k, acc.s); }
  __device__ __forceinline__ static RowMap of(const RowRes& r) { return make(r.a, r.b); }
  __device__ __forceinline__ RowRes result() const { return RowRes{k, s}; }
  __device__ __forceinline__ float operator()(float x) const {
    return __builtin_amdgcn_exp2f(__builtin_fmaf(x, LOG2E_F, -k)) * rs;
  }
  // log of the row's sum of exponentials: (k + log2 s) ln 2
  __device__ __forceinline__ float lse() const { return (k + __builtin_amdgcn_logf(s)) * LN2_F; }
};

// Softmax chains of one thread that share one exponent k (every chain's k is
// the same): raised once per loop iteration to cover the iteration's largest
// element, the chains' sums rescaled exactly, so that each element then costs
// one fused multiply-add, one exp2 and one addition instead of a compare and
// a branch of its own.
template <int NA>
__device__ __forceinline__ void raise_shared(Acc<ACC_SOFTMAX> (&acc)[NA], float m) {
  const float y = m * LOG2E_F;
  if (y > acc[0].k) {
    const float kn = __builtin_ceilf(y), d = acc[0].k - kn;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      acc[j].s = scale_pow2(acc[j].s, d);
      acc[j].k = kn;
    }
  }
}

// A thread's held vectors r[k] (those with first + k * stride < nvec) into
// softmax chains that share one exponent: one maximum over all of them, one
// raise (raise_shared), then per element a fused multiply-add, an exp2 and an
// addition.
template <int DTI, int NA, int KB>
__device__ __forceinline__ void softmax_add_held(Acc<ACC_SOFTMAX> (&acc)[NA], const u4 (&r)[KB], int64_t first,
                                                 int64_t stride, int64_t nvec) {
  constexpr int VEC = Elem<DTI>::VEC;
  float m = -3.0e38f;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    if (first + (int64_t)k * stride < nvec) {
      float x[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int c = 0; c < VEC; ++c) m = fmaxf(m, x[c]);
    }
  }
  raise_shared<NA>(acc, m);
  const float nk = -acc[0].k;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    if (first + (int64_t)k * stride < nvec) {
      float x[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[(k * VEC + c) % NA].s += __builtin_amdgcn_exp2f(__builtin_fmaf(x[c], LOG2E_F, nk));
    }
  }
}

// ---- resident rows -------------------------------------------------------------------------
// A row of at most RES_MAX_SEGMENTS segments of 2^RES_LOG2 elements crosses
// HBM twice instead of three times: each segment is one work item, held in
// one block's registers from its read to its write. The blocks of a row
// publish their segment sums, each waits until it sees all of them, merges
// them in a fixed order (the same in every block of the row, so that every
// block divides by the same bits) and divides its segment from registers.
//
// Progress: blocks take items from a counter (CNT_DISPENSE) in item order, a
// row's items are consecutive, a block takes an item only once it has
// finished the previous one, and it publishes its sum before it waits. Every row
// before the one holding the last item taken therefore has all its items in
// running blocks, each of which publishes: their waits end. Only that last
// row can wait on items not yet taken, and at most RES_MAX_SEGMENTS - 1 of
// its blocks wait while the others take its remaining items. The wait is
// still bounded: after RES_SPIN_LIMIT polls a block flags NRM_DEVERR_STALL
// and goes on, and every wait of the call gives up once that flag is set,
// so the kernel always ends.
//
// A partial travels as tagged 64-bit words (this call's number in the high
// half, a binary32 in the low half; two words for the two-float kinds),
// written and read with agent-scope atomics, which are coherent across the
// XCDs' L2 caches. A word is valid when its tag is this call's number: no
// slot is cleared between calls and no fence orders one word after another.
constexpr uint32_t RES_SPIN_LIMIT = 1u << 18;

template <int ACC>
struct Tagged {
  static constexpr int WORDS = ACC == NRM_ACC_F32 ? 1 : 2;
  __device__ __forceinline__ static void split(const Acc<ACC>& v, float (&f)[2]) {
    if constexpr (ACC == NRM_ACC_F32) {
      f[0] = v.s;
      f[1] = 0.0f;
    } else if constexpr (ACC == NRM_ACC_KAHAN) {
      f[0] = v.hi;
      f[1] = v.lo;
    } else {
      f[0] = v.k;
      f[1] = v.s;
    }
  }
  __device__ __forceinline__ static Acc<ACC> join(const float (&f)[2]) {
    Acc<ACC> v;
    if constexpr (ACC == NRM_ACC_F32) {
      v.s = f[0];
    } else if constexpr (ACC == NRM_ACC_KAHAN) {
      v.hi = f[0];
      v.lo = f[1];
    } else {
      v.k = f[0];
      v.s = f[1];
    }
    return v;
  }
};

// Where one row's segments meet: segment s's tagged words at slots[2 s] and
// slots[2 s + 1]; the count of segments that have published (0 between
// calls); the row's merged total, two tagged words. The last segment to
// arrive merges all partials and publishes the total; the others wait for
// that one word, so a row's blocks poll one location each instead of every
// block polling every partial.
struct ResExchange {
  unsigned long long* slots;
  unsigned long long* total;
  unsigned* arrivals;
  uint32_t ep;                // this call's number
  int* error;                 // device error word (NRM_DEVERR_STALL)
  unsigned long long* stall;  // the number of the last call in which a wait gave up
  unsigned long long* call;   // when set: the call counter the last arrival moves on
};

template <int ACC>
__device__ __forceinline__ void publish_tagged(unsigned long long* words, uint32_t ep, const Acc<ACC>& v) {
  float f[2];
  Tagged<ACC>::split(v, f);
#pragma unroll
  for (int w = 0; w < Tagged<ACC>::WORDS; ++w)
    __hip_atomic_store(words + w, ((unsigned long long)ep << 32) | bits_f32(f[w]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// A bounded wait has run out: flag it for the host and for this call's other
// waits.
__device__ __forceinline__ void give_up(const ResExchange& x) {
  atomicOr(x.error, NRM_DEVERR_STALL);
  __hip_atomic_store(x.stall, (unsigned long long)x.ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool given_up(const ResExchange& x, uint32_t spin) {
  return (spin & 255) == 255 && __hip_atomic_load(x.stall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == x.ep;
}

// One thread: wait for the row's total (bounded), and return it.
template <int ACC>
__device__ __forceinline__ Acc<ACC> wait_total(const ResExchange& x) {
  float f[2] = {0.0f, 0.0f};
  for (uint32_t spin = 0;; ++spin) {
    bool ok = true;
#pragma unroll
    for (int w = 0; w < Tagged<ACC>::WORDS; ++w) {
      const unsigned long long v = __hip_atomic_load(x.total + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      f[w] = f32_bits((uint32_t)v);
      ok = ok && (uint32_t)(v >> 32) == x.ep;
    }
    if (ok) break;
    if (spin >= RES_SPIN_LIMIT) {
      give_up(x);
      break;
    }
    if (given_up(x, spin)) break;
    __builtin_amdgcn_s_sleep(1);
  }
  return Tagged<ACC>::join(f);
}

// Wavefront 0 (all 64 lanes) of the last block to arrive: read the row's
// nseg <= 64 * PER_LANE partials (each has been published; a word not yet
// visible is read again), lane l taking segments l, l + 64, ..., then merge
// them: each lane its own pairwise, then the wavefront tree. Every lane
// returns the row's total; the order depends only on nseg.
template <int ACC, int PER_LANE>
__device__ __forceinline__ Acc<ACC> gather_row(const ResExchange& x, int nseg) {
  const int lane = threadIdx.x & 63;
  float f[PER_LANE][2];
  bool have[PER_LANE];
#pragma unroll
  for (int j = 0; j < PER_LANE; ++j) {
    f[j][0] = f[j][1] = 0.0f;
    have[j] = lane + 64 * j >= nseg;
  }
  for (uint32_t spin = 0;; ++spin) {
    bool all = true;
#pragma unroll
    for (int j = 0; j < PER_LANE; ++j) {
      if (!have[j]) {
        bool ok = true;
#pragma unroll
        for (int w = 0; w < Tagged<ACC>::WORDS; ++w) {
          const unsigned long long v = __hip_atomic_load(x.slots + 2 * (lane + 64 * j) + w, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
          f[j][w] = f32_bits((uint32_t)v);
          ok = ok && (uint32_t)(v >> 32) == x.ep;
        }
        have[j] = ok;
      }
      all = all && have[j];
    }
    if (__all(all)) break;
    if (spin >= RES_SPIN_LIMIT) {
      if (lane == 0) give_up(x);
      break;
    }
    if (given_up(x, spin)) break;  // another wait of this call already gave up
    __builtin_amdgcn_s_sleep(1);
  }
  Acc<ACC> v[PER_LANE];
#pragma unroll
  for (int j = 0; j < PER_LANE; ++j) {
    if (lane + 64 * j < nseg && have[j]) v[j] = Tagged<ACC>::join(f[j]);
    else v[j].zero();
  }
#pragma unroll
  for (int st = 1; st < PER_LANE; st <<= 1)
#pragma unroll
    for (int j = 0; j + st < PER_LANE; j += 2 * st) v[j].merge(v[j + st]);
  return wave_reduce<ACC>(v[0]);
}

// One resident segment of 2^LOG2 elements held by a BLOCK-thread block:
// read into registers, block sum, exchange with the row's other segments,
// divide from the registers, write. The row's result (RowMap) is left in
// *s_bcast; lse, when given, receives the softmax row's log-sum-exp (from
// segment 0).
//
// DIRECT: every block of the row reads all partials itself (one round trip:
// the lowest latency for a single row of few segments) instead of waiting for
// the last arrival's total (fewer polls: the better throughput for a batch);
// the arrival count then only finds the last block, which moves the call
// number on.
template <int DTI, int DTO, int ACC, int BLOCK, int LOG2, int PER_LANE, bool DIRECT = false>
__device__ __forceinline__ void resident_unit(const RowDesc& d, int seg, const ResExchange& x, Acc<ACC>* slots,
                                              RowRes* s_bcast, float* lse_row) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int KB = (1 << LOG2) / (BLOCK * VEC);
  static_assert(KB >= 1 && KB * BLOCK * VEC == (1 << LOG2), "a segment is whole vectors per thread");
  // chains per thread: 8 binary32, 4 of the two-float kinds (registers)
  constexpr int NA_MAX = ACC == NRM_ACC_F32 ? 8 : 4;
  constexpr int NA = KB * VEC < NA_MAX ? KB * VEC : NA_MAX;
  const int t = threadIdx.x;
  const int64_t S = int64_t(1) << LOG2;
  const int64_t b = (int64_t)seg << LOG2;
  const int64_t n = d.n - b < S ? d.n - b : S;
  const int nseg = (int)((d.n + S - 1) >> LOG2);
  const char* in_seg = d.in + b * Elem<DTI>::SIZE;
  char* out_seg = d.out + b * Elem<DTO>::SIZE;
  const Geom g = geometry<DTI>(in_seg, n);
  const u4* body = reinterpret_cast<const u4*>(in_seg + g.head * Elem<DTI>::SIZE);
  const bool has_head = t < g.head;
  const int64_t ti = g.tail_begin + t;
  const bool has_tail = ti < n;
  u4 r[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int64_t v = t + (int64_t)k * BLOCK;
    if (v < g.nvec) r[k] = load_vec<true>(body + v);
  }
  const float xh = has_head ? load_one<DTI>(in_seg, t) : 0.0f;
  const float xt = has_tail ? load_one<DTI>(in_seg, ti) : 0.0f;
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  if constexpr (ACC == ACC_SOFTMAX) {
    softmax_add_held<DTI, NA, KB>(acc, r, t, BLOCK, g.nvec);
  } else {
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      if (t + (int64_t)k * BLOCK < g.nvec) {
        float xv[VEC];
        widen<DTI>(r[k], xv);
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[(k * VEC + c) % NA].add(xv[c]);
      }
    }
  }
  if (has_head) acc[0].add(xh);
  if (has_tail) acc[0].add(xt);
  merge_chains<ACC, NA>(acc);
  const Acc<ACC> tot = block_reduce<ACC>(acc[0], slots);
  if (nseg == 1) {
    if (t == 0) {
      const RowMap<ACC> f0 = RowMap<ACC>::of(tot);
      *s_bcast = f0.result();
      if constexpr (ACC == ACC_SOFTMAX) {
        if (lse_row) *lse_row = f0.lse();
      }
    }
  } else if (DIRECT && t < 64) {
    if (t == 0) publish_tagged<ACC>(x.slots + 2 * seg, x.ep, tot);
    const Acc<ACC> total = gather_row<ACC, PER_LANE>(x, nseg);
    if (t == 0) {
      const RowMap<ACC> f0 = RowMap<ACC>::of(total);
      *s_bcast = f0.result();
      if constexpr (ACC == ACC_SOFTMAX) {
        if (lse_row && seg == 0) *lse_row = f0.lse();
      }
      // after this block's reads of the tags: the last one moves the call on
      if (__hip_atomic_fetch_add(x.arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)nseg - 1) {
        __hip_atomic_store(x.arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (x.call) __hip_atomic_fetch_add(x.call, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  } else if (t < 64) {
    unsigned prev = 0;
    if (t == 0) {
      publish_tagged<ACC>(x.slots + 2 * seg, x.ep, tot);
      prev = __hip_atomic_fetch_add(x.arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = (unsigned)__builtin_amdgcn_readfirstlane((int)prev);
    Acc<ACC> total;
    if (prev == (unsigned)nseg - 1) {
      // the last to arrive: every segment has published; the count goes back
      // to 0 for the next call, and the merged total is published once
      if (t == 0) __hip_atomic_store(x.arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      total = gather_row<ACC, PER_LANE>(x, nseg);
      if (t == 0) {
        publish_tagged<ACC>(x.total, x.ep, total);
        if (x.call) __hip_atomic_fetch_add(x.call, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else if (t == 0) {
      total = wait_total<ACC>(x);
    }
    if (t == 0) {
      const RowMap<ACC> f0 = RowMap<ACC>::of(total);
      *s_bcast = f0.result();
      if constexpr (ACC == ACC_SOFTMAX) {
        if (lse_row && seg == 0) *lse_row = f0.lse();
      }
    }
  }
  lds_barrier();
  const RowMap<ACC> f = RowMap<ACC>::of(*s_bcast);
  const bool vec_ok = out_vector_ok<DTI, DTO>(out_seg, g.head);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int64_t v = t + (int64_t)k * BLOCK;
    if (v < g.nvec) {
      float xv[VEC], q[VEC];
      widen<DTI>(r[k], xv);
#pragma unroll
      for (int c = 0; c < VEC; ++c) q[c] = f(xv[c]);
      store_quotients<DTI, DTO>(out_seg, g.head, v, vec_ok, q);
    }
  }
  if (has_head) store_one<DTO>(out_seg, t, f(xh));
  if (has_tail) store_one<DTO>(out_seg, ti, f(xt));
}

template <int ACC>
__device__ __forceinline__ void dispatch_resident(const RowDesc& d, int seg, const ResExchange& x, Acc<ACC>* slots,
                                                  RowRes* s_bcast, float* lse_row) {
  if constexpr (ACC == ACC_SOFTMAX) {
    resident_unit<NRM_F32, NRM_F32, ACC, RES_BLOCK, RES_LOG2, 1>(d, seg, x, slots, s_bcast, lse_row);
  } else {
#define NRM_RU(I, O) return resident_unit<I, O, ACC, RES_BLOCK, RES_LOG2, 1>(d, seg, x, slots, s_bcast, lse_row)
    switch (d.in_dt * 3 + d.out_dt) {
      case NRM_F32 * 3 + NRM_F32: NRM_RU(NRM_F32, NRM_F32);
      case NRM_F32 * 3 + NRM_BF16: NRM_RU(NRM_F32, NRM_BF16);
      case NRM_F32 * 3 + NRM_F16: NRM_RU(NRM_F32, NRM_F16);
      case NRM_BF16 * 3 + NRM_F32: NRM_RU(NRM_BF16, NRM_F32);
      case NRM_BF16 * 3 + NRM_BF16: NRM_RU(NRM_BF16, NRM_BF16);
      case NRM_BF16 * 3 + NRM_F16: NRM_RU(NRM_BF16, NRM_F16);
      case NRM_F16 * 3 + NRM_F32: NRM_RU(NRM_F16, NRM_F32);
      case NRM_F16 * 3 + NRM_BF16: NRM_RU(NRM_F16, NRM_BF16);
      default: NRM_RU(NRM_F16, NRM_F16);
    }
#undef NRM_RU
  }
}

}  // namespace
}  // namespace nrm
