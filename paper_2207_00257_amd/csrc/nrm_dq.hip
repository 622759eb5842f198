// The serving device queue's persistent kernel (the protocol and the shared
// layouts are described in nrm_dq.h; the server's executor is in
// nrm_server.cpp). A request of up to 2^20 elements runs as resident
// segments with the batched path's exchange (nrm_rows.h); a longer one, when
// the server keeps it in the kernel, as parts summed, merged and divided.
#include <stddef.h>

#include "nrm_batch.h"
#include "nrm_device.h"
#include "nrm_dq.h"
#include "nrm_rows.h"

namespace nrm {
namespace {

using namespace dev;

// ---- device queue: the server's persistent kernel -----------------------------------------
// The protocol is described in nrm_dq.h. Wavefront 0 of a block takes a
// ticket (the next unit number) and waits until the unit is published; the
// block holding the ticket equal to the published count is the one that
// polls the host (at most one block reads host memory at a time) and copies
// new requests into the device ring. Progress follows the resident rows'
// argument: units are taken in order and a request's units are consecutive,
// a block takes a ticket only after finishing its previous unit, and it
// publishes before it waits; a long request's dividing units wait only on
// its summing units, all of which were taken before them. Every wait is
// bounded: the exchange waits by RES_SPIN_LIMIT polls, the poller by the idle
// limit, the launch's slice or the host's stop word, and a waiting block by
// the exit word the poller sets when it ends, or by four idle limits of its
// own.

// Blocks whose ticket is more than this many units past the published count
// poll it at the slowest rate.
constexpr unsigned long long DQ_NEAR = 16;

struct DqClaim {
  RowDesc d;
  long long part;  // the unit's index within its request
  unsigned long long seq;
  int units;
  int slot;
  int exit;
  int pad;
};

__device__ __forceinline__ unsigned long long dq_now() { return (unsigned long long)wall_clock64(); }

__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_sys(const uint64_t* p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// What a block remembers between its claims (in LDS, written by lane 0 of
// wavefront 0): the largest published unit count it has seen, and the
// request of its last unit. Unit numbers are never reused, so a unit inside
// the remembered request's range belongs to it, and that request cannot have
// completed while one of its units is still to run.
struct DqCache {
  unsigned long long pub;
  unsigned long long first, units;
  unsigned long long w[7];  // the request's ring entry: in, out, n, dtypes, key, seq, slot
  int slot;
  int pad;
};

// The poller (wavefront 0 of the block holding the ticket equal to the
// published unit count): read the next DQ_BATCH lines of the publish ring and
// the host's stop word in one round trip (lane 4 i + k: word k of request
// pub_reqs + i; lane 4 DQ_BATCH: the stop word), take the leading requests
// whose four words all carry their tag, copy them into the device ring with
// their unit numbers, then publish the new unit count. The first of them
// holds the poller's own unit: it goes into the block's cache, which spares
// the lookup. Returns whether there were any; *stop receives the stop word.
constexpr int DQ_BATCH = 15;
static_assert(4 * DQ_BATCH < 64, "one wavefront reads the lines and the stop word");

__device__ __forceinline__ bool dq_copy_new(const DqArgs& a, unsigned long long* stop, DqCache* m) {
  DqDev* q = a.dev;
  const DqHost* h = a.host;
  const int lane = threadIdx.x;
  const int i = lane >> 2, k = lane & 3;
  unsigned long long done = lane == 0 ? ld_agent(&q->pub_reqs) : 0;
  done = uniform_u64(done);
  unsigned long long word = 0;
  if (i < DQ_BATCH) word = ld_sys(&h->pub[(done + i) % DQ_PUB].w[k]);
  else if (lane == 4 * DQ_BATCH) word = ld_sys(&h->stop);
  *stop = uniform_u64((unsigned long long)__builtin_amdgcn_readlane((int)(uint32_t)word, 4 * DQ_BATCH));
  const bool ok = i < DQ_BATCH && (word >> DQ_TAG_SHIFT) == dq_pub_tag(done + i);
  // requests are taken in order: stop at the first with a word missing
  const unsigned long long bad = __ballot(i < DQ_BATCH && !ok) | (~0ull << (4 * DQ_BATCH));
  const int cnt = __builtin_ctzll(bad) / 4;
  if (cnt == 0) return false;
  const unsigned long long low = word & ((1ull << DQ_TAG_SHIFT) - 1);
  // n is word 2 of each request: every lane of request i learns its n and
  // the units of the requests before it
  unsigned long long first = uniform_u64(ld_agent(&q->pub_units)), my_first = 0, my_units = 0;
  for (int j = 0; j < cnt; ++j) {
    const int64_t nj = (int64_t)uniform_u64(
        ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(low >> 32), 4 * j + 2) << 32) |
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)low, 4 * j + 2));
    const unsigned long long uj = (unsigned long long)dq_units(nj);
    if (i == j) {
      my_first = first;
      my_units = uj;
    }
    first += uj;
  }
  if (i < cnt) {
    // word 3: in_dtype | out_dtype << 8 | slot << 16
    const unsigned long long w3 = (unsigned long long)(uint32_t)__shfl((int)(uint32_t)low, 4 * i + 3);
    const int slot = (int)((w3 >> 16) & (DQ_RING - 1));
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(&q->ring[slot]);
    if (k < 3) {
      st_agent(dst + k, low);  // in, out, n
    } else {
      st_agent(dst + 3, (w3 & 0xFF) | ((w3 >> 8) & 0xFF) << 32);  // in_dt, out_dt
      const unsigned long long key = (my_first << DQ_KEY_UNIT_BITS) | my_units;
      st_agent(dst + offsetof(DqReq, key) / 8, key);
      st_agent(dst + offsetof(DqReq, seq) / 8, done + i);
      st_agent(dst + offsetof(DqReq, slot) / 8, (unsigned long long)slot);
      st_agent(&q->key[slot], key);
      // the slot's previous request has completed: its counters start from 0
      // (they are 0 already unless one of its waits gave up)
      __hip_atomic_store(&q->arrivals[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&q->finished[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  // request 0's entry, as the lanes of request 0 wrote it to the ring
  const unsigned long long w0 = uniform_u64(((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(low >> 32), 0) << 32) |
                                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)low, 0));
  const unsigned long long w1 = uniform_u64(((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(low >> 32), 1) << 32) |
                                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)low, 1));
  const unsigned long long w2 = uniform_u64(((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(low >> 32), 2) << 32) |
                                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)low, 2));
  const unsigned long long w3 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)low, 3);
  const unsigned long long first0 = uniform_u64(ld_agent(&q->pub_units));
  const unsigned long long units0 = (unsigned long long)dq_units((int64_t)w2);
  // the copies before the counts: a block that sees the new unit count finds
  // its request in the ring
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (lane == 0) {
    m->w[0] = w0;
    m->w[1] = w1;
    m->w[2] = w2;
    m->w[3] = (w3 & 0xFF) | ((w3 >> 8) & 0xFF) << 32;
    m->w[offsetof(DqReq, key) / 8] = (first0 << DQ_KEY_UNIT_BITS) | units0;
    m->w[offsetof(DqReq, seq) / 8] = done;
    m->w[offsetof(DqReq, slot) / 8] = (w3 >> 16) & (DQ_RING - 1);
    m->first = first0;
    m->units = units0;
    m->slot = (int)((w3 >> 16) & (DQ_RING - 1));
    st_agent(&q->pub_reqs, done + cnt);
    st_agent(&q->last_seen, dq_now());
    __hip_atomic_store(&q->pub_units, first, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  return true;
}

// Wavefront 0: take the next ticket, wait until its unit is published (or
// the kernel ends), and find the unit's request. Fills *c (c->exit when the
// block is to end).
__device__ __forceinline__ void dq_claim(const DqArgs& a, DqClaim* c, DqCache* m) {
  DqDev* q = a.dev;
  const int lane = threadIdx.x;
  unsigned long long u = 0;
  if (lane == 0) u = __hip_atomic_fetch_add(&q->next_unit, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  u = uniform_u64(u);
  if (u >= uniform_u64(m->pub)) {
    const unsigned long long t_start = dq_now();
    for (uint32_t spin = 0;; ++spin) {
      unsigned long long pub = lane == 0 ? ld_agent(&q->pub_units) : 0;
      pub = uniform_u64(pub);
      if (u < pub) {
        if (lane == 0) m->pub = pub;
        break;
      }
      bool end = false;
      if (u == pub) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the previous poller's counts
        unsigned long long stop = 0;
        if (dq_copy_new(a, &stop, m)) continue;
        unsigned long long last = 0, ex = 0, born = 0;
        if (lane == 0) {
          last = ld_agent(&q->last_seen);
          ex = ld_agent(&q->exit_epoch);
          born = ld_agent(&q->launched_at);
        }
        last = uniform_u64(last);
        ex = uniform_u64(ex);
        born = uniform_u64(born);
        const unsigned long long now = dq_now();
        // idle for idle_ticks, or this launch has run its slice (so that a
        // kernel queued behind it on its hardware queue waits at most that
        // long; the host starts the next launch)
        end = stop != 0 || ex == a.epoch || (now > last && now - last > a.idle_ticks) ||
              (a.slice_ticks != 0 && now > born && now - born > a.slice_ticks);
        if (!end) __builtin_amdgcn_s_sleep(2);
      } else if ((spin & 7) == 7) {
        unsigned long long ex = lane == 0 ? ld_agent(&q->exit_epoch) : 0;
        ex = uniform_u64(ex);
        const unsigned long long now = dq_now();
        end = ex == a.epoch || now - t_start > 4 * a.idle_ticks;
      } else if (u - pub > DQ_NEAR) {
        // far from the published count: poll rarely, so that hundreds of idle
        // blocks do not load one word hundreds of millions of times a second
        // (that channel then slows every transfer striped across it)
        __builtin_amdgcn_s_sleep(127);
      } else {
        __builtin_amdgcn_s_sleep(16);
      }
      if (end) {
        if (lane == 0) {
          st_agent(&q->exit_epoch, a.epoch);
          c->exit = 1;
        }
        return;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the ring entries copied before the unit count
  }
  const unsigned long long mfirst = uniform_u64(m->first), munits = uniform_u64(m->units);
  if (!(munits > 0 && mfirst <= u && u < mfirst + munits)) {
    // lane s looks at slot s: the published request whose units hold u (the
    // ranges of different requests never overlap; a request's entry stays
    // until the request has completed, and u is one of its units)
    // (every lane reads its slot's whole entry in the same round trip; a slot
    // being rewritten for a newer request cannot match u, whose request was
    // copied before the unit count this block has seen)
    bool found = false;
    for (uint32_t spin = 0; spin < RES_SPIN_LIMIT; ++spin) {
      const unsigned long long* e = reinterpret_cast<const unsigned long long*>(&q->ring[lane]);
      unsigned long long w[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) w[k] = ld_agent(e + k);
      const unsigned long long key = w[offsetof(DqReq, key) / 8];
      const unsigned long long first = key >> DQ_KEY_UNIT_BITS, units = key & ((1ull << DQ_KEY_UNIT_BITS) - 1);
      const bool mine = units > 0 && first <= u && u < first + units;
      const unsigned long long hit = __ballot(mine);
      if (hit) {
        const int src = __builtin_ctzll(hit);
        if (lane == src) {
#pragma unroll
          for (int k = 0; k < 7; ++k) m->w[k] = w[k];
          m->first = first;
          m->units = units;
          m->slot = src;
        }
        found = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!found) {
      // cannot happen while the host keeps its side of the protocol; skip the unit
      if (lane == 0) {
        atomicOr(&q->error, NRM_DEVERR_ROW);
        c->d.n = 0;
        c->units = 0;
        c->exit = 0;
      }
      return;
    }
  }
  if (lane == 0) {
    // the entry's words: in, out, n, dtypes, key, seq, slot
    c->d.in = reinterpret_cast<const char*>(m->w[0]);
    c->d.out = reinterpret_cast<char*>(m->w[1]);
    c->d.n = (int64_t)m->w[2];
    c->d.in_dt = (int32_t)(uint32_t)m->w[3];
    c->d.out_dt = (int32_t)(uint32_t)(m->w[3] >> 32);
    c->part = (long long)(u - m->first);
    c->seq = m->w[5];
    c->units = (int)m->units;
    c->slot = m->slot;
    c->exit = 0;
  }
}

// Sum of part `part` (2^DQ_LONG_LOG2 elements) of a long request: temporal
// loads, so that the request's dividing units find it in the last-level cache.
// The result is valid in thread 0.
template <int DTI, int ACC>
__device__ __forceinline__ Acc<ACC> dq_part_sum(const RowDesc& d, int64_t part, Acc<ACC>* slots) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int KB = (1 << RES_LOG2) / (RES_BLOCK * VEC);
  constexpr int CH = 1 << (DQ_LONG_LOG2 - RES_LOG2);
  constexpr int NA = ACC == NRM_ACC_F32 ? 8 : 4;
  const int t = threadIdx.x;
  const int64_t b = part << DQ_LONG_LOG2;
  const int64_t n = d.n - b < (int64_t(1) << DQ_LONG_LOG2) ? d.n - b : (int64_t(1) << DQ_LONG_LOG2);
  const char* in_seg = d.in + b * Elem<DTI>::SIZE;
  const Geom g = geometry<DTI>(in_seg, n);
  const u4* body = reinterpret_cast<const u4*>(in_seg + g.head * Elem<DTI>::SIZE);
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
#pragma unroll 1
  for (int ch = 0; ch < CH; ++ch) {
    u4 r[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int64_t v = (int64_t)ch * KB * RES_BLOCK + t + (int64_t)k * RES_BLOCK;
      if (v < g.nvec) r[k] = load_vec<false>(body + v);
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int64_t v = (int64_t)ch * KB * RES_BLOCK + t + (int64_t)k * RES_BLOCK;
      if (v < g.nvec) {
        float xv[VEC];
        widen<DTI>(r[k], xv);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[(k * VEC + e) % NA].add(xv[e]);
      }
    }
  }
  if (t < g.head) acc[0].add(load_one<DTI>(in_seg, t));
  if (g.tail_begin + t < n) acc[0].add(load_one<DTI>(in_seg, g.tail_begin + t));
  merge_chains<ACC, NA>(acc);
  return block_reduce<ACC>(acc[0], slots);
}

// Divide part `part` of a long request by the request's sum S.
template <int DTI, int DTO, int ACC>
__device__ __forceinline__ void dq_part_map(const RowDesc& d, int64_t part, const RowMap<ACC>& f) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int KB = (1 << RES_LOG2) / (RES_BLOCK * VEC);
  constexpr int CH = 1 << (DQ_LONG_LOG2 - RES_LOG2);
  const int t = threadIdx.x;
  const int64_t b = part << DQ_LONG_LOG2;
  const int64_t n = d.n - b < (int64_t(1) << DQ_LONG_LOG2) ? d.n - b : (int64_t(1) << DQ_LONG_LOG2);
  const char* in_seg = d.in + b * Elem<DTI>::SIZE;
  char* out_seg = d.out + b * Elem<DTO>::SIZE;
  const Geom g = geometry<DTI>(in_seg, n);
  const u4* body = reinterpret_cast<const u4*>(in_seg + g.head * Elem<DTI>::SIZE);
  const bool vec_ok = out_vector_ok<DTI, DTO>(out_seg, g.head);
#pragma unroll 1
  for (int ch = 0; ch < CH; ++ch) {
    u4 r[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int64_t v = (int64_t)ch * KB * RES_BLOCK + t + (int64_t)k * RES_BLOCK;
      if (v < g.nvec) r[k] = load_vec<true>(body + v);
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int64_t v = (int64_t)ch * KB * RES_BLOCK + t + (int64_t)k * RES_BLOCK;
      if (v < g.nvec) {
        float xv[VEC], qv[VEC];
        widen<DTI>(r[k], xv);
#pragma unroll
        for (int e = 0; e < VEC; ++e) qv[e] = f(xv[e]);
        store_quotients<DTI, DTO>(out_seg, g.head, v, vec_ok, qv);
      }
    }
  }
  if (t < g.head) store_one<DTO>(out_seg, t, f(load_one<DTI>(in_seg, t)));
  if (g.tail_begin + t < n) store_one<DTO>(out_seg, g.tail_begin + t, f(load_one<DTI>(in_seg, g.tail_begin + t)));
}

// One unit of a long request: a summing unit (part < m) publishes its part's
// sum, and the last of the request's parts to arrive merges all m in a fixed
// order and publishes the total; a dividing unit (part >= m) waits for the
// total and divides its part. Returns whether the unit wrote outputs.
// Wavefront 0 of the last part to arrive: the request's m <= DQ_MAX_PARTS
// part sums, lane l taking parts l, l + 64, ..., requested four slices of 64
// at a time; a slice with a word not yet visible is read again (bounded, as
// every wait here). Then each lane's pairwise merge and the wavefront tree:
// the same order as gather_row. Not inlined: it runs once per long request,
// and inlined its registers would crowd the resident units' (the kernel
// spilled).
template <int ACC>
__device__ __noinline__ Acc<ACC> gather_parts(ResExchange x, int m) {
  constexpr int PER = DQ_MAX_PARTS / 64;
  constexpr int G = 4;  // slices requested at once
  constexpr int W = Tagged<ACC>::WORDS;
  const int lane = threadIdx.x & 63;
  Acc<ACC> v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) v[j].zero();
#pragma unroll
  for (int j0 = 0; j0 < PER; j0 += G) {
    if (64 * j0 >= m) break;
    unsigned long long w[G][W];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int s = lane + 64 * (j0 + g);
#pragma unroll
      for (int k = 0; k < W; ++k)
        w[g][k] = s < m ? __hip_atomic_load(x.slots + 2 * s + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int s = lane + 64 * (j0 + g);
      bool ok = true;
#pragma unroll
      for (int k = 0; k < W; ++k) ok = ok && (s >= m || (uint32_t)(w[g][k] >> 32) == x.ep);
      for (uint32_t spin = 0; !__all(ok); ++spin) {
        if (spin >= RES_SPIN_LIMIT) {
          if (lane == 0) give_up(x);
          break;
        }
        if (given_up(x, spin)) break;
        __builtin_amdgcn_s_sleep(1);
        if (!ok) {
          ok = true;
#pragma unroll
          for (int k = 0; k < W; ++k) {
            w[g][k] = __hip_atomic_load(x.slots + 2 * s + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = ok && (uint32_t)(w[g][k] >> 32) == x.ep;
          }
        }
      }
      if (s < m && ok) {
        float f[2] = {f32_bits((uint32_t)w[g][0]), W > 1 ? f32_bits((uint32_t)w[g][W - 1]) : 0.0f};
        v[j0 + g] = Tagged<ACC>::join(f);
      }
    }
  }
#pragma unroll
  for (int st = 1; st < PER; st <<= 1)
#pragma unroll
    for (int j = 0; j + st < PER; j += 2 * st) v[j].merge(v[j + st]);
  return wave_reduce<ACC>(v[0]);
}

template <int ACC>
__device__ __forceinline__ Acc<ACC> dispatch_part_sum(const RowDesc& d, int64_t part, Acc<ACC>* slots) {
  if (d.in_dt == NRM_F32) return dq_part_sum<NRM_F32, ACC>(d, part, slots);
  if (d.in_dt == NRM_BF16) return dq_part_sum<NRM_BF16, ACC>(d, part, slots);
  return dq_part_sum<NRM_F16, ACC>(d, part, slots);
}

template <int ACC>
__device__ __forceinline__ void dispatch_part_map(const RowDesc& d, int64_t part, const RowMap<ACC>& f) {
#define NRM_DM(I, O) return dq_part_map<I, O, ACC>(d, part, f)
  switch (d.in_dt * 3 + d.out_dt) {
    case NRM_F32 * 3 + NRM_F32: NRM_DM(NRM_F32, NRM_F32);
    case NRM_F32 * 3 + NRM_BF16: NRM_DM(NRM_F32, NRM_BF16);
    case NRM_F32 * 3 + NRM_F16: NRM_DM(NRM_F32, NRM_F16);
    case NRM_BF16 * 3 + NRM_F32: NRM_DM(NRM_BF16, NRM_F32);
    case NRM_BF16 * 3 + NRM_BF16: NRM_DM(NRM_BF16, NRM_BF16);
    case NRM_BF16 * 3 + NRM_F16: NRM_DM(NRM_BF16, NRM_F16);
    case NRM_F16 * 3 + NRM_F32: NRM_DM(NRM_F16, NRM_F32);
    case NRM_F16 * 3 + NRM_BF16: NRM_DM(NRM_F16, NRM_BF16);
    default: NRM_DM(NRM_F16, NRM_F16);
  }
#undef NRM_DM
}

// One unit of a long request: a summing unit (part < m) publishes its part's
// sum, and the last of the request's parts to arrive merges all m in a fixed
// order and publishes the total; a dividing unit (part >= m) waits for the
// total and divides its part. Only the loops depend on the dtypes; the
// exchange is shared by all of them. Returns whether the unit wrote outputs.
template <int ACC>
__device__ __forceinline__ bool dq_long_unit(const RowDesc& d, int64_t part, int m, const ResExchange& x,
                                             Acc<ACC>* slots, RowRes* s_bcast) {
  const int t = threadIdx.x;
  if (part < m) {
    const Acc<ACC> tot = dispatch_part_sum<ACC>(d, part, slots);
    if (t < 64) {
      unsigned prev = 0;
      if (t == 0) {
        publish_tagged<ACC>(x.slots + 2 * part, x.ep, tot);
        prev = __hip_atomic_fetch_add(x.arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      prev = (unsigned)__builtin_amdgcn_readfirstlane((int)prev);
      if (prev == (unsigned)m - 1) {
        if (t == 0) __hip_atomic_store(x.arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const Acc<ACC> total = gather_parts<ACC>(x, m);
        if (t == 0) publish_tagged<ACC>(x.total, x.ep, total);
      }
    }
    return false;
  }
  if (t == 0) *s_bcast = RowMap<ACC>::of(wait_total<ACC>(x)).result();
  lds_barrier();
  dispatch_part_map<ACC>(d, part - m, RowMap<ACC>::of(*s_bcast));
  return true;
}

// After a unit that wrote outputs: make its stores visible beyond the XCD's
// L2 (to the host, DMA engines and later kernels), count it, and let the
// request's last such unit write the completion word into host memory.
__device__ __forceinline__ void dq_finish(const DqArgs& a, const DqClaim& c, unsigned target) {
  // every wavefront waits for its own stores to reach the L2 before the
  // barrier (the barrier's workgroup-scope release does not wait for global
  // stores), so that thread 0's write-back below covers the whole unit
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    DqDev* q = a.dev;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    // a one-unit request needs no count: its unit is the last
    const unsigned prev =
        target == 1 ? 0u : __hip_atomic_fetch_add(&q->finished[c.slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == target - 1) {
      if (target > 1) __hip_atomic_store(&q->finished[c.slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
      const unsigned long long tag = dq_tag(c.seq);
      DqHost* h = a.host;
      if (ld_agent(&q->stall) == tag)
        __hip_atomic_store(reinterpret_cast<unsigned long long*>(&h->stalled[c.slot]), tag, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(reinterpret_cast<unsigned long long*>(&h->done[c.slot]), tag, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

template <int ACC>
__global__ void __launch_bounds__(RES_BLOCK) __attribute__((amdgpu_waves_per_eu(4, 4))) dq_kernel(DqArgs a) {
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ RowRes s_bcast;
  __shared__ DqClaim s_c;
  __shared__ DqCache s_cache;
  DqDev* q = a.dev;
  if (threadIdx.x == 0) {
    s_cache.pub = 0;
    s_cache.units = 0;
  }
  for (;;) {
    if (threadIdx.x < 64) dq_claim(a, &s_c, &s_cache);
    lds_barrier();
    // the same in every thread: scalar registers, so that the branches on the
    // unit's kind are uniform and their bodies do not share registers
    DqClaim c;
    c.d.in = reinterpret_cast<const char*>(uniform_u64(reinterpret_cast<unsigned long long>(s_c.d.in)));
    c.d.out = reinterpret_cast<char*>(uniform_u64(reinterpret_cast<unsigned long long>(s_c.d.out)));
    c.d.n = (int64_t)uniform_u64((unsigned long long)s_c.d.n);
    c.d.in_dt = __builtin_amdgcn_readfirstlane(s_c.d.in_dt);
    c.d.out_dt = __builtin_amdgcn_readfirstlane(s_c.d.out_dt);
    c.part = (long long)uniform_u64((unsigned long long)s_c.part);
    c.seq = uniform_u64(s_c.seq);
    c.units = __builtin_amdgcn_readfirstlane(s_c.units);
    c.slot = __builtin_amdgcn_readfirstlane(s_c.slot);
    c.exit = __builtin_amdgcn_readfirstlane(s_c.exit);
    if (c.exit) return;
    if (c.units == 0) {
      lds_barrier();  // s_c is written again by the next claim
      continue;
    }
    const uint32_t tag = dq_tag(c.seq);
    const ResExchange x{q->tagged[c.slot], q->total[c.slot], &q->arrivals[c.slot], tag, &q->error, &q->stall,
                        nullptr};
    if (c.d.n <= DQ_RESIDENT_MAX) {
      dispatch_resident<ACC>(c.d, (int)c.part, x, slots, &s_bcast, nullptr);
      dq_finish(a, c, (unsigned)c.units);
    } else {
      const int m = c.units / 2;
      if (dq_long_unit<ACC>(c.d, c.part, m, x, slots, &s_bcast)) dq_finish(a, c, (unsigned)m);
      else lds_barrier();  // slots and s_c are reused by the next unit
    }
  }
}

__global__ void dq_hold_kernel(const DqHost* h, unsigned long long max_ticks) {
  const unsigned long long t0 = dq_now();
  while (ld_sys(&h->hold) == 0 && dq_now() - t0 < max_ticks) __builtin_amdgcn_s_sleep(20);
}

__global__ void dq_touch_kernel() {}

__global__ void dq_reset_kernel(DqDev* q) {
  st_agent(&q->next_unit, ld_agent(&q->pub_units));
  st_agent(&q->exit_epoch, 0ull);
  const unsigned long long now = dq_now();
  st_agent(&q->last_seen, now);
  st_agent(&q->launched_at, now);
}

}  // namespace

hipError_t launch_dq_hold(const DqHost* host, unsigned long long max_ticks, hipStream_t s) {
  hipLaunchKernelGGL(dq_hold_kernel, dim3(1), dim3(1), 0, s, host, max_ticks);
  return hipGetLastError();
}

hipError_t launch_dq_touch(hipStream_t s) {
  hipLaunchKernelGGL(dq_touch_kernel, dim3(1), dim3(1), 0, s);
  return hipGetLastError();
}

hipError_t launch_dq(const DqArgs& a, int acc, int64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(dq_reset_kernel, dim3(1), dim3(1), 0, s, a.dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (acc == NRM_ACC_KAHAN)
    hipLaunchKernelGGL((dq_kernel<NRM_ACC_KAHAN>), dim3((unsigned)blocks), dim3(RES_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((dq_kernel<NRM_ACC_F32>), dim3((unsigned)blocks), dim3(RES_BLOCK), 0, s, a);
  return hipGetLastError();
}

}  // namespace nrm
