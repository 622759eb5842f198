// Internal interface between the C-ABI layer (nrm_api.cpp) and the HIP
// kernels (nrm_kernels.hip). Not installed, not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrm.h"

namespace nrm {

// Reduction kinds of the batched kernels: the two public accumulation modes
// (nrm_accum) and the row softmax's (exponent, scaled sum) pairs.
constexpr int ACC_SOFTMAX = 2;

// Element sizes of the storage dtypes (nrm_dtype order: F32, BF16, F16).
inline int dtype_size(int dt) { return dt == NRM_F32 ? 4 : 2; }
// Elements per 16-byte vector.
inline int dtype_vec(int dt) { return 16 / dtype_size(dt); }

// Independent accumulator chains per thread in the reduce kernel: one per
// element of the U vectors a thread loads per iteration, capped so that the
// chains stay in registers (32 plain; 16 for the two-float chains:
// compensated pairs, and the softmax kind's exponent and sum).
__host__ __device__ constexpr int accumulators(int dt, int acc, int unroll) {
  return (unroll * (16 / (dt == NRM_F32 ? 4 : 2))) < (acc == NRM_ACC_F32 ? 32 : 16)
             ? unroll * (16 / (dt == NRM_F32 ? 4 : 2))
             : (acc == NRM_ACC_F32 ? 32 : 16);
}
// Additions each chain receives per loop iteration.
__host__ __device__ constexpr int adds_per_iteration(int dt, int acc, int unroll) {
  return unroll * (16 / (dt == NRM_F32 ? 4 : 2)) / accumulators(dt, acc, unroll);
}
// Plain binary32 mode: additions a chain receives before the thread sums its
// chains into its running total and restarts them.
constexpr int CHAIN_ADDS = 16;

// Height (longest path of additions) of one thread's summation tree in plain
// mode after `iters` loop iterations: a chain of CHAIN_ADDS (+1 for the head
// or tail element), the pairwise merge of the chains, and one addition into
// the running total per flush.
inline int64_t thread_tree_height(int dt, int acc, int unroll, int64_t iters) {
  int na = accumulators(dt, acc, unroll), lg = 0;
  while ((1 << lg) < na) ++lg;
  int flush = CHAIN_ADDS / adds_per_iteration(dt, acc, unroll);
  return CHAIN_ADDS + 1 + lg + (iters + flush - 1) / flush;
}

// Plan of one plain normalize call, fully resolved on the host.
struct PlainPlan {
  const void* in;
  void* out;
  int64_t n;
  int in_dt, out_dt, acc;
  int64_t head;       // elements before the input's first 128-byte line
  int64_t nvec;       // 16-byte input vectors in the aligned body
  int64_t tail_begin; // first element after the body
  bool vector_map;    // out is aligned like in, so the map can use vector stores
  // reduce kernel
  int block;          // threads per block (multiple of 64, <= 1024)
  int unroll;         // 16-byte vectors per thread per iteration
  int64_t grid;       // blocks
  int64_t chunk;      // vectors per block (layout CHUNK; multiple of block * unroll)
  int64_t tile;       // vectors per tile (layout TILE; multiple of block * unroll)
  int layout;         // NRM_LAYOUT_*
  bool fused;         // no grid-wide ticket: every map block merges the partials
  int reduce_nt;      // non-temporal hint on loads
  int64_t keep_from;  // vectors from this index on are loaded with a temporal hint
  // map kernel
  int map_block;
  int map_unroll;
  int64_t map_grid;
  int64_t map_chunk;  // map units per block (layout CHUNK)
  int64_t map_tile;   // map units per tile (layout TILE)
  int64_t map_units;  // map units in the body: 16-byte vectors, or 8-byte halves
                      // for a 2-byte input with binary32 output
  int map_layout;
  int map_nt;
  int reverse_map;
};

// Device workspace of the plain path: per-block partials, the completion
// ticket of the grid combine, and the hoisted sum.
struct PlainWorkspace {
  void* partials;     // float[grid] or float2[grid] (compensated)
  unsigned* ticket;   // zero between calls
  float* sum;         // the invariant, one float (compensated: hi, lo)
};

hipError_t launch_reduce(const PlainPlan& p, const PlainWorkspace& ws, hipStream_t s);

// Forward NLL loss (nrm_nll.hip): one reduce launch of `grid` blocks (two
// Acc partials each in `partials`) and, unless reduction is none, a one-block
// combine.
struct NllPlan {
  const float* logp;
  const int64_t* target;
  const float* weight;
  int64_t n, c, ignore;
  int reduction, acc;
  float* out;
  float* total_weight;
  int64_t grid;
};
int64_t nll_grid(int64_t n, int64_t max_grid);

// The plain path's single-launch form for small n (nrm_batched.hip): one block
// holds up to small_capacity(in_dt) elements in registers.
int64_t small_capacity(int in_dt);
hipError_t launch_small(const void* in, int in_dt, void* out, int out_dt, int64_t n, int acc, float* sum_out,
                        hipStream_t s);

// The plain path's single-launch form for mid-size n (nrm_batched.hip): one
// block per segment of the input held in registers across an exchange of the
// segment sums; n <= plain_resident_capacity(). Workspace, zero-initialized:
// the segments' tagged partials (16 bytes each), the merged total, the
// arrival count, the call number, the stall marker and error word, and the
// sum for nrm_get_last_sum.
struct PlainResidentWs {
  unsigned long long* slots;  // 2 x 256 words
  unsigned long long* total;  // 2 words
  unsigned* arrivals;         // 0 between calls
  unsigned long long* call;
  unsigned long long* stall;
  int* error;
  float* sum_out;
};
int64_t plain_resident_capacity();
hipError_t launch_plain_resident(const void* in, int in_dt, void* out, int out_dt, int64_t n, int acc,
                                 const PlainResidentWs& w, hipStream_t s);

// The Fig. 9-shaped tile kernel in one of its three forms (nrm_layerforward.hip).
hipError_t launch_layerforward(int form, float* hidden, const float* input, float* output, int64_t rows,
                               hipStream_t s);
hipError_t launch_nll(const NllPlan& p, void* partials, int* error, hipStream_t s);
hipError_t launch_form(int form, float* out, const float* in, int64_t n, int block, hipStream_t s);
hipError_t launch_map(const PlainPlan& p, const PlainWorkspace& ws, hipStream_t s);

// Bandwidth ceilings for measurement (nrm_ceiling.hip): kind 0 copies `bytes`
// from src to dst, kind 1 reads them (dst: a word per block, rarely written).
hipError_t launch_ceiling(int kind, void* dst, const void* src, int64_t bytes, int64_t grid, hipStream_t s);

}  // namespace nrm
