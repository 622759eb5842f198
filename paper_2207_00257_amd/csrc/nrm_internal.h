// Internal interface between the C-ABI layer (nrm_api.cpp) and the HIP
// kernels (nrm_kernels.hip). Not installed, not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrm.h"

namespace nrm {

// Element sizes of the storage dtypes (nrm_dtype order: F32, BF16, F16).
inline int dtype_size(int dt) { return dt == NRM_F32 ? 4 : 2; }
// Elements per 16-byte vector.
inline int dtype_vec(int dt) { return 16 / dtype_size(dt); }

// Independent accumulator chains per thread in the reduce kernel: one per
// element of the U vectors a thread loads per iteration, capped so that the
// chains stay in registers (32 plain, 16 compensated pairs).
__host__ __device__ constexpr int accumulators(int dt, int acc, int unroll) {
  return (unroll * (16 / (dt == NRM_F32 ? 4 : 2))) < (acc == NRM_ACC_KAHAN ? 16 : 32)
             ? unroll * (16 / (dt == NRM_F32 ? 4 : 2))
             : (acc == NRM_ACC_KAHAN ? 16 : 32);
}
// Additions each chain receives per loop iteration.
__host__ __device__ constexpr int adds_per_iteration(int dt, int acc, int unroll) {
  return unroll * (16 / (dt == NRM_F32 ? 4 : 2)) / accumulators(dt, acc, unroll);
}

// Plan of one plain normalize call, fully resolved on the host.
struct PlainPlan {
  const void* in;
  void* out;
  int64_t n;
  int in_dt, out_dt, acc;
  int64_t head;       // elements before the first 16-byte aligned input vector
  int64_t nvec;       // 16-byte input vectors in the aligned body
  int64_t tail_begin; // first element after the body
  bool vector_map;    // out is aligned like in, so the map can use vector stores
  int block;          // threads per block (multiple of 64, <= 1024)
  int unroll;         // 16-byte vectors per thread per iteration
  int map_unroll;
  int64_t grid;       // reduce blocks
  int64_t chunk;      // reduce: vectors per block (multiple of block * unroll)
  int64_t map_grid;
  int64_t map_chunk;  // map: vectors per block (multiple of block * map_unroll)
  int layout;         // NRM_LAYOUT_*
  int reverse_map;
  int nt_loads;       // non-temporal hint on the map's loads
};

// Device workspace of the plain path: per-block partials, the completion
// ticket of the grid combine, and the hoisted sum.
struct PlainWorkspace {
  void* partials;     // float[grid] or float2[grid] (compensated)
  unsigned* ticket;   // zero between calls
  float* sum;         // the invariant, one float (compensated: hi, lo)
};

hipError_t launch_reduce(const PlainPlan& p, const PlainWorkspace& ws, hipStream_t s);
hipError_t launch_map(const PlainPlan& p, const PlainWorkspace& ws, hipStream_t s);

}  // namespace nrm
