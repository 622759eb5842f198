// Bandwidth ceilings for the measurement: a plain device copy and a plain
// read-only sweep over the same bytes as a normalize call, timed in the same
// run, so that normalize can be reported as a fraction of what this machine's HBM
// actually delivers, not only of the published 8 TB/s. They are not part of
// the normalize path.
//
// Both stream 16-byte vectors with non-temporal hints (nothing is reused) in
// the divide map's own shape: tiles of 1024 vectors (16 KiB), block b taking
// tiles b, b + grid, ..., two vectors per thread per tile; the read sweep
// folds what it reads into one word per thread so that the loads cannot be
// removed, and stores it only when it has a value no input here produces.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrm_internal.h"

namespace nrm {
namespace {

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

constexpr int CEIL_BLOCK = 512;
constexpr int CEIL_U = 2;
constexpr int64_t CEIL_TILE = CEIL_BLOCK * CEIL_U;  // vectors per tile

__global__ void __launch_bounds__(CEIL_BLOCK) ceiling_copy_kernel(u4v* dst, const u4v* src, int64_t nvec) {
  for (int64_t base = (int64_t)blockIdx.x * CEIL_TILE; base < nvec; base += (int64_t)gridDim.x * CEIL_TILE) {
    u4v v[CEIL_U];
#pragma unroll
    for (int u = 0; u < CEIL_U; ++u) {
      const int64_t j = base + threadIdx.x + (int64_t)u * CEIL_BLOCK;
      if (j < nvec) v[u] = __builtin_nontemporal_load(src + j);
    }
#pragma unroll
    for (int u = 0; u < CEIL_U; ++u) {
      const int64_t j = base + threadIdx.x + (int64_t)u * CEIL_BLOCK;
      if (j < nvec) __builtin_nontemporal_store(v[u], dst + j);
    }
  }
}

__global__ void __launch_bounds__(CEIL_BLOCK) ceiling_read_kernel(const u4v* src, int64_t nvec, unsigned* sink) {
  unsigned acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * CEIL_TILE; base < nvec; base += (int64_t)gridDim.x * CEIL_TILE) {
#pragma unroll
    for (int u = 0; u < CEIL_U; ++u) {
      const int64_t j = base + threadIdx.x + (int64_t)u * CEIL_BLOCK;
      if (j < nvec) {
        const u4v v = __builtin_nontemporal_load(src + j);
        acc += v.x ^ v.y ^ v.z ^ v.w;
      }
    }
  }
  if (acc == 0x9e3779b9u) sink[blockIdx.x] = acc;
}

}  // namespace

hipError_t launch_ceiling(int kind, void* dst, const void* src, int64_t bytes, int64_t grid, hipStream_t s) {
  const int64_t nvec = bytes / 16;
  const int64_t tiles = (nvec + CEIL_TILE - 1) / CEIL_TILE;
  const int64_t g = grid < tiles ? grid : tiles;
  if (g < 1) return hipSuccess;
  if (kind == 0)
    hipLaunchKernelGGL(ceiling_copy_kernel, dim3((unsigned)g), dim3(CEIL_BLOCK), 0, s, static_cast<u4v*>(dst),
                       static_cast<const u4v*>(src), nvec);
  else
    hipLaunchKernelGGL(ceiling_read_kernel, dim3((unsigned)g), dim3(CEIL_BLOCK), 0, s, static_cast<const u4v*>(src),
                       nvec, static_cast<unsigned*>(dst));
  return hipGetLastError();
}

}  // namespace nrm
