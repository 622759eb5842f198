// A synthetic layer-forward tile kernel with the shape of the example the
// paper uses for barrier elimination and memory-to-register promotion across
// barriers (arXiv 2207.00257, Sec. IV-A and IV-B, Fig. 9), in three forms, to
// measure on gfx950 what those transformations remove.
//
// hidden is an R x 16 binary32 matrix and input an R-vector (R a multiple of
// 16); one 256-thread block (tx = column 0..15, ty = row 0..15) per tile of 16
// rows. Thread tx == 0 of each row loads input into node[ty]; every thread
// forms hidden * node[ty] in the shared tile; a halving tree over ty (four
// steps, a block barrier after each) leaves each column's sum in tile row 0;
// every row is written back to hidden and thread tx == 0 of row ty writes
// column ty's sum to output.
//
//   FORM_PRINTED    the barriers of the example as analysed: one after the
//                   node load, one after the tile store, one after the
//                   multiply, one per tree step, one after the write-back.
//   FORM_ELIMINATED without the two barriers the memory-effect rule of
//                   Sec. IV-A proves redundant: the first (no access after it
//                   touches what was written before it until the next
//                   barrier) and the last (only the thread's own global store
//                   precedes it; the read after it is of the tile, last
//                   written before the tree's final barrier).
//   FORM_PROMOTED   also without the shared store that only the same thread
//                   reads back across a barrier (Sec. IV-B): the loaded value
//                   stays in a register and the tile is written once.
//   FORM_REGISTERS  the end point of that promotion: each thread keeps one
//                   column of one tile in registers and runs the same tree
//                   there (no shared memory, no barrier); a block holds 16
//                   tiles.
// The four forms perform the same arithmetic in the same order: their
// results are bitwise equal. The barriers here are __syncthreads(), whose
// workgroup-scope release also waits for the wavefront's outstanding global
// stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrm.h"
#include "nrm_internal.h"

namespace nrm {
namespace {

constexpr int LF = 16;  // tile side

template <int FORM>
__global__ void __launch_bounds__(LF * LF) layerforward_kernel(float* hidden, const float* input, float* output) {
  __shared__ float node[LF];
  __shared__ float tile[LF][LF];
  const int tx = threadIdx.x % LF, ty = threadIdx.x / LF;
  const int64_t row = (int64_t)blockIdx.x * LF + ty;
  const int64_t idx = row * LF + tx;
  if (tx == 0) node[ty] = input[row];
  if constexpr (FORM == NRM_LF_PRINTED) __syncthreads();
  if constexpr (FORM == NRM_LF_PROMOTED) {
    const float h = hidden[idx];
    __syncthreads();  // node[] crosses threads
    tile[ty][tx] = h * node[ty];
  } else {
    tile[ty][tx] = hidden[idx];
    __syncthreads();
    tile[ty][tx] = tile[ty][tx] * node[ty];
  }
  __syncthreads();
#pragma unroll
  for (int s = 1; s <= 4; ++s) {
    const int step = 1 << s;
    if ((ty & (step - 1)) == 0) tile[ty][tx] += tile[ty + step / 2][tx];
    __syncthreads();
  }
  hidden[idx] = tile[ty][tx];
  if constexpr (FORM == NRM_LF_PRINTED) __syncthreads();
  if (tx == 0) output[(int64_t)blockIdx.x * LF + ty] = tile[0][ty];
}

// One thread per tile column: 16 tiles per 256-thread block. The products
// are rounded on their own, as the other forms round them on their way
// through the shared tile: no contraction of a product into the first tree
// addition.
__global__ void __launch_bounds__(LF * LF) layerforward_registers_kernel(float* hidden, const float* input,
                                                                         float* output, int64_t tiles) {
#pragma clang fp contract(off)
  const int64_t tile = (int64_t)blockIdx.x * LF + threadIdx.x / LF;
  const int x = threadIdx.x % LF;
  if (tile >= tiles) return;
  float p[LF];
#pragma unroll
  for (int y = 0; y < LF; ++y) {
    const int64_t row = tile * LF + y;
    p[y] = hidden[row * LF + x] * input[row];
  }
#pragma unroll
  for (int s = 1; s <= 4; ++s) {
    const int step = 1 << s;
#pragma unroll
    for (int y = 0; y < LF; y += step) p[y] += p[y + step / 2];
  }
#pragma unroll
  for (int y = 0; y < LF; ++y) hidden[(tile * LF + y) * LF + x] = p[y];
  output[tile * LF + x] = p[0];
}

}  // namespace

hipError_t launch_layerforward(int form, float* hidden, const float* input, float* output, int64_t rows,
                               hipStream_t s) {
  const dim3 grid((unsigned)(rows / LF)), block(LF * LF);
  switch (form) {
    case NRM_LF_PRINTED:
      hipLaunchKernelGGL(layerforward_kernel<NRM_LF_PRINTED>, grid, block, 0, s, hidden, input, output);
      break;
    case NRM_LF_ELIMINATED:
      hipLaunchKernelGGL(layerforward_kernel<NRM_LF_ELIMINATED>, grid, block, 0, s, hidden, input, output);
      break;
    case NRM_LF_PROMOTED:
      hipLaunchKernelGGL(layerforward_kernel<NRM_LF_PROMOTED>, grid, block, 0, s, hidden, input, output);
      break;
    default: {
      const int64_t tiles = rows / LF;
      hipLaunchKernelGGL(layerforward_registers_kernel, dim3((unsigned)((tiles + LF - 1) / LF)), block, 0, s, hidden,
                         input, output, tiles);
      break;
    }
  }
  return hipGetLastError();
}

}  // namespace nrm
