// A synthetic layer-forward tile kernel with the shape of the example the
// paper uses for barrier elimination and for memory-to-register promotion
// across barriers (arXiv 2207.00257, Sec. IV-A and IV-B, Fig. 9), written
// from what it computes, to measure on gfx950 what those transformations
// remove.
//
// What it computes, per tile of 16 rows of the R x 16 binary32 matrix
// `hidden` (one 256-thread block per tile): the products
// p[y][x] = hidden[y][x] * input[y], a halving tree over y that leaves in row
// y the sum of p over rows y .. y + L(y) - 1 (L(y) the largest power of two
// dividing y, 16 for y = 0), every row written back to hidden, and the
// column sums (row 0) to output.
//
// The block runs it as stages that meet in LDS:
//   SCALE  the tile's 16 input values into LDS (the first 16 threads, one
//          coalesced load);
//   STAGE  every thread its hidden element into the LDS tile;
//   SCALE_TILE  every thread multiplies its tile element by its row's scale;
//   TREE   four halving levels; level s adds row y + 2^(s-1) into row y for
//          y a multiple of 2^s, the 16 >> s active rows times 16 columns
//          packed onto the block's first threads;
//   WRITE  every thread its tile element back to hidden;
//   EMIT   the first 16 threads the tile's row 0 to output.
// A barrier between two stages is needed only when a location one thread
// accesses on one side is written by another thread on the other side (Sec.
// IV-A's rule; reads on both sides do not conflict). Here that fails for two
// of them: after SCALE (before it only input is read and the scale written;
// STAGE reads hidden and writes the tile, and the next barrier follows), and
// after WRITE (WRITE reads the tile and writes hidden; EMIT reads the tile
// and writes output). The forms:
//   NRM_LF_ALL_BARRIERS  a barrier after every stage and tree level;
//   NRM_LF_ELIMINATED    without those two;
//   NRM_LF_PROMOTED      also STAGE and SCALE_TILE as one stage: the tile
//                        element crossed the barrier between them only to be
//                        read back by the thread that wrote it (Sec. IV-B), so
//                        it stays in a register and the tile is written once;
//   NRM_LF_REGISTERS     no LDS at all: each thread keeps one column of one
//                        tile in registers and runs the tree there; a block
//                        holds 16 tiles.
// Every form performs the same roundings in the same order: their results are
// bitwise equal. The barriers are __syncthreads(); on gfx950 their
// workgroup-scope fences wait for LDS operations (a block's wavefronts share
// one CU), not for global stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrm.h"
#include "nrm_internal.h"

namespace nrm {
namespace {

constexpr int SIDE = 16;             // rows per tile and columns of hidden
constexpr int THREADS = SIDE * SIDE;

template <int FORM>
__device__ __forceinline__ void stage_sync(bool needed_by_rule) {
  if (needed_by_rule || FORM == NRM_LF_ALL_BARRIERS) __syncthreads();
}

template <int FORM>
__global__ void __launch_bounds__(THREADS) layerforward_tile_kernel(float* hidden, const float* input,
                                                                    float* output) {
  __shared__ float scale[SIDE];
  __shared__ float tile[SIDE * SIDE];  // row-major: element (y, x) at y * SIDE + x
  const int t = threadIdx.x;
  const int64_t first_row = (int64_t)blockIdx.x * SIDE;
  float* hid = hidden + first_row * SIDE;  // the tile's 256 elements, contiguous

  if (t < SIDE) scale[t] = input[first_row + t];  // SCALE
  if constexpr (FORM == NRM_LF_PROMOTED) {
    const float h = hid[t];
    stage_sync<FORM>(true);                     // scale[] crosses threads
    tile[t] = h * scale[t / SIDE];              // STAGE + SCALE_TILE
  } else {
    stage_sync<FORM>(false);                    // removable: no conflict across it
    tile[t] = hid[t];                           // STAGE
    stage_sync<FORM>(true);                     // scale[] crosses threads
    tile[t] = tile[t] * scale[t / SIDE];        // SCALE_TILE
  }
  stage_sync<FORM>(true);
#pragma unroll
  for (int s = 1; s <= 4; ++s) {                // TREE
    const int span = 1 << s;
    if (t < (SIDE >> s) * SIDE) {
      const int y = (t / SIDE) * span, x = t % SIDE;
      tile[y * SIDE + x] += tile[(y + span / 2) * SIDE + x];
    }
    stage_sync<FORM>(true);
  }
  hid[t] = tile[t];                             // WRITE
  stage_sync<FORM>(false);                      // removable: reads of the tile on both sides
  if (t < SIDE) output[first_row + t] = tile[t];  // EMIT (row 0)
}

// One thread per tile column: 16 tiles per 256-thread block. The products
// are rounded on their own, as the LDS forms round them on their way through
// the tile: no contraction of a product into the first tree addition.
__global__ void __launch_bounds__(THREADS) layerforward_registers_kernel(float* hidden, const float* input,
                                                                         float* output, int64_t tiles) {
#pragma clang fp contract(off)
  const int64_t tile = (int64_t)blockIdx.x * SIDE + threadIdx.x / SIDE;
  const int x = threadIdx.x % SIDE;
  if (tile >= tiles) return;
  float p[SIDE];
#pragma unroll
  for (int y = 0; y < SIDE; ++y) {
    const int64_t row = tile * SIDE + y;
    p[y] = hidden[row * SIDE + x] * input[row];
  }
#pragma unroll
  for (int s = 1; s <= 4; ++s) {
    const int span = 1 << s;
#pragma unroll
    for (int y = 0; y < SIDE; y += span) p[y] += p[y + span / 2];
  }
#pragma unroll
  for (int y = 0; y < SIDE; ++y) hidden[(tile * SIDE + y) * SIDE + x] = p[y];
  output[tile * SIDE + x] = p[0];
}

}  // namespace

hipError_t launch_layerforward(int form, float* hidden, const float* input, float* output, int64_t rows,
                               hipStream_t s) {
  const dim3 grid((unsigned)(rows / SIDE)), block(THREADS);
  switch (form) {
    case NRM_LF_ALL_BARRIERS:
      hipLaunchKernelGGL(layerforward_tile_kernel<NRM_LF_ALL_BARRIERS>, grid, block, 0, s, hidden, input, output);
      break;
    case NRM_LF_ELIMINATED:
      hipLaunchKernelGGL(layerforward_tile_kernel<NRM_LF_ELIMINATED>, grid, block, 0, s, hidden, input, output);
      break;
    case NRM_LF_PROMOTED:
      hipLaunchKernelGGL(layerforward_tile_kernel<NRM_LF_PROMOTED>, grid, block, 0, s, hidden, input, output);
      break;
    default: {
      const int64_t tiles = rows / SIDE;
      hipLaunchKernelGGL(layerforward_registers_kernel, dim3((unsigned)((tiles + SIDE - 1) / SIDE)), block, 0, s,
                         hidden, input, output, tiles);
      break;
    }
  }
  return hipGetLastError();
}

}  // namespace nrm
