// The two un-hoisted forms of normalize (arXiv 2207.00257, Fig. 1), kept on
// the GPU only to measure what hoisting the invariant sum buys:
//
//   naive_kernel     every thread computes the whole sum itself, then divides
//                    its element: O(n^2) work (Fig. 1 as printed).
//   perblock_kernel  thread 0 of every block computes the sum into block-
//                    shared memory, the block meets at a barrier, then every
//                    thread divides: O(n^2 / B) work (the shared-memory variant
//                    in Fig. 1's comments; Fig. 3).
//
// Each per-thread sum is a Kahan-compensated binary32 chain over the input in
// index order, so the results stay within the library's error bound even for
// these long chains. These are not performance paths.
#include "nrm_device.h"

namespace nrm {
namespace {

using namespace dev;

__device__ __forceinline__ float sum_whole(const float* in, int64_t n) {
  Acc<NRM_ACC_KAHAN> a;
  a.zero();
  for (int64_t j = 0; j < n; ++j) a.add(in[j]);
  return a.value();
}

__global__ void __launch_bounds__(1024) naive_kernel(float* out, const float* in, int64_t n) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float val = sum_whole(in, n);  // recomputed by every thread
  if (tid < n) out[tid] = in[tid] / val;
}

__global__ void __launch_bounds__(1024) perblock_kernel(float* out, const float* in, int64_t n) {
  __shared__ float val;
  if (threadIdx.x == 0) val = sum_whole(in, n);  // once per block
  __syncthreads();
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < n) out[tid] = in[tid] / val;
}

}  // namespace

hipError_t launch_form(int form, float* out, const float* in, int64_t n, int block, hipStream_t s) {
  const int64_t grid = (n + block - 1) / block;
  if (form == NRM_FORM_NAIVE)
    hipLaunchKernelGGL(naive_kernel, dim3(grid), dim3(block), 0, s, out, in, n);
  else
    hipLaunchKernelGGL(perblock_kernel, dim3(grid), dim3(block), 0, s, out, in, n);
  return hipGetLastError();
}

}  // namespace nrm
