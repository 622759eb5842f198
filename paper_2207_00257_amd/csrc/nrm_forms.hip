// The two un-hoisted forms of normalize (arXiv 2207.00257, Fig. 1 and its
// caption), kept on the GPU only to measure what hoisting the invariant sum
// buys. Both divide every element by the sum of all elements; they differ in
// how often that sum is computed:
//
//   naive     once per thread: each thread reads the whole input itself and
//             divides its own element, O(n^2) work in total;
//   perblock  once per block: the block's first wavefront reads the whole
//             input (64 lanes, 16-byte vectors), merges its lanes, and leaves
//             the sum in LDS; after one block barrier every thread divides its
//             element, O(n^2 / B) work in total.
//
// The sums are Kahan-compensated binary32 (one chain per thread, or per lane
// merged by TwoSum), so the results stay within the library's error bound
// even for these long chains. These are not performance paths.
#include "nrm_device.h"

namespace nrm {
namespace {

using namespace dev;

// Sum of in[0..n) into a compensated chain: lane `lane` of `lanes` takes the
// 16-byte vectors lane, lane + lanes, ... of the input's aligned body; lane 0
// also takes the unaligned head and the tail.
__device__ __forceinline__ Acc<NRM_ACC_KAHAN> sum_strided(const float* in, int64_t n, int lane, int lanes) {
  Acc<NRM_ACC_KAHAN> a;
  a.zero();
  const int64_t mis = (int64_t)((reinterpret_cast<uintptr_t>(in) & 15) / 4);
  const int64_t head = mis ? (4 - mis < n ? 4 - mis : n) : 0;
  const int64_t nvec = (n - head) / 4;
  const u4* body = reinterpret_cast<const u4*>(in + head);
  for (int64_t v = lane; v < nvec; v += lanes) {
    const u4 r = body[v];
    a.add(f32_bits(r[0]));
    a.add(f32_bits(r[1]));
    a.add(f32_bits(r[2]));
    a.add(f32_bits(r[3]));
  }
  if (lane == 0) {
    for (int64_t i = 0; i < head; ++i) a.add(in[i]);
    for (int64_t i = head + 4 * nvec; i < n; ++i) a.add(in[i]);
  }
  return a;
}

__global__ void __launch_bounds__(1024) naive_kernel(float* out, const float* in, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float sum = sum_strided(in, n, 0, 1).value();  // this thread's own pass over the input
  if (i < n) out[i] = in[i] / sum;
}

__global__ void __launch_bounds__(1024) perblock_kernel(float* out, const float* in, int64_t n) {
  __shared__ float block_sum;
  if (threadIdx.x < 64) {
    const Acc<NRM_ACC_KAHAN> total = wave_reduce<NRM_ACC_KAHAN>(sum_strided(in, n, threadIdx.x, 64));
    if (threadIdx.x == 0) block_sum = total.value();
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] / block_sum;
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
