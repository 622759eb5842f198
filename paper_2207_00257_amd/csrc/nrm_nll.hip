// Forward negative log-likelihood loss on gfx950: the loss kernel the paper
// translated because it synchronises with a block barrier (arXiv 2207.00257,
// Sec. V-B), written from the loss's definition. For N samples, C classes,
// log-probabilities logp[N][C] (row-major binary32), targets t[N] (int64)
// and class weights w[C] (binary32, all 1 when absent):
//     loss_n = -w[t_n] logp[n][t_n]  (0 for t_n == ignore_index),
//     none: out[n] = loss_n;  sum: out = sum loss_n;  mean: out = sum / sum w[t_n].
// Like normalize (Fig. 1) it reduces invariants once (two: the loss and the
// weight total) and then maps (here the one division).
//
//   nll_reduce_kernel   grid-stride over samples, U per thread per
//                       iteration: the targets are read coalesced, then the
//                       U gathers logp[n*C + t_n] and w[t_n] are in flight
//                       together; independent loss and weight chains per
//                       thread, a DPP wavefront reduce, one LDS slot per
//                       wavefront, two partials per block (plain stores).
//                       For reduction none it writes each loss_n instead.
//   nll_combine_kernel  one block merges each partial array in a fixed order
//                       (combine_partials) and writes the result: the kernel
//                       boundary is the grid-wide barrier.
// A target outside [0, C) that is not ignore_index contributes nothing and
// sets NRM_DEVERR_TARGET in the device error word.
#include "nrm_batch.h"
#include "nrm_device.h"

namespace nrm {
namespace {

using namespace dev;

constexpr int NLL_BLOCK = 256;
constexpr int NLL_U = 4;

struct NllArgs {
  const float* logp;
  const int64_t* target;
  const float* weight;  // NULL: all 1
  int64_t n, c, ignore;
  int reduction;
  void* partials;       // [2 * gridDim.x] Acc: the loss partials, then the weight partials
  float* out;
  float* total_weight;  // NULL: not written
  int* error;
};

template <int ACC>
__global__ void __launch_bounds__(NLL_BLOCK) nll_reduce_kernel(NllArgs a) {
  __shared__ Acc<ACC> slots[NLL_BLOCK / 64];
  Acc<ACC> ls[NLL_U], ws[NLL_U];
#pragma unroll
  for (int u = 0; u < NLL_U; ++u) {
    ls[u].zero();
    ws[u].zero();
  }
  bool bad = false;
  const int64_t B = blockDim.x, step = (int64_t)gridDim.x * B * NLL_U;
  for (int64_t base = (int64_t)blockIdx.x * B * NLL_U + threadIdx.x; base < a.n; base += step) {
    int64_t t[NLL_U];
#pragma unroll
    for (int u = 0; u < NLL_U; ++u) {
      const int64_t i = base + u * B;
      t[u] = i < a.n ? a.target[i] : a.ignore;
    }
    float x[NLL_U], w[NLL_U];
    bool keep[NLL_U];
#pragma unroll
    for (int u = 0; u < NLL_U; ++u) {
      const int64_t i = base + u * B;
      const bool in_range = t[u] >= 0 && t[u] < a.c;
      keep[u] = i < a.n && t[u] != a.ignore && in_range;
      bad |= i < a.n && t[u] != a.ignore && !in_range;
      x[u] = keep[u] ? a.logp[i * a.c + t[u]] : 0.0f;
      w[u] = keep[u] ? (a.weight ? a.weight[t[u]] : 1.0f) : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < NLL_U; ++u) {
      const int64_t i = base + u * B;
      const float l = -(w[u] * x[u]);  // one rounding: the product
      if (a.reduction == NRM_NLL_NONE) {
        if (i < a.n) a.out[i] = keep[u] ? l : 0.0f;
      } else if (keep[u]) {
        ls[u].add(l);
        ws[u].add(w[u]);
      }
    }
  }
  if (bad) atomicOr(a.error, NRM_DEVERR_TARGET);
  if (a.reduction == NRM_NLL_NONE) return;
  merge_chains<ACC, NLL_U>(ls);
  merge_chains<ACC, NLL_U>(ws);
  const Acc<ACC> L = block_reduce<ACC>(ls[0], slots);
  lds_barrier();  // slots are reused
  const Acc<ACC> W = block_reduce<ACC>(ws[0], slots);
  Acc<ACC>* part = static_cast<Acc<ACC>*>(a.partials);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = L;
    part[gridDim.x + blockIdx.x] = W;
  }
}

template <int ACC>
__global__ void __launch_bounds__(1024) nll_combine_kernel(NllArgs a, int64_t parts) {
  __shared__ Acc<ACC> tree[COMBINE_TILE];
  __shared__ Acc<ACC> tiles[MAX_COMBINE_TILES];
  const Acc<ACC>* part = static_cast<const Acc<ACC>*>(a.partials);
  const Acc<ACC> L = combine_partials<ACC>(part, parts, tree, tiles);
  lds_barrier();  // the trees are reused
  const Acc<ACC> W = combine_partials<ACC>(part + parts, parts, tree, tiles);
  if (threadIdx.x == 0) {
    const float l = L.value(), w = W.value();
    a.out[0] = a.reduction == NRM_NLL_MEAN ? l / w : l;
    if (a.total_weight) a.total_weight[0] = w;
  }
}

template <int ACC>
hipError_t launch_acc(const NllPlan& p, void* partials, int* error, hipStream_t s) {
  NllArgs a;
  a.logp = p.logp;
  a.target = p.target;
  a.weight = p.weight;
  a.n = p.n;
  a.c = p.c;
  a.ignore = p.ignore;
  a.reduction = p.reduction;
  a.partials = partials;
  a.out = p.out;
  a.total_weight = p.total_weight;
  a.error = error;
  hipLaunchKernelGGL((nll_reduce_kernel<ACC>), dim3(p.grid), dim3(NLL_BLOCK), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.reduction == NRM_NLL_NONE) return e;
  hipLaunchKernelGGL((nll_combine_kernel<ACC>), dim3(1), dim3(1024), 0, s, a, p.grid);
  return hipGetLastError();
}

}  // namespace

int64_t nll_grid(int64_t n, int64_t max_grid) {
  const int64_t per_block = (int64_t)NLL_BLOCK * NLL_U;
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return g < max_grid ? g : max_grid;
}

hipError_t launch_nll(const NllPlan& p, void* partials, int* error, hipStream_t s) {
  return p.acc == NRM_ACC_KAHAN ? launch_acc<NRM_ACC_KAHAN>(p, partials, error, s)
                                : launch_acc<NRM_ACC_F32>(p, partials, error, s);
}

}  // namespace nrm
