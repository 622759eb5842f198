/*
 * FP64 CPU oracle for the forward negative log-likelihood loss.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library and its Python binding) never calls it, and this file shares no
 * code, header, table or helper with that path.
 *
 * What it computes. The NLL-loss forward is the PyTorch kernel the paper
 * translated with its compiler because it synchronises with a block barrier
 * (arXiv 2207.00257, Sec. V-B); it is written here from the loss's
 * definition, not from any implementation. For N samples with C classes,
 * log-probabilities logp[N][C] (row-major binary32), class targets t[N]
 * (int64) and optional class weights w[C] (binary32; all 1 when absent):
 *     loss_n = -w[t_n] * logp[n][t_n]   for t_n != ignore_index, else 0,
 *     total_weight = sum over the kept samples of w[t_n],
 *     reduction none: out[n] = loss_n;  sum: out = sum_n loss_n;
 *     mean: out = (sum_n loss_n) / total_weight  (0/0 = NaN when every
 *     sample is ignored).
 * The sums are the reduce, the division the map over the one output: the
 * shape of the paper's normalize (Fig. 1), with two invariants. Binary64
 * arithmetic (the product of two binary32 values is exact in binary64), sums
 * in sample order. A target outside [0, C) that is not ignore_index is an
 * argument error.
 *
 * Parity status: pinned by CPU tests against closed forms, exact rational
 * arithmetic, torch.nn.functional.nll_loss in float64 and invariants.
 */
#include <math.h>
#include <stdint.h>

enum { ORC_NLL_OK = 0, ORC_NLL_EINVAL = -1 };
enum { ORC_NLL_NONE = 0, ORC_NLL_SUM = 1, ORC_NLL_MEAN = 2 };

/* out: n values for reduction none, else one; total_weight may be NULL. */
int oracle_nll_loss(const float* logp, const int64_t* target, const float* weight, int64_t n, int64_t c,
                    int64_t ignore_index, int reduction, double* out, double* total_weight) {
  if (n < 0 || c < 1 || !out || (n > 0 && (!logp || !target))) return ORC_NLL_EINVAL;
  if (reduction != ORC_NLL_NONE && reduction != ORC_NLL_SUM && reduction != ORC_NLL_MEAN) return ORC_NLL_EINVAL;
  double loss = 0.0, wsum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t t = target[i];
    if (t == ignore_index) {
      if (reduction == ORC_NLL_NONE) out[i] = 0.0;
      continue;
    }
    if (t < 0 || t >= c) return ORC_NLL_EINVAL;
    const double w = weight ? (double)weight[t] : 1.0;
    const double l = -w * (double)logp[i * c + t];
    if (reduction == ORC_NLL_NONE) out[i] = l;
    loss += l;
    wsum += w;
  }
  if (reduction == ORC_NLL_SUM) out[0] = loss;
  if (reduction == ORC_NLL_MEAN) out[0] = loss / wsum;
  if (total_weight) *total_weight = wsum;
  return ORC_NLL_OK;
}
