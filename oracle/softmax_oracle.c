/*
 * FP64 CPU oracle for the row softmax and log-sum-exp of a ragged batch.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library and its Python binding) never calls it, and this file shares no
 * code, header, table or helper with that path.
 *
 * What it computes. For every CSR row r = [offsets[r], offsets[r+1]) of a
 * binary32 array x:
 *     softmax_i = exp(x_i) / sum_j exp(x_j),       lse_r = log(sum_j exp(x_j)).
 * Softmax is one of the aggregation kernels the paper's PyTorch integration
 * had to provide (arXiv 2207.00257, Sec. V-B). It has the shape of the paper's
 * running example (Fig. 1, Sec. II-A, Sec. IV-C): a quantity that is invariant
 * across a row (here the pair: row maximum, sum of exponentials) is computed
 * once per row, then an element-wise map uses it.
 *
 * How: through the identity exp(x_i) / sum_j exp(x_j) = exp(x_i - m) /
 * sum_j exp(x_j - m), with m the row maximum, which keeps every exponential
 * in (0, 1] (no overflow for any finite input); lse_r = m + log(sum_j
 * exp(x_j - m)). Binary64 arithmetic from the exactly widened binary32
 * inputs; the maximum is exact, the sum runs in index order. An empty row has
 * no outputs and lse = -inf (the log of an empty sum). Inputs are finite;
 * a non-finite input yields whatever these formulas give (NaN for inf - inf).
 *
 * Parity status: pinned by CPU tests against closed forms (constant rows,
 * one- and two-element rows, the logistic function), invariants (a shift of a
 * row leaves its softmax and moves its lse by the shift) and an independent
 * library implementation.
 */
#include <math.h>
#include <stdint.h>

enum { ORC_SM_OK = 0, ORC_SM_EINVAL = -1 };

/* The row maximum (exact). */
static double row_max(const float* x, int64_t b, int64_t e) {
  double m = (double)x[b];
  for (int64_t j = b + 1; j < e; ++j)
    if ((double)x[j] > m) m = (double)x[j];
  return m;
}

/* sum_j exp(x_j - m) over the row, in index order. */
static double row_sum_exp(const float* x, int64_t b, int64_t e, double m) {
  double s = 0.0;
  for (int64_t j = b; j < e; ++j) s += exp((double)x[j] - m);
  return s;
}

/* Softmax of every row into out (binary64, one value per element of x) and
 * the log-sum-exp of every row into lse (may be NULL). offsets has rows + 1
 * non-decreasing entries starting at >= 0. */
int oracle_softmax_batched(const float* x, const int64_t* offsets, int64_t rows, double* out,
                           double* lse) {
  if (rows < 0 || (rows > 0 && (!x || !offsets || !out))) return ORC_SM_EINVAL;
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t b = offsets[r], e = offsets[r + 1];
    if (b < 0 || e < b) return ORC_SM_EINVAL;
    if (e == b) {
      if (lse) lse[r] = -INFINITY;
      continue;
    }
    const double m = row_max(x, b, e);
    const double s = row_sum_exp(x, b, e, m);
    for (int64_t i = b; i < e; ++i) out[i] = exp((double)x[i] - m) / s;
    if (lse) lse[r] = m + log(s);
  }
  return ORC_SM_OK;
}
