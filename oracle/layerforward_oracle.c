/*
 * FP64 CPU oracle for the barrier-elimination example: a synthetic layer-
 * forward tile kernel with the shape of the example the paper analyses
 * (arXiv 2207.00257, Sec. IV-A and IV-B, Fig. 9).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library and its Python binding) never calls it, and this file shares no
 * code, header, table or helper with that path.
 *
 * What it computes. hidden is an R x 16 binary32 matrix (R a multiple of 16)
 * and input an R-vector, cut into tiles of 16 consecutive rows. In tile b,
 * with rows j = 16 b + y (y = 0..15) and columns x = 0..15, let
 *     p[y][x] = hidden[j][x] * input[j]            (the product step),
 * then the tile is reduced over y by a halving tree: at step s = 1..4 the
 * rows y with y mod 2^s == 0 add row y + 2^(s-1). When the tree is done, row
 * y holds the sum of p over rows y .. y + L(y) - 1, where L(y) is the largest
 * power of two dividing y (16 for y = 0): row 0 holds the column sums. The
 * kernel writes every row back into hidden and the 16 column sums of tile b
 * into output[16 b .. 16 b + 15]. Those are the values computed here, in
 * binary64, each sum in row order.
 *
 * Parity status: pinned by CPU tests against closed forms (all-ones and
 * one-hot tiles), an independent matrix-vector product for the column sums,
 * and block sums over the power-of-two row ranges for the tree's rows.
 */
#include <stdint.h>

enum { ORC_LF_OK = 0, ORC_LF_EINVAL = -1 };
enum { LF_TILE = 16 };

/* Largest power of two dividing y, or LF_TILE for y == 0. */
static int span_of(int y) { return y == 0 ? LF_TILE : (y & -y); }

/* new_hidden: R x 16 (the rows after the tree), output: R (16 column sums
 * per tile). */
int oracle_layerforward(const float* hidden, const float* input, int64_t rows, double* new_hidden,
                        double* output) {
  if (rows < 0 || rows % LF_TILE || (rows > 0 && (!hidden || !input || !new_hidden || !output)))
    return ORC_LF_EINVAL;
  for (int64_t b = 0; b < rows / LF_TILE; ++b) {
    for (int y = 0; y < LF_TILE; ++y) {
      const int span = span_of(y);
      for (int x = 0; x < LF_TILE; ++x) {
        double s = 0.0;
        for (int k = y; k < y + span; ++k) {
          const int64_t j = b * LF_TILE + k;
          s += (double)hidden[j * LF_TILE + x] * (double)input[j];
        }
        new_hidden[(b * LF_TILE + y) * LF_TILE + x] = s;
        if (y == 0) output[b * LF_TILE + x] = s;
      }
    }
  }
  return ORC_LF_OK;
}
