/* Drives every exported function of the C oracle (oracle/*.c) over small
 * inputs and their edge cases (empty, one element, empty CSR rows, every
 * storage type, invalid arguments), so that tests/test_sched_cpu.py can run
 * the oracle under AddressSanitizer and UndefinedBehaviorSanitizer. The
 * values themselves are pinned elsewhere; here only a few invariants are
 * checked. Exit status 0: no check failed (the sanitizers abort on their
 * own findings). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_decode(const void* in, int dtype, int64_t n, double* out);
double oracle_sum(const void* in, int dtype, int64_t n);
int oracle_normalize(const void* in, int dtype, int64_t n, double* out, double* sum_out);
int oracle_normalize_naive(const void* in, int dtype, int64_t n, double* out);
int oracle_normalize_perblock(const void* in, int dtype, int64_t n, int64_t block, double* out);
int oracle_normalize_batched(const void* in, int dtype, const int64_t* offsets, int64_t rows, double* out,
                             double* sums);
uint16_t oracle_round_bf16_one(double x);
int oracle_round_bf16(const double* x, int64_t n, uint16_t* out);
int oracle_softmax_batched(const float* x, const int64_t* offsets, int64_t rows, double* out, double* lse);
int oracle_nll_loss(const float* logp, const int64_t* target, const float* weight, int64_t n, int64_t c,
                    int64_t ignore_index, int reduction, double* out, double* total_weight);
int oracle_layerforward(const float* hidden, const float* input, int64_t rows, double* new_hidden,
                        double* output);

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

/* malloc'd exactly n elements (so that the sanitizer sees any overrun) */
static void* exact(size_t bytes) { return malloc(bytes ? bytes : 1); }

int main(void) {
  static const int64_t sizes[] = {0, 1, 2, 3, 17, 64, 257, 1000};
  for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]); ++si) {
    const int64_t n = sizes[si];
    float* f = exact(sizeof(float) * (size_t)n);
    uint16_t* h = exact(sizeof(uint16_t) * (size_t)n);
    double* out = exact(sizeof(double) * (size_t)n);
    uint16_t* r16 = exact(sizeof(uint16_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
      f[i] = 0.5f + (float)((i * 37) % 101) / 101.0f;
      h[i] = (uint16_t)(0x3F00 + (i * 13) % 200); /* positive BF16 and FP16 patterns */
    }
    for (int dt = 0; dt < 3; ++dt) {
      const void* in = dt == 0 ? (const void*)f : (const void*)h;
      double s = 0.0;
      CHECK(oracle_decode(in, dt, n, out) == 0);
      const double tot = oracle_sum(in, dt, n);
      CHECK(oracle_normalize(in, dt, n, out, &s) == 0);
      CHECK(s == tot);
      if (n > 0) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) acc += out[i];
        CHECK(fabs(acc - 1.0) < 1e-12);
      }
      CHECK(oracle_normalize_naive(in, dt, n, out) == 0);
      CHECK(oracle_normalize_perblock(in, dt, n, 64, out) == 0);
      CHECK(oracle_round_bf16(out, n, r16) == 0);
    }
    /* CSR rows over the same array: an empty row first and last */
    int64_t offs[5] = {0, 0, n / 3, n, n};
    double sums[4];
    CHECK(oracle_normalize_batched(f, 0, offs, 4, out, sums) == 0);
    double lse[4];
    CHECK(oracle_softmax_batched(f, offs, 4, out, lse) == 0);
    free(f);
    free(h);
    free(out);
    free(r16);
  }
  /* invalid arguments are rejected, not read */
  double d;
  CHECK(oracle_normalize(NULL, 0, -1, &d, NULL) != 0);
  CHECK(oracle_normalize(NULL, 7, 3, &d, NULL) != 0);
  int64_t bad[3] = {0, 5, 2};
  float x[8] = {1, 2, 3, 4, 5, 6, 7, 8};
  double o8[8];
  CHECK(oracle_normalize_batched(x, 0, bad, 2, o8, NULL) != 0);
  CHECK(oracle_softmax_batched(x, bad, 2, o8, NULL) != 0);
  (void)oracle_round_bf16_one(1.0 / 3.0);
  (void)oracle_round_bf16_one(NAN);
  (void)oracle_round_bf16_one(INFINITY);
  /* NLL loss: 5 samples, 4 classes, one ignored */
  float logp[20];
  for (int i = 0; i < 20; ++i) logp[i] = -0.25f * (float)(i % 7) - 0.1f;
  int64_t target[5] = {0, 3, -100, 2, 1};
  float w[4] = {1.0f, 0.5f, 2.0f, 1.5f};
  double loss[5], tw;
  CHECK(oracle_nll_loss(logp, target, w, 5, 4, -100, 0, loss, NULL) == 0);
  CHECK(oracle_nll_loss(logp, target, w, 5, 4, -100, 1, loss, &tw) == 0);
  CHECK(oracle_nll_loss(logp, target, NULL, 5, 4, -100, 2, loss, &tw) == 0);
  CHECK(oracle_nll_loss(logp, target, w, 0, 4, -100, 2, loss, &tw) == 0);
  CHECK(oracle_nll_loss(logp, target, w, 5, 0, -100, 0, loss, NULL) != 0);
  /* layer forward: two tiles */
  float* hid = exact(sizeof(float) * 32 * 16);
  float in32[32];
  for (int i = 0; i < 32 * 16; ++i) hid[i] = 0.5f + (float)(i % 9) / 9.0f;
  for (int i = 0; i < 32; ++i) in32[i] = 0.0625f;
  double* nh = exact(sizeof(double) * 32 * 16);
  double out32[32];
  CHECK(oracle_layerforward(hid, in32, 32, nh, out32) == 0);
  CHECK(oracle_layerforward(hid, in32, 17, nh, out32) != 0);
  free(hid);
  free(nh);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("oracle_san: all passed\n");
  return 0;
}
