/*
 * FP64 CPU oracle for normalize(out, in, n): out[i] = in[i] / sum(in[0..n)).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library and its Python binding) never calls it, and this file shares no
 * code, header, table or helper with that path.
 *
 * What it follows (arXiv 2207.00257):
 *   - Fig. 1 (the `normalize` kernel and its `launch`): every thread computes
 *     sum(in, n) itself and then writes in[tid] / sum for tid < n. This is
 *     oracle_normalize_naive below, O(n^2) work.
 *   - The commented-out shared-memory variant of Fig. 1 and its MLIR form in
 *     Fig. 3: thread 0 of each block computes the sum into block-shared storage,
 *     a block barrier follows, then every thread divides. O(n^2 / B) work. This
 *     is oracle_normalize_perblock.
 *   - Fig. 1 caption, Sec. II-A (GPU Compilation) and Sec. IV-C (parallel
 *     loop-invariant code motion): the sum is loop-invariant, so it may be
 *     computed once before the parallel loop, giving O(n) work without changing
 *     the result. This is oracle_normalize, the reference every test uses.
 *   - The body of `sum` is elided in the paper. Here it is the plain definition
 *     sum_{j<n} in[j], accumulated sequentially in index order in binary64.
 *     All three forms call the same sum routine, so they agree bit for bit:
 *     that agreement is the legality claim of the hoist made executable.
 *
 * Precision: every input element is first widened exactly to binary64 from its
 * storage type (FP32, BF16 or FP16, decoded here from the IEEE bit layouts);
 * the sum and the division are binary64 with IEEE semantics (x/0 -> +-inf,
 * 0/0 -> NaN, NaN propagates). Build with -ffp-contract=off and without
 * -ffast-math so the compiler keeps this arithmetic as written.
 *
 * Ragged batched form: rows are CSR slices [offsets[r], offsets[r+1]) of one
 * flat array; each row is normalized on its own (the batched workload defined
 * for this library: a batch of independent normalize calls).
 *
 * Parity status of every function is pinned by CPU tests against closed
 * forms, exact rational arithmetic, brute force and library decoders.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

enum { ORC_F32 = 0, ORC_BF16 = 1, ORC_F16 = 2 };
enum { ORC_OK = 0, ORC_EINVAL = -1 };

/* ---- exact widening from storage types (IEEE 754 bit layouts) ---------- */

/* binary32 -> binary64 is exact; the cast is the definition. */
static double widen_f32(const float* p, int64_t i) { return (double)p[i]; }

/* bfloat16 is the top half of a binary32: sign(1) exponent(8) fraction(7).
 * Decode the fields directly: value = (-1)^s * 2^(e-127) * (1 + f/128) for
 * 0 < e < 255, 2^-126 * f/128 for e == 0, inf/NaN for e == 255. */
static double decode_bf16(uint16_t h) {
  int s = (h >> 15) & 1;
  int e = (h >> 7) & 0xFF;
  int f = h & 0x7F;
  double v;
  if (e == 0xFF) {
    v = f ? NAN : INFINITY;
  } else if (e == 0) {
    v = ldexp((double)f, -126 - 7);
  } else {
    v = ldexp(128.0 + (double)f, e - 127 - 7);
  }
  return s ? -v : v;
}

/* binary16: sign(1) exponent(5) fraction(10), bias 15. */
static double decode_f16(uint16_t h) {
  int s = (h >> 15) & 1;
  int e = (h >> 10) & 0x1F;
  int f = h & 0x3FF;
  double v;
  if (e == 0x1F) {
    v = f ? NAN : INFINITY;
  } else if (e == 0) {
    v = ldexp((double)f, -14 - 10);
  } else {
    v = ldexp(1024.0 + (double)f, e - 15 - 10);
  }
  return s ? -v : v;
}

static double load(const void* in, int dtype, int64_t i) {
  switch (dtype) {
    case ORC_F32: return widen_f32((const float*)in, i);
    case ORC_BF16: return decode_bf16(((const uint16_t*)in)[i]);
    default: return decode_f16(((const uint16_t*)in)[i]);
  }
}

static int valid_dtype(int dtype) { return dtype == ORC_F32 || dtype == ORC_BF16 || dtype == ORC_F16; }

int oracle_decode(const void* in, int dtype, int64_t n, double* out) {
  if (n < 0 || !valid_dtype(dtype) || (n > 0 && (!in || !out))) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i) out[i] = load(in, dtype, i);
  return ORC_OK;
}

/* ---- the elided `sum` of Fig. 1: sum_{j<n} in[j], sequential binary64 --- */

static double sum_seq(const void* in, int dtype, int64_t begin, int64_t end) {
  double s = 0.0;
  for (int64_t j = begin; j < end; ++j) s += load(in, dtype, j);
  return s;
}

double oracle_sum(const void* in, int dtype, int64_t n) {
  if (n <= 0 || !valid_dtype(dtype) || !in) return 0.0;
  return sum_seq(in, dtype, 0, n);
}

/* ---- hoisted form: the invariant sum once, then the element-wise divide -- */

int oracle_normalize(const void* in, int dtype, int64_t n, double* out, double* sum_out) {
  if (n < 0 || !valid_dtype(dtype) || (n > 0 && (!in || !out))) return ORC_EINVAL;
  double s = n > 0 ? sum_seq(in, dtype, 0, n) : 0.0;
  for (int64_t i = 0; i < n; ++i) out[i] = load(in, dtype, i) / s;
  if (sum_out) *sum_out = s;
  return ORC_OK;
}

/* ---- Fig. 1 as written: each thread of a <<<ceil(n/32), 32>>> launch calls
 * sum itself. Thread ids enumerate [0, 32*ceil(n/32)) once each (the element-
 * wise reading of the kernel: every out[i], i < n, is written exactly once). */

int oracle_normalize_naive(const void* in, int dtype, int64_t n, double* out) {
  if (n < 0 || !valid_dtype(dtype) || (n > 0 && (!in || !out))) return ORC_EINVAL;
  const int64_t block = 32;
  const int64_t grid = (n + block - 1) / block;
  for (int64_t b = 0; b < grid; ++b) {
    for (int64_t t = 0; t < block; ++t) {
      double val = sum_seq(in, dtype, 0, n); /* recomputed by every thread */
      int64_t tid = b * block + t;
      if (tid < n) out[tid] = load(in, dtype, tid) / val;
    }
  }
  return ORC_OK;
}

/* ---- the shared-memory variant (Fig. 1 comments, Fig. 3): one sum per block
 * stored in block-shared storage, a barrier, then all threads divide. The
 * barrier is implicit in running the two phases one after the other. */

int oracle_normalize_perblock(const void* in, int dtype, int64_t n, int64_t block, double* out) {
  if (n < 0 || block <= 0 || !valid_dtype(dtype) || (n > 0 && (!in || !out))) return ORC_EINVAL;
  const int64_t grid = (n + block - 1) / block;
  for (int64_t b = 0; b < grid; ++b) {
    double shared_val = sum_seq(in, dtype, 0, n); /* thread 0 of block b */
    /* barrier */
    for (int64_t t = 0; t < block; ++t) {
      int64_t tid = b * block + t;
      if (tid < n) out[tid] = load(in, dtype, tid) / shared_val;
    }
  }
  return ORC_OK;
}

/* ---- ragged batched: independent hoisted normalize per CSR row ---------- */

int oracle_normalize_batched(const void* in, int dtype, const int64_t* offsets, int64_t rows,
                             double* out, double* row_sums) {
  if (rows < 0 || !valid_dtype(dtype) || (rows > 0 && !offsets)) return ORC_EINVAL;
  for (int64_t r = 0; r < rows; ++r) {
    int64_t b = offsets[r], e = offsets[r + 1];
    if (b < 0 || e < b) return ORC_EINVAL;
  }
  for (int64_t r = 0; r < rows; ++r) {
    int64_t b = offsets[r], e = offsets[r + 1];
    double s = e > b ? sum_seq(in, dtype, b, e) : 0.0;
    for (int64_t i = b; i < e; ++i) out[i] = load(in, dtype, i) / s;
    if (row_sums) row_sums[r] = s;
  }
  return ORC_OK;
}

/* ---- round binary64 to the nearest bfloat16, ties to even -------------
 * Used to state which BF16 output is the correctly rounded one. Works on the
 * exact binary64 value (no detour through binary32, which could round twice).
 * bfloat16 has 8 significant bits, exponent range as binary32. */

uint16_t oracle_round_bf16_one(double x) {
  if (isnan(x)) return 0x7FC0;
  uint16_t sign = signbit(x) ? 0x8000 : 0;
  double a = fabs(x);
  if (isinf(a)) return sign | 0x7F80;
  if (a == 0.0) return sign;
  /* quantum of the bfloat16 binade containing a (subnormals: 2^-133) */
  int e;
  frexp(a, &e); /* a = m * 2^e, 0.5 <= m < 1, so the leading bit is 2^(e-1) */
  int lead = e - 1;
  if (lead < -126) lead = -126;
  double q = ldexp(1.0, lead - 7);
  double k = a / q; /* exact: a has at most 53 bits, q is a power of two */
  double kf = floor(k);
  double rem = k - kf; /* exact */
  double kr;
  if (rem > 0.5) kr = kf + 1.0;
  else if (rem < 0.5) kr = kf;
  else kr = fmod(kf, 2.0) == 0.0 ? kf : kf + 1.0;
  double r = kr * q;
  /* encode r: overflow beyond the largest finite bfloat16 rounds to inf */
  const double maxbf = ldexp(255.0, 127 - 7); /* (2 - 2^-7) * 2^127 */
  if (r > maxbf) return sign | 0x7F80;
  if (r < ldexp(1.0, -126)) {
    /* subnormal or rounded up to the smallest normal */
    int64_t f = (int64_t)(r / ldexp(1.0, -133));
    return sign | (uint16_t)f; /* f == 128 encodes the smallest normal */
  }
  int re;
  double rm = frexp(r, &re); /* r = rm * 2^re */
  int biased = re - 1 + 127;
  int64_t frac = (int64_t)ldexp(rm, 8) - 128; /* 8 significant bits */
  return sign | (uint16_t)(biased << 7) | (uint16_t)frac;
}

int oracle_round_bf16(const double* x, int64_t n, uint16_t* out) {
  if (n < 0 || (n > 0 && (!x || !out))) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i) out[i] = oracle_round_bf16_one(x[i]);
  return ORC_OK;
}
