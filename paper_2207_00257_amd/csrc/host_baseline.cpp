// Host-side comparison points for the benchmark, built into their own
// library (libnrm_host.so) and loaded only by the benchmark's CPU leg: the
// library behind include/nrm.h never calls them and has no CPU path.
//
//   nrm_host_normalize_mt  the hoisted normalize of arXiv 2207.00257 (Fig. 1
//                          with the sum computed once, Sec. IV-C) as a
//                          multicore CPU program, the kind of code the
//                          paper's transformation emits for a CPU: each of T
//                          threads sums a contiguous chunk in binary64, the
//                          T partials are added in thread order, then the
//                          threads divide their chunks in binary32.
//   nrm_host_copy_mt       a plain multi-threaded copy: the host memory
//                          ceiling the normalize above is compared with.
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

namespace {

template <class F>
void run_chunks(int64_t n, int threads, F&& f) {
  if (threads < 1) threads = 1;
  std::vector<std::thread> pool;
  pool.reserve((size_t)threads);
  const int64_t per = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const int64_t b = std::min<int64_t>(n, (int64_t)t * per), e = std::min<int64_t>(n, b + per);
    pool.emplace_back([&f, t, b, e] { f(t, b, e); });
  }
  for (auto& th : pool) th.join();
}

}  // namespace

extern "C" {

// out[i] = in[i] / S, S = sum of in[0..n) in binary64 (per-thread partials
// added in thread order), divided in binary32. Returns S through *sum.
// Returns 0, or -1 for bad arguments.
int nrm_host_normalize_mt(float* out, const float* in, int64_t n, int threads, double* sum) {
  if (n < 0 || (n > 0 && (!in || !out)) || threads < 1) return -1;
  std::vector<double> part((size_t)threads, 0.0);
  run_chunks(n, threads, [&](int t, int64_t b, int64_t e) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = b;
    for (; i + 4 <= e; i += 4) {
      s0 += in[i];
      s1 += in[i + 1];
      s2 += in[i + 2];
      s3 += in[i + 3];
    }
    for (; i < e; ++i) s0 += in[i];
    part[(size_t)t] = (s0 + s1) + (s2 + s3);
  });
  double s = 0.0;
  for (double p : part) s += p;
  const float sf = (float)s;
  run_chunks(n, threads, [&](int, int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) out[i] = in[i] / sf;
  });
  if (sum) *sum = s;
  return 0;
}

// Copies `bytes` bytes from src to dst with `threads` threads.
int nrm_host_copy_mt(void* dst, const void* src, int64_t bytes, int threads) {
  if (bytes < 0 || (bytes > 0 && (!dst || !src)) || threads < 1) return -1;
  char* d = static_cast<char*>(dst);
  const char* s = static_cast<const char*>(src);
  run_chunks(bytes, threads, [&](int, int64_t b, int64_t e) { std::memcpy(d + b, s + b, (size_t)(e - b)); });
  return 0;
}

}  // extern "C"
