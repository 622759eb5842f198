// Ragged batched normalize on gfx950: every row of a batch is normalized on
// its own, out_r[i] = in_r[i] / sum(in_r), with the per-row sum hoisted out
// of the element-wise divide exactly as in the plain path (arXiv 2207.00257,
// Fig. 1 and Sec. IV-C), in one persistent launch sequence for the batch.
//
//   batch_count_kernel   (batches of more than 4096 rows of capacity) one
//                        block per round of 1024 rows: the round's counts,
//                        so that the planner's blocks need not scan every
//                        round themselves.
//   batch_plan_kernel    one block per round of 1024 rows: resolves the row
//                        table (from CSR offsets or a descriptor table),
//                        validates it, classifies rows, and by exclusive
//                        scans writes its round's part of the work-item
//                        table (first the tiles of every long row,
//                        ceil(n / tile) each and consecutive per row, then
//                        one item per short row, n <= short_max), of the
//                        long rows' descriptors and starts, and of phase 2's
//                        chunk table.
//   batch_wave_kernel    rows of 0 < n <= wave_max (at most 2048) elements,
//                        one per wavefront (four per wavefront, 16 lanes
//                        each, up to 256), statically: read into registers,
//                        summed across the lanes, divided and written, with
//                        no barrier and no work claim.
//   batch_resident_kernel  rows of up to 2^20 elements held on chip in
//                        segments of 2^14 (one block each) between their read
//                        and their write.
//   batch_phase1_kernel  persistent blocks walk the items. A single-pass item
//                        keeps its row in registers: one read, block sum,
//                        divide, one write. A tile item writes its partial.
//   batch_rowsum_kernel  one block per long row merges the row's tile
//                        partials in a fixed order into the row's sum (the
//                        kernel boundary is the barrier that makes the
//                        partials visible).
//   batch_phase2_kernel  persistent blocks divide equal chunks of the long
//                        rows' concatenation by their rows' sums, so every
//                        block moves the same number of elements.
// Both persistent phases walk their work blockIdx.x, blockIdx.x + gridDim.x,
// ... and fetch the next unit's descriptor while the current one streams.
//
// All per-call inputs are read through fixed pointers (a header and the row
// table in pinned host memory, read once by the planner), so the launches
// can be captured once in a hipGraph and replayed for any batch that fits
// the workspace. A row's summation order
// depends only on its length, its start alignment modulo 128 bytes, its
// dtypes, the accumulation mode and the launch parameters: never on the
// other rows or its position in the batch.
#include "nrm_batch.h"
#include "nrm_device.h"
#include "nrm_rows.h"

namespace nrm {
namespace {

using namespace dev;

// The lse output of a softmax call (device float[rows]), or NULL.
__device__ __forceinline__ float* lse_out(const BatchArgs& a) { return reinterpret_cast<float*>(a.cnt[CNT_LSE]); }

// ---- planner ---------------------------------------------------------------------

constexpr int PLAN_THREADS = 1024;

__device__ __forceinline__ bool valid_dt(int dt) { return dt == NRM_F32 || dt == NRM_BF16 || dt == NRM_F16; }

// Tiles are 2^tile_log2 elements: a shift, not a 64-bit division (which the
// GPU emulates in about a hundred instructions, per lane).
__device__ __forceinline__ int64_t long_tiles(int64_t n, int64_t short_max, int tile_log2) {
  return n <= short_max ? 0 : (n + (int64_t(1) << tile_log2) - 1) >> tile_log2;
}

// A value the same in every lane, moved to scalar registers, so that
// arithmetic on it (a 64-bit division, say) runs once per wavefront.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The raw description of one row: its two CSR offsets, or its table entry.
union RawRow {
  RowDesc d;
  struct {
    int64_t b, e;
  } o;
};

// Loads only, so that several rounds' rows can be in flight at once.
__device__ __forceinline__ RawRow fetch_row(const BatchHeader* h, int64_t r) {
  RawRow x;
  if (h->mode == BATCH_CSR) {
    x.o.b = h->offsets[r];
    x.o.e = h->offsets[r + 1];
  } else {
    x.d = h->table[r];
  }
  return x;
}

// Resolve and validate a fetched row; returns it with n = 0 if invalid.
__device__ __forceinline__ RowDesc resolve_row(const BatchHeader* h, const RawRow& x, int& err) {
  RowDesc d;
  if (h->mode == BATCH_CSR) {
    const int64_t b = x.o.b, e = x.o.e;
    const int si = h->csr_in_dt == NRM_F32 ? 4 : 2, so = h->csr_out_dt == NRM_F32 ? 4 : 2;
    d.in = h->csr_in + b * si;
    d.out = h->csr_out + b * so;
    d.n = e - b;
    d.in_dt = h->csr_in_dt;
    d.out_dt = h->csr_out_dt;
    if (b < 0 || e < b || e > h->capacity) {
      err |= NRM_DEVERR_OFFSETS;
      d.n = 0;
    }
  } else {
    d = x.d;
    if (d.n < 0 || !valid_dt(d.in_dt) || !valid_dt(d.out_dt) || (d.n > 0 && (!d.in || !d.out))) {
      err |= NRM_DEVERR_ROW;
      d.n = 0;
    }
  }
  return d;
}

// Per-row counters of the planner: tile items, single-pass item, long row,
// elements of a long row.
constexpr int NCNT = 4;
constexpr int PLAN_WAVES = PLAN_THREADS / 64;

// Wavefront scans with DPP lane moves (a few cycles a step, no LDS):
// row_shr by 1, 2, 4 and 8 scans each row of 16 lanes (lanes shifted in from
// outside the row read 0); the totals of rows 0..2 (lanes 15, 31, 47) are then
// added to the rows after them. A 64-bit value moves as two 32-bit halves.
template <int N>
__device__ __forceinline__ uint32_t row_shr(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x110 + N, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t row_scan32(uint32_t x) {
  x += row_shr<1>(x);
  x += row_shr<2>(x);
  x += row_shr<4>(x);
  x += row_shr<8>(x);
  return x;
}

template <int N>
__device__ __forceinline__ void add_shr64(uint32_t& lo, uint32_t& hi) {
  const uint32_t slo = row_shr<N>(lo), shi = row_shr<N>(hi);
  const uint32_t nlo = lo + slo;
  hi = hi + shi + (nlo < lo ? 1u : 0u);
  lo = nlo;
}

__device__ __forceinline__ uint64_t row_scan64(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  add_shr64<1>(lo, hi);
  add_shr64<2>(lo, hi);
  add_shr64<4>(lo, hi);
  add_shr64<8>(lo, hi);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t lane_value64(uint64_t x, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_scan32(uint32_t x, int lane) {
  x = row_scan32(x);
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
  if (lane >= 16) x += r0;
  if (lane >= 32) x += r1;
  if (lane >= 48) x += r2;
  return x;
}

__device__ __forceinline__ uint64_t wave_scan64(uint64_t x, int lane) {
  x = row_scan64(x);
  const uint64_t r0 = lane_value64(x, 15), r1 = lane_value64(x, 31), r2 = lane_value64(x, 47);
  if (lane >= 16) x += r0;
  if (lane >= 32) x += r1;
  if (lane >= 48) x += r2;
  return x;
}

// Inclusive block-wide scan of the NCNT counters, and their block totals in
// last. Each wavefront scans its lanes and leaves its totals in sc; after one
// barrier every wavefront scans the PLAN_WAVES (= 16, one DPP row) totals
// itself and adds those of the wavefronts before it. The first three
// counters of one round fit 32 bits (at most PLAN_THREADS * MAX_ROW_TILES);
// the element count takes 64. The caller must pass a barrier before sc is
// written again.
static_assert(PLAN_WAVES == 16, "the cross-wavefront scan is one DPP row");
__device__ __forceinline__ void scan_counts(int64_t (&v)[NCNT], int64_t (&last)[NCNT], int64_t (*sc)[PLAN_WAVES]) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int k = 0; k < NCNT - 1; ++k) v[k] = (int64_t)wave_scan32((uint32_t)v[k], lane);
  v[NCNT - 1] = (int64_t)wave_scan64((uint64_t)v[NCNT - 1], lane);
  if (lane == 63)
    for (int k = 0; k < NCNT; ++k) sc[k][wave] = v[k];
  lds_barrier();
#pragma unroll
  for (int k = 0; k < NCNT - 1; ++k) {
    const uint32_t w = row_scan32(lane < PLAN_WAVES ? (uint32_t)sc[k][lane] : 0u);
    if (wave > 0) v[k] += (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)w, wave - 1);
    last[k] = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)w, PLAN_WAVES - 1);
  }
  const uint64_t w = row_scan64(lane < PLAN_WAVES ? (uint64_t)sc[NCNT - 1][lane] : 0u);
  if (wave > 0) v[NCNT - 1] += (int64_t)lane_value64(w, wave - 1);
  last[NCNT - 1] = (int64_t)lane_value64(w, PLAN_WAVES - 1);
}

// Block totals of the NCNT per-thread 64-bit values v (any magnitude, unlike
// scan_counts' 32-bit counters), the same in every thread. The caller must
// pass a barrier before sc is written again.
__device__ __forceinline__ void block_totals(const int64_t (&v)[NCNT], int64_t (&tot)[NCNT],
                                             int64_t (*sc)[PLAN_WAVES]) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int k = 0; k < NCNT; ++k) {
    const int64_t w = (int64_t)wave_scan64((uint64_t)v[k], lane);
    if (lane == 63) sc[k][wave] = w;
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < NCNT; ++k) {
    int64_t x = 0;
#pragma unroll
    for (int j = 0; j < PLAN_WAVES; ++j) x += sc[k][j];
    tot[k] = uniform64(x);  // the same in every lane: scalar registers
  }
}

// Items of a row that is not long: one single-pass item, or with resident
// rows one per segment of 2^RES_LOG2 elements; a row of the short rows'
// kernel (0 < n <= wave_max) has none.
__device__ __forceinline__ void row_counts(int64_t n, const BatchArgs& a, int64_t (&v)[NCNT]) {
  const bool wave = n > 0 && n <= a.wave_max;
  v[0] = wave ? 0 : long_tiles(n, a.short_max, a.tile_log2);
  v[1] = (!wave && n > 0 && n <= a.short_max) ? (a.res_on ? (n + (int64_t(1) << RES_LOG2) - 1) >> RES_LOG2 : 1) : 0;
  v[2] = v[0] > 0 ? 1 : 0;
  v[3] = v[0] > 0 ? n : 0;
}

// For each of S values x[u]: the last j in [0, PLAN_THREADS) with
// ex[j] <= x[u], for a non-decreasing ex with ex[0] = 0 <= x[u] (the thread
// whose range [ex[j], ex[j] + count) holds x[u]). The S binary searches are
// interleaved so that their dependent LDS reads overlap.
template <int S, typename T>
__device__ __forceinline__ void last_le(const T* ex, const int64_t (&x)[S], int (&j)[S]) {
#pragma unroll
  for (int u = 0; u < S; ++u) j[u] = 0;
#pragma unroll
  for (int step = PLAN_THREADS / 2; step > 0; step >>= 1)
#pragma unroll
    for (int u = 0; u < S; ++u)
      if ((int64_t)ex[j[u] + step] <= x[u]) j[u] += step;
}

constexpr int PLAN_SEARCHES = 4;  // binary searches in flight per thread

// Rows are taken PLAN_THREADS at a time ("rounds"), row q * PLAN_THREADS + t
// in thread t (coalesced reads of the offsets or of the table). Block b owns
// round b: it alone stores that round's resolved rows and writes its part of
// the tables; blocks past the last round return at once (the grid is sized
// for the workspace's row capacity, so that a captured graph fits any batch).
//
// Pass 1: resolve and validate the round's rows and count, by a block scan,
// their tile items, single-pass items, long rows and long-row elements. A
// block needs the totals before its own round and the grand totals. Up to
// PLAN_SPLIT_ROWS rows of capacity each block scans all rounds itself (a few
// us per round; rows fetched PLAN_ROUNDS rounds at a time, one round trip)
// and the blocks never wait on one another. Above, the counting launch has
// left every round's totals, and each block scans only its own round and
// adds up the others' totals (every thread a share of the rounds, then the
// block): the planner's time no longer grows with the rounds.
//
// Pass 2 (own round only): each short row's item and each long row's first
// item, descriptor and start in the long rows' concatenation (one thread per
// row); then, cooperatively, the round's tile items and its chunks of the
// chunk table, each entry finding its row by a binary search over the
// round's scan in LDS.
//
// Phase 2 covers the concatenation of the long rows in equal chunks, about
// G * m of them for G phase-2 blocks (m chunks per block, each at most about
// one tile, a multiple of 64 elements, at least one full block-iteration), so
// that every block moves the same number of elements however the row lengths
// fall.
constexpr int PLAN_ROUNDS = 4;
static_assert(PLAN_THREADS == PLAN_ROUND_ROWS, "a round is one planner block's rows");

// A fetched row resolved and validated as the planner takes it: n = 0 if it
// is invalid (error bits in e) or has more tiles than a row's combine merges.
__device__ __forceinline__ RowDesc plan_row(const BatchArgs& a, const BatchHeader* h, const RawRow& x, int& e) {
  RowDesc d = resolve_row(h, x, e);
  if (long_tiles(d.n, a.short_max, a.tile_log2) > MAX_ROW_TILES) {
    e |= NRM_DEVERR_ROW;
    d.n = 0;
  }
  return d;
}

// The split planner's first launch: block b counts round b's tile items,
// single-pass items, long rows and long-row elements and leaves the totals
// in round_agg[4 b ..]; block 0 also copies the header to device memory for
// the planner's blocks. Errors are left to the planner, which resolves the
// same rows again.
__global__ void __launch_bounds__(PLAN_THREADS) batch_count_kernel(BatchArgs a) {
  __shared__ int64_t sc[NCNT][PLAN_WAVES];
  __shared__ BatchHeader hs;
  const int t = threadIdx.x;
  const int64_t own = blockIdx.x;
  if (t == 0) {
    hs = *a.hdr;  // one read of the header (pinned host memory)
    if (own == 0) *a.hdr_dev = hs;  // read by the planner after the kernel boundary
  }
  lds_barrier();
  const int64_t nrows = hs.nrows;
  if (nrows < 0 || nrows > a.cap_rows) return;  // the planner reports it
  if (own >= (nrows + PLAN_THREADS - 1) / PLAN_THREADS) return;
  const int64_t r = own * PLAN_THREADS + t;
  RowDesc d;
  d.n = 0;
  if (r < nrows) {
    int e = 0;
    d = plan_row(a, &hs, fetch_row(&hs, r), e);
  }
  int64_t v[NCNT], last[NCNT];
  row_counts(d.n, a, v);
  scan_counts(v, last, sc);
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NCNT; ++k) a.round_agg[own * NCNT + k] = last[k];
  }
}

template <bool SPLIT>
__global__ void __launch_bounds__(PLAN_THREADS) batch_plan_kernel(BatchArgs a) {
  __shared__ int64_t sc[NCNT][PLAN_WAVES];
  __shared__ BatchHeader hs;
  __shared__ int32_t ex_tile[PLAN_THREADS];  // the own round's exclusive scans
  __shared__ int32_t ex_lrow[PLAN_THREADS];
  __shared__ int64_t ex_elem[PLAN_THREADS];
  __shared__ int32_t ex_short[PLAN_THREADS];
  const int t = threadIdx.x;
  const int64_t own = blockIdx.x;
  // one read of the header: from pinned host memory, or split, from the
  // counting launch's copy in device memory
  if (t == 0) hs = SPLIT ? *a.hdr_dev : *a.hdr;
  lds_barrier();
  const BatchHeader* h = &hs;
  const int64_t nrows = h->nrows;
  if (nrows < 0 || nrows > a.cap_rows) {
    if (own == 0 && t == 0) {
      atomicOr(a.error, NRM_DEVERR_CAPACITY);
      for (int k = 0; k < CNT_DISPENSE; ++k) a.cnt[k] = 0;  // the call number stays
      a.cnt[CNT_ROWS] = 0;
    }
    return;
  }
  const int64_t rounds = (nrows + PLAN_THREADS - 1) / PLAN_THREADS;
  if (own > 0 && own >= rounds) return;  // block 0 stays: it writes the counters
  int err = 0;
  // validate row q * PLAN_THREADS + t (fetched as x); n = 0 if invalid or
  // past the end. Only the owner of the round stores the row and records
  // its errors.
  auto resolve = [&](int64_t q, const RawRow& x, bool mine) -> RowDesc {
    const int64_t r = q * PLAN_THREADS + t;
    RowDesc d;
    d.n = 0;
    if (r >= nrows) return d;
    int e = 0;
    d = plan_row(a, h, x, e);
    if (mine) {
      err |= e;
      a.rows[r] = d;
      if (d.n == 0 && h->lse) h->lse[r] = -__builtin_inff();  // the log of an empty sum
    }
    return d;
  };
  auto fetch = [&](int64_t q) {
    const int64_t r = q * PLAN_THREADS + t;
    RawRow x;
    if (r < nrows) x = fetch_row(h, r);
    return x;
  };

  // pass 1
  int64_t carry[NCNT] = {0, 0, 0, 0};
  int64_t c_own[NCNT] = {0, 0, 0, 0}, incl_own[NCNT] = {0, 0, 0, 0}, last_own[NCNT] = {0, 0, 0, 0};
  RowDesc d_own;
  d_own.n = 0;
  if constexpr (SPLIT) {
    // the own round's rows and scan; the totals of the rounds before it and
    // of all rounds from the counting launch (every thread sums every
    // PLAN_THREADS-th round, then the block adds them up)
    if (own < rounds) {
      d_own = resolve(own, fetch(own), true);
      row_counts(d_own.n, a, incl_own);
      scan_counts(incl_own, last_own, sc);
      lds_barrier();  // sc is rewritten below
    }
    int64_t before[NCNT] = {0, 0, 0, 0}, all[NCNT] = {0, 0, 0, 0};
    for (int64_t q = t; q < rounds; q += PLAN_THREADS)
#pragma unroll
      for (int k = 0; k < NCNT; ++k) {
        const int64_t x = a.round_agg[q * NCNT + k];
        all[k] += x;
        before[k] += q < own ? x : 0;
      }
    block_totals(before, c_own, sc);
    lds_barrier();
    block_totals(all, carry, sc);
  }
  for (int64_t q0 = 0; !SPLIT && q0 < rounds; q0 += PLAN_ROUNDS) {
    RawRow fetched[PLAN_ROUNDS];
#pragma unroll
    for (int k = 0; k < PLAN_ROUNDS; ++k)
      if (q0 + k < rounds) fetched[k] = fetch(q0 + k);
#pragma unroll
    for (int k = 0; k < PLAN_ROUNDS; ++k) {
      const int64_t q = q0 + k;
      if (q < rounds) {
        const bool mine = q == own;
        const RowDesc d = resolve(q, fetched[k], mine);
        int64_t incl[NCNT], last[NCNT];
        row_counts(d.n, a, incl);
        scan_counts(incl, last, sc);
        lds_barrier();  // sc is rewritten by the next scan
        if (mine) {
          d_own = d;
          for (int c = 0; c < NCNT; ++c) {
            c_own[c] = carry[c];
            incl_own[c] = incl[c];
            last_own[c] = last[c];
          }
        }
        for (int c = 0; c < NCNT; ++c) carry[c] = uniform64(carry[c] + last[c]);  // scalar registers
      }
    }
  }
  const int64_t total_long = carry[0], total = carry[0] + carry[1], n_lrows = carry[2], elems = carry[3];

  // phase-2 chunks: G * m of them when the workspace holds that many
  int64_t chunk = 1, n_chunks = 0;
  if (elems > 0) {
    const int64_t G = a.map_grid;
    int64_t m = (elems + G * a.tile - 1) / (G * a.tile);
    int64_t most = G * (m > 0 ? m : 1);
    if (most > a.cap_chunks) most = a.cap_chunks;
    chunk = (elems + most - 1) / most;
    if (chunk < a.min_chunk) chunk = a.min_chunk;  // small batches: fewer, fully used blocks
    chunk = (chunk + 63) / 64 * 64;  // rows that start on a line keep their chunks on lines
    n_chunks = (elems + chunk - 1) / chunk;
  }

  // pass 2, the own round
  if (total <= a.cap_items && own < rounds) {
    const int64_t q = own, r = q * PLAN_THREADS + t;
    const int64_t(&incl)[NCNT] = incl_own;
    const int64_t(&c)[NCNT] = c_own;
    const int64_t(&last)[NCNT] = last_own;
    int64_t v[NCNT];
    row_counts(d_own.n, a, v);
    ex_tile[t] = (int32_t)(incl[0] - v[0]);  // at most PLAN_THREADS * MAX_ROW_TILES
    ex_lrow[t] = (int32_t)(incl[2] - v[2]);
    ex_elem[t] = incl[3] - v[3];
    ex_short[t] = (int32_t)(incl[1] - v[1]);  // at most PLAN_THREADS * RES_MAX_SEGMENTS
    if (v[2]) {
      const int64_t k = c[2] + incl[2] - 1;
      a.lrow_first[k] = c[0] + incl[0] - v[0];
      a.lrows[k] = d_own;
      a.lstart[k] = c[3] + incl[3] - v[3];
    }
    lds_barrier();
    constexpr int SN = PLAN_SEARCHES;
    for (int64_t i0 = t; i0 < last[0]; i0 += SN * PLAN_THREADS) {
      int64_t x[SN];
      int j[SN];
#pragma unroll
      for (int u = 0; u < SN; ++u) x[u] = i0 + u * PLAN_THREADS < last[0] ? i0 + u * PLAN_THREADS : 0;
      last_le<SN>(ex_tile, x, j);
#pragma unroll
      for (int u = 0; u < SN; ++u)
        if (i0 + u * PLAN_THREADS < last[0])
          a.items[c[0] + x[u]] = Item{(int32_t)(q * PLAN_THREADS + j[u]), (int32_t)(x[u] - ex_tile[j[u]])};
    }
    // the round's single-pass items, or its resident rows' segments
    for (int64_t i0 = t; i0 < last[1]; i0 += SN * PLAN_THREADS) {
      int64_t x[SN];
      int j[SN];
#pragma unroll
      for (int u = 0; u < SN; ++u) x[u] = i0 + u * PLAN_THREADS < last[1] ? i0 + u * PLAN_THREADS : 0;
      last_le<SN>(ex_short, x, j);
#pragma unroll
      for (int u = 0; u < SN; ++u)
        if (i0 + u * PLAN_THREADS < last[1])
          a.items[total_long + c[1] + x[u]] = Item{(int32_t)(q * PLAN_THREADS + j[u]), (int32_t)(x[u] - ex_short[j[u]])};
    }
    // the chunks whose first element lies in this round's long rows (c[],
    // last[] and chunk are the same in every lane: divide once per wavefront)
    const int64_t c3 = uniform64(c[3]), ch = uniform64(chunk);
    int64_t ce = (c3 + uniform64(last[3]) + ch - 1) / ch;
    if (ce > n_chunks) ce = n_chunks;
    for (int64_t c0 = (c3 + ch - 1) / ch + t; c0 < ce; c0 += SN * PLAN_THREADS) {
      int64_t x[SN];
      int j[SN];
#pragma unroll
      for (int u = 0; u < SN; ++u) x[u] = c0 + u * PLAN_THREADS < ce ? (c0 + u * PLAN_THREADS) * ch - c3 : 0;
      last_le<SN>(ex_elem, x, j);
#pragma unroll
      for (int u = 0; u < SN; ++u)
        if (c0 + u * PLAN_THREADS < ce) a.chunk_lrow[c0 + u * PLAN_THREADS] = (int32_t)(c[2] + ex_lrow[j[u]]);
    }
  }
  if (err) atomicOr(a.error, err);
  if (own == 0 && t == 0) {
    if (total > a.cap_items) {
      atomicOr(a.error, NRM_DEVERR_CAPACITY);
      for (int k = 0; k < CNT_DISPENSE; ++k) a.cnt[k] = 0;  // the call number stays
      a.cnt[CNT_ROWS] = 0;
    } else {
      a.cnt[CNT_ROWS] = nrows;
      a.cnt[CNT_ITEMS] = total;
      a.cnt[CNT_LONG_ITEMS] = total_long;
      a.cnt[CNT_LONG_ROWS] = n_lrows;
      a.cnt[CNT_LONG_ELEMS] = elems;
      a.cnt[CNT_CHUNK] = chunk;
      a.cnt[CNT_CHUNKS] = n_chunks;
      a.cnt[CNT_LSE] = reinterpret_cast<int64_t>(h->lse);
    }
    // a new call: the resident kernel hands out its units from 0 and tags its
    // partials with a number no earlier call of this workspace used (the
    // workspace starts at 0; the count skips 0 when it wraps)
    a.cnt[CNT_DISPENSE] = 0;
    const uint32_t ep = (uint32_t)a.cnt[CNT_EPOCH] + 1u;
    a.cnt[CNT_EPOCH] = ep ? ep : 1u;
  }
}

// ---- single-pass rows (held in registers) --------------------------------------------

template <int DTI, int DTO, int ACC, int KB>
__device__ __forceinline__ void single_pass(const RowDesc& d, Acc<ACC>* slots, RowRes* s_bcast, float* lse,
                                            int64_t row) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int NA = accumulators(DTI, ACC, KB);
  const int B = blockDim.x, t = threadIdx.x;
  const Geom g = geometry<DTI>(d.in, d.n);
  const u4* body = reinterpret_cast<const u4*>(d.in + g.head * Elem<DTI>::SIZE);
  u4 r[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int64_t v = t + (int64_t)k * B;
    if (v < g.nvec) r[k] = load_vec<false>(body + v);
  }
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  if constexpr (ACC == ACC_SOFTMAX) {
    softmax_add_held<DTI, NA, KB>(acc, r, t, B, g.nvec);
  } else {
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      if (t + (int64_t)k * B < g.nvec) {
        float x[VEC];
        widen<DTI>(r[k], x);
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[(k * VEC + c) % NA].add(x[c]);
      }
    }
  }
  if (t < g.head) acc[0].add(load_one<DTI>(d.in, t));
  if (t < d.n - g.tail_begin) acc[0].add(load_one<DTI>(d.in, g.tail_begin + t));
  merge_chains<ACC, NA>(acc);
  Acc<ACC> tot = block_reduce<ACC>(acc[0], slots);
  if (t == 0) {
    const RowMap<ACC> f0 = RowMap<ACC>::of(tot);
    *s_bcast = f0.result();
    if constexpr (ACC == ACC_SOFTMAX) {
      if (lse) lse[row] = f0.lse();
    }
  }
  lds_barrier();
  const RowMap<ACC> f = RowMap<ACC>::of(*s_bcast);
  const bool vec_ok = out_vector_ok<DTI, DTO>(d.out, g.head);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int64_t v = t + (int64_t)k * B;
    if (v < g.nvec) {
      float x[VEC], q[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int c = 0; c < VEC; ++c) q[c] = f(x[c]);
      store_quotients<DTI, DTO>(d.out, g.head, v, vec_ok, q);
    }
  }
  if (t < g.head) store_one<DTO>(d.out, t, f(load_one<DTI>(d.in, t)));
  if (t < d.n - g.tail_begin) {
    const int64_t i = g.tail_begin + t;
    store_one<DTO>(d.out, i, f(load_one<DTI>(d.in, i)));
  }
}

// ---- tiles of long rows ------------------------------------------------------------

// Sum of elements [b, e) of a row; valid in thread 0. NT: non-temporal loads
// (a temporal tile stays in the last-level cache for phase 2).
template <int DTI, int ACC, int U, bool NT>
__device__ __forceinline__ Acc<ACC> tile_reduce(const char* in_row, int64_t b, int64_t e,
                                                Acc<ACC>* slots) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int NA = accumulators(DTI, ACC, U);
  constexpr int FLUSH = CHAIN_ADDS / adds_per_iteration(DTI, ACC, U);
  const char* seg = in_row + b * Elem<DTI>::SIZE;
  const int64_t n = e - b;
  const Geom g = geometry<DTI>(seg, n);
  const u4* p = reinterpret_cast<const u4*>(seg + g.head * Elem<DTI>::SIZE) + threadIdx.x;
  const int64_t B = blockDim.x, step = B * U;
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  Acc<ACC> run;
  run.zero();
  int since_flush = 0;
  // the unaligned head and the short tail, loaded before the stream so their
  // latency overlaps it
  const bool has_head = (int64_t)threadIdx.x < g.head;
  const bool has_tail = (int64_t)threadIdx.x < n - g.tail_begin;
  const float xh = has_head ? load_one<DTI>(seg, threadIdx.x) : 0.0f;
  const float xt = has_tail ? load_one<DTI>(seg, g.tail_begin + threadIdx.x) : 0.0f;
  for (int64_t base = 0; base < g.nvec; base += step) {
    if (base + step <= g.nvec) {
      u4 r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load_vec<NT>(p + base + u * B);
      if constexpr (ACC == ACC_SOFTMAX) {
        // full iterations keep the chains' k equal (see raise_shared); only
        // the last iteration of a tile can be partial, and it and the head
        // and tail raise their chains element by element
        float x[U][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) widen<DTI>(r[u], x[u]);
        float m = x[0][0];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int c = 0; c < VEC; ++c) m = fmaxf(m, x[u][c]);
        raise_shared<NA>(acc, m);
        const float nk = -acc[0].k;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int c = 0; c < VEC; ++c)
            acc[(u * VEC + c) % NA].s += __builtin_amdgcn_exp2f(__builtin_fmaf(x[u][c], LOG2E_F, nk));
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float x[VEC];
          widen<DTI>(r[u], x);
#pragma unroll
          for (int c = 0; c < VEC; ++c) acc[(u * VEC + c) % NA].add(x[c]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (base + u * B + (int64_t)threadIdx.x < g.nvec) {
          float x[VEC];
          widen<DTI>(load_vec<NT>(p + base + u * B), x);
#pragma unroll
          for (int c = 0; c < VEC; ++c) acc[(u * VEC + c) % NA].add(x[c]);
        }
      }
    }
    if constexpr (ACC != NRM_ACC_KAHAN) {
      if (++since_flush == FLUSH) {
        since_flush = 0;
        merge_chains<ACC, NA>(acc);
        run.merge(acc[0]);
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k].zero();
      }
    }
  }
  if (has_head) acc[0].add(xh);
  if (has_tail) acc[0].add(xt);
  merge_chains<ACC, NA>(acc);
  run.merge(acc[0]);
  return block_reduce<ACC>(run, slots);
}

// out[i] = f(in[i]) for elements [b, e) of a row.
template <int DTI, int DTO, int U, class F>
__device__ __forceinline__ void tile_map(const RowDesc& d, int64_t b, int64_t e, const F& f) {
  constexpr int VEC = Elem<DTI>::VEC;
  const char* in_seg = d.in + b * Elem<DTI>::SIZE;
  char* out_seg = d.out + b * Elem<DTO>::SIZE;
  const int64_t n = e - b;
  const Geom g = geometry<DTI>(in_seg, n);
  const u4* body = reinterpret_cast<const u4*>(in_seg + g.head * Elem<DTI>::SIZE);
  const bool vec_ok = out_vector_ok<DTI, DTO>(out_seg, g.head);
  const int64_t B = blockDim.x, step = B * U;
  const bool has_head = (int64_t)threadIdx.x < g.head;
  const int64_t ti = g.tail_begin + threadIdx.x;
  const bool has_tail = ti < n;
  const float xh = has_head ? load_one<DTI>(in_seg, threadIdx.x) : 0.0f;
  const float xt = has_tail ? load_one<DTI>(in_seg, ti) : 0.0f;
  for (int64_t base = 0; base < g.nvec; base += step) {
    const int64_t v0 = base + threadIdx.x;
    if (base + step <= g.nvec) {
      u4 r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load_vec<true>(body + v0 + u * B);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float x[VEC], q[VEC];
        widen<DTI>(r[u], x);
#pragma unroll
        for (int c = 0; c < VEC; ++c) q[c] = f(x[c]);
        store_quotients<DTI, DTO>(out_seg, g.head, v0 + u * B, vec_ok, q);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (v0 + u * B < g.nvec) {
          float x[VEC], q[VEC];
          widen<DTI>(load_vec<true>(body + v0 + u * B), x);
#pragma unroll
          for (int c = 0; c < VEC; ++c) q[c] = f(x[c]);
          store_quotients<DTI, DTO>(out_seg, g.head, v0 + u * B, vec_ok, q);
        }
      }
    }
  }
  if (has_head) store_one<DTO>(out_seg, threadIdx.x, f(xh));
  if (has_tail) store_one<DTO>(out_seg, ti, f(xt));
}

// ---- dtype dispatch of one item --------------------------------------------------------
// The softmax kind is binary32 in and out only (the host rejects anything else).

template <int ACC, int KB>
__device__ __forceinline__ void dispatch_single(const RowDesc& d, Acc<ACC>* slots, RowRes* s_bcast, float* lse,
                                                int64_t row) {
  if constexpr (ACC == ACC_SOFTMAX) {
    single_pass<NRM_F32, NRM_F32, ACC, KB>(d, slots, s_bcast, lse, row);
  } else {
#define NRM_SP(I, O) single_pass<I, O, ACC, KB>(d, slots, s_bcast, lse, row)
    switch (d.in_dt * 3 + d.out_dt) {
      case NRM_F32 * 3 + NRM_F32: NRM_SP(NRM_F32, NRM_F32); break;
      case NRM_F32 * 3 + NRM_BF16: NRM_SP(NRM_F32, NRM_BF16); break;
      case NRM_F32 * 3 + NRM_F16: NRM_SP(NRM_F32, NRM_F16); break;
      case NRM_BF16 * 3 + NRM_F32: NRM_SP(NRM_BF16, NRM_F32); break;
      case NRM_BF16 * 3 + NRM_BF16: NRM_SP(NRM_BF16, NRM_BF16); break;
      case NRM_BF16 * 3 + NRM_F16: NRM_SP(NRM_BF16, NRM_F16); break;
      case NRM_F16 * 3 + NRM_F32: NRM_SP(NRM_F16, NRM_F32); break;
      case NRM_F16 * 3 + NRM_BF16: NRM_SP(NRM_F16, NRM_BF16); break;
      default: NRM_SP(NRM_F16, NRM_F16); break;
    }
#undef NRM_SP
  }
}

template <int ACC, int U, bool NT>
__device__ __forceinline__ Acc<ACC> dispatch_tile_reduce(const RowDesc& d, int64_t b, int64_t e,
                                                         Acc<ACC>* slots) {
  if constexpr (ACC == ACC_SOFTMAX) {
    return tile_reduce<NRM_F32, ACC, U, NT>(d.in, b, e, slots);
  } else {
    switch (d.in_dt) {
      case NRM_F32: return tile_reduce<NRM_F32, ACC, U, NT>(d.in, b, e, slots);
      case NRM_BF16: return tile_reduce<NRM_BF16, ACC, U, NT>(d.in, b, e, slots);
      default: return tile_reduce<NRM_F16, ACC, U, NT>(d.in, b, e, slots);
    }
  }
}

template <int ACC, int U>
__device__ __forceinline__ void dispatch_tile_map(const RowDesc& d, int64_t b, int64_t e, const RowMap<ACC>& f) {
  if constexpr (ACC == ACC_SOFTMAX) {
    tile_map<NRM_F32, NRM_F32, U>(d, b, e, f);
  } else {
#define NRM_TM(I, O) tile_map<I, O, U>(d, b, e, f)
    switch (d.in_dt * 3 + d.out_dt) {
      case NRM_F32 * 3 + NRM_F32: NRM_TM(NRM_F32, NRM_F32); break;
      case NRM_F32 * 3 + NRM_BF16: NRM_TM(NRM_F32, NRM_BF16); break;
      case NRM_F32 * 3 + NRM_F16: NRM_TM(NRM_F32, NRM_F16); break;
      case NRM_BF16 * 3 + NRM_F32: NRM_TM(NRM_BF16, NRM_F32); break;
      case NRM_BF16 * 3 + NRM_BF16: NRM_TM(NRM_BF16, NRM_BF16); break;
      case NRM_BF16 * 3 + NRM_F16: NRM_TM(NRM_BF16, NRM_F16); break;
      case NRM_F16 * 3 + NRM_F32: NRM_TM(NRM_F16, NRM_F32); break;
      case NRM_F16 * 3 + NRM_BF16: NRM_TM(NRM_F16, NRM_BF16); break;
      default: NRM_TM(NRM_F16, NRM_F16); break;
    }
#undef NRM_TM
  }
}

// Persistent blocks take the resident items (after the long rows' tiles in
// the item table) one at a time from the counter.
template <int ACC>
__global__ void __launch_bounds__(RES_BLOCK) __attribute__((amdgpu_waves_per_eu(4, 4))) batch_resident_kernel(BatchArgs a) {
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ RowRes s_bcast;
  __shared__ int64_t s_claim;
  const int64_t begin = a.cnt[CNT_LONG_ITEMS], units = a.cnt[CNT_ITEMS] - begin;
  if (units <= 0) return;
  const uint32_t ep = (uint32_t)a.cnt[CNT_EPOCH];
  float* lse = lse_out(a);
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(a.cnt + CNT_DISPENSE);
  if (threadIdx.x == 0)
    s_claim = (int64_t)__hip_atomic_fetch_add(counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  lds_barrier();
  int64_t u = s_claim;
  while (u < units) {
    const int64_t item = begin + u;
    const Item it = a.items[item];
    const RowDesc d = a.rows[it.row];
    // the row's items are consecutive: its first segment is item - tile
    const int64_t first = item - it.tile;
    const ResExchange x{a.tagged + 2 * first, a.rowtot + 2 * first, a.arrivals + first, ep, a.error,
                        reinterpret_cast<unsigned long long*>(a.cnt + CNT_STALL), nullptr};
    dispatch_resident<ACC>(d, it.tile, x, slots, &s_bcast, lse ? lse + it.row : nullptr);
    // the next item once this one is done (claiming it as soon as the row's
    // sum was known, to overlap the claim with the writes, measured slower)
    lds_barrier();  // slots, s_bcast and s_claim are reused
    if (threadIdx.x == 0)
      s_claim = (int64_t)__hip_atomic_fetch_add(counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lds_barrier();
    u = s_claim;
  }
}

// ---- the persistent phases ------------------------------------------------------------------

template <int ACC, int U, int KB>
__global__ void __launch_bounds__(1024) batch_phase1_kernel(BatchArgs a) {
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ RowRes s_bcast;
  const int64_t n_long = a.cnt[CNT_LONG_ITEMS];
  // with resident rows the items after the long rows' tiles are the
  // resident kernel's
  const int64_t n_items = a.res_on ? n_long : a.cnt[CNT_ITEMS];
  const int64_t keep_item = n_long - a.keep_tiles;
  float* lse = lse_out(a);
  Acc<ACC>* part = reinterpret_cast<Acc<ACC>*>(a.partials);
  const int64_t G = gridDim.x;
  int64_t item = blockIdx.x;
  if (item >= n_items) return;
  Item it = a.items[item];
  RowDesc d = a.rows[it.row];
  Item it_next = item + G < n_items ? a.items[item + G] : it;
  while (true) {
    // Two deep: the next item's descriptor (its index is already here) and
    // the index of the one after are fetched while this item streams.
    const int64_t next = item + G;
    RowDesc d_next = d;
    Item it_after = it_next;
    if (next < n_items) {
      d_next = a.rows[it_next.row];
      if (next + G < n_items) it_after = a.items[next + G];
    }
    if (item >= n_long) {
      dispatch_single<ACC, KB>(d, slots, &s_bcast, lse, it.row);
    } else {
      const int64_t b = (int64_t)it.tile * a.tile;
      const int64_t e = b + a.tile < d.n ? b + a.tile : d.n;
      // the last keep_tiles tiles are read with a temporal hint: phase 2
      // finds them in the last-level cache
      const Acc<ACC> p = item >= keep_item ? dispatch_tile_reduce<ACC, U, false>(d, b, e, slots)
                                           : dispatch_tile_reduce<ACC, U, true>(d, b, e, slots);
      if (threadIdx.x == 0) part[item] = p;  // read after the kernel boundary
    }
    if (next >= n_items) break;
    it = it_next;
    d = d_next;
    it_next = it_after;
    item = next;
    lds_barrier();  // the block's LDS is reused by the next item
  }
}

// Each long row's result from its tile partials, in a fixed order that
// depends only on the number of tiles (combine_partials: one wavefront for up
// to 1024 partials, the LDS tree beyond). One block per long row at a time.
template <int ACC>
__global__ void __launch_bounds__(1024) batch_rowsum_kernel(BatchArgs a) {
  __shared__ Acc<ACC> tree[COMBINE_TILE];
  __shared__ Acc<ACC> tiles[MAX_COMBINE_TILES];
  const int64_t n_lrows = a.cnt[CNT_LONG_ROWS];
  float* lse = lse_out(a);
  const Acc<ACC>* part = reinterpret_cast<const Acc<ACC>*>(a.partials);
  for (int64_t k = blockIdx.x; k < n_lrows; k += gridDim.x) {
    const int64_t first = a.lrow_first[k];
    const int64_t count = (a.lrows[k].n + a.tile - 1) >> a.tile_log2;
    Acc<ACC> tot = combine_partials<ACC>(part + first, count, tree, tiles);
    if (threadIdx.x == 0) {
      const RowMap<ACC> f = RowMap<ACC>::of(tot);
      a.lsum[k] = f.result();
      if constexpr (ACC == ACC_SOFTMAX) {
        if (lse) lse[a.items[first].row] = f.lse();
      }
    }
    lds_barrier();  // the trees are reused by the next row
  }
}

// Phase 2 walks equal chunks of the long rows' concatenation: chunk c covers
// positions [c * chunk, (c + 1) * chunk) and starts in long row
// chunk_lrow[c]; a chunk that reaches past its row's end continues in the
// following long rows.
template <int ACC, int U>
__global__ void __launch_bounds__(1024) batch_phase2_kernel(BatchArgs a) {
  const int64_t elems = a.cnt[CNT_LONG_ELEMS], chunk = a.cnt[CNT_CHUNK], n_chunks = a.cnt[CNT_CHUNKS];
  const int64_t G = gridDim.x;
  int64_t c = blockIdx.x;
  if (c >= n_chunks) return;
  int64_t k = a.chunk_lrow[c];
  RowDesc d = a.lrows[k];
  int64_t start = a.lstart[k];
  RowRes R = a.lsum[k];
  int64_t k_next = c + G < n_chunks ? a.chunk_lrow[c + G] : k;
  while (true) {
    // Two deep, as in phase 1: the next chunk's row (its index is already
    // here) and the index of the one after.
    const int64_t next = c + G;
    RowDesc d_next = d;
    int64_t start_next = start;
    RowRes R_next = R;
    int64_t k_after = k_next;
    if (next < n_chunks) {
      d_next = a.lrows[k_next];
      start_next = a.lstart[k_next];
      R_next = a.lsum[k_next];
      if (next + G < n_chunks) k_after = a.chunk_lrow[next + G];
    }
    int64_t pos = c * chunk;
    const int64_t end = pos + chunk < elems ? pos + chunk : elems;
    while (true) {
      const int64_t e = end - start < d.n ? end - start : d.n;
      dispatch_tile_map<ACC, U>(d, pos - start, e, RowMap<ACC>::of(R));
      pos = start + e;
      if (pos >= end) break;
      ++k;  // the chunk continues in the next long row
      d = a.lrows[k];
      start = a.lstart[k];
      R = a.lsum[k];
    }
    if (next >= n_chunks) break;
    c = next;
    k = k_next;
    d = d_next;
    start = start_next;
    R = R_next;
    k_next = k_after;
  }
}

template <int ACC, int U>
hipError_t phase1_kb(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  switch (p.short_regs) {
    case 1: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 1>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    case 2: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 2>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    case 4: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 4>), dim3(p.grid), dim3(p.block), 0, s, a); break;
    default: hipLaunchKernelGGL((batch_phase1_kernel<ACC, U, 8>), dim3(p.grid), dim3(p.block), 0, s, a); break;
  }
  return hipGetLastError();
}

template <int ACC>
hipError_t phase1_u(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  switch (p.unroll) {
    case 1: return phase1_kb<ACC, 1>(p, a, s);
    case 2: return phase1_kb<ACC, 2>(p, a, s);
    case 4: return phase1_kb<ACC, 4>(p, a, s);
    default: return phase1_kb<ACC, 8>(p, a, s);
  }
}

constexpr int64_t ROWSUM_GRID = 1024;

template <int ACC>
hipError_t rowsum_acc(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  // one 64-thread block per long row at a time; more blocks than this only
  // add dispatch work for small batches
  const int64_t grid = p.grid < ROWSUM_GRID ? p.grid : ROWSUM_GRID;
  hipLaunchKernelGGL((batch_rowsum_kernel<ACC>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <int ACC>
hipError_t phase2_acc(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  switch (p.map_unroll) {
    case 1: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 1>), dim3(p.map_grid), dim3(p.map_block), 0, s, a); break;
    case 2: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 2>), dim3(p.map_grid), dim3(p.map_block), 0, s, a); break;
    case 4: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 4>), dim3(p.map_grid), dim3(p.map_block), 0, s, a); break;
    default: hipLaunchKernelGGL((batch_phase2_kernel<ACC, 8>), dim3(p.map_grid), dim3(p.map_block), 0, s, a); break;
  }
  return hipGetLastError();
}

// ---- short rows, one wavefront each ----------------------------------------------------
// A row of 0 < n <= wave_max elements (at most WAVE_MAX_ELEMS) is taken by one
// wavefront: its head, 16-byte vectors and tail are read into registers, summed
// in each lane's chains and across the lanes by DPP moves (no LDS, no barrier,
// no work claim), divided from the registers and written: two HBM transfers,
// and a wavefront never waits for another. The wavefronts walk the batch's
// rows statically (batch_wave_kernel below) and skip the rows the other
// kernels take. A row's summation order depends only on its length, its
// start alignment and its dtypes.
template <int DTI, int DTO, int ACC>
__device__ __forceinline__ void wave_row(const RowDesc& d, float* lse) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int KW = (int)(WAVE_MAX_ELEMS / (64 * VEC));
  constexpr int NA = ACC == NRM_ACC_F32 ? 8 : 4;  // chains per lane (few: registers go to the held row)
  const int lane = threadIdx.x & 63;
  const Geom g = geometry<DTI>(d.in, d.n);
  const u4* body = reinterpret_cast<const u4*>(d.in + g.head * Elem<DTI>::SIZE);
  u4 r[KW];
#pragma unroll
  for (int k = 0; k < KW; ++k)
    if (lane + k * 64 < g.nvec) r[k] = load_vec<false>(body + lane + k * 64);
  const bool has_head = lane < g.head;
  const bool has_tail = lane < d.n - g.tail_begin;
  const float xh = has_head ? load_one<DTI>(d.in, lane) : 0.0f;
  const float xt = has_tail ? load_one<DTI>(d.in, g.tail_begin + lane) : 0.0f;
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  if constexpr (ACC == ACC_SOFTMAX) {
    softmax_add_held<DTI, NA, KW>(acc, r, lane, 64, g.nvec);
  } else {
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      if (lane + k * 64 < g.nvec) {
        float x[VEC];
        widen<DTI>(r[k], x);
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[(k * VEC + c) % NA].add(x[c]);
      }
    }
  }
  if (has_head) acc[0].add(xh);
  if (has_tail) acc[0].add(xt);
  merge_chains<ACC, NA>(acc);
  const RowMap<ACC> f = RowMap<ACC>::of(wave_reduce<ACC>(acc[0]));  // the same in every lane
  if constexpr (ACC == ACC_SOFTMAX) {
    if (lse && lane == 0) *lse = f.lse();
  }
  const bool vec_ok = out_vector_ok<DTI, DTO>(d.out, g.head);
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int64_t v = lane + k * 64;
    if (v < g.nvec) {
      float x[VEC], q[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int c = 0; c < VEC; ++c) q[c] = f(x[c]);
      store_quotients<DTI, DTO>(d.out, g.head, v, vec_ok, q);
    }
  }
  if (has_head) store_one<DTO>(d.out, lane, f(xh));
  if (has_tail) store_one<DTO>(d.out, g.tail_begin + lane, f(xt));
}

template <int ACC>
__device__ __forceinline__ void dispatch_wave(const RowDesc& d, float* lse) {
  if constexpr (ACC == ACC_SOFTMAX) {
    wave_row<NRM_F32, NRM_F32, ACC>(d, lse);
  } else {
#define NRM_WR(I, O) wave_row<I, O, ACC>(d, lse)
    switch (d.in_dt * 3 + d.out_dt) {
      case NRM_F32 * 3 + NRM_F32: NRM_WR(NRM_F32, NRM_F32); break;
      case NRM_F32 * 3 + NRM_BF16: NRM_WR(NRM_F32, NRM_BF16); break;
      case NRM_F32 * 3 + NRM_F16: NRM_WR(NRM_F32, NRM_F16); break;
      case NRM_BF16 * 3 + NRM_F32: NRM_WR(NRM_BF16, NRM_F32); break;
      case NRM_BF16 * 3 + NRM_BF16: NRM_WR(NRM_BF16, NRM_BF16); break;
      case NRM_BF16 * 3 + NRM_F16: NRM_WR(NRM_BF16, NRM_F16); break;
      case NRM_F16 * 3 + NRM_F32: NRM_WR(NRM_F16, NRM_F32); break;
      case NRM_F16 * 3 + NRM_BF16: NRM_WR(NRM_F16, NRM_BF16); break;
      default: NRM_WR(NRM_F16, NRM_F16); break;
    }
#undef NRM_WR
  }
}

// Rows of at most WAVE_QUARTER_MAX elements go four to a wavefront: each
// row of 16 lanes (a DPP row) takes one, so four such rows are in flight
// per wavefront instead of one. The head before the first 16-byte boundary
// (fewer than one vector) and the tail are one element per lane; each lane
// holds at most WAVE_QUARTER_MAX / (16 VEC) vectors; the sum is the 16
// lanes' chains merged by row16_reduce, in every lane of the row.
constexpr int64_t WAVE_QUARTER_MAX = 256;

// What a row of 16 lanes holds of its row between its loads and the rest,
// so that a wavefront's next group of rows can be loaded while the current
// one is summed and written: at most four 16-byte vectors per lane, and the
// lane's head and tail elements.
struct QuarterHeld {
  u4 r[4];
  float xh, xt;
};
static_assert(WAVE_QUARTER_MAX / (16 * 4) <= 4, "a lane holds at most four vectors");

template <int DTI>
struct QuarterGeom {
  int64_t head, nvec, tail_begin;
  __device__ __forceinline__ explicit QuarterGeom(const RowDesc& d) {
    const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(d.in) & 15);
    head = mis ? (16 - mis) / Elem<DTI>::SIZE : 0;
    if (head > d.n) head = d.n;
    nvec = (d.n - head) / Elem<DTI>::VEC;
    tail_begin = head + nvec * Elem<DTI>::VEC;
  }
};

template <int DTI>
__device__ __forceinline__ void quarter_load(const RowDesc& d, QuarterHeld& q) {
  constexpr int KQ = (int)(WAVE_QUARTER_MAX / (16 * Elem<DTI>::VEC));
  const int j = threadIdx.x & 15;
  const QuarterGeom<DTI> g(d);
  const u4* body = reinterpret_cast<const u4*>(d.in + g.head * Elem<DTI>::SIZE);
#pragma unroll
  for (int k = 0; k < KQ; ++k)
    if (j + k * 16 < g.nvec) q.r[k] = load_vec<false>(body + j + k * 16);
  q.xh = j < g.head ? load_one<DTI>(d.in, j) : 0.0f;
  q.xt = j < d.n - g.tail_begin ? load_one<DTI>(d.in, g.tail_begin + j) : 0.0f;
}

template <int DTI, int DTO, int ACC>
__device__ __forceinline__ void quarter_finish(const RowDesc& d, const QuarterHeld& q, float* lse) {
  constexpr int VEC = Elem<DTI>::VEC;
  constexpr int KQ = (int)(WAVE_QUARTER_MAX / (16 * VEC));
  constexpr int NA = ACC == NRM_ACC_F32 ? 8 : 4;
  const int j = threadIdx.x & 15;
  const QuarterGeom<DTI> g(d);
  const bool has_head = j < g.head;
  const bool has_tail = j < d.n - g.tail_begin;
  u4 r[KQ];
#pragma unroll
  for (int k = 0; k < KQ; ++k) r[k] = q.r[k];
  Acc<ACC> acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k].zero();
  if constexpr (ACC == ACC_SOFTMAX) {
    softmax_add_held<DTI, NA, KQ>(acc, r, j, 16, g.nvec);
  } else {
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
      if (j + k * 16 < g.nvec) {
        float x[VEC];
        widen<DTI>(r[k], x);
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[(k * VEC + c) % NA].add(x[c]);
      }
    }
  }
  if (has_head) acc[0].add(q.xh);
  if (has_tail) acc[0].add(q.xt);
  merge_chains<ACC, NA>(acc);
  const RowMap<ACC> f = RowMap<ACC>::of(row16_reduce<ACC>(acc[0]));  // the same in the row's 16 lanes
  if constexpr (ACC == ACC_SOFTMAX) {
    if (lse && j == 0) *lse = f.lse();
  }
  const bool vec_ok = out_vector_ok<DTI, DTO>(d.out, g.head);
#pragma unroll
  for (int k = 0; k < KQ; ++k) {
    const int64_t v = j + k * 16;
    if (v < g.nvec) {
      float x[VEC], qv[VEC];
      widen<DTI>(r[k], x);
#pragma unroll
      for (int c = 0; c < VEC; ++c) qv[c] = f(x[c]);
      store_quotients<DTI, DTO>(d.out, g.head, v, vec_ok, qv);
    }
  }
  if (has_head) store_one<DTO>(d.out, j, f(q.xh));
  if (has_tail) store_one<DTO>(d.out, g.tail_begin + j, f(q.xt));
}

// The dtype switches of a row of each 16-lane group: they may differ between
// the groups (row tables), never within one.
template <int ACC>
__device__ __forceinline__ void dispatch_quarter_load(const RowDesc& d, QuarterHeld& q) {
  if (ACC == ACC_SOFTMAX || d.in_dt == NRM_F32) quarter_load<NRM_F32>(d, q);
  else if (d.in_dt == NRM_BF16) quarter_load<NRM_BF16>(d, q);
  else quarter_load<NRM_F16>(d, q);
}

template <int ACC>
__device__ __forceinline__ void dispatch_quarter_finish(const RowDesc& d, const QuarterHeld& q, float* lse) {
  if constexpr (ACC == ACC_SOFTMAX) {
    quarter_finish<NRM_F32, NRM_F32, ACC>(d, q, lse);
  } else {
#define NRM_QR(I, O) quarter_finish<I, O, ACC>(d, q, lse)
    switch (d.in_dt * 3 + d.out_dt) {
      case NRM_F32 * 3 + NRM_F32: NRM_QR(NRM_F32, NRM_F32); break;
      case NRM_F32 * 3 + NRM_BF16: NRM_QR(NRM_F32, NRM_BF16); break;
      case NRM_F32 * 3 + NRM_F16: NRM_QR(NRM_F32, NRM_F16); break;
      case NRM_BF16 * 3 + NRM_F32: NRM_QR(NRM_BF16, NRM_F32); break;
      case NRM_BF16 * 3 + NRM_BF16: NRM_QR(NRM_BF16, NRM_BF16); break;
      case NRM_BF16 * 3 + NRM_F16: NRM_QR(NRM_BF16, NRM_F16); break;
      case NRM_F16 * 3 + NRM_F32: NRM_QR(NRM_F16, NRM_F32); break;
      case NRM_F16 * 3 + NRM_BF16: NRM_QR(NRM_F16, NRM_BF16); break;
      default: NRM_QR(NRM_F16, NRM_F16); break;
    }
#undef NRM_QR
  }
}

// Two static walks, one after the other (their registers are not live at
// once): wavefront w of W first takes the groups of four consecutive rows
// 4w, 4(w + W), ..., and runs the group's rows of at most WAVE_QUARTER_MAX
// elements, each on its 16 lanes, all at once, with the next group's rows
// loaded before the current group is summed and written; then it takes rows
// w, w + W, ... and runs those of WAVE_QUARTER_MAX < n <= wave_max elements
// on the whole wavefront, fetching the next descriptor while a row streams.
template <int ACC>
__global__ void __launch_bounds__(WAVE_BLOCK) batch_wave_kernel(BatchArgs a) {
  const int64_t nrows = a.cnt[CNT_ROWS], wmax = a.wave_max;
  float* lse = lse_out(a);
  const int grp = (threadIdx.x & 63) >> 4;
  const int64_t W = (int64_t)gridDim.x * (WAVE_BLOCK / 64);
  const int64_t w = (int64_t)blockIdx.x * (WAVE_BLOCK / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (4 * w < nrows) {
    // two groups in flight: the next group's rows are loaded (and the
    // descriptors of the one after fetched) before the current group is
    // summed and written
    const auto quarter = [&](const RowDesc& x) { return x.n > 0 && x.n <= WAVE_QUARTER_MAX && x.n <= wmax; };
    const auto desc = [&](int64_t r) {
      RowDesc x;
      x.n = 0;
      if (r < nrows) x = a.rows[r];
      return x;
    };
    int64_t g = 4 * w;
    RowDesc d = desc(g + grp), dn = desc(g + 4 * W + grp);
    QuarterHeld q;
    if (quarter(d)) dispatch_quarter_load<ACC>(d, q);
    while (true) {
      const int64_t next = g + 4 * W;
      QuarterHeld qn;
      if (quarter(dn)) dispatch_quarter_load<ACC>(dn, qn);
      const RowDesc dnn = desc(next + 4 * W + grp);
      if (quarter(d)) dispatch_quarter_finish<ACC>(d, q, lse ? lse + g + grp : nullptr);
      if (next >= nrows) break;
      g = next;
      d = dn;
      dn = dnn;
      q = qn;
    }
  }
  if (wmax <= WAVE_QUARTER_MAX || w >= nrows) return;
  int64_t r = w;
  RowDesc d = a.rows[r];
  while (true) {
    const int64_t next = r + W;
    RowDesc d_next = d;
    if (next < nrows) d_next = a.rows[next];
    if (d.n > WAVE_QUARTER_MAX && d.n <= wmax) dispatch_wave<ACC>(d, lse ? lse + r : nullptr);
    if (next >= nrows) break;
    r = next;
    d = d_next;
  }
}

template <int ACC>
hipError_t launch_phases(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  if (p.wave_grid > 0) {
    hipLaunchKernelGGL((batch_wave_kernel<ACC>), dim3((unsigned)p.wave_grid), dim3(WAVE_BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.res_grid > 0) {
    hipLaunchKernelGGL((batch_resident_kernel<ACC>), dim3((unsigned)p.res_grid), dim3(RES_BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipError_t e = phase1_u<ACC>(p, a, s);
  if (e != hipSuccess) return e;
  e = rowsum_acc<ACC>(p, a, s);
  if (e != hipSuccess) return e;
  return phase2_acc<ACC>(p, a, s);
}

// ---- the plain path's single-launch form for small n ---------------------------------
// One 1024-thread block holds the whole input in registers (SMALL_ELEMS
// elements: 16 vectors per thread for binary32, 8 for 2-byte inputs, which
// keeps the widened values in registers), reduces it, and divides from the
// registers: one read, one write, one launch. The sum is left in sum_out for
// nrm_get_last_sum.
constexpr int64_t SMALL_ELEMS = 65536;

template <int DTI, int DTO, int ACC>
__global__ void __launch_bounds__(1024) small_normalize_kernel(RowDesc d, float* sum_out) {
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ RowRes s_bcast;
  constexpr int KB = (int)(SMALL_ELEMS / 1024 / Elem<DTI>::VEC);
  single_pass<DTI, DTO, ACC, KB>(d, slots, &s_bcast, nullptr, 0);
  if (threadIdx.x == 0) sum_out[0] = s_bcast.a;  // single_pass ended after the broadcast's barrier
}

template <int ACC>
hipError_t small_acc(const RowDesc& d, float* sum_out, hipStream_t s) {
#define NRM_SK(I, O) hipLaunchKernelGGL((small_normalize_kernel<I, O, ACC>), dim3(1), dim3(1024), 0, s, d, sum_out)
  switch (d.in_dt * 3 + d.out_dt) {
    case NRM_F32 * 3 + NRM_F32: NRM_SK(NRM_F32, NRM_F32); break;
    case NRM_F32 * 3 + NRM_BF16: NRM_SK(NRM_F32, NRM_BF16); break;
    case NRM_F32 * 3 + NRM_F16: NRM_SK(NRM_F32, NRM_F16); break;
    case NRM_BF16 * 3 + NRM_F32: NRM_SK(NRM_BF16, NRM_F32); break;
    case NRM_BF16 * 3 + NRM_BF16: NRM_SK(NRM_BF16, NRM_BF16); break;
    case NRM_BF16 * 3 + NRM_F16: NRM_SK(NRM_BF16, NRM_F16); break;
    case NRM_F16 * 3 + NRM_F32: NRM_SK(NRM_F16, NRM_F32); break;
    case NRM_F16 * 3 + NRM_BF16: NRM_SK(NRM_F16, NRM_BF16); break;
    default: NRM_SK(NRM_F16, NRM_F16); break;
  }
#undef NRM_SK
  return hipGetLastError();
}

// ---- the plain path's single-launch form for mid-size n ---------------------------------
// n in (small_n, 2^20]: one block of PRES_BLOCK threads per segment of
// 2^PRES_LOG2 elements (at most PRES_MAX_SEGMENTS blocks), each held in
// registers from its read to its write while the blocks exchange their
// segment sums as the resident rows of a batch do: two transfers and one
// launch instead of three transfers and two launches. The grid is the
// row's segments, so every block of the launch must be able to run at once
// (256 blocks of 256 threads: one per CU on MI355X). The call number that
// tags the partials lives in the workspace; the last block to arrive moves
// it on (every block read it before arriving), so consecutive calls on one
// workspace never read each other's partials.
constexpr int PRES_BLOCK = 256;
constexpr int PRES_LOG2 = 12;
constexpr int PRES_MAX_SEGMENTS = 256;

template <int DTI, int DTO, int ACC, bool DIRECT>
__global__ void __launch_bounds__(PRES_BLOCK) plain_resident_kernel(RowDesc d, PlainResidentWs w) {
  __shared__ Acc<ACC> slots[MAX_WAVES];
  __shared__ RowRes s_bcast;
  // the tag is never 0, the value of a slot that was never written; the last
  // block to arrive moves the call number on once every block has read it
  const unsigned long long call = __hip_atomic_load(w.call, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const ResExchange x{w.slots, w.total, w.arrivals, (uint32_t)(call % 0xFFFFFFFFull) + 1u, w.error, w.stall, w.call};
  resident_unit<DTI, DTO, ACC, PRES_BLOCK, PRES_LOG2, DIRECT ? 1 : PRES_MAX_SEGMENTS / 64, DIRECT>(
      d, blockIdx.x, x, slots, &s_bcast, nullptr);
  if (threadIdx.x == 0 && blockIdx.x == 0) w.sum_out[0] = s_bcast.a;  // the invariant, for nrm_get_last_sum
}

// Rows of at most 64 segments exchange directly (one lane per segment).
constexpr int PRES_DIRECT_MAX = 64;

template <int ACC, bool DIRECT>
hipError_t plain_resident_acc(const RowDesc& d, const PlainResidentWs& w, hipStream_t s) {
  const unsigned grid = (unsigned)((d.n + (int64_t(1) << PRES_LOG2) - 1) >> PRES_LOG2);
#define NRM_PR(I, O) \
  hipLaunchKernelGGL((plain_resident_kernel<I, O, ACC, DIRECT>), dim3(grid), dim3(PRES_BLOCK), 0, s, d, w)
  switch (d.in_dt * 3 + d.out_dt) {
    case NRM_F32 * 3 + NRM_F32: NRM_PR(NRM_F32, NRM_F32); break;
    case NRM_F32 * 3 + NRM_BF16: NRM_PR(NRM_F32, NRM_BF16); break;
    case NRM_F32 * 3 + NRM_F16: NRM_PR(NRM_F32, NRM_F16); break;
    case NRM_BF16 * 3 + NRM_F32: NRM_PR(NRM_BF16, NRM_F32); break;
    case NRM_BF16 * 3 + NRM_BF16: NRM_PR(NRM_BF16, NRM_BF16); break;
    case NRM_BF16 * 3 + NRM_F16: NRM_PR(NRM_BF16, NRM_F16); break;
    case NRM_F16 * 3 + NRM_F32: NRM_PR(NRM_F16, NRM_F32); break;
    case NRM_F16 * 3 + NRM_BF16: NRM_PR(NRM_F16, NRM_BF16); break;
    default: NRM_PR(NRM_F16, NRM_F16); break;
  }
#undef NRM_PR
  return hipGetLastError();
}


}  // namespace

int64_t small_capacity(int) { return SMALL_ELEMS; }
int64_t plain_resident_capacity() { return (int64_t)PRES_MAX_SEGMENTS << PRES_LOG2; }

hipError_t launch_plain_resident(const void* in, int in_dt, void* out, int out_dt, int64_t n, int acc,
                                 const PlainResidentWs& w, hipStream_t s) {
  RowDesc d;
  d.in = static_cast<const char*>(in);
  d.out = static_cast<char*>(out);
  d.n = n;
  d.in_dt = in_dt;
  d.out_dt = out_dt;
  const bool direct = ((n + (int64_t(1) << PRES_LOG2) - 1) >> PRES_LOG2) <= PRES_DIRECT_MAX;
  if (acc == NRM_ACC_KAHAN)
    return direct ? plain_resident_acc<NRM_ACC_KAHAN, true>(d, w, s) : plain_resident_acc<NRM_ACC_KAHAN, false>(d, w, s);
  return direct ? plain_resident_acc<NRM_ACC_F32, true>(d, w, s) : plain_resident_acc<NRM_ACC_F32, false>(d, w, s);
}

hipError_t launch_small(const void* in, int in_dt, void* out, int out_dt, int64_t n, int acc, float* sum_out,
                        hipStream_t s) {
  RowDesc d;
  d.in = static_cast<const char*>(in);
  d.out = static_cast<char*>(out);
  d.n = n;
  d.in_dt = in_dt;
  d.out_dt = out_dt;
  return acc == NRM_ACC_KAHAN ? small_acc<NRM_ACC_KAHAN>(d, sum_out, s) : small_acc<NRM_ACC_F32>(d, sum_out, s);
}

hipError_t launch_batch(const BatchPlan& p, const BatchArgs& a, hipStream_t s) {
  // one block per round of the workspace's row capacity (blocks past the
  // batch's last round return at once)
  const int64_t plan_blocks = (a.cap_rows + PLAN_THREADS - 1) / PLAN_THREADS;
  const dim3 plan_grid((unsigned)(plan_blocks > 0 ? plan_blocks : 1));
  if (a.split_plan) {
    hipLaunchKernelGGL(batch_count_kernel, plan_grid, dim3(PLAN_THREADS), 0, s, a);
    const hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  if (a.split_plan)
    hipLaunchKernelGGL(batch_plan_kernel<true>, plan_grid, dim3(PLAN_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL(batch_plan_kernel<false>, plan_grid, dim3(PLAN_THREADS), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (p.acc) {
    case NRM_ACC_KAHAN: return launch_phases<NRM_ACC_KAHAN>(p, a, s);
    case ACC_SOFTMAX: return launch_phases<ACC_SOFTMAX>(p, a, s);
    default: return launch_phases<NRM_ACC_F32>(p, a, s);
  }
}

}  // namespace nrm
