// Internal interface of the ragged batched path: the device-side header and
// row table a batch is described by, the workspace pointers the kernels use,
// and the launch plan. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrm.h"

namespace nrm {

// One row as the kernels see it (same layout as the public nrm_row).
struct RowDesc {
  const char* in;
  char* out;
  int64_t n;
  int32_t in_dt;
  int32_t out_dt;
};
static_assert(sizeof(RowDesc) == sizeof(nrm_row), "RowDesc must match nrm_row");

enum { BATCH_CSR = 0, BATCH_TABLE = 1 };

// Per-call inputs, written by the host into pinned memory that the planner
// reads in place, so that a captured graph replays with new contents.
struct BatchHeader {
  int64_t nrows;
  int32_t mode;            // BATCH_CSR or BATCH_TABLE
  int32_t csr_in_dt, csr_out_dt;
  int32_t pad;
  const int64_t* offsets;  // CSR: rows + 1 offsets (device)
  const char* csr_in;
  char* csr_out;
  int64_t capacity;        // CSR: elements addressable through csr_in / csr_out
  const RowDesc* table;    // TABLE: the row table (pinned host memory)
  float* lse;              // softmax: each row's log-sum-exp (device), or NULL
};

// Device error bits (OR-ed by the planner, read by nrm_get_device_error).
enum {
  NRM_DEVERR_OFFSETS = 1,   // CSR offsets negative, decreasing or past capacity
  NRM_DEVERR_ROW = 2,       // a table row with n < 0, bad dtype, NULL pointer, or too many tiles
  NRM_DEVERR_CAPACITY = 4,  // more rows or work items than the workspace holds
  NRM_DEVERR_TARGET = 8,    // NLL loss: a target outside [0, C) that is not ignore_index
  NRM_DEVERR_STALL = 16,    // a resident row's segments did not all arrive within the spin limit
};

constexpr int64_t MAX_ROW_TILES = 65536;  // partials the per-row combine merges

// One work item: a tile of a long row, or a whole short row (tile 0).
struct Item {
  int32_t row;
  int32_t tile;
};

// Counters the planner leaves for the later kernels (device memory).
enum {
  CNT_ITEMS = 0,       // all work items of phase 1
  CNT_LONG_ITEMS = 1,  // the leading items that are tiles of long rows
  CNT_LONG_ROWS = 2,   // long rows
  CNT_LONG_ELEMS = 3,  // elements in long rows: the length of phase 2's range
  CNT_CHUNK = 4,       // elements per phase-2 chunk
  CNT_CHUNKS = 5,      // phase-2 chunks
  CNT_LSE = 6,         // softmax: the header's lse pointer, for the kernels after the planner
  CNT_DISPENSE = 7,    // resident units handed out so far (set to 0 by the planner)
  CNT_EPOCH = 8,       // this call's number: tags the resident rows' published partials
  CNT_STALL = 9,       // the number of the last call in which a resident wait gave up
  CNT_ROWS = 10,       // the batch's rows (0 when the planner rejected the batch)
  CNT_COUNT = 11,
};

// One row's reduction result: the sum (a) for normalize, or the exponent and
// the scaled sum (a = k, b = s) for softmax.
struct RowRes {
  float a, b;
};

// Kernel arguments: workspace pointers, fixed for a context's workspace.
struct BatchArgs {
  const BatchHeader* hdr;
  RowDesc* rows;         // resolved rows [cap_rows]
  Item* items;           // [cap_items]: the long rows' tiles first, then the short rows
  int64_t* lrow_first;   // [cap_rows]: first item (and partial) of each long row, in row order
  RowDesc* lrows;        // [cap_rows]: the long rows' descriptors, in row order
  int64_t* lstart;       // [cap_rows]: each long row's first position in the long rows' concatenation
  RowRes* lsum;          // [cap_rows]: each long row's result (written between the phases)
  int32_t* chunk_lrow;   // [cap_chunks]: the long row in which each phase-2 chunk starts
  int64_t* cnt;          // [CNT_COUNT]
  int* error;            // [1]
  void* partials;        // [cap_items] x 8 bytes
  int64_t cap_rows;
  int64_t cap_items;
  int64_t cap_chunks;
  int64_t tile;          // elements per tile of a long row: 2^tile_log2
  int tile_log2;
  int64_t short_max;     // rows with n <= short_max take one pass
  int64_t map_grid;      // phase 2 blocks: the chunks are sized to a multiple of it
  int64_t min_chunk;     // elements of one full phase-2 block-iteration: the smallest chunk
  int64_t keep_tiles;    // phase 1 reads the last this many long-row tiles with a temporal hint
  // resident rows (res_on): a row of n <= short_max elements is cut into
  // segments of 2^RES_LOG2 elements, one work item each, each held in one
  // block's registers from its read to its write
  int res_on;
  unsigned long long* tagged;  // [2 * cap_items]: each segment's partial, two tagged words
  unsigned long long* rowtot;  // [2 * cap_items]: a resident row's total at its first item, two tagged words
  unsigned* arrivals;          // [cap_items]: a resident row's published segments at its first item (0 between calls)
  // short rows: a row of 0 < n <= wave_max elements is taken by one
  // wavefront of the short rows' kernel (0: none; at most WAVE_MAX_ELEMS)
  int64_t wave_max;
  // split planner (split_plan): a counting kernel leaves each round's counter
  // totals here, so that the planner's blocks scan only their own round
  int split_plan;
  int64_t* round_agg;          // [ceil(cap_rows / PLAN_ROUND_ROWS) * 4]
  BatchHeader* hdr_dev;        // the header, copied to device memory by the counting launch
};

// The planner takes rows PLAN_ROUND_ROWS at a time (a "round", one block).
// Up to PLAN_SPLIT_ROWS rows of capacity every planner block scans every
// round itself (one launch); above, a counting launch first leaves each
// round's totals, and each planner block scans its own round only.
constexpr int64_t PLAN_ROUND_ROWS = 1024;
constexpr int64_t PLAN_SPLIT_ROWS = 4096;

// Elements of one resident segment: 512 threads x 8 vectors of 4 binary32
// (4 vectors of 8 for 2-byte inputs); two blocks fit a CU's registers.
constexpr int RES_LOG2 = 14;
constexpr int RES_BLOCK = 512;
constexpr int RES_MAX_SEGMENTS = 64;  // one wavefront lane per segment in the merge

// The short rows' kernel: blocks of WAVE_BLOCK threads, rows of at most
// WAVE_MAX_ELEMS elements (2048 binary32: eight 16-byte vectors per lane).
constexpr int WAVE_BLOCK = 256;
constexpr int64_t WAVE_MAX_ELEMS = 2048;

struct BatchPlan {
  int acc;
  int block;
  int unroll;       // tile reduce: vectors per thread per iteration
  int map_unroll;   // tile map
  int short_regs;   // vectors per thread held for a single-pass row
  int64_t grid;     // persistent blocks of phase 1 and of the row sums
  int map_block;    // phase 2
  int64_t map_grid;
  int64_t res_grid; // persistent blocks of the resident-row kernel (0: none launched)
  int64_t wave_grid; // blocks of the short rows' kernel (0: none launched)
};

hipError_t launch_batch(const BatchPlan& p, const BatchArgs& a, hipStream_t s);

}  // namespace nrm
