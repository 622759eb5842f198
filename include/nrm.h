/*
 * nrm.h - C ABI of the MI355X (gfx950) normalize library, libnrm.so.
 *
 * normalize(out, in, n) computes out[i] = in[i] / sum_{j<n} in[j] for every
 * i in [0, n): the running example of arXiv 2207.00257 (Fig. 1, the
 * `normalize` kernel and its host-side `launch`). The sum is loop-invariant
 * across the kernel's threads; this library computes it once per call, as the
 * parallel loop-invariant code motion of Sec. IV-C and the O(N) form named in
 * the Fig. 1 caption and Sec. II-A do, instead of once per thread (O(N^2)) or
 * once per block (O(N^2/B), the shared-memory variant in Fig. 1's comments).
 *
 * Execution: a block-level partial reduction (wavefront DPP reduce, one LDS
 * slot per wavefront, one block barrier), a deterministic fixed-order combine
 * of the block partials behind a grid-wide barrier (the last block to finish
 * combines), then a coalesced 16-byte-vector divide map. Results are
 * bitwise reproducible for a given (n, pointer alignment, dtypes,
 * accumulation mode, parameters).
 *
 * Conventions for every entry point:
 *  - Data pointers (in, out, offsets) are DEVICE pointers in the current HIP
 *    device's memory. The caller owns them; the library never frees them.
 *  - Calls are stream-ordered and asynchronous: NRM_OK means the work was
 *    enqueued (the paper's `launch` is likewise a kernel launch). Results are
 *    visible after the stream is synchronized.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *  - Sizes are int64_t. n == 0 returns NRM_OK and writes nothing.
 *  - Argument errors are detected on the host before anything is enqueued.
 *  - out == in (same address, same element size) is allowed: the result is
 *    the hoisted definition, the sum of the original input. Any other overlap
 *    of the input and output byte ranges is NRM_EOVERLAP.
 *  - The library owns only its workspace (per-block partials, the combine
 *    ticket, the sum), held by a context; workspace grows on demand with
 *    hipMalloc, which is stream-synchronizing the first time a size is seen.
 *  - Calls that share a context must be ordered (same stream, or synchronized
 *    between streams): they share its workspace. A context's host-side state
 *    is locked for the duration of each call, so host threads may share a
 *    context (the default context of a device is shared by every thread that
 *    passes ctx NULL); the ordering rule still applies to their device work
 *    (the basic forms all use the null stream, which orders them).
 *  - Floating point: IEEE binary32 accumulation (or compensated binary32), a
 *    correctly rounded binary32 division, round-to-nearest-even conversions to
 *    BF16/FP16. No FP64 on the GPU. For non-negative inputs the relative error
 *    of every output against the exact quotient is at most gamma_h + u, where
 *    h <= max_height + 26 is the height of the summation tree, u = 2^-24 and
 *    gamma_h = h u / (1 - h u) (default max_height 36: h <= 62, bound 3.8e-6);
 *    compensated accumulation brings the sum's error to a few u whatever the
 *    size.
 */
#ifndef NRM_H
#define NRM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every entry point. */
typedef enum {
  NRM_OK = 0,
  NRM_EINVAL = -1,      /* bad argument: n < 0, NULL pointer with n > 0, bad enum or parameter */
  NRM_EOVERLAP = -2,    /* in and out overlap without being the same array */
  NRM_ENOMEM = -3,      /* workspace allocation failed */
  NRM_EHIP = -4,        /* a HIP runtime call failed; see nrm_last_error() */
  NRM_EUNSUPPORTED = -5,/* dtype pair or mode not supported */
  NRM_EDEVICE = -6      /* the device flagged invalid data (e.g. decreasing offsets) */
} nrm_status;

/* Storage types of in and out. */
typedef enum { NRM_F32 = 0, NRM_BF16 = 1, NRM_F16 = 2 } nrm_dtype;

/* Accumulation of the sum: plain binary32 in many independent chains, or
 * binary32 Kahan-compensated chains combined with error-free transformations
 * (TwoSum). */
typedef enum { NRM_ACC_F32 = 0, NRM_ACC_KAHAN = 1 } nrm_accum;

/* How blocks cover the input: each block a contiguous chunk; the grid
 * strides over the input one block-iteration at a time; or the input is cut
 * into tiles of 2^tile_log2 elements (rounded up to whole block-iterations)
 * and block b streams tiles b, b + grid, b + 2 grid, ... */
typedef enum { NRM_LAYOUT_CHUNK = 0, NRM_LAYOUT_STRIDE = 1, NRM_LAYOUT_TILE = 2 } nrm_layout;

/* Launch parameters of the plain path. Start from nrm_default_params() and
 * change fields; nrm_set_params validates every field. Changing them changes
 * the summation tree, hence the low bits of the result (always within the
 * stated error bound), never its definition. */
typedef struct {
  /* reduce kernel */
  int32_t block;        /* threads per block: 64..1024, multiple of 64 */
  int32_t unroll;       /* 16-byte vectors per thread per iteration: 1, 2, 4 or 8 */
  int32_t grid;         /* blocks (upper bound; raised when the height bound needs more) */
  int32_t layout;       /* nrm_layout */
  int32_t reduce_nt;    /* 1: non-temporal hint on the reduce's loads */
  int32_t max_height;   /* bound on the additions along any path of one thread's summation
                           tree, 24..40; the whole tree then has height <= max_height + 26
                           (wavefront 6, block <= 4, grid combine <= 16), so that
                           gamma_h + u < 4e-6 even at the cap (h = 66: 3.99e-6) */
  /* map kernel */
  int32_t map_block;    /* threads per block: 64..1024, multiple of 64 */
  int32_t map_unroll;   /* 16-byte vectors per thread per iteration: 1, 2, 4 or 8 */
  int32_t map_grid;     /* blocks (upper bound) */
  int32_t map_layout;   /* nrm_layout */
  int32_t map_nt;       /* 1: non-temporal hint on the map's loads */
  int32_t reverse_map;  /* 1: each block walks its share from the end (reuse of recently read lines) */
  int32_t reduce_keep_mib; /* 0..4096: the reduce reads the last this many MiB of the input with a
                              temporal hint (the rest non-temporal), so that the map finds them in
                              the last-level cache (256 MB on MI355X: a larger tail thrashes it and
                              gains nothing) */
  int32_t tile_log2;    /* layout TILE (either kernel): log2 of the elements per tile, 10..22 */
  int32_t fused_combine;/* 1: the reduce ends without a grid-wide ticket or fence and every map
                           block merges the reduce's partials itself, in the same fixed order
                           (height 10), so all blocks divide by the same value. Taken when the
                           reduce has at most 1024 blocks and out is aligned like in; otherwise
                           the last reduce block combines as with 0. */
  int32_t small_n;      /* 0..2^16: n up to this runs as one launch of one 1024-thread block that
                           reads the input once into registers (16 binary32 or 8 2-byte vectors
                           per thread), reduces it, and divides from the registers: one read,
                           one write, one launch. Default 0 (never): the resident form below was
                           faster per call at every size */
  int32_t resident_n;   /* 0..2^20: n in (small_n, resident_n] runs as one launch of one 256-thread
                           block per 4096 elements, each block holding its elements in registers
                           while the blocks exchange their sums: one read, one write, one launch
                           (all n / 4096 blocks must be able to run at once: one per CU). Up to 64
                           blocks every block reads every block's sum; beyond, the last block to
                           arrive publishes the total. Default 2^18; 0: never */
} nrm_params;

/* Launch parameters of the ragged batched path. Start from
 * nrm_default_batch_params(). A row's result depends on these, on its length,
 * dtypes and start alignment modulo 16 bytes, never on the other rows. */
typedef struct {
  int32_t block;       /* threads per block: 64..1024, multiple of 64 */
  int32_t unroll;      /* tile sums: 16-byte vectors per thread per iteration: 1, 2, 4, 8 */
  int32_t map_unroll;  /* tile divides: 16-byte vectors per thread per iteration: 1, 2, 4, 8 */
  int32_t grid;        /* persistent blocks of the planner-fed phase 1 (sums, single-pass rows) */
  int32_t tile_log2;   /* a long row is cut into tiles of 2^tile_log2 elements: 10..22 */
  int32_t short_regs;  /* 16-byte vectors per thread held in registers by a single-pass row:
                          1, 2, 4 or 8; rows with n <= block * short_regs * 4 take one pass
                          (one read, one write) */
  int32_t graph;       /* 1 (default): capture the launch sequence once per staging buffer in a
                          hipGraph and replay it (captured on a stream of the library's own, on
                          first use); 0: launch the kernels one by one */
  int32_t map_block;   /* threads per block of the divide phase: 64..1024, multiple of 64 */
  int32_t map_grid;    /* persistent blocks G of the divide phase: the long rows' concatenation is
                          cut into about G * m equal chunks of at most about one tile each, so
                          that every block divides the same number of elements */
  int32_t keep_mib;    /* 0..4096: phase 1 reads the long rows' last tiles, up to this many MiB,
                          with a temporal hint (the rest non-temporal), so that the divide phase
                          finds them in the last-level cache (256 MB on MI355X) */
  int32_t resident_segments; /* 0..64: a row of n <= resident_segments * 2^14 elements crosses HBM
                                twice instead of three times: each of its segments of 2^14 elements
                                is held in one block's registers from its read to its write while the
                                row's blocks exchange their segment sums. 0: off (such rows take the
                                single-pass or tile path) */
  int32_t resident_grid;     /* persistent 512-thread blocks of the resident rows' kernel, 1..2^20 and
                                at least resident_segments: a row's blocks wait for each other, so the
                                device must be able to run that many of them at once (two per CU fit) */
  int32_t wave_max;          /* 0..2048: a row of 0 < n <= wave_max elements is taken by one wavefront
                                (64 lanes), or for n <= 256 by a quarter of one (16 lanes, four such
                                rows per wavefront at once): read into registers, summed across the
                                lanes by DPP moves with no LDS, barrier or work claim, divided from
                                the registers and written (two HBM transfers). 0: off (such rows take
                                the resident or single-pass path) */
  int32_t wave_grid;         /* 256-thread blocks of the short rows' kernel, 1..2^20; its W wavefronts
                                take the rows statically (wavefront w: rows w, w + W, ...) */
} nrm_batch_params;

/* One row of a batch given as a table: `in` and `out` are device arrays of
 * n elements of in_dtype / out_dtype; the row is normalized on its own. */
typedef struct {
  const void* in;
  void* out;
  int64_t n;
  int32_t in_dtype;
  int32_t out_dtype;
} nrm_row;

typedef struct nrm_ctx nrm_ctx;

/* ---- the basic forms: FP32 in and out, default context, null stream ------- */

/* out[i] = in[i] / sum(in[0..n)) for i in [0, n). Fig. 1 semantics with the
 * sum hoisted (Sec. IV-C). in, out: device arrays of n floats. */
int normalize(float* out, const float* in, int64_t n);

/* Ragged batched, CSR form: row r in [0, rows) is the slice
 * [offsets[r], offsets[r+1]) of both `in` and `out`, normalized on its own.
 * offsets: DEVICE array of rows + 1 int64, offsets[0] >= 0, non-decreasing;
 * empty rows are allowed. FP32, default context, null stream. The library
 * reads offsets[rows] back to the host (synchronizing the null stream) to
 * size its workspace and to bound every row; rows that violate the rules are
 * skipped and reported by nrm_get_device_error. */
int normalize_batched(float* out, const float* in, const int64_t* offsets, int64_t rows);

/* ---- allocation-free plain form ------------------------------------------ */

/* For callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc. Computes exactly what
 * nrm_normalize_ex does on a context of the current device whose parameters
 * are the library's defaults for it (same kernels, same launch parameters,
 * same bits; the tuning cache is not read), but takes no context
 * and calls no hipMalloc, hipFree or other allocating routine: the workspace
 * (block partials, combine ticket, sum, the mid-size form's exchange slots)
 * is a fixed array of
 * NRM_NOALLOC_SCRATCH_BYTES bytes in the library's code object, one copy per
 * device, held until the process ends. The first call on a device looks up
 * that device's copy and enqueues one tiny kernel on `stream` to clear the
 * ticket.
 *   in, out:  device arrays of n elements of in_dtype / out_dtype, as for
 *             nrm_normalize_ex (same overlap, alignment and dtype rules);
 *   accum:    NRM_ACC_F32 or NRM_ACC_KAHAN;  stream: hipStream_t or NULL.
 * Limit: the call may use at most 16384 reduce blocks (one 8-byte partial
 * each); with the default parameters that holds for every n <= 2^34. A larger
 * n returns NRM_EINVAL before anything is enqueued.
 * All calls on one device share that device's array and it keeps the last
 * call's contents: calls that overlap in time on one device (unordered
 * streams, several host threads) race on it and give wrong results; order
 * them (one stream, or events). Asynchronous like every other call. */
#define NRM_NOALLOC_SCRATCH_BYTES 135680
int nrm_normalize_noalloc(void* out, int out_dtype, const void* in, int in_dtype, int64_t n, int accum,
                          void* stream);

/* ---- contexts ------------------------------------------------------------ */

/* Create a context on HIP device `device` (-1: the current device). The
 * context owns workspace on that device and the launch parameters. Until
 * nrm_set_params is called on it, each plain call takes the launch
 * parameters the autotuner stored for its key (device architecture, dtypes,
 * accumulation, size class floor(log2 n)) in the tuning cache, the JSON file
 * named by $NRM_TUNE_CACHE or else tuned/plain.json next to libnrm.so, and
 * the library defaults where the cache has no entry. */
int nrm_create(nrm_ctx** ctx, int device);
/* Free the context's workspace. Waits for the device to be idle first. */
int nrm_destroy(nrm_ctx* ctx);
/* The library's default launch parameters (tuned for MI355X). */
int nrm_default_params(nrm_params* params);
/* Replace the context's launch parameters (from then on they apply to every
 * call, in place of the tuning cache); NRM_EINVAL if any field is out of range. */
int nrm_set_params(nrm_ctx* ctx, const nrm_params* params);
int nrm_get_params(const nrm_ctx* ctx, nrm_params* params);

/* ---- extended plain form ------------------------------------------------- */

/* normalize with storage dtypes, accumulation mode, context and stream.
 * in: n elements of in_dtype; out: n elements of out_dtype. Supported:
 * every pair of {F32, BF16, F16}. ctx NULL: the default context of the
 * current device. */
int nrm_normalize_ex(nrm_ctx* ctx, void* out, int out_dtype, const void* in, int in_dtype,
                     int64_t n, int accum, void* stream);

/* ---- forward NLL loss ----------------------------------------------------- */

/* The forward negative log-likelihood loss: the loss kernel the paper
 * translated because it synchronises with a block barrier (arXiv 2207.00257,
 * Sec. V-B), defined from the loss. N samples, C classes:
 *     loss_n = -weight[t_n] * logp[n * C + t_n]   (0 when t_n == ignore_index),
 *     NRM_NLL_NONE: out[n] = loss_n (N floats);
 *     NRM_NLL_SUM:  out[0] = sum_n loss_n;
 *     NRM_NLL_MEAN: out[0] = sum_n loss_n / sum over kept n of weight[t_n]
 *                   (0/0 = NaN when every sample is ignored).
 * Like normalize (Fig. 1) it reduces invariants once (the loss and the
 * weight total), then maps (the one division).
 *   logp:   device binary32 [N][C], row-major;   target: device int64 [N];
 *   weight: device binary32 [C], or NULL for all 1;
 *   out:    device binary32, N (none) or 1 (sum, mean);
 *   total_weight: device binary32 [1] receiving the kept weights' sum
 *           (sum and mean), or NULL.
 * accum: NRM_ACC_F32 or NRM_ACC_KAHAN for the two sums. Per-sample losses are
 * the correctly rounded products; with non-negative weights the sums add
 * non-negative terms, within gamma_h of the exact sum for the summation
 * tree's height h (see DESIGN). A target outside [0, C) that is not
 * ignore_index contributes nothing (0 for none) and is reported by
 * nrm_get_device_error. Outputs must not overlap the inputs (NRM_EOVERLAP).
 * ctx NULL: the default context of the current device. */
typedef enum { NRM_NLL_NONE = 0, NRM_NLL_SUM = 1, NRM_NLL_MEAN = 2 } nrm_reduction;
int nrm_nll_loss(nrm_ctx* ctx, float* out, float* total_weight, const float* logp, const int64_t* target,
                 const float* weight, int64_t n, int64_t classes, int64_t ignore_index, int reduction, int accum,
                 void* stream);

/* ---- barrier elimination, for measurement --------------------------------- */

/* A synthetic layer-forward tile kernel with the shape of the paper's
 * barrier-elimination example (arXiv 2207.00257, Sec. IV-A and IV-B, Fig. 9),
 * to measure what removing barriers saves on the GPU. hidden: device binary32
 * R x 16 (row-major), updated in place; input: device binary32 [R]; output:
 * device binary32 [R]; R a multiple of 16, R / 16 <= 2^31 - 1. Per tile of 16
 * rows (one 256-thread block): p[y][x] = hidden[16 b + y][x] * input[16 b + y],
 * a halving tree over y (row y ends with the sum of p over rows y .. y + L(y)
 * - 1, L(y) the largest power of two dividing y, 16 for y = 0), every row
 * written back to hidden, and output[16 b + x] = the column sums (tile row 0).
 *   NRM_LF_ALL_BARRIERS  a block barrier after every stage (scale load, tile
 *                        load, scaling, each tree level, write-back);
 *   NRM_LF_ELIMINATED    without the two barriers that Sec. IV-A's rule finds
 *                        no conflicting access across (after the scale load
 *                        and after the write-back);
 *   NRM_LF_PROMOTED      also without the shared store/load a thread makes
 *                        only to itself across a barrier (Sec. IV-B);
 *   NRM_LF_REGISTERS     the tile kept in registers, one thread per column:
 *                        no shared memory and no barrier.
 * The forms compute the same values bit for bit (products rounded to binary32,
 * the tree's additions in the same order). hidden, input and output must not
 * overlap (NRM_EOVERLAP). */
typedef enum { NRM_LF_ALL_BARRIERS = 0, NRM_LF_ELIMINATED = 1, NRM_LF_PROMOTED = 2, NRM_LF_REGISTERS = 3 } nrm_lf_form;
int nrm_layerforward(int form, float* hidden, const float* input, float* output, int64_t rows, void* stream);

/* ---- the un-hoisted forms, for measurement ------------------------------- */

/* Fig. 1's two slower forms on the GPU: NRM_FORM_NAIVE, every thread sums the
 * whole input itself (O(n^2) work); NRM_FORM_PERBLOCK, the first wavefront of
 * each block sums it into block-shared memory, a block barrier, then every
 * thread divides (O(n^2 / block)). FP32, 1 <= n <= 2^20, block 64..1024
 * (multiple of 64). The sums are Kahan-compensated binary32 chains. They
 * exist to measure what the hoisted form saves; they are not fast paths. */
typedef enum { NRM_FORM_NAIVE = 1, NRM_FORM_PERBLOCK = 2 } nrm_form;
int nrm_normalize_form(int form, float* out, const float* in, int64_t n, int block, void* stream);

/* ---- extended batched forms ---------------------------------------------- */

/* CSR form with dtypes, accumulation, context and stream. `capacity` is the
 * number of elements `in` and `out` hold: every row must lie inside
 * [0, capacity), which the device checks (rows outside are skipped and
 * flagged). capacity < 0: read offsets[rows] back and use it (synchronizes
 * `stream`). The workspace is sized for rows and capacity. */
int nrm_normalize_batched_ex(nrm_ctx* ctx, void* out, int out_dtype, const void* in, int in_dtype,
                             const int64_t* offsets, int64_t rows, int64_t capacity, int accum,
                             void* stream);

/* Row softmax and log-sum-exp of a ragged batch, on the same planner and
 * persistent phases as the batched normalize. Softmax is one of the
 * aggregation kernels the paper's PyTorch integration carries (arXiv
 * 2207.00257, Sec. V-B); it has normalize's shape (Fig. 1): a row-invariant
 * pair is reduced once per row, then every element is mapped. For every CSR
 * row r = [offsets[r], offsets[r+1]) of the binary32 array in:
 *     out[i] = exp(in[i]) / sum_{j in r} exp(in[j]),
 *     lse[r] = log(sum_{j in r} exp(in[j])).
 * The invariant pair is a base-2 exponent k >= every in[j] log2(e) and the
 * sum s of exp2(in[j] log2(e) - k), each term in (0, 1], reduced with exact
 * power-of-two rescaling (no rounding added when the maximum moves); then
 * out[i] = exp2(in[i] log2(e) - k) times the correctly rounded 1/s, and
 * lse[r] = (k + log2 s) ln 2.
 *   in, out:  device binary32, `capacity` elements each (capacity < 0: read
 *             offsets[rows] back, which synchronizes `stream`); in == out
 *             computes in place, any other overlap is NRM_EOVERLAP.
 *   offsets:  device int64[rows + 1]; rows outside [0, capacity) are skipped
 *             and flagged on the device (nrm_get_device_error).
 *   lse:      device float[rows], or NULL; empty rows get -inf. It must not
 *             overlap in or out.
 * Inputs are finite with |in| < 1e38. Accuracy (u = 2^-24): each output is
 * within a relative (2|x| + |x - m| + 7) u + e_s of the exact value (x its
 * input, m the row maximum), where e_s, the relative error of s, is at most
 * the same quantity averaged over the row with the softmax weights plus
 * gamma_62 (the summation tree's height bound); lse within e_s + 4 u (|lse| + 1).
 * Outputs below 2^-125 may be flushed to zero (a term exp2(.) below 2^-126
 * flushes, and s >= 1/2). Returns NRM_OK or an error
 * code; the call itself is asynchronous on `stream`. ctx NULL: the default
 * context of the current device. */
int nrm_softmax_batched(nrm_ctx* ctx, float* out, const float* in, const int64_t* offsets, int64_t rows,
                        int64_t capacity, float* lse, void* stream);

/* Table form: `rows` is a HOST array of nrows descriptors (device data
 * pointers), staged in the context's pinned memory, which the device reads in
 * place; rows may mix dtypes. Rows are validated on the host. The context
 * keeps four such staging buffers and uses them in turn (the CSR forms stage
 * their arguments the same way): a call blocks the host only while the call
 * four before it on the same context has not finished. */
int nrm_normalize_rows(nrm_ctx* ctx, const nrm_row* rows, int64_t nrows, int accum, void* stream);

/* Reserve batched workspace for up to max_rows rows and max_elems elements
 * in total (optional: calls grow it on demand, which synchronizes the
 * device; a captured graph needs a fixed workspace). */
int nrm_batch_reserve(nrm_ctx* ctx, int64_t max_rows, int64_t max_elems);

int nrm_default_batch_params(nrm_batch_params* params);
int nrm_set_batch_params(nrm_ctx* ctx, const nrm_batch_params* params);
int nrm_get_batch_params(const nrm_ctx* ctx, nrm_batch_params* params);

/* Synchronize `stream`, then return NRM_EDEVICE if a batched call on this
 * context found invalid rows or ran out of workspace since the last check
 * (and clear the flag), else NRM_OK. nrm_last_error() names the cause. */
int nrm_get_device_error(nrm_ctx* ctx, void* stream);

/* ---- continuous-batching server --------------------------------------------- */

/* A normalize request: `in` is a device array of n elements of in_dtype that
 * stays valid until the request completes; the output is allocated by the
 * server. t_arrival_ns: for nrm_server_submit, the arrival time on the
 * steady clock in ns (0: now); for nrm_server_replay, the offset of the
 * scheduled arrival from the start of the replay. */
typedef struct {
  int64_t id;
  const void* in;
  int64_t n;
  int32_t in_dtype;
  int32_t out_dtype;
  int64_t t_arrival_ns;
} nrm_request;

typedef struct {
  int64_t id;
  void* out;             /* device output (valid until released when hold_outputs) */
  int64_t t_arrival_ns;  /* scheduled arrival (steady clock, ns) */
  int64_t t_launch_ns;   /* when its batch was launched */
  int64_t t_done_ns;     /* when its completion was observed */
  int32_t status;
  int32_t pad;
} nrm_completion;

typedef struct {
  int32_t slots;             /* concurrent batches (each its own stream, workspace, graph): 1..64 */
  int32_t batching;          /* 1: one ragged batched launch per admitted group; 0: one plain call per request */
  int32_t graph;             /* 1: batched launches replay a captured hipGraph */
  int32_t accum;             /* nrm_accum */
  int32_t hold_outputs;      /* 1: outputs (and their budget) stay until nrm_server_release */
  int32_t use_batch_params;  /* 1: use batch_params for the slots, else the library defaults */
  int32_t single_plain;      /* 1: a group of one request runs the plain path (two kernels
                                instead of the batched four); its bits then match the plain
                                path rather than the batched one, both within the error bound */
  int32_t spread;            /* 1: waiting requests are spread over the free slots, each free slot
                                taking ceil(waiting / free slots) of them in arrival order, so that
                                requests run alone and concurrently while slots are free and are
                                grouped only when the queue outgrows the slots; 0: the first free
                                slot takes all it can */
  int32_t idle_spin_us;      /* 0..10^6: after its last activity the scheduler thread keeps polling
                                (yielding) this long before it blocks, so that an arrival within
                                that time is picked up without a thread wake-up */
  int32_t min_batch_rows;    /* 1..2^20: with batching, a group of fewer requests runs as one plain
                                call per request on its slot (a small call is one launch; the batched
                                call costs its planner and five kernels whatever the group's size) */
  int64_t budget_bytes;      /* HBM admission budget: input + output bytes of admitted requests */
  int64_t arena_bytes;       /* device arena for outputs (0: two thirds of the budget) */
  int64_t max_batch_rows;    /* requests per batch */
  int64_t max_batch_elems;   /* elements per batch (a single larger request still runs alone) */
  nrm_batch_params batch_params;
  int32_t device_queue;      /* 1: no launch per request: one persistent kernel polls a ring of
                                published requests in pinned host memory and runs each one as it
                                arrives (batching, graph, single_plain, spread, min_batch_rows and
                                batch_params do not apply); each request of n <= 2^20 elements
                                crosses HBM twice, a longer one three times; n <= 2^25; slots
                                (1..64) bounds the requests in flight. While the kernel is
                                resident, a kernel the caller queues on a stream that shares its
                                hardware queue (the runtime spreads streams over a few such
                                queues) waits until it ends: dq_slice_us, or dq_idle_us after the
                                last request if sooner; the server's own streams are probed apart
                                from it at creation.
                                0: launches per batch or request as above */
  int32_t dq_blocks;         /* device queue: persistent blocks of 512 threads (0: two per compute
                                unit); at least 64 must be able to run at once */
  int64_t dq_idle_us;        /* device queue: the kernel ends after this long (1..10^7 us) without a
                                new request and is started again by the next one */
  int64_t dq_plain_above;    /* device queue: a request of more elements than this (1..2^25) runs
                                as the plain two-kernel call on its slot's own stream instead (the
                                default, 2^20, keeps in the kernel the requests it holds in
                                registers, which it serves fastest); 2^25: every request in the
                                kernel. dq_blocks 0 then means one block per compute unit, which
                                leaves room for those calls, and two when every request stays */
  int64_t dq_slice_us;       /* device queue: each launch of the kernel ends after this long (0: no
                                limit; 0..10^7 us, default 10^4) and the next request starts the
                                next, so that a kernel queued behind it on its hardware queue waits
                                at most about this long */
} nrm_server_config;

typedef struct {
  int64_t in_flight;   /* submitted and not completed */
  int64_t queued;      /* waiting for admission */
  int64_t held;        /* completed, output not released */
  int64_t budget_used; /* bytes */
  int64_t batches;
  int64_t launches;    /* library calls made (batched calls or plain calls) */
  int64_t replaying;
  int64_t failed;      /* requests completed with an error status */
} nrm_server_counters;

typedef struct nrm_server nrm_server;

int nrm_server_default_config(nrm_server_config* cfg);
/* Start a server on `device` (-1: current): allocates the output arena and
 * one context, stream and event per slot, and starts the scheduler thread. */
int nrm_server_create(nrm_server** server, int device, const nrm_server_config* cfg);
/* Queue requests now (thread-safe). A request larger than the budget is
 * NRM_EINVAL; otherwise it waits until memory and a slot free up. */
int nrm_server_submit(nrm_server* server, const nrm_request* reqs, int64_t count);
/* Submit a trace from a background thread at its scheduled times (open
 * loop; requests sorted by t_arrival_ns). *t0_ns receives the start time. */
int nrm_server_replay(nrm_server* server, const nrm_request* reqs, int64_t count, int64_t* t0_ns);
/* Move up to max completions into out; *count receives how many. Each
 * completion carries its own status: a request whose launch or execution
 * failed completes with that error (its output is not valid and its memory is
 * already released); poll itself fails only on bad arguments. */
int nrm_server_poll(nrm_server* server, nrm_completion* out, int64_t max, int64_t* count);
/* NRM_OK if no request has failed so far, else the first failure's status,
 * with its text in nrm_last_error(). */
int nrm_server_last_failure(nrm_server* server);
/* Release a held output (hold_outputs = 1). */
int nrm_server_release(nrm_server* server, int64_t id);
int nrm_server_stats(nrm_server* server, nrm_server_counters* counters);
/* Stop accepting replays, finish all queued and in-flight work, free everything. */
int nrm_server_destroy(nrm_server* server);

/* ---- diagnostics and measurement ------------------------------------------ */

/* The hoisted sum S of the last plain call on this context, as the kernels
 * used it (binary32; compensated mode: hi + lo rounded once), read after
 * synchronizing `stream`. ctx NULL: the default context. */
int nrm_get_last_sum(nrm_ctx* ctx, void* stream, float* sum);

/* Measurement only, not part of normalize: the bandwidth ceilings a call is
 * compared with in the same run. NRM_CEILING_COPY copies `bytes` from src to
 * dst (the traffic of the divide map: one read and one write per byte);
 * NRM_CEILING_READ reads `bytes` of src (the traffic of the reduce) and may
 * write one 4-byte word per block to dst (a device buffer of at least 4 * grid
 * bytes). 16-byte vectors, non-temporal hints, each of `grid` blocks (512
 * threads) taking one contiguous chunk. bytes: a multiple of 16; src and dst
 * 16-byte aligned, not overlapping; grid 1..2^20. Asynchronous on `stream`. */
typedef enum { NRM_CEILING_COPY = 0, NRM_CEILING_READ = 1 } nrm_ceiling_kind;
int nrm_ceiling(int kind, void* dst, const void* src, int64_t bytes, int64_t grid, void* stream);

/* The tuning cache's parameters for a call key (architecture name such as
 * "gfx950", dtypes, accumulation, n): writes them over nrm_default_params()
 * and returns 1, or returns 0 (params = the defaults) when the cache has no
 * entry for the key. No HIP call. */
int nrm_tuned_params(const char* arch, int in_dtype, int out_dtype, int accum, int64_t n, nrm_params* params);

/* Static text for a status code. */
const char* nrm_status_string(int status);
/* Detail of the last error on the calling thread (HIP error text), or "". */
const char* nrm_last_error(void);

/* Kernel timing: while enabled, every plain call records HIP events around
 * its reduce and map kernels on the call's stream (batched calls: around the
 * whole call). nrm_kernel_times
 * synchronizes those events and returns the summed durations (ms) and the
 * number of calls recorded since timing was last enabled (the last 1024 calls
 * are kept). */
int nrm_set_timing(nrm_ctx* ctx, int enable);
int nrm_kernel_times(nrm_ctx* ctx, double* reduce_ms, double* map_ms, int64_t* calls);
/* The same for batched calls: summed duration of each call's whole launch
 * sequence (staging copy, planner, both phases), and the number of calls. */
int nrm_batch_times(nrm_ctx* ctx, double* total_ms, int64_t* calls);

#ifdef __cplusplus
}
#endif

#endif /* NRM_H */
