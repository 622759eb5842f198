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
 *    between streams): they share its workspace.
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

/* How blocks cover the input: each block a contiguous chunk, or the grid
 * strides over the input one block-iteration at a time. */
typedef enum { NRM_LAYOUT_CHUNK = 0, NRM_LAYOUT_STRIDE = 1 } nrm_layout;

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
                           tree, 24..48; the whole tree then has height <= max_height + 26
                           (wavefront 6, block <= 4, grid combine <= 16) */
  /* map kernel */
  int32_t map_block;    /* threads per block: 64..1024, multiple of 64 */
  int32_t map_unroll;   /* 16-byte vectors per thread per iteration: 1, 2, 4 or 8 */
  int32_t map_grid;     /* blocks (upper bound) */
  int32_t map_layout;   /* nrm_layout */
  int32_t map_nt;       /* 1: non-temporal hint on the map's loads */
  int32_t reverse_map;  /* 1: each block walks its share from the end (reuse of recently read lines) */
  int32_t reserved[4];
} nrm_params;

typedef struct nrm_ctx nrm_ctx;

/* ---- the spec forms: FP32 in and out, default context, null stream -- */

/* out[i] = in[i] / sum(in[0..n)) for i in [0, n). Fig. 1 semantics with the
 * sum hoisted (Sec. IV-C). in, out: device arrays of n floats. */
int normalize(float* out, const float* in, int64_t n);

/* ---- contexts ------------------------------------------------------------ */

/* Create a context on HIP device `device` (-1: the current device). The
 * context owns workspace on that device and the launch parameters. */
int nrm_create(nrm_ctx** ctx, int device);
/* Free the context's workspace. Waits for the device to be idle first. */
int nrm_destroy(nrm_ctx* ctx);
/* The library's default launch parameters (tuned for MI355X). */
int nrm_default_params(nrm_params* params);
/* Replace the context's launch parameters; NRM_EINVAL if any field is out of range. */
int nrm_set_params(nrm_ctx* ctx, const nrm_params* params);
int nrm_get_params(const nrm_ctx* ctx, nrm_params* params);

/* ---- extended plain form ------------------------------------------------- */

/* normalize with storage dtypes, accumulation mode, context and stream.
 * in: n elements of in_dtype; out: n elements of out_dtype. Supported:
 * every pair of {F32, BF16, F16}. ctx NULL: the default context of the
 * current device. */
int nrm_normalize_ex(nrm_ctx* ctx, void* out, int out_dtype, const void* in, int in_dtype,
                     int64_t n, int accum, void* stream);

/* ---- diagnostics and measurement ------------------------------------------ */

/* Static text for a status code. */
const char* nrm_status_string(int status);
/* Detail of the last error on the calling thread (HIP error text), or "". */
const char* nrm_last_error(void);

/* Kernel timing: while enabled, every plain call records HIP events around
 * its reduce and map kernels on the call's stream. nrm_kernel_times
 * synchronizes those events and returns the summed durations (ms) and the
 * number of calls recorded since timing was last enabled (the last 1024 calls
 * are kept). */
int nrm_set_timing(nrm_ctx* ctx, int enable);
int nrm_kernel_times(nrm_ctx* ctx, double* reduce_ms, double* map_ms, int64_t* calls);

#ifdef __cplusplus
}
#endif

#endif /* NRM_H */
