// Internal interface of the device queue: the server's persistent-kernel
// executor (nrm_server.cpp) and the kernel that runs it (nrm_dq.hip).
// Not part of the public ABI.
//
// The host publishes each admitted request into a ring in pinned, coherent
// host memory; one persistent kernel polls the ring, copies new requests into
// device memory, and its blocks take the requests' work units from a ticket
// counter in order. A request of
// n <= DQ_RESIDENT_MAX elements is one unit per resident segment (held in a
// block's registers from its read to its write, as the resident rows of a
// batch are); a longer one is m units that each sum one part of 2^DQ_LONG_LOG2
// elements, then m units that divide those parts by the request's sum. The
// last unit of a request to finish writes the request's completion word into
// host memory, which the host polls: no kernel launch per request.
#pragma once

#include <stdint.h>

#include "nrm_batch.h"

namespace nrm {

constexpr int DQ_RING = 64;            // requests in flight at most (one wavefront lane each)
constexpr int DQ_LONG_LOG2 = 15;       // elements of one part of a long request: 2^15
constexpr int DQ_MAX_PARTS = 1024;     // parts of a long request (16 partials per lane in the merge)
constexpr int64_t DQ_RESIDENT_MAX = (int64_t)RES_MAX_SEGMENTS << RES_LOG2;  // 2^20
constexpr int64_t DQ_MAX_N = (int64_t)DQ_MAX_PARTS << DQ_LONG_LOG2;         // 2^25
constexpr int DQ_KEY_UNIT_BITS = 12;   // a ring key packs (first unit << 12) | units

// Units of a request of n elements (n >= 1, n <= DQ_MAX_N).
__host__ __device__ inline int64_t dq_units(int64_t n) {
  if (n <= DQ_RESIDENT_MAX) return (n + (int64_t(1) << RES_LOG2) - 1) >> RES_LOG2;
  return 2 * ((n + (int64_t(1) << DQ_LONG_LOG2) - 1) >> DQ_LONG_LOG2);
}

// A request in the kernel's device ring (64 bytes), copied from its published
// words; the kernel numbers its units (key) as it copies.
struct DqReq {
  RowDesc d;       // in, out, n, dtypes
  uint64_t key;    // (first unit << DQ_KEY_UNIT_BITS) | units
  uint64_t seq;    // request number, from 0
  int32_t slot;    // the completion word the request reports to
  int32_t pad;
  uint64_t pad2;
};
static_assert(sizeof(DqReq) == 64, "a request is one 64-byte line");

// Pinned, coherent host memory shared by the host and the kernel. The host
// publishes request r as four words in line r % DQ_PUB, each carrying the
// request's 16-bit tag in its top bits (in, out, n, and the dtypes and slot
// below the tag), so that one read of a line tells the kernel whether the
// whole request is there: no counter to read first, no ordering between the
// words. A line is reused only after its request was copied (a request not
// copied yet is in flight, and at most DQ_RING are).
constexpr int DQ_PUB = 2 * DQ_RING;
constexpr int DQ_TAG_SHIFT = 48;  // device and host addresses, and n, fit below
struct DqPubLine {
  uint64_t w[4];
  uint64_t pad[4];
};
struct DqHost {
  uint64_t stop;                // host: 1 = end once nothing new is published
  uint64_t hold;                // host: 1 = end dq_hold (the stream probe at set-up)
  uint64_t pad0[14];
  DqPubLine pub[DQ_PUB];        // host
  uint64_t done[DQ_RING];       // per slot: tag of the last request completed there (device)
  uint64_t stalled[DQ_RING];    // per slot: tag of a request whose wait gave up (device)
};

// The 16-bit tag of request r in its published words (never 0).
__host__ __device__ inline uint64_t dq_pub_tag(uint64_t r) { return r % 0xFFFFull + 1; }

// The kernel's state in device memory (zeroed once, kept across launches).
struct DqDev {
  unsigned long long next_unit;   // tickets handed out
  unsigned long long pub_units;   // units of the requests copied so far
  unsigned long long pub_reqs;    // requests copied so far
  unsigned long long exit_epoch;  // set to the launch's number when it ends
  unsigned long long last_seen;   // device clock when new requests were last copied (or the launch began)
  unsigned long long stall;       // tag of the last request whose wait gave up
  int error;                      // NRM_DEVERR_* bits
  int pad;
  unsigned long long launched_at; // device clock when this launch began
  unsigned long long pad1[8];
  DqReq ring[DQ_RING];                    // by slot, copied from the host's
  unsigned long long key[DQ_RING];        // ring[i].key, also read alone in the lookup
  unsigned arrivals[DQ_RING];             // parts or segments that have published (0 between requests)
  unsigned finished[DQ_RING];             // units whose outputs are written (0 between requests)
  unsigned long long total[DQ_RING][2];   // the request's sum, tagged words
  unsigned long long tagged[DQ_RING][2 * DQ_MAX_PARTS];  // each part's or segment's partial, tagged words
};

struct DqArgs {
  DqHost* host;             // device address of the pinned block
  DqDev* dev;
  unsigned long long epoch; // this launch's number (>= 1)
  unsigned long long idle_ticks;  // device clock ticks without new requests before the kernel ends
  unsigned long long slice_ticks; // device clock ticks after which the launch ends (0: none)
};

// The tag of request seq in the exchange words (never 0, the value of a word
// that was never written).
__host__ __device__ inline uint32_t dq_tag(uint64_t seq) { return (uint32_t)(seq % 0xFFFFFFFFull) + 1u; }

// Reset the ticket counter to the copied units and clear the exit flag, then
// run the persistent kernel with `blocks` blocks of RES_BLOCK threads.
hipError_t launch_dq(const DqArgs& a, int acc, int64_t blocks, hipStream_t s);

// Set-up probe of which streams share the kernel's hardware queue (a kernel
// queued behind the persistent one on a shared queue would wait for it to
// end): dq_hold keeps stream s busy until host->hold is set or max_ticks of
// the device clock pass; dq_touch is an empty kernel.
hipError_t launch_dq_hold(const DqHost* host, unsigned long long max_ticks, hipStream_t s);
hipError_t launch_dq_touch(hipStream_t s);

}  // namespace nrm
