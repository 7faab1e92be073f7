// Internal definitions of the gfx950 flow-shop bounding library (not part of
// the C ABI).  Device tables follow Table I of the paper: PTM (times), LM
// (lags), JM (Johnson order per machine pair), MM (pairs); the per-node RM
// (releases) and QM (tails) are computed on the device from each prefix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/fspbb.h"

namespace fspbb {

constexpr int kMaxJobs = 512;      // largest n (bit masks fit a 16-word register vector)
constexpr int kMaxMachines = 32;   // largest m
constexpr int kGroup = 128;        // nodes per scan group in the 16-bit path (64 lanes x 2 halves)

// Per-slot record of the general 32-bit kernel, in Johnson-with-lags order of
// its pair: job word (j >> 5), job bit (j & 31), E = lag + a, C = b - a
// (a = p[j][k], b = p[j][l]).  The pair scan is then s <- max(s, E) + C over
// unscheduled jobs, where s = timeOnM2 - timeOnM1 of Fig. 2.
struct Rec32 {
    uint32_t word, bit;
    int32_t E, C;
};

// Per-slot record of the 16-bit scan: LDS byte offset of the job's mask row
// (j * 256) and (E << 16) | (C & 0xffff).  Padding slots point at an all-zero
// row, so they leave the state unchanged.
struct Rec16 {
    uint32_t joff;
    uint32_t ce;
};

// Per-slot record of the 32-bit scan with masks in LDS: the job's mask-row
// offset (j * 256) and E, C as in Rec32.  npad slots per pair; padding slots
// point at the all-zero row n with E = C = 0.
struct RecW {
    uint32_t joff;
    int32_t E, C;
};

// Largest tail whose 16 bits, read as a half-precision number, are a finite
// value below the largest finite half (0x7bff): non-negative finite halves
// order like their bit patterns, so minima of such tails can be taken with
// the packed half-precision minimum.
constexpr int32_t kTailsHalfMax = 0x7bfe;

// Kernel-side view of an instance (passed by value).
struct DevTables {
    int32_t n, m, P;
    int32_t npad;             // slots per pair in rec16 (n rounded up to 4)
    int32_t heads;            // 1: releases are the earliest starts of unscheduled jobs
    int32_t tails16ok;        // 1: every tail is below 65536, so tails16 is exact; 2: also at most
                              // kTailsHalfMax, so the tails order like their bits read as halves
    const int32_t *p32;       // (n+1) x 32, zero-padded; row n is zero (PTM)
    const int32_t *colsum32;  // 32: sum over all jobs of p[j][k], zero-padded
    const int32_t *tails32;   // n x 32: Q[j][l] = sum_{h>l} p[j][h], zero-padded
    const uint32_t *tails16;  // n x 16: (Q[j][2c], Q[j][2c+1]) as 16-bit halves (16-bit path)
    const uint32_t *tord;     // n x 32: rank r, machine l: (job << 16) | low 16 bits of its tail, the
                              // r-th job by increasing tail on machine l (ties by job)
    const int32_t *pairs;     // P x 2: (k, l), k < l, lexicographic (MM)
    const Rec32 *rec32;       // P x n
    const Rec32 *rec32sm;     // n x P: the same records slot-major (wave-per-node kernel)
    const Rec16 *rec16;       // P x npad
    const RecW *recw;         // P x npad (32-bit scan with LDS masks)
    unsigned long long *bad;  // invalid-node counter
};

}  // namespace fspbb

// Event triples recorded around one bound launch (start, after decode, after scan).
struct TimingRecord {
    hipEvent_t ev[3];
};

struct fsp_instance_s {
    int32_t n, m, P;
    int32_t max_value;
    int32_t packed16;
    int32_t flags;
    int device;
    int64_t table_bytes;
    void *dev_blob;
    fspbb::DevTables dt;
    // host copies (kept for the host-side search code)
    int32_t *p_host;
    // optional kernel timing
    int timing = 0;
    std::vector<TimingRecord> *timing_log = nullptr;
};

namespace fspbb {
// Launchers (bound_*.hip).  Return a HIP error code.
hipError_t launch_bound_lane32(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths,
                               int64_t N, int32_t *out_lb, hipStream_t s);
// sort_depths: decode the nodes in depth order (a counting sort first), which
// evens out the per-lane prefix loops of pools of mixed depths.
hipError_t launch_bound_packed(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths,
                               int64_t N, int32_t *out_lb, hipStream_t s, bool sort_depths = true);
// The same over a caller-provided workspace (256-byte aligned, at least
// packed_workspace_bytes(I, N) bytes); allocates nothing when marks is false
// (the timing marks create events).
size_t packed_workspace_bytes(const fsp_instance_s *I, int64_t N);
hipError_t launch_bound_packed_ws(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N,
                                  int32_t *out_lb, hipStream_t s, bool sort_depths, void *ws, bool marks);

hipError_t launch_bound_wavepair(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths,
                                 int64_t N, int32_t *out_lb, hipStream_t s);

void set_last_error(hipError_t e);

// Stream-ordered device allocation.  stream_free keeps released blocks (up to
// 16 GiB) for a later stream_alloc on the same device and stream; other
// requests come from a library-owned memory pool of the current device whose
// release threshold is unbounded (pool_alloc; memory freed to it stays in it
// across stream synchronizations).  Every block from stream_alloc is released
// with stream_free, on the stream whose work last used it.
hipError_t stream_alloc(void **ptr, size_t bytes, hipStream_t s);
hipError_t stream_free(void *ptr, hipStream_t s);
hipError_t pool_alloc(void **ptr, size_t bytes, hipStream_t s);

// Pinned host buffers from a small process-wide cache: allocating and freeing
// pinned memory maps and unmaps pages and can wait for the device (a
// millisecond or more per call), so released buffers are kept for reuse.
// pinned_get returns a buffer of at least `bytes` and its capacity in *cap;
// pinned_put takes it back (the caller has synchronized every copy that
// reads or writes it).
hipError_t pinned_get(void **ptr, size_t *cap, size_t bytes);
void pinned_put(void *ptr, size_t cap);

// Records event `which` (0 = start, 1 = after decode, 2 = after scan) of the
// current launch when timing is on.  which = 0 opens a new record.
void timing_mark(fsp_instance_s *I, int which, hipStream_t s);
}  // namespace fspbb
