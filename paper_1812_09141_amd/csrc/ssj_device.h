// Device-side declarations shared by the kernels and the host runtime of libssj.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssj {

constexpr int kClasses = 5;      // length classes of |r| + |s|
constexpr int kBlock = 256;      // threads per workgroup of every verify kernel
constexpr int kWave = 64;        // CDNA wavefront width

// Per-request device counters.  Every verify launch leaves them zeroed again
// (the last workgroup to finish resets them), so a request never needs a
// memset before it runs, also not inside a captured graph.
struct alignas(256) Counters {
    unsigned long long out_count;   // passing pairs appended so far
    unsigned int err;               // != 0: an id was out of range
    unsigned int done;              // workgroups finished (last-block detection)
    unsigned int head[kClasses];    // work-stealing cursors per class queue
    unsigned int tail[kClasses];    // entries per class queue (written by classify)
    unsigned int pad[64 - 4 - 2 * kClasses];
};

// Everything one verification launch needs.
struct VerifyArgs {
    const int32_t* tok;        // collection tokens
    const uint2* desc;         // {start, len} per set
    uint32_t n_sets;
    uint32_t n;                // candidate pairs
    const int2* cand;          // (r, s) pairs
    unsigned long long tn;     // t_num
    unsigned long long tsum;   // t_num + t_den
    int2* out;                 // passing pairs
    unsigned long long cap;    // capacity of out in pairs
    Counters* ctr;             // zeroed counters (left zeroed on exit)
    long long* d_count;        // result count, -1 on an id error
    uint32_t* queues;          // kClasses queues of qcap entries (bucketed mode)
    uint32_t qcap;
    uint32_t bounds[kClasses]; // inclusive upper bound of |r|+|s| per class
    int lanes[kClasses];       // lanes per pair, per class
    int order[kClasses];       // class processing order (heaviest first)
};

// Launch helpers (defined in kernels.hip).  All return hipSuccess or the
// launch error.
hipError_t launch_build_desc(const int64_t* d_offsets, uint2* d_desc, int64_t n_sets,
                             hipStream_t st);
hipError_t launch_verify_direct(const VerifyArgs& a, int lanes, int grid, hipStream_t st);
hipError_t launch_classify(const VerifyArgs& a, int grid, hipStream_t st);
hipError_t launch_verify_bucketed(const VerifyArgs& a, int grid, hipStream_t st);

// Kernel entry points, for occupancy queries and graph capture.
const void* kernel_verify_bucketed();
const void* kernel_verify_direct(int lanes);
const void* kernel_classify();

bool lanes_supported(int lanes);

}  // namespace ssj
