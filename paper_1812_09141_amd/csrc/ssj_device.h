// Device-side declarations shared by the kernels and the host runtime of libssj.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssj {

constexpr int kClasses = 5;      // length classes of |r| + |s|
constexpr int kSpillQ = kClasses;  // queue of the thread-per-pair merges cut off by the budget
constexpr int kQueues = kClasses + 1;  // deferred-class queues, then the spill queue
constexpr int kBlock = 256;      // threads per workgroup of every verify kernel
constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kMaxReq = 16;      // requests per launch
constexpr int kHeadTokens = 6;   // leading tokens kept in each 32-byte set record
constexpr unsigned kWaveStage = 8 * kWave;  // staged output pairs per wavefront (in-order kernel)

// How a request turns set sizes into its required overlap alpha (the
// equivalent overlap of paper Table 1).
enum OverlapRule : uint32_t {
    kLinear = 0,    // alpha = ceil(num * (|r| + |s|) / den): Jaccard, Dice
    kCosine = 1,    // alpha = least o with o^2 * den^2 >= num^2 * |r| * |s|
    kConstant = 2,  // alpha = num: Overlap
};

// One verification request inside a launch.
struct Request {
    const int2* cand;          // (r, s) pairs
    int2* out;                 // passing pairs
    long long* d_count;        // result count, -1 on an id error
    unsigned long long cap;    // capacity of out in pairs
    unsigned long long num;    // threshold terms of the overlap rule
    unsigned long long den;
    uint32_t n;                // pairs
    uint32_t rule;             // OverlapRule
    // A grouped request (the C / C_O layout of paper Sec. 3.3.1) has no
    // cand: its candidates are the s ids sids[0..n), and group g = {probe id,
    // exclusive end into sids} covers sids[end(g-1) .. end(g)) with end(-1)
    // = 0.  chunk_g[t] is the first group whose end exceeds t * kWave (the
    // group of the chunk's first candidate), written by the launch's group
    // pre-pass.
    const int32_t* sids;
    const int2* groups;
    uint32_t* chunk_g;
    uint32_t n_groups;
    // division by den without a divide (kLinear, dividends below 2^32):
    // q = (t + ((x - t) >> (dshift & 0xff))) >> (dshift >> 8), t = mulhi(dmagic, x)
    uint32_t dmagic;
    uint32_t dshift;
    uint32_t pad;
};

// Per-launch device counters.  Every launch leaves them zeroed again (its
// final one-workgroup kernel resets them), so no memset is needed before a
// launch, also not inside a captured graph.
struct alignas(256) Counters {
    unsigned long long out_count[kMaxReq];  // passing pairs appended so far
    unsigned int err[kMaxReq];              // != 0: an id was out of range
    unsigned int head[kQueues];             // work-stealing cursors of the queues
    unsigned int tail[kQueues];             // entries in each queue
    unsigned int pad[64 - kMaxReq - 2 * kQueues];
};

// Everything one launch needs (passed by value as the kernel argument).
struct LaunchArgs {
    const int32_t* tok;                  // tokens of the collection of the r side of each pair
    const uint4* heads;                  // its set records: {start, len, tok0, tok1}, {tok2..tok5}
    const int32_t* tok_s;                // the same for the s side (an R-S join's second
    const uint4* heads_s;                // collection; the same collection in a self-join)
    Counters* ctr;
    uint32_t* queues;                    // kQueues queues of qcap global pair indices
    uint32_t qcap;
    uint32_t n_sets;                     // sets of the r-side collection
    uint32_t n_sets_s;                   // sets of the s-side collection
    int n_req;
    int defer_from;                      // first deferred class (kClasses: none)
    int inline_lanes;                    // lanes per pair in the in-order kernel
    int hard_lanes;                      // lanes finishing long merges (inline_lanes == 1)
    uint32_t defer_cap;                  // LDS queue entries per deferred class and wavefront (>= 2 chunks)
    uint32_t cosine;                     // != 0: some request uses the Cosine rule
    uint32_t spill_iters;                // window steps a thread-per-pair merge may take in the
                                         // in-order kernel before it is queued for the deferred
                                         // kernel (0xffffffff: no limit)
    int spill_lanes;                     // lanes per pair of the spill queue
    uint32_t staged;                     // != 0: thread-per-pair merges through the window
                                         // ring in LDS, their loads two steps ahead
                                         // (merge_ring); spill_iters counts window steps
    uint32_t grouped;                    // != 0: every request of the launch is grouped
    uint32_t* probes;                    // grouped launches that defer: the probe id of every
                                         // queued pair, by global pair index
    uint4* spill_state;                  // launches whose merges spill: {i, j, o, 0} of every
                                         // spilled merge by global pair index, from which the
                                         // deferred kernel resumes it (nullptr: it restarts)
    const uint32_t* chunk_g;             // grouped launches: every request's chunk_g, by global
                                         // chunk index (req[r].chunk_g = chunk_g + tile_off[r])
    uint32_t group_off[kMaxReq + 1];     // grouped launches: prefix sums of per-request groups
    uint32_t tile_off[kMaxReq + 1];      // prefix sums of per-request chunks (of kWave pairs)
    uint32_t pair_off[kMaxReq + 1];      // prefix sums of per-request pairs
    uint32_t bounds[kClasses];           // inclusive upper bound of |r|+|s| per class
    int lanes[kClasses];                 // lanes per pair of each deferred class
    Request req[kMaxReq];
};

// Launch helpers (defined in kernels.hip).  Return hipSuccess or the launch
// error.
// Set records (2 x uint4 per set) on the device from the CSR offsets (for
// the lengths), the start of each set in the device token array and that
// array.
hipError_t launch_build_heads(const int64_t* d_offsets, const uint32_t* d_start, const int32_t* d_tok,
                              uint4* d_heads, int64_t n_sets, hipStream_t st);
// Group pre-pass of a grouped launch (a.grouped): writes every request's
// chunk_g and checks its group ends (not decreasing, none above n, the last
// one n); malformed ends set the request's error flag, which the launch's
// finalize kernel reports.  Candidates no group covers are verified with
// probe id -1, an id error.
hipError_t launch_group_chunks(const LaunchArgs& a, hipStream_t st);
// The in-order kernel: every pair of a class below defer_from is verified
// with inline_lanes lanes; the others are queued for launch_verify_deferred,
// and so is every thread-per-pair merge still undecided after spill_iters
// window steps.
hipError_t launch_verify_tiles(const LaunchArgs& a, int grid, hipStream_t st);
// Drains the queues (needed only when defer_from < kClasses or merges spill).
hipError_t launch_verify_deferred(const LaunchArgs& a, int grid, hipStream_t st);
// Dynamic LDS of the in-order kernel for a.defer_from / a.spill_iters / a.defer_cap.
size_t tiles_lds_bytes(const LaunchArgs& a);
// Publishes the request counts and resets the counters (always last).
hipError_t launch_finalize(const LaunchArgs& a, hipStream_t st);
// Zeroes n 32-bit words of device memory with a fill kernel.
hipError_t launch_clear_words(uint32_t* d_words, size_t n, hipStream_t st);

// The in-order kernel of a mapping: lanes per pair and hard lanes, or the
// window-ring thread-per-pair merge (staged, lanes 1, hard_lanes 0); for a
// flat or a grouped launch (grouped launches have no window-ring instance:
// staged selects the plain one).
const void* kernel_verify_tiles(int lanes, int hard_lanes, bool staged, bool deferring, bool cosine, bool grouped);
const void* kernel_verify_deferred(bool cosine, bool grouped);
const void* kernel_finalize();

// LDS queues of a wavefront of the in-order kernel: one per deferred class,
// one more for spilled merges.
__host__ __device__ inline int wave_queues(int defer_from, bool spill) { return kClasses - defer_from + (spill ? 1 : 0); }
__host__ __device__ inline bool spilling(const LaunchArgs& a) { return a.spill_iters != 0xffffffffu; }

bool lanes_supported(int lanes);              // deferred classes: 1..64 or kBlock
bool inline_supported(int lanes, int hard_lanes, bool staged);  // in-order kernel: 1..64; 0/8/16 hard
                                                                 // lanes with 1; staged with 1 and 0

}  // namespace ssj
