// Host runtime of libssj: the C ABI, the HBM collection store, device scratch
// and launch management (plans, batching, graph replay, autotuning) and the
// streaming request loop.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <ctime>
#include <deque>
#include <new>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "ssj.h"
#include "ssj_device.h"
#include "filter.h"

namespace {

thread_local std::string tl_error;

int set_error(int code, const std::string& msg) {
    tl_error = msg;
    return code;
}

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

constexpr uint64_t kDefaultBudget = 4ull << 30;
// The allocation-free entry point's device scratch: a counter block, then the
// deferral queues for up to SSJ_NOALLOC_MAX_PAIRS pairs.
constexpr size_t kNoAllocQueueWords = (size_t)ssj::kQueues * SSJ_NOALLOC_MAX_PAIRS;
constexpr size_t kNoAllocBytes = sizeof(ssj::Counters) + kNoAllocQueueWords * sizeof(uint32_t);
constexpr int kMaxDevices = 64;
constexpr int64_t kMaxLaunchPairs = ((int64_t)1 << 31) - 1;  // pairs per launch
constexpr int kMaxSpillIters = 1 << 20;
constexpr int kMaxWgPerCu = 64;
// device bytes per candidate pair of a request: the pair, a worst-case output
// pair, and its queue entries
constexpr size_t kBytesPerPair = 8 + 8 + 4 * ssj::kQueues;
// host-buffer verification: candidates pass through a ring of two pinned
// buffers of kRingPiece pairs, at most kMaxPieces pieces per device batch
constexpr int64_t kRingPiece = (int64_t)1 << 20;
constexpr int64_t kMaxPieces = 64;
// a stream slot may always hold this many pairs, whatever the budget leaves
constexpr int64_t kSlotFloor = 1024;
constexpr int64_t kSlotResults = (int64_t)1 << 16;  // pinned result pairs per slot at start

// Threshold range of a similarity function (SSJ_SIM_*): 0 < t_den < 2^31,
// 0 <= t_num < 2^31, and t <= 1 for the normalised functions.
bool valid_threshold(int sim, int64_t t_num, int64_t t_den) {
    if (sim < SSJ_SIM_JACCARD || sim > SSJ_SIM_OVERLAP) return false;
    if (t_den <= 0 || t_den > INT32_MAX || t_num < 0 || t_num > INT32_MAX) return false;
    return sim == SSJ_SIM_OVERLAP || t_num <= t_den;
}

const char* kThresholdError =
    "bad similarity function or threshold: need 0 < t_den < 2^31, 0 <= t_num < 2^31, "
    "and t_num <= t_den except for SSJ_SIM_OVERLAP";

// The request's required-overlap rule (paper Table 1 in integers):
//   Jaccard  ceil(t_num (|r|+|s|) / (t_num + t_den))
//   Dice     ceil(t_num (|r|+|s|) / (2 t_den))
//   Cosine   least o with o^2 t_den^2 >= t_num^2 |r| |s|
//   Overlap  ceil(t_num / t_den)
// Magic number and shifts for dividing 32-bit dividends by d (1 <= d <
// 2^32) with one high multiply (Granlund and Montgomery, "Division by
// Invariant Integers using Multiplication", PLDI 1994, the unsigned round-up
// method): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, then
// floor(x / d) = (t + ((x - t) >> min(l, 1))) >> max(l - 1, 0) with t the
// high word of m x.
void division_magic(unsigned long long d, ssj::Request& R) {
    int l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    const unsigned __int128 num = ((unsigned __int128)1 << 32) * (((unsigned __int128)1 << l) - d);
    R.dmagic = (uint32_t)(num / d + 1u);
    R.dshift = (uint32_t)std::min(l, 1) | ((uint32_t)std::max(l - 1, 0) << 8);
}

void overlap_rule(int sim, int64_t t_num, int64_t t_den, ssj::Request& R) {
    switch (sim) {
        case SSJ_SIM_DICE:
            R.rule = ssj::kLinear;
            R.num = (unsigned long long)t_num;
            R.den = 2ull * (unsigned long long)t_den;
            break;
        case SSJ_SIM_COSINE:
            R.rule = ssj::kCosine;
            R.num = (unsigned long long)t_num;
            R.den = (unsigned long long)t_den;
            break;
        case SSJ_SIM_OVERLAP:
            R.rule = ssj::kConstant;
            R.num = (unsigned long long)((t_num + t_den - 1) / t_den);
            R.den = 1ull;
            break;
        default:
            R.rule = ssj::kLinear;
            R.num = (unsigned long long)t_num;
            R.den = (unsigned long long)(t_num + t_den);
            break;
    }
    // every den here is below 2^32 (thresholds below 2^31)
    division_magic(R.den, R);
}

template <class T>
hipError_t grow(T*& p, size_t& cap, size_t need) {
    if (need <= cap && p) return hipSuccess;
    size_t n = std::max<size_t>(need, cap + cap / 2);
    n = std::max<size_t>(n, 1024);
    if (p) {
        // the old buffer may still be read by work queued on any stream
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        e = hipFree(p);
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc((void**)&p, n * sizeof(T));
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = n;
    return hipSuccess;
}

// Device scratch of one launch in flight: counters and deferred queues.
struct Scratch {
    ssj::Counters* d_ctr = nullptr;
    uint32_t* d_queues = nullptr;
    size_t q_cap = 0;  // entries (kQueues x per-queue capacity)
    uint32_t* d_chunk_g = nullptr;  // grouped launches: first group of every chunk
    size_t chunk_cap = 0;
    uint32_t* d_probes = nullptr;   // grouped launches that defer: probe id per queued pair
    size_t probes_cap = 0;
    // launches whose merges spill: the merge state of every spilled pair, so
    // that the deferred kernel resumes it (only where resume is set: the
    // context's own scratch; stream slots and the allocation-free entry point
    // restart spilled merges instead of holding 16 bytes per pair)
    bool resume = false;
    uint4* d_spill = nullptr;
    size_t spill_cap = 0;
};

struct GraphKey {
    int inline_lanes, hard_lanes, staged, defer_from, spill, cosine, grid1, grid2;
    bool operator<(const GraphKey& o) const {
        return std::tie(inline_lanes, hard_lanes, staged, defer_from, spill, cosine, grid1, grid2) <
               std::tie(o.inline_lanes, o.hard_lanes, o.staged, o.defer_from, o.spill, o.cosine, o.grid1,
                        o.grid2);
    }
};

// A launch as a graph of kernel nodes (in-order, [deferred], finalize) whose
// arguments are replaced before every replay.
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t nodes[3] = {nullptr, nullptr, nullptr};
    hipKernelNodeParams params[3] = {};
    int n_nodes = 0;
};

}  // namespace

// Scratch of ssj_verify_device_noalloc, one copy per device for the life of
// the process.  Host code never passes this name to a kernel: it takes the
// array's device address from hipGetSymbolAddress (noalloc_scratch) and
// uses that.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of scratch, per device (null: not set up)

}  // namespace

struct ssj_coll {
    ssj_ctx* ctx = nullptr;
    int32_t* d_tok = nullptr;
    uint4* d_heads = nullptr;  // 32-byte record per set: start, len, first tokens
    int64_t n_sets = 0;
    int64_t n_tokens = 0;
    int64_t max_len = 0;
    uint64_t dev_bytes = 0;  // device bytes of its tokens and set records
    mutable std::atomic<int> inflight{0};  // stream requests not yet finished
};

struct StreamEngine;

struct ssj_ctx {
    int device = 0;
    std::string device_key;   // architecture, name and compute units (tuning cache key)
    std::string tune_cache;   // tuning cache file ("" = none)
    uint64_t budget = kDefaultBudget;
    std::atomic<uint64_t> resident{0};  // device bytes of the uploaded collections (within budget)
    int n_slots = 4;
    int queue_depth = 64;
    int n_cu = 0;
    // in-order kernel workgroups per CU, limited by registers and by its
    // dynamic LDS: [4 * mapping index + 2 * cosine + deferring][deferred classes]
    // [8 * mapping + 4 * grouped + 2 * cosine + deferring][LDS queues per wavefront]
    int occ_tiles[8 * 9][ssj::kQueues + 1] = {};
    int occ_deferred2[4] = {0};  // [2 * grouped + cosine]
    ssj_plan plan{};
    std::mutex mu;  // default scratch, host staging, collections, plan, graphs
    // also held while the plan changes (after mu), so that the stream engine,
    // which holds its own lock, can read the plan without taking mu (the
    // lock order is mu, then the engine's lock)
    std::mutex plan_mu;
    hipStream_t stream = nullptr;  // the context's own stream (host-buffer calls)
    hipStream_t copy_stream = nullptr;  // host-to-device copies of the host-buffer path's pieces
    Scratch def;
    // host-buffer verify staging
    int2* d_cand = nullptr;
    size_t cand_cap = 0;
    int2* d_out = nullptr;
    size_t out_cap = 0;
    long long* d_count = nullptr;
    long long* h_count = nullptr;  // pinned
    // the pinned ring of the host-buffer path (allocated on first use), one
    // event per buffer (its last copy to the device, on copy_stream),
    // per-piece counts
    int2* h_ring[2] = {nullptr, nullptr};
    hipEvent_t ring_ev[2] = {nullptr, nullptr};
    long long* d_counts = nullptr;  // kMaxPieces
    long long* h_counts = nullptr;  // pinned, kMaxPieces
    uint64_t ring_seq = 0;
    // grouped candidates: host-call staging of groups and s ids, and the
    // flat pairs they expand to (with one word per 64 candidates)
    int2* d_groups = nullptr;
    size_t groups_cap = 0;
    int32_t* d_sids = nullptr;
    size_t sids_cap = 0;
    int2* d_pairs = nullptr;
    size_t pairs_cap = 0;
    // GPU candidate generation (prefix index and probe counts)
    struct {
        uint32_t *plen = nullptr, *pre = nullptr, *pos = nullptr, *pos2 = nullptr;
        unsigned long long *keys = nullptr, *keys2 = nullptr, *counts = nullptr, *off = nullptr,
                           *items = nullptr, *istart = nullptr;
        uint2 *probes = nullptr, *range = nullptr;
        unsigned char* temp = nullptr;
        size_t plen_cap = 0, pre_cap = 0, pos_cap = 0, pos2_cap = 0, counts_cap = 0, off_cap = 0,
               keys_cap = 0, keys2_cap = 0, probes_cap = 0, temp_cap = 0, items_cap = 0, istart_cap = 0,
               range_cap = 0;
    } flt;
    std::atomic<bool> failed{false};
    std::vector<ssj_coll*> colls;
    std::map<GraphKey, GraphEntry> graphs;
    hipStream_t capture_stream = nullptr;
    // kernel timing (ssj_timing_*): every timing_period-th launch is timed
    std::atomic<int> timing_period{0};
    std::atomic<uint64_t> timing_tick{0};
    std::mutex tmu;
    std::vector<hipEvent_t> ev_pool;
    // sampled launches: start / end of the in-order kernel, start / end of
    // the deferred kernel (null when none ran)
    std::vector<std::array<hipEvent_t, 4>> ev_pending;
    double t_inorder_ms = 0.0, t_deferred_ms = 0.0;
    int64_t t_launches = 0;
    std::unique_ptr<StreamEngine> engine;
    Scratch noalloc;  // views into this device's copy of scratch (owned by nobody)
};

namespace {

int hip_fail(ssj_ctx* ctx, const char* what, hipError_t e) {
    if (ctx) ctx->failed = true;
    return set_error(SSJ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(ctx, expr)                                   \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) return hip_fail((ctx), #expr, _e); \
    } while (0)

// index of an in-order mapping in occ_tiles
int inline_index(int lanes, int hard_lanes, int staged) {
    if (staged) return 8;
    if (lanes == 1) return hard_lanes == 0 ? 0 : (hard_lanes == 8 ? 6 : 7);
    switch (lanes) {
        case 4: return 1;
        case 8: return 2;
        case 16: return 3;
        case 32: return 4;
        case 64: return 5;
        default: return 0;
    }
}

// in-order mappings: by lanes, hard lanes and staging (the window ring)
constexpr int kMappings = 9;
const int kInlineLanes[kMappings] = {1, 4, 8, 16, 32, 64, 1, 1, 1};
const int kInlineHard[kMappings] = {0, 0, 0, 0, 0, 0, 8, 16, 0};
const int kInlineStaged[kMappings] = {0, 0, 0, 0, 0, 0, 0, 0, 1};

int scratch_init(ssj_ctx* ctx, Scratch& s) {
    HIP_OR_FAIL(ctx, hipMalloc((void**)&s.d_ctr, sizeof(ssj::Counters)));
    HIP_OR_FAIL(ctx, hipMemset(s.d_ctr, 0, sizeof(ssj::Counters)));
    HIP_OR_FAIL(ctx, hipDeviceSynchronize());
    return SSJ_OK;
}

void scratch_free(Scratch& s) {
    if (s.d_ctr) (void)hipFree(s.d_ctr);
    if (s.d_queues) (void)hipFree(s.d_queues);
    if (s.d_chunk_g) (void)hipFree(s.d_chunk_g);
    if (s.d_probes) (void)hipFree(s.d_probes);
    if (s.d_spill) (void)hipFree(s.d_spill);
    s = Scratch{};
}

void default_plan(ssj_plan& p) {
    p.inline_lanes = 1;
    p.hard_lanes = 0;
    p.defer_from = 3;
    const int lanes[ssj::kClasses] = {4, 16, 64, ssj::kBlock, ssj::kBlock};
    for (int q = 0; q < ssj::kClasses; ++q) p.lanes[q] = lanes[q];
    p.use_graph = 0;
    p.spill_iters = 0;
    p.spill_lanes = 16;
    p.wg_per_cu = 0;
    p.staged = 0;
}

bool plan_valid(const ssj_plan& p) {
    if (p.staged != 0 && p.staged != 1) return false;
    if (!ssj::inline_supported(p.inline_lanes, p.hard_lanes, p.staged != 0)) return false;
    if (p.defer_from < 0 || p.defer_from > ssj::kClasses) return false;
    for (int q = 0; q < ssj::kClasses; ++q)
        if (!ssj::lanes_supported(p.lanes[q])) return false;
    if (p.spill_iters < 0 || p.spill_iters > kMaxSpillIters || !ssj::lanes_supported(p.spill_lanes))
        return false;
    if (p.spill_iters > 0 && (p.inline_lanes != 1 || p.hard_lanes != 0)) return false;
    if (p.wg_per_cu < 0 || p.wg_per_cu > kMaxWgPerCu) return false;
    return true;
}

// A plan runs the deferred kernel when it defers classes or cuts merges off.
bool plan_two_kernels(const ssj_plan& p) { return p.defer_from < ssj::kClasses || p.spill_iters > 0; }

hipEvent_t timing_event(ssj_ctx* ctx) {
    std::lock_guard<std::mutex> g(ctx->tmu);
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    // no system-scope fence on completion: the events only time kernels
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// One request of a launch, host side.
struct Req {
    const int2* d_cand;
    int64_t n;
    int64_t t_num, t_den;
    int2* d_out;
    int64_t out_cap;
    long long* d_count;
    int sim = SSJ_SIM_JACCARD;
    // grouped request (d_cand unused): s ids and groups {probe id, end}
    const int32_t* d_sids = nullptr;
    const int2* d_groups = nullptr;
    int64_t n_groups = 0;
    bool grouped = false;
};

int check_req(const Req& r) {
    if (!valid_threshold(r.sim, r.t_num, r.t_den)) return set_error(SSJ_EINVAL, kThresholdError);
    if (r.n < 0) return set_error(SSJ_EINVAL, "negative candidate count");
    if (r.out_cap < 0) return set_error(SSJ_EINVAL, "negative output capacity");
    if (!r.d_count || (r.n > 0 && !r.d_cand)) return set_error(SSJ_EINVAL, "null device buffer");
    if (r.out_cap > 0 && !r.d_out) return set_error(SSJ_EINVAL, "out_cap > 0 with a null output buffer");
    return SSJ_OK;
}

// Workgroups of a kBlock-thread kernel that one compute unit holds at once
// as far as vector registers go: each workgroup puts one wavefront on each of
// the four SIMDs, and a SIMD has 512 registers per lane, allocated to a
// wavefront in blocks of 16 (measured on gfx950: a kernel with 70 registers
// runs 6 wavefronts per SIMD, where blocks of 8 would allow 7).
int vgpr_limited_blocks(const void* f) {
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, f) != hipSuccess || attr.numRegs <= 0) return 1 << 20;
    const int alloc = (attr.numRegs + 15) / 16 * 16;
    return std::max(1, std::min(8, 512 / alloc));
}

// Workgroups of the in-order kernel that the device holds at once per
// compute unit.
int tiles_occupancy(const ssj_ctx* ctx, const ssj_plan& plan, bool cosine, bool grouped = false) {
    const bool deferring = plan_two_kernels(plan);
    const int nq = ssj::wave_queues(plan.defer_from, plan.spill_iters > 0);
    return std::max(1, ctx->occ_tiles[8 * inline_index(plan.inline_lanes, plan.hard_lanes, plan.staged) +
                                      (grouped ? 4 : 0) + (cosine ? 2 : 0) + (deferring ? 1 : 0)][nq]);
}

// Workgroups of the in-order kernel: one per kBlock / kWave chunks, at most
// plan.wg_per_cu per compute unit, or what the device holds at once.
int grid_tiles(const ssj_ctx* ctx, const ssj_plan& plan, bool cosine, bool grouped, int64_t n_chunks) {
    const int per_cu = plan.wg_per_cu > 0 ? plan.wg_per_cu : tiles_occupancy(ctx, plan, cosine, grouped);
    const int64_t cap = (int64_t)ctx->n_cu * per_cu;
    const int64_t per_wg = ssj::kBlock / ssj::kWave;
    return (int)std::max<int64_t>(1, std::min<int64_t>((n_chunks + per_wg - 1) / per_wg, cap));
}

int grid_deferred(const ssj_ctx* ctx, bool cosine, bool grouped) {
    return ctx->n_cu * std::max(1, ctx->occ_deferred2[(grouped ? 2 : 0) + (cosine ? 1 : 0)]);
}

int launch_graph(ssj_ctx* ctx, const ssj::LaunchArgs& a, int g1, int g2, bool two,
                 hipStream_t st) {
    GraphKey key{a.inline_lanes, a.hard_lanes, (int)a.staged, a.defer_from, ssj::spilling(a) ? 1 : 0,
                 (int)a.cosine, g1, two ? g2 : 0};
    ssj::LaunchArgs args = a;
    void* kparams[] = {&args};
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        GraphEntry ge;
        HIP_OR_FAIL(ctx, hipGraphCreate(&ge.graph, 0));
        // (grouped launches do not use graphs)
        const void* funcs[3] = {ssj::kernel_verify_tiles(a.inline_lanes, a.hard_lanes, a.staged != 0, two,
                                                         a.cosine != 0, false),
                                ssj::kernel_verify_deferred(a.cosine != 0, false), ssj::kernel_finalize()};
        const int grids[3] = {g1, g2, 1};
        const int blocks[3] = {ssj::kBlock, ssj::kBlock, ssj::kWave};
        for (int k = 0; k < 3; ++k) {
            if (k == 1 && !two) continue;
            hipKernelNodeParams p{};
            p.func = const_cast<void*>(funcs[k]);
            p.gridDim = dim3((unsigned)grids[k]);
            p.blockDim = dim3((unsigned)blocks[k]);
            p.sharedMemBytes = k == 0 ? (unsigned)ssj::tiles_lds_bytes(a) : 0u;
            p.kernelParams = kparams;
            p.extra = nullptr;
            hipGraphNode_t dep = ge.n_nodes ? ge.nodes[ge.n_nodes - 1] : nullptr;
            HIP_OR_FAIL(ctx, hipGraphAddKernelNode(&ge.nodes[ge.n_nodes], ge.graph, dep ? &dep : nullptr,
                                                   dep ? 1 : 0, &p));
            ge.params[ge.n_nodes] = p;
            ++ge.n_nodes;
        }
        HIP_OR_FAIL(ctx, hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
        it = ctx->graphs.emplace(key, ge).first;
    } else {
        GraphEntry& ge = it->second;
        for (int k = 0; k < ge.n_nodes; ++k) {
            hipKernelNodeParams p = ge.params[k];
            p.kernelParams = kparams;
            HIP_OR_FAIL(ctx, hipGraphExecKernelNodeSetParams(ge.exec, ge.nodes[k], &p));
        }
    }
    HIP_OR_FAIL(ctx, hipGraphLaunch(it->second.exec, st));
    return SSJ_OK;
}

// Enqueues one launch verifying up to kMaxReq requests already on the device:
// r ids index coll, s ids coll_s (null: coll, a self-join).
int enqueue_launch(ssj_ctx* ctx, const ssj_coll* coll, Scratch& sc, const Req* reqs, int n_req,
                   hipStream_t st, const ssj_plan& plan, bool allow_graph = true,
                   const ssj_coll* coll_s = nullptr, bool allow_timing = true) {
    const ssj_coll* cs = coll_s ? coll_s : coll;
    ssj::LaunchArgs a{};
    a.tok = coll->d_tok;
    a.heads = coll->d_heads;
    a.tok_s = cs->d_tok;
    a.heads_s = cs->d_heads;
    a.ctr = sc.d_ctr;
    a.n_sets = (uint32_t)coll->n_sets;
    a.n_sets_s = (uint32_t)cs->n_sets;
    a.n_req = n_req;
    a.defer_from = plan.defer_from;
    a.inline_lanes = plan.inline_lanes;
    a.hard_lanes = plan.hard_lanes;
    a.spill_iters = plan.spill_iters > 0 ? (uint32_t)plan.spill_iters : 0xffffffffu;
    a.spill_lanes = plan.spill_lanes;
    a.staged = plan.staged ? 1u : 0u;
    // in-order work unit: a chunk of kWave pairs of one request per wavefront
    const uint64_t tile_pairs = (uint64_t)ssj::kWave;
    a.defer_cap = (uint32_t)(2 * tile_pairs);
    const uint32_t bounds[ssj::kClasses] = SSJ_CLASS_BOUNDS;
    for (int q = 0; q < ssj::kClasses; ++q) {
        a.bounds[q] = bounds[q];
        a.lanes[q] = plan.lanes[q];
    }
    // a launch is grouped when its requests are (callers never mix the two);
    // grouped launches have no window-ring instance
    a.grouped = n_req > 0 && reqs[0].grouped ? 1u : 0u;
    if (a.grouped) a.staged = 0u;
    uint64_t tiles = 0, pairs = 0, groups = 0;
    for (int r = 0; r < n_req; ++r) {
        const Req& q = reqs[r];
        a.tile_off[r] = (uint32_t)tiles;
        a.pair_off[r] = (uint32_t)pairs;
        a.group_off[r] = (uint32_t)groups;
        ssj::Request& R = a.req[r];
        R.cand = q.d_cand;
        R.out = q.d_out;
        R.d_count = q.d_count;
        R.cap = (unsigned long long)q.out_cap;
        overlap_rule(q.sim, q.t_num, q.t_den, R);
        if (R.rule == ssj::kCosine) a.cosine = 1u;
        R.n = (uint32_t)q.n;
        if (a.grouped) {
            // a request without candidates has nothing to verify: its groups
            // are not read (nor checked)
            R.sids = q.d_sids;
            R.groups = q.d_groups;
            R.n_groups = q.n > 0 ? (uint32_t)q.n_groups : 0u;
            groups += R.n_groups;
        }
        tiles += ((uint64_t)q.n + tile_pairs - 1) / tile_pairs;
        pairs += (uint64_t)q.n;
    }
    a.tile_off[n_req] = (uint32_t)tiles;
    a.pair_off[n_req] = (uint32_t)pairs;
    a.group_off[n_req] = (uint32_t)groups;
    const bool two = plan_two_kernels(plan);
    if (two) {
        HIP_OR_FAIL(ctx, grow(sc.d_queues, sc.q_cap, (size_t)ssj::kQueues * std::max<uint64_t>(pairs, 1)));
    }
    if (two && sc.resume && ssj::spilling(a)) {
        HIP_OR_FAIL(ctx, grow(sc.d_spill, sc.spill_cap, (size_t)std::max<uint64_t>(pairs, 1)));
        a.spill_state = sc.d_spill;
    }
    if (a.grouped) {
        HIP_OR_FAIL(ctx, grow(sc.d_chunk_g, sc.chunk_cap, (size_t)std::max<uint64_t>(tiles, 1)));
        a.chunk_g = sc.d_chunk_g;
        for (int r = 0; r < n_req; ++r) a.req[r].chunk_g = sc.d_chunk_g + a.tile_off[r];
        if (two) {
            HIP_OR_FAIL(ctx, grow(sc.d_probes, sc.probes_cap, (size_t)std::max<uint64_t>(pairs, 1)));
            a.probes = sc.d_probes;
        }
    }
    a.queues = sc.d_queues;
    a.qcap = (uint32_t)(sc.q_cap / ssj::kQueues);
    const int g1 = grid_tiles(ctx, plan, a.cosine != 0, a.grouped != 0, (int64_t)tiles);
    const int g2 = grid_deferred(ctx, a.cosine != 0, a.grouped != 0);

    std::array<hipEvent_t, 4> ev{nullptr, nullptr, nullptr, nullptr};
    const int period = ctx->timing_period.load();
    const bool timing = allow_timing && period > 0 && (ctx->timing_tick.fetch_add(1) % (uint64_t)period) == 0;
    if (timing) {
        // marker events right before and after each verification kernel (the
        // finalize kernel is not timed)
        for (int k = 0; k < (two ? 4 : 2); ++k) {
            ev[k] = timing_event(ctx);
            if (!ev[k]) return hip_fail(ctx, "hipEventCreate", hipErrorOutOfMemory);
        }
    }
    // grouped launches start with the group pre-pass (outside the graph and
    // the timing events, which cover the verification kernels)
    if (a.grouped) HIP_OR_FAIL(ctx, ssj::launch_group_chunks(a, st));
    if (plan.use_graph && allow_graph && !timing && !a.grouped) {
        int rc = launch_graph(ctx, a, g1, g2, two, st);
        if (rc != SSJ_OK) return rc;
    } else {
        if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev[0], st));
        HIP_OR_FAIL(ctx, ssj::launch_verify_tiles(a, g1, st));
        if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev[1], st));
        if (two) {
            if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev[2], st));
            HIP_OR_FAIL(ctx, ssj::launch_verify_deferred(a, g2, st));
            if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev[3], st));
        }
        HIP_OR_FAIL(ctx, ssj::launch_finalize(a, st));
    }
    if (timing) {
        std::lock_guard<std::mutex> g(ctx->tmu);
        ctx->ev_pending.push_back(ev);
    }
    return SSJ_OK;
}

// Budget bytes left for candidate buffers next to the resident collections.
uint64_t free_budget(const ssj_ctx* ctx) {
    const uint64_t r = ctx->resident.load();
    return r < ctx->budget ? ctx->budget - r : 0u;
}

int check_ctx(ssj_ctx* ctx) {
    if (!ctx) return set_error(SSJ_EINVAL, "null context");
    if (ctx->failed) return set_error(SSJ_EDEVICE, "context failed after a HIP error");
    return SSJ_OK;
}

int check_coll(ssj_ctx* ctx, const ssj_coll* coll) {
    if (!coll) return set_error(SSJ_EINVAL, "null collection");
    if (coll->ctx != ctx) return set_error(SSJ_EINVAL, "collection does not belong to this context");
    return SSJ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Streaming: requests are copied to pinned staging at submit; an engine
// thread admits batches of them into free slots (each slot owns device
// buffers sized from the HBM budget and its own stream), one launch per
// batch, and collects the results.
struct StreamReq {
    uint64_t ticket = 0;
    const ssj_coll* coll = nullptr;
    int64_t t_num = 0, t_den = 1;
    int sim = SSJ_SIM_JACCARD;
    int64_t n = 0;
    int2* h_cand = nullptr;       // pinned copy of the candidates
    size_t h_cand_bytes = 0;
    // a request is verified in parts (it may be split across slots and launches);
    // it is finished when every candidate was admitted and every admitted part
    // has completed
    int64_t parts_admitted = 0, parts_done = 0, next_part_off = 0;
    bool finished = false;
    std::vector<int2> result;
    int status = SSJ_PENDING;    // SSJ_PENDING until every part is done
    bool bad_id = false;         // a part reported an id out of range
    bool failed = false;         // a part hit a device failure
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
};

struct SlotPart {
    StreamReq* req;
    int64_t off, n;         // range of the request's candidates
    int64_t dev_off;        // offset in the slot's device buffers
    int64_t res_off;        // offset of its results in the slot's pinned result buffer
};

// A slot: a stream and the device buffers of one launch in flight.  The
// buffers are sized on demand (to the largest batch the slot has taken) within
// the part of the HBM budget that the collections and the other slots leave.
struct StreamSlot {
    hipStream_t stream = nullptr;
    Scratch sc;
    int2* d_cand = nullptr;
    int2* d_out = nullptr;
    long long* d_count = nullptr;
    long long* h_count = nullptr;    // pinned, kMaxReq entries
    int2* h_out = nullptr;           // pinned results of the batch, h_cap pairs (grown on demand)
    int64_t h_cap = 0;
    size_t cand_cap = 0, out_cap = 0;  // pairs d_cand and d_out hold
    int64_t cap = 0;                 // pairs all device buffers hold
    uint64_t held = 0;               // device bytes of d_cand, d_out and the queues
    hipEvent_t ev = nullptr;
    int state = 0;                   // 0 idle, 1 running, 2 reading results, 3 results on host
    std::vector<SlotPart> parts;
    const ssj_coll* coll = nullptr;
};

struct StreamEngine {
    ssj_ctx* ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_space, cv_done;
    std::deque<StreamReq*> pending;     // not fully admitted
    int reserved = 0;                   // queue places taken by submits still copying their candidates
    std::unordered_map<uint64_t, StreamReq*> table;
    std::vector<StreamSlot> slots;
    uint64_t held = 0;                  // device bytes held by all slots' buffers
    uint64_t next_ticket = 1;
    bool stop = false;
    bool paused = false;                // ssj_stream_pause: admit nothing (until stop)
    std::thread worker;
    // pinned staging pool by size class (powers of two)
    std::map<size_t, std::vector<void*>> pool;
    // pinned result buffers outgrown by their slot: freed at stop (a
    // hipHostFree would wait for the whole device inside the engine loop)
    std::vector<void*> retired_host;
    // statistics (ssj_stream_stats)
    uint64_t slot_grows = 0, result_grows = 0;
    double slot_grow_ms = 0.0, result_grow_ms = 0.0, longest_pass_ms = 0.0;
};

namespace {

// A pooled pinned buffer of at least bytes (E->mu held): one of the
// power-of-two size class holding bytes, else an idle one of a larger class
// (*cls: the class it returns to), else null: the caller then allocates one
// of *cls bytes after releasing the lock, since a pinned allocation can take
// milliseconds and stalls the runtime's other work meanwhile.
void* pinned_take(StreamEngine* E, size_t bytes, size_t* cls) {
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    *cls = c;
    for (auto it = E->pool.lower_bound(c); it != E->pool.end(); ++it) {
        if (it->second.empty()) continue;
        void* p = it->second.back();
        it->second.pop_back();
        *cls = it->first;
        return p;
    }
    return nullptr;
}

void pinned_put(StreamEngine* E, void* p, size_t cls) {
    if (p) E->pool[cls].push_back(p);
}

// Called with E->mu held after a part of r completed (or r was abandoned).
void maybe_finish(StreamEngine* E, StreamReq* r) {
    if (r->finished || r->next_part_off < r->n || r->parts_done < r->parts_admitted) return;
    r->finished = true;
    r->status = r->failed ? SSJ_EDEVICE : (r->bad_id ? SSJ_EINVAL : SSJ_OK);
    r->t_done = now_ns();
    pinned_put(E, r->h_cand, r->h_cand_bytes);
    r->h_cand = nullptr;
    r->coll->inflight.fetch_sub(1);
}

void fail_slot(StreamEngine* E, StreamSlot& s) {
    E->ctx->failed = true;
    for (auto& p : s.parts) {
        p.req->failed = true;
        ++p.req->parts_done;
        maybe_finish(E, p.req);
    }
    s.parts.clear();
    s.state = 0;
    E->cv_done.notify_all();
}

// Called with E->mu held.  Fills idle slot s with parts of pending requests
// and enqueues their copies, one launch, and the count read-back.
// Grows slot s's device buffers to hold at least n pairs (the slot is idle;
// grow() synchronises the device before it releases an old buffer).
// A slot buffer of at least need elements from the device's stream-ordered
// pool, on the slot's stream.  The slot is idle when it grows, so its old
// buffer goes back to the pool in stream order; neither step waits for the
// other slots' work (hipFree and hipDeviceSynchronize would), and once the
// pool holds the memory (it keeps what is freed) neither reaches the driver.
template <class T>
hipError_t slot_realloc(T*& p, size_t& cap, size_t need, hipStream_t st) {
    if (need <= cap && p) return hipSuccess;
    if (p) {
        const hipError_t e = hipFreeAsync(p, st);
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    const hipError_t e = hipMallocAsync((void**)&p, need * sizeof(T), st);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = need;
    return hipSuccess;
}

bool slot_grow(StreamEngine* E, StreamSlot& s, int64_t n) {
    const auto t0 = std::chrono::steady_clock::now();
    E->held -= s.held;
    s.held = 0;
    s.cap = 0;
    if (slot_realloc(s.d_cand, s.cand_cap, (size_t)n, s.stream) != hipSuccess) return false;
    if (slot_realloc(s.d_out, s.out_cap, (size_t)n, s.stream) != hipSuccess) return false;
    if (slot_realloc(s.sc.d_queues, s.sc.q_cap, (size_t)ssj::kQueues * (size_t)n, s.stream) != hipSuccess)
        return false;
    s.cap = (int64_t)std::min({s.cand_cap, s.out_cap, s.sc.q_cap / (size_t)ssj::kQueues});
    s.held = (uint64_t)(s.cand_cap + s.out_cap) * sizeof(int2) + (uint64_t)s.sc.q_cap * sizeof(uint32_t);
    E->held += s.held;
    E->slot_grows += 1;
    E->slot_grow_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return true;
}

bool admit(StreamEngine* E, StreamSlot& s) {
    ssj_ctx* ctx = E->ctx;
    s.parts.clear();
    if (E->pending.empty()) return true;
    s.coll = E->pending.front()->coll;
    // pairs this slot may hold: its own buffers plus the budget that the
    // collections and the other slots' buffers leave (at least kSlotFloor)
    const uint64_t others = E->held - s.held;
    const uint64_t spare = free_budget(ctx);
    const int64_t room = std::min<int64_t>(
        kMaxLaunchPairs,
        std::max<int64_t>(kSlotFloor, (int64_t)((spare > others ? spare - others : 0) / kBytesPerPair)));
    int64_t want = 0;
    {
        int k = 0;
        for (StreamReq* r : E->pending) {
            if (r->coll != s.coll || k++ >= ssj::kMaxReq || want >= room) break;
            want += r->n - r->next_part_off;
        }
        want = std::min(want, room);
    }
    if (want > s.cap) {
        // to the batch's size, or twice the old size when that fits (fewer
        // regrowths while batch sizes vary)
        const int64_t n = std::min(room, std::max(want, 2 * s.cap));
        if (!slot_grow(E, s, n)) return false;
    }
    int64_t used = 0;
    while (!E->pending.empty() && (int)s.parts.size() < ssj::kMaxReq) {
        StreamReq* r = E->pending.front();
        if (r->coll != s.coll) break;  // one collection per launch
        const int64_t left = r->n - r->next_part_off;
        const int64_t take = std::min(left, s.cap - used);
        if (take <= 0 && left > 0) break;
        if (r->t_admit == 0) r->t_admit = now_ns();
        s.parts.push_back(SlotPart{r, r->next_part_off, take, used, 0});
        r->parts_admitted += 1;
        r->next_part_off += take;
        used += take;
        if (r->next_part_off >= r->n) E->pending.pop_front();
        if (used >= s.cap) break;
    }
    E->cv_space.notify_all();
    std::vector<Req> reqs;
    for (auto& p : s.parts) {
        if (p.n > 0 &&
            hipMemcpyAsync(s.d_cand + p.dev_off, p.req->h_cand + p.off, (size_t)p.n * 8,
                           hipMemcpyHostToDevice, s.stream) != hipSuccess)
            return false;
        reqs.push_back(Req{s.d_cand + p.dev_off, p.n, p.req->t_num, p.req->t_den,
                           s.d_out + p.dev_off, p.n, s.d_count + reqs.size(), p.req->sim});
    }
    ssj_plan plan;
    {
        std::lock_guard<std::mutex> g(ctx->plan_mu);
        plan = ctx->plan;
    }
    if (enqueue_launch(ctx, s.coll, s.sc, reqs.data(), (int)reqs.size(), s.stream, plan, false) != SSJ_OK)
        return false;
    if (hipMemcpyAsync(s.h_count, s.d_count, sizeof(long long) * reqs.size(), hipMemcpyDeviceToHost,
                       s.stream) != hipSuccess)
        return false;
    if (hipEventRecord(s.ev, s.stream) != hipSuccess) return false;
    s.state = 1;
    return true;
}

// Called with E->mu held; slot state 1 and its event complete: copy back the
// passing pairs (their number is now known) into the slot's pinned result
// buffer, part after part.
bool read_counts(StreamEngine* E, StreamSlot& s) {
    int64_t total = 0;
    for (size_t k = 0; k < s.parts.size(); ++k) {
        s.parts[k].res_off = total;
        total += std::max<long long>(0, s.h_count[k]);
    }
    if (total > s.h_cap) {
        // results are usually few (the buffer starts at kSlotResults pairs);
        // it grows to the largest batch result, the old one retired
        const auto t0 = std::chrono::steady_clock::now();
        const int64_t n = std::max<int64_t>(total, 2 * s.h_cap);
        if (s.h_out) E->retired_host.push_back(s.h_out);
        s.h_out = nullptr;
        s.h_cap = 0;
        if (hipHostMalloc((void**)&s.h_out, (size_t)n * sizeof(int2), hipHostMallocDefault) != hipSuccess) {
            s.h_out = nullptr;
            return false;
        }
        s.h_cap = n;
        E->result_grows += 1;
        E->result_grow_ms +=
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    bool any = false;
    for (size_t k = 0; k < s.parts.size(); ++k) {
        const long long c = s.h_count[k];
        if (c > 0) {
            if (hipMemcpyAsync(s.h_out + s.parts[k].res_off, s.d_out + s.parts[k].dev_off, (size_t)c * 8,
                               hipMemcpyDeviceToHost, s.stream) != hipSuccess)
                return false;
            any = true;
        }
    }
    if (any) {
        if (hipEventRecord(s.ev, s.stream) != hipSuccess) return false;
        s.state = 2;
    } else {
        s.state = 3;
    }
    return true;
}

// Called with E->mu held; results of the slot are on the host.
void complete_slot(StreamEngine* E, StreamSlot& s) {
    for (size_t k = 0; k < s.parts.size(); ++k) {
        SlotPart& p = s.parts[k];
        StreamReq* r = p.req;
        const long long c = s.h_count[k];
        if (c < 0) {
            r->bad_id = true;
        } else if (c > 0) {
            r->result.insert(r->result.end(), s.h_out + p.res_off, s.h_out + p.res_off + c);
        }
        ++r->parts_done;
        maybe_finish(E, r);
    }
    s.parts.clear();
    s.state = 0;
    E->cv_done.notify_all();
}

void engine_loop(StreamEngine* E) {
    (void)hipSetDevice(E->ctx->device);
    // the loop polls slot events while work is in flight: a 1 us timer slack
    // keeps its short sleeps short (the default slack of 50 us would add
    // about that much to every slot state change, three per request)
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(E->mu);
    for (;;) {
        const auto t_pass = std::chrono::steady_clock::now();
        bool busy = false;
        for (auto& s : E->slots) {
            if (s.state == 1 || s.state == 2) {
                busy = true;
                const hipError_t q = hipEventQuery(s.ev);
                if (q == hipSuccess) {
                    if (s.state == 1) {
                        if (!read_counts(E, s)) fail_slot(E, s);
                    } else {
                        s.state = 3;
                    }
                } else if (q != hipErrorNotReady) {
                    fail_slot(E, s);
                }
            }
            if (s.state == 3) complete_slot(E, s);
            if (s.state == 0 && !E->pending.empty() && !E->ctx->failed && (!E->paused || E->stop)) {
                if (!admit(E, s)) {
                    fail_slot(E, s);
                } else if (s.state == 1) {
                    busy = true;
                }
            }
        }
        if (E->ctx->failed) {
            // nothing more can run: fail whatever waits
            while (!E->pending.empty()) {
                StreamReq* r = E->pending.front();
                E->pending.pop_front();
                r->failed = true;
                // the rest is never admitted; parts in flight finish in their slot
                r->next_part_off = r->n;
                maybe_finish(E, r);
            }
            E->cv_done.notify_all();
            E->cv_space.notify_all();
        }
        E->longest_pass_ms = std::max(
            E->longest_pass_ms,
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_pass).count());
        if (E->stop && !busy && E->pending.empty()) break;
        if (busy) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(5));
            lk.lock();
        } else {
            E->cv_work.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
}

// Takes this device's address of scratch (once per device, with the device
// current) and clears its counter block with a fill kernel; the context
// keeps views of it.  Every launch's finalize kernel leaves the counters at
// zero again.
int noalloc_setup(ssj_ctx* ctx) {
    if (ctx->device >= kMaxDevices) return set_error(SSJ_EINVAL, "device ordinal too large");
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch_ptr[ctx->device]) {
            HIP_OR_FAIL(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return hip_fail(ctx, "hipGetSymbolAddress", hipErrorInvalidSymbol);
            HIP_OR_FAIL(ctx, ssj::launch_clear_words(reinterpret_cast<uint32_t*>(ptr),
                                                     sizeof(ssj::Counters) / sizeof(uint32_t), ctx->stream));
            HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
            g_scratch_ptr[ctx->device] = ptr;
        }
        ptr = g_scratch_ptr[ctx->device];
    }
    ctx->noalloc.d_ctr = reinterpret_cast<ssj::Counters*>(ptr);
    ctx->noalloc.d_queues = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(ptr) +
                                                        sizeof(ssj::Counters));
    ctx->noalloc.q_cap = kNoAllocQueueWords;
    return SSJ_OK;
}

int engine_start(ssj_ctx* ctx) {
    auto E = std::make_unique<StreamEngine>();
    E->ctx = ctx;
    E->slots.resize((size_t)ctx->n_slots);
    // the slots' device buffers come from the device's stream-ordered pool,
    // which keeps freed memory for later allocations instead of returning it
    // to the driver
    hipMemPool_t pool = nullptr;
    HIP_OR_FAIL(ctx, hipDeviceGetDefaultMemPool(&pool, ctx->device));
    uint64_t keep = UINT64_MAX;
    HIP_OR_FAIL(ctx, hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    // per slot: a stream, counters and count buffers; the candidate, output
    // and queue buffers are sized by the first batches the slot admits
    for (auto& s : E->slots) {
        HIP_OR_FAIL(ctx, hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
        int rc = scratch_init(ctx, s.sc);
        if (rc != SSJ_OK) return rc;
        HIP_OR_FAIL(ctx, hipMalloc((void**)&s.d_count, sizeof(long long) * ssj::kMaxReq));
        HIP_OR_FAIL(ctx, hipHostMalloc((void**)&s.h_count, sizeof(long long) * ssj::kMaxReq, hipHostMallocDefault));
        HIP_OR_FAIL(ctx, hipHostMalloc((void**)&s.h_out, sizeof(int2) * kSlotResults, hipHostMallocDefault));
        s.h_cap = kSlotResults;
        HIP_OR_FAIL(ctx, hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    }
    StreamEngine* raw = E.get();
    ctx->engine = std::move(E);
    raw->worker = std::thread(engine_loop, raw);
    return SSJ_OK;
}

void engine_stop(ssj_ctx* ctx) {
    StreamEngine* E = ctx->engine.get();
    if (!E) return;
    {
        std::lock_guard<std::mutex> g(E->mu);
        E->stop = true;
    }
    E->cv_work.notify_all();
    E->cv_space.notify_all();
    if (E->worker.joinable()) E->worker.join();
    for (auto& s : E->slots) {
        if (s.stream) {
            if (s.d_cand) (void)hipFreeAsync(s.d_cand, s.stream);
            if (s.d_out) (void)hipFreeAsync(s.d_out, s.stream);
            if (s.sc.d_queues) (void)hipFreeAsync(s.sc.d_queues, s.stream);
            s.sc.d_queues = nullptr;
            (void)hipStreamSynchronize(s.stream);
        }
        scratch_free(s.sc);
        if (s.d_count) (void)hipFree(s.d_count);
        if (s.h_count) (void)hipHostFree(s.h_count);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    for (auto& kv : E->table) {
        if (kv.second->h_cand) (void)hipHostFree(kv.second->h_cand);
        delete kv.second;
    }
    for (auto& kv : E->pool)
        for (void* p : kv.second) (void)hipHostFree(p);
    for (void* p : E->retired_host) (void)hipHostFree(p);
    ctx->engine.reset();
}

}  // namespace

extern "C" {

const char* ssj_last_error(ssj_ctx*) { return tl_error.c_str(); }

int ssj_init(const ssj_opts* opts, ssj_ctx** out) {
    if (!out) return set_error(SSJ_EINVAL, "null output pointer");
    *out = nullptr;
    ssj_opts o{};
    if (opts) o = *opts;
    int n_dev = 0;
    hipError_t e = hipGetDeviceCount(&n_dev);
    if (e != hipSuccess || n_dev <= 0) return set_error(SSJ_EDEVICE, "no HIP device available");
    if (o.device < 0 || o.device >= n_dev) return set_error(SSJ_EINVAL, "device ordinal out of range");
    if (o.n_slots < 0 || o.n_slots > 64 || o.queue_depth < 0 || o.queue_depth > (1 << 20))
        return set_error(SSJ_EINVAL, "n_slots must be in [0, 64], queue_depth in [0, 2^20]");
    ssj_ctx* ctx = new (std::nothrow) ssj_ctx();
    if (!ctx) return set_error(SSJ_ENOMEM, "host allocation failed");
    ctx->device = o.device;
    ctx->budget = o.hbm_budget ? o.hbm_budget : kDefaultBudget;
    ctx->n_slots = o.n_slots ? o.n_slots : 4;
    ctx->queue_depth = o.queue_depth ? o.queue_depth : 64;
    default_plan(ctx->plan);
    int rc = SSJ_OK;
    do {
        if ((e = hipSetDevice(ctx->device)) != hipSuccess) { rc = hip_fail(ctx, "hipSetDevice", e); break; }
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, ctx->device)) != hipSuccess) { rc = hip_fail(ctx, "hipGetDeviceProperties", e); break; }
        ctx->n_cu = prop.multiProcessorCount;
        // architecture and compute units: the marketing name is not part of
        // it (it reads empty under some profiling tools)
        ctx->device_key = std::string(prop.gcnArchName) + "/" + std::to_string(ctx->n_cu) + "cu";
        for (char& ch : ctx->device_key)
            if (ch == '"' || ch == '\\' || ch == '|' || (unsigned char)ch < 32) ch = '_';
        for (int k = 0; k < 8 * kMappings && rc == SSJ_OK; ++k) {
            const bool deferring = (k & 1) != 0;
            const void* f = ssj::kernel_verify_tiles(kInlineLanes[k / 8], kInlineHard[k / 8],
                                                     kInlineStaged[k / 8] != 0, deferring, (k & 2) != 0,
                                                     (k & 4) != 0);
            // by the number of LDS queues per wavefront (deferred classes,
            // plus the spill queue)
            for (int nd = deferring ? 1 : 0; nd <= (deferring ? ssj::kQueues : 0) && rc == SSJ_OK; ++nd) {
                ssj::LaunchArgs la{};
                la.defer_from = nd <= ssj::kClasses ? ssj::kClasses - nd : 0;
                la.spill_iters = nd <= ssj::kClasses ? 0xffffffffu : 1u;
                la.defer_cap = 2 * ssj::kWave;
                la.staged = (uint32_t)kInlineStaged[k / 8];
                la.inline_lanes = kInlineLanes[k / 8];
                int occ = 0;
                if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, ssj::kBlock, ssj::tiles_lds_bytes(la))) != hipSuccess)
                    rc = hip_fail(ctx, "hipOccupancyMaxActiveBlocksPerMultiprocessor", e);
                ctx->occ_tiles[k][nd] = std::min(occ, vgpr_limited_blocks(f));
            }
        }
        if (rc != SSJ_OK) break;
        for (int k = 0; k < 4 && rc == SSJ_OK; ++k) {
            int occ = 0;
            const void* f = ssj::kernel_verify_deferred((k & 1) != 0, (k & 2) != 0);
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, ssj::kBlock, 0)) != hipSuccess)
                rc = hip_fail(ctx, "hipOccupancyMaxActiveBlocksPerMultiprocessor", e);
            ctx->occ_deferred2[k] = std::min(occ, vgpr_limited_blocks(f));
        }
        if (rc != SSJ_OK) break;
        if ((e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess) { rc = hip_fail(ctx, "hipStreamCreate", e); break; }
        if ((rc = scratch_init(ctx, ctx->def)) != SSJ_OK) break;
        ctx->def.resume = true;
        if ((rc = noalloc_setup(ctx)) != SSJ_OK) break;
        if ((e = hipMalloc((void**)&ctx->d_count, sizeof(long long))) != hipSuccess) { rc = hip_fail(ctx, "hipMalloc", e); break; }
        if ((e = hipHostMalloc((void**)&ctx->h_count, sizeof(long long), hipHostMallocDefault)) != hipSuccess) { rc = hip_fail(ctx, "hipHostMalloc", e); break; }
        rc = engine_start(ctx);
    } while (0);
    if (rc != SSJ_OK) {
        const std::string msg = tl_error;
        ssj_shutdown(ctx);
        tl_error = msg;
        return rc;
    }
    *out = ctx;
    return SSJ_OK;
}

int ssj_shutdown(ssj_ctx* ctx) {
    if (!ctx) return SSJ_OK;
    (void)hipSetDevice(ctx->device);
    engine_stop(ctx);
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        for (ssj_coll* c : ctx->colls) {
            if (c->d_tok) (void)hipFree(c->d_tok);
            if (c->d_heads) (void)hipFree(c->d_heads);
            delete c;
        }
        ctx->colls.clear();
        scratch_free(ctx->def);
        if (ctx->d_cand) (void)hipFree(ctx->d_cand);
        if (ctx->d_out) (void)hipFree(ctx->d_out);
        if (ctx->d_groups) (void)hipFree(ctx->d_groups);
        if (ctx->d_sids) (void)hipFree(ctx->d_sids);
        if (ctx->d_pairs) (void)hipFree(ctx->d_pairs);
        for (void* q : {(void*)ctx->flt.plen, (void*)ctx->flt.pre, (void*)ctx->flt.pos, (void*)ctx->flt.pos2,
                        (void*)ctx->flt.counts, (void*)ctx->flt.off, (void*)ctx->flt.keys,
                        (void*)ctx->flt.keys2, (void*)ctx->flt.probes, (void*)ctx->flt.temp,
                        (void*)ctx->flt.items, (void*)ctx->flt.istart, (void*)ctx->flt.range})
            if (q) (void)hipFree(q);
        if (ctx->d_count) (void)hipFree(ctx->d_count);
        if (ctx->h_count) (void)hipHostFree(ctx->h_count);
        if (ctx->copy_stream) (void)hipStreamSynchronize(ctx->copy_stream);
        for (int k = 0; k < 2; ++k) {
            if (ctx->h_ring[k]) (void)hipHostFree(ctx->h_ring[k]);
            if (ctx->ring_ev[k]) (void)hipEventDestroy(ctx->ring_ev[k]);
        }
        if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
        if (ctx->d_counts) (void)hipFree(ctx->d_counts);
        if (ctx->h_counts) (void)hipHostFree(ctx->h_counts);
        for (auto& kv : ctx->graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        }
        ctx->graphs.clear();
        if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
        if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    }
    for (auto& ev : ctx->ev_pending)
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
    return SSJ_OK;
}

int ssj_upload_collection(ssj_ctx* ctx, const int64_t* offsets, int64_t n_sets,
                          const int32_t* tokens, int64_t n_tokens, ssj_coll** out) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if (!out) return set_error(SSJ_EINVAL, "null output pointer");
    *out = nullptr;
    if (!offsets || n_sets < 0 || n_sets >= INT32_MAX)
        return set_error(SSJ_EINVAL, "n_sets must be in [0, 2^31 - 1) with offsets given");
    if (n_tokens < 0 || n_tokens >= ((int64_t)1 << 32) || (n_tokens > 0 && !tokens))
        return set_error(SSJ_EINVAL, "n_tokens must be in [0, 2^32) with tokens given");
    if (offsets[0] != 0 || offsets[n_sets] != n_tokens)
        return set_error(SSJ_EINVAL, "offsets[0] must be 0 and offsets[n_sets] == n_tokens");
    int64_t max_len = 0;
    for (int64_t i = 0; i < n_sets; ++i) {
        const int64_t b = offsets[i], e = offsets[i + 1];
        if (e <= b) {
            return set_error(SSJ_EINVAL, "set " + std::to_string(i) +
                                             " is empty or offsets decrease (sets must be non-empty)");
        }
        if (e > n_tokens) return set_error(SSJ_EINVAL, "offset beyond n_tokens");
        if (tokens[b] < 0) return set_error(SSJ_EINVAL, "negative token in set " + std::to_string(i));
        for (int64_t k = b + 1; k < e; ++k) {
            if (tokens[k] <= tokens[k - 1])
                return set_error(SSJ_EINVAL, "tokens of set " + std::to_string(i) +
                                                 " are not strictly increasing");
        }
        max_len = std::max(max_len, e - b);
    }
    // Device layout: every set starts on a 16-byte boundary (a multiple of 4
    // tokens), so a lane can read 4 consecutive tokens of a set with one
    // aligned 16-byte load; the slots after a set's end hold -1.
    std::vector<uint32_t> start;
    std::vector<int32_t> padded;
    uint64_t n_dev = 0;
    try {
        start.resize((size_t)std::max<int64_t>(n_sets, 1));
        for (int64_t i = 0; i < n_sets; ++i) {
            start[(size_t)i] = (uint32_t)n_dev;
            n_dev += ((uint64_t)(offsets[i + 1] - offsets[i]) + 3u) & ~(uint64_t)3u;
            if (n_dev >= ((uint64_t)1 << 32))
                return set_error(SSJ_EINVAL, "collection too large: tokens padded to 16-byte set starts must stay below 2^32");
        }
        padded.assign((size_t)std::max<uint64_t>(n_dev, 4), -1);
        for (int64_t i = 0; i < n_sets; ++i)
            std::memcpy(padded.data() + start[(size_t)i], tokens + offsets[i],
                        (size_t)(offsets[i + 1] - offsets[i]) * 4);
    } catch (const std::bad_alloc&) {
        return set_error(SSJ_ENOMEM, "host allocation failed");
    }
    std::lock_guard<std::mutex> g(ctx->mu);
    // the collections resident at once must fit the HBM budget (what is left
    // of it bounds the candidate buffers of each call)
    const uint64_t bytes = (uint64_t)padded.size() * 4u + (uint64_t)std::max<int64_t>(n_sets, 1) * 32u;
    if (ctx->resident.load() + bytes > ctx->budget)
        return set_error(SSJ_ENOMEM, "the collection (" + std::to_string(bytes) + " device bytes) does not fit "
                                     "the HBM budget next to the resident collections (" +
                                     std::to_string(ctx->resident.load()) + " of " + std::to_string(ctx->budget) +
                                     " bytes)");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    ssj_coll* c = new (std::nothrow) ssj_coll();
    if (!c) return set_error(SSJ_ENOMEM, "host allocation failed");
    c->dev_bytes = bytes;
    c->ctx = ctx;
    c->n_sets = n_sets;
    c->n_tokens = n_tokens;
    c->max_len = max_len;
    int64_t* d_off = nullptr;
    uint32_t* d_start = nullptr;
    hipError_t e = hipSuccess;
    do {
        if ((e = hipMalloc((void**)&c->d_tok, padded.size() * 4)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&c->d_heads, (size_t)std::max<int64_t>(n_sets, 1) * 32)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&d_off, (size_t)(n_sets + 1) * 8)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&d_start, start.size() * 4)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(c->d_tok, padded.data(), padded.size() * 4, hipMemcpyHostToDevice, ctx->stream)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(d_off, offsets, (size_t)(n_sets + 1) * 8, hipMemcpyHostToDevice, ctx->stream)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(d_start, start.data(), start.size() * 4, hipMemcpyHostToDevice, ctx->stream)) != hipSuccess) break;
        if ((e = ssj::launch_build_heads(d_off, d_start, c->d_tok, c->d_heads, n_sets, ctx->stream)) != hipSuccess) break;
        if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) break;
    } while (0);
    if (d_off) (void)hipFree(d_off);
    if (d_start) (void)hipFree(d_start);
    if (e != hipSuccess) {
        if (c->d_tok) (void)hipFree(c->d_tok);
        if (c->d_heads) (void)hipFree(c->d_heads);
        delete c;
        if (e == hipErrorOutOfMemory) return set_error(SSJ_ENOMEM, "device allocation failed");
        return hip_fail(ctx, "upload", e);
    }
    {
        std::unique_lock<std::mutex> ek;
        if (ctx->engine) ek = std::unique_lock<std::mutex>(ctx->engine->mu);
        ctx->colls.push_back(c);
        ctx->resident += bytes;
    }
    *out = c;
    return SSJ_OK;
}

int ssj_free_collection(ssj_ctx* ctx, ssj_coll* coll) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    std::lock_guard<std::mutex> g(ctx->mu);
    {
        // submits take their place in flight under the engine's lock, so a
        // request is either counted here or submitted after the collection is
        // gone from ctx->colls (and then refused by the submit's lookup)
        std::unique_lock<std::mutex> ek;
        if (ctx->engine) ek = std::unique_lock<std::mutex>(ctx->engine->mu);
        if (coll->inflight.load() != 0) return set_error(SSJ_EAGAIN, "collection has requests in flight");
        auto it = std::find(ctx->colls.begin(), ctx->colls.end(), coll);
        if (it == ctx->colls.end()) return set_error(SSJ_EINVAL, "unknown collection");
        ctx->colls.erase(it);
        ctx->resident -= coll->dev_bytes;
    }
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (coll->d_tok) (void)hipFree(coll->d_tok);
    if (coll->d_heads) (void)hipFree(coll->d_heads);
    delete coll;
    return SSJ_OK;
}

int ssj_collection_info(const ssj_coll* coll, int64_t* n_sets, int64_t* n_tokens, int64_t* max_len) {
    if (!coll) return set_error(SSJ_EINVAL, "null collection");
    if (n_sets) *n_sets = coll->n_sets;
    if (n_tokens) *n_tokens = coll->n_tokens;
    if (max_len) *max_len = coll->max_len;
    return SSJ_OK;
}

int ssj_get_plan(ssj_ctx* ctx, ssj_plan* plan) {
    if (!ctx || !plan) return set_error(SSJ_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    *plan = ctx->plan;
    return SSJ_OK;
}

int ssj_set_plan(ssj_ctx* ctx, const ssj_plan* plan) {
    if (!ctx || !plan) return set_error(SSJ_EINVAL, "null argument");
    if (!plan_valid(*plan))
        return set_error(SSJ_EINVAL, "inline_lanes must be 1, 4, 8, 16, 32 or 64 (hard_lanes 0, 8 "
                                     "or 16 with 1 lane, else 0); defer_from in [0, 5]; "
                                     "lanes and spill_lanes 1, 4, 8, 16, 32, 64 or 256; "
                                     "spill_iters in [0, 2^20], > 0 only with 1 lane and "
                                     "hard_lanes 0; wg_per_cu in [0, 64]; staged 0 or 1, "
                                     "1 only with 1 lane and hard_lanes 0");
    std::lock_guard<std::mutex> g(ctx->mu);
    std::lock_guard<std::mutex> gp(ctx->plan_mu);
    ctx->plan = *plan;
    return SSJ_OK;
}

int ssj_timing_enable(ssj_ctx* ctx, int period) {
    if (!ctx) return set_error(SSJ_EINVAL, "null context");
    if (period < 0) return set_error(SSJ_EINVAL, "negative timing period");
    ctx->timing_period = period;
    ctx->timing_tick = 0;
    return SSJ_OK;
}

int ssj_timing_read(ssj_ctx* ctx, int reset, double* inorder_ms, double* deferred_ms,
                    int64_t* launches) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    std::lock_guard<std::mutex> g(ctx->tmu);
    for (auto& ev : ctx->ev_pending) {
        float a = 0.f, b = 0.f;
        HIP_OR_FAIL(ctx, hipEventSynchronize(ev[1]));
        HIP_OR_FAIL(ctx, hipEventElapsedTime(&a, ev[0], ev[1]));
        if (ev[2]) {
            HIP_OR_FAIL(ctx, hipEventSynchronize(ev[3]));
            HIP_OR_FAIL(ctx, hipEventElapsedTime(&b, ev[2], ev[3]));
        }
        ctx->t_inorder_ms += a;
        ctx->t_deferred_ms += b;
        ctx->t_launches += 1;
        for (auto e : ev)
            if (e) ctx->ev_pool.push_back(e);
    }
    ctx->ev_pending.clear();
    if (inorder_ms) *inorder_ms = ctx->t_inorder_ms;
    if (deferred_ms) *deferred_ms = ctx->t_deferred_ms;
    if (launches) *launches = ctx->t_launches;
    if (reset) {
        ctx->t_inorder_ms = ctx->t_deferred_ms = 0.0;
        ctx->t_launches = 0;
    }
    return SSJ_OK;
}

int ssj_verify_batch_device(ssj_ctx* ctx, const ssj_coll* coll, const ssj_request* reqs,
                            int n_reqs, void* hip_stream) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    if (n_reqs < 0 || n_reqs > ssj::kMaxReq || (n_reqs > 0 && !reqs))
        return set_error(SSJ_EINVAL, "n_reqs must be in [0, SSJ_MAX_BATCH]");
    std::vector<Req> v((size_t)n_reqs);
    int64_t total = 0;
    for (int i = 0; i < n_reqs; ++i) {
        v[i] = Req{reinterpret_cast<const int2*>(reqs[i].d_cand), reqs[i].n_cand, reqs[i].t_num,
                   reqs[i].t_den, reinterpret_cast<int2*>(reqs[i].d_out), reqs[i].out_cap,
                   reinterpret_cast<long long*>(reqs[i].d_count), reqs[i].sim};
        if ((rc = check_req(v[i])) != SSJ_OK) return rc;
        total += v[i].n;
        if (total > kMaxLaunchPairs) return set_error(SSJ_EINVAL, "a batch must hold fewer than 2^31 pairs");
    }
    if (n_reqs == 0) return SSJ_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    return enqueue_launch(ctx, coll, ctx->def, v.data(), n_reqs, (hipStream_t)hip_stream, ctx->plan);
}

namespace {

// Device-buffer verification of flat pairs, r ids in coll, s ids in coll_s.
int verify_device(ssj_ctx* ctx, const ssj_coll* coll, const ssj_coll* coll_s, const ssj_pair* d_cand,
                  int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* d_out,
                  int64_t out_cap, int64_t* d_count, void* hip_stream) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_s)) != SSJ_OK) return rc;
    Req r{reinterpret_cast<const int2*>(d_cand), n_cand, t_num, t_den, reinterpret_cast<int2*>(d_out),
          out_cap, reinterpret_cast<long long*>(d_count), sim};
    if ((rc = check_req(r)) != SSJ_OK) return rc;
    if (n_cand > kMaxLaunchPairs) return set_error(SSJ_EINVAL, "n_cand must be below 2^31 per device call");
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    return enqueue_launch(ctx, coll, ctx->def, &r, 1, (hipStream_t)hip_stream, ctx->plan, true, coll_s);
}

// A grouped request (candidates read in place by the verification kernels).
void grouped_req(Req& r, const int2* d_groups, int64_t n_groups, const int32_t* d_sids, int64_t n_cand, int sim,
                 int64_t t_num, int64_t t_den, int2* d_out, int64_t out_cap, long long* d_count) {
    r = Req{nullptr, n_cand, t_num, t_den, d_out, out_cap, d_count, sim};
    r.d_sids = d_sids;
    r.d_groups = d_groups;
    r.n_groups = n_groups;
    r.grouped = true;
}

// Enqueues the verification of grouped candidates already on the device
// (ctx->mu held).
int enqueue_groups(ssj_ctx* ctx, const ssj_coll* R, const ssj_coll* S, const int2* d_groups,
                   int64_t n_groups, const int32_t* d_sids, int64_t n_cand, int sim, int64_t t_num,
                   int64_t t_den, int2* d_out, int64_t out_cap, long long* d_count, hipStream_t st) {
    Req r;
    grouped_req(r, d_groups, n_groups, d_sids, n_cand, sim, t_num, t_den, d_out, out_cap, d_count);
    return enqueue_launch(ctx, R, ctx->def, &r, 1, st, ctx->plan, true, S);
}

}  // namespace

int ssj_verify_device_sim(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand,
                          int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* d_out,
                          int64_t out_cap, int64_t* d_count, void* hip_stream) {
    return verify_device(ctx, coll, coll, d_cand, n_cand, sim, t_num, t_den, d_out, out_cap, d_count,
                         hip_stream);
}

int ssj_verify_rs_device(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                         const ssj_pair* d_cand, int64_t n_cand, int sim, int64_t t_num,
                         int64_t t_den, ssj_pair* d_out, int64_t out_cap, int64_t* d_count,
                         void* hip_stream) {
    return verify_device(ctx, coll_r, coll_s, d_cand, n_cand, sim, t_num, t_den, d_out, out_cap,
                         d_count, hip_stream);
}

int ssj_verify_groups_device(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                             const ssj_group* d_groups, int64_t n_groups, const int32_t* d_cand,
                             int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* d_out,
                             int64_t out_cap, int64_t* d_count, void* hip_stream) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_r)) != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_s)) != SSJ_OK) return rc;
    if (!valid_threshold(sim, t_num, t_den)) return set_error(SSJ_EINVAL, kThresholdError);
    if (n_groups < 0 || n_cand < 0 || out_cap < 0) return set_error(SSJ_EINVAL, "negative size");
    if (n_cand > kMaxLaunchPairs || n_groups > kMaxLaunchPairs)
        return set_error(SSJ_EINVAL, "n_cand and n_groups must be below 2^31 per device call");
    if (!d_count || (n_cand > 0 && !d_cand) || (n_groups > 0 && !d_groups))
        return set_error(SSJ_EINVAL, "null device buffer");
    if (out_cap > 0 && !d_out) return set_error(SSJ_EINVAL, "out_cap > 0 with a null output buffer");
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    return enqueue_groups(ctx, coll_r, coll_s, reinterpret_cast<const int2*>(d_groups), n_groups, d_cand,
                          n_cand, sim, t_num, t_den, reinterpret_cast<int2*>(d_out), out_cap,
                          reinterpret_cast<long long*>(d_count), (hipStream_t)hip_stream);
}

int ssj_verify_groups_batch_device(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                                   const ssj_group_request* reqs, int n_reqs, void* hip_stream) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_r)) != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_s)) != SSJ_OK) return rc;
    if (n_reqs < 0 || n_reqs > ssj::kMaxReq || (n_reqs > 0 && !reqs))
        return set_error(SSJ_EINVAL, "n_reqs must be in [0, SSJ_MAX_BATCH]");
    int64_t total = 0, total_groups = 0;
    for (int i = 0; i < n_reqs; ++i) {
        const ssj_group_request& q = reqs[i];
        if (!valid_threshold(q.sim, q.t_num, q.t_den)) return set_error(SSJ_EINVAL, kThresholdError);
        if (q.n_groups < 0 || q.n_cand < 0 || q.out_cap < 0) return set_error(SSJ_EINVAL, "negative size");
        total_groups += q.n_groups;
        if (q.n_groups > kMaxLaunchPairs || total_groups > kMaxLaunchPairs)
            return set_error(SSJ_EINVAL, "the groups of a batch must stay below 2^31");
        if (!q.d_count || (q.n_cand > 0 && !q.d_cand) || (q.n_groups > 0 && !q.d_groups))
            return set_error(SSJ_EINVAL, "null device buffer");
        if (q.out_cap > 0 && !q.d_out) return set_error(SSJ_EINVAL, "out_cap > 0 with a null output buffer");
        total += q.n_cand;
        if (total > kMaxLaunchPairs) return set_error(SSJ_EINVAL, "a batch must hold fewer than 2^31 candidates");
    }
    if (n_reqs == 0) return SSJ_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<Req> v((size_t)n_reqs);
    for (int i = 0; i < n_reqs; ++i) {
        const ssj_group_request& q = reqs[i];
        grouped_req(v[i], reinterpret_cast<const int2*>(q.d_groups), q.n_groups, q.d_cand, q.n_cand, q.sim,
                    q.t_num, q.t_den, reinterpret_cast<int2*>(q.d_out), q.out_cap,
                    reinterpret_cast<long long*>(q.d_count));
    }
    return enqueue_launch(ctx, coll_r, ctx->def, v.data(), n_reqs, st, ctx->plan, true, coll_s);
}

namespace {

// GPU prefix-filter candidates of coll at t = t_num / t_den into ctx->d_pairs;
// *n_cand receives their number (three host synchronisations on st: the index
// size, the probe work items and the candidate count).  ctx->mu held.
int gpu_candidates(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den, bool positional,
                   hipStream_t st, int64_t* n_cand) {
    auto& F = ctx->flt;
    const uint32_t n = (uint32_t)coll->n_sets;
    const uint64_t num = (uint64_t)t_num, den = (uint64_t)t_den;
    *n_cand = 0;
    if (n == 0) return SSJ_OK;
    auto temp_for = [&](size_t need) -> hipError_t { return grow(F.temp, F.temp_cap, std::max<size_t>(need, 1)); };
    HIP_OR_FAIL(ctx, grow(F.plen, F.plen_cap, (size_t)n + 1));
    HIP_OR_FAIL(ctx, grow(F.pre, F.pre_cap, (size_t)n + 1));
    size_t tb = 0;
    HIP_OR_FAIL(ctx, ssj::filter_prefix_lengths(coll->d_heads, n, num, den, F.plen, F.pre, nullptr, &tb, st));
    HIP_OR_FAIL(ctx, temp_for(tb));
    tb = F.temp_cap;
    HIP_OR_FAIL(ctx, ssj::filter_prefix_lengths(coll->d_heads, n, num, den, F.plen, F.pre, F.temp, &tb, st));
    uint32_t m = 0;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_count, F.pre + n, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    std::memcpy(&m, ctx->h_count, sizeof(uint32_t));
    if (m == 0) return SSJ_OK;
    HIP_OR_FAIL(ctx, grow(F.keys, F.keys_cap, m));
    HIP_OR_FAIL(ctx, grow(F.keys2, F.keys2_cap, m));
    HIP_OR_FAIL(ctx, grow(F.pos, F.pos_cap, m));
    HIP_OR_FAIL(ctx, grow(F.pos2, F.pos2_cap, m));
    HIP_OR_FAIL(ctx, grow(F.probes, F.probes_cap, m));
    HIP_OR_FAIL(ctx, grow(F.range, F.range_cap, m));
    HIP_OR_FAIL(ctx, grow(F.items, F.items_cap, (size_t)m + 1));
    HIP_OR_FAIL(ctx, grow(F.istart, F.istart_cap, (size_t)m + 1));
    tb = 0;
    HIP_OR_FAIL(ctx, ssj::filter_build_index(coll->d_heads, coll->d_tok, n, m, F.plen, F.pre, F.keys, F.pos,
                                             F.keys2, F.pos2, F.probes, nullptr, &tb, st));
    size_t tb2 = 0;
    HIP_OR_FAIL(ctx, ssj::filter_probe_items(coll->d_heads, coll->d_tok, F.probes, m, F.keys2, F.range, F.items,
                                             F.istart, nullptr, &tb2, st));
    HIP_OR_FAIL(ctx, temp_for(std::max(tb, tb2)));
    tb = F.temp_cap;
    HIP_OR_FAIL(ctx, ssj::filter_build_index(coll->d_heads, coll->d_tok, n, m, F.plen, F.pre, F.keys, F.pos,
                                             F.keys2, F.pos2, F.probes, F.temp, &tb, st));
    tb = F.temp_cap;
    HIP_OR_FAIL(ctx, ssj::filter_probe_items(coll->d_heads, coll->d_tok, F.probes, m, F.keys2, F.range, F.items,
                                             F.istart, F.temp, &tb, st));
    unsigned long long items64 = 0;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_count, F.istart + m, sizeof(items64), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    std::memcpy(&items64, ctx->h_count, sizeof(items64));
    // (prefixes that many sets share make the probe work grow as the square of
    // those sets)
    if (items64 >= ((unsigned long long)1 << 31)) return set_error(SSJ_ENOMEM, "too many prefix meetings");
    const uint32_t n_items = (uint32_t)items64;
    HIP_OR_FAIL(ctx, grow(F.counts, F.counts_cap, (size_t)n_items + 1));
    HIP_OR_FAIL(ctx, grow(F.off, F.off_cap, (size_t)n_items + 1));
    tb = 0;
    HIP_OR_FAIL(ctx, ssj::filter_scan_counts(F.counts, F.off, n_items, nullptr, &tb, st));
    HIP_OR_FAIL(ctx, temp_for(tb));
    HIP_OR_FAIL(ctx, ssj::filter_probe(coll->d_heads, coll->d_tok, F.probes, m, n_items, F.keys2, F.pos2, F.plen,
                                       F.range, F.istart, num, den, positional, F.counts, nullptr, nullptr, 0, st));
    tb = F.temp_cap;
    HIP_OR_FAIL(ctx, ssj::filter_scan_counts(F.counts, F.off, n_items, F.temp, &tb, st));
    unsigned long long total = 0;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_count, F.off + n_items, sizeof(total), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    std::memcpy(&total, ctx->h_count, sizeof(total));
    if (total > (unsigned long long)kMaxLaunchPairs)
        return set_error(SSJ_ENOMEM, "more than 2^31 candidates");
    HIP_OR_FAIL(ctx, grow(ctx->d_pairs, ctx->pairs_cap, std::max<size_t>((size_t)total, 1)));
    HIP_OR_FAIL(ctx, ssj::filter_probe(coll->d_heads, coll->d_tok, F.probes, m, n_items, F.keys2, F.pos2, F.plen,
                                       F.range, F.istart, num, den, positional, nullptr, F.off, ctx->d_pairs, total,
                                       st));
    *n_cand = (int64_t)total;
    return SSJ_OK;
}

int check_filter_args(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    if (!valid_threshold(SSJ_SIM_JACCARD, t_num, t_den) || t_num == 0)
        return set_error(SSJ_EINVAL, "the prefix filter needs 0 < t_num <= t_den < 2^31");
    return SSJ_OK;
}

}  // namespace

int ssj_candidates_device(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den, int positional,
                          ssj_pair* d_out, int64_t out_cap, int64_t* d_count, void* hip_stream) {
    int rc = check_filter_args(ctx, coll, t_num, t_den);
    if (rc != SSJ_OK) return rc;
    if (out_cap < 0 || !d_count || (out_cap > 0 && !d_out)) return set_error(SSJ_EINVAL, "bad output buffer");
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    int64_t n = 0;
    if ((rc = gpu_candidates(ctx, coll, t_num, t_den, positional != 0, st, &n)) != SSJ_OK) return rc;
    const int64_t k = std::min(n, out_cap);
    if (k > 0) HIP_OR_FAIL(ctx, hipMemcpyAsync(d_out, ctx->d_pairs, (size_t)k * 8, hipMemcpyDeviceToDevice, st));
    *ctx->h_count = n;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(d_count, ctx->h_count, sizeof(long long), hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));  // h_count is reused
    return SSJ_OK;
}

int ssj_join_device(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den, int positional,
                    ssj_pair* d_out, int64_t out_cap, int64_t* d_count, void* hip_stream) {
    int rc = check_filter_args(ctx, coll, t_num, t_den);
    if (rc != SSJ_OK) return rc;
    if (out_cap < 0 || !d_count || (out_cap > 0 && !d_out)) return set_error(SSJ_EINVAL, "bad output buffer");
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    int64_t n = 0;
    if ((rc = gpu_candidates(ctx, coll, t_num, t_den, positional != 0, st, &n)) != SSJ_OK) return rc;
    Req r{ctx->d_pairs, n, t_num, t_den, reinterpret_cast<int2*>(d_out), out_cap,
          reinterpret_cast<long long*>(d_count), SSJ_SIM_JACCARD};
    return enqueue_launch(ctx, coll, ctx->def, &r, 1, st, ctx->plan);
}

int ssj_join(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den, int positional, ssj_pair* out,
             int64_t out_cap, int64_t* out_n) {
    int rc = check_filter_args(ctx, coll, t_num, t_den);
    if (rc != SSJ_OK) return rc;
    if (out_cap < 0 || !out_n || (out_cap > 0 && !out)) return set_error(SSJ_EINVAL, "bad output buffer");
    *out_n = 0;
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    int64_t n = 0;
    if ((rc = gpu_candidates(ctx, coll, t_num, t_den, positional != 0, st, &n)) != SSJ_OK) return rc;
    HIP_OR_FAIL(ctx, grow(ctx->d_out, ctx->out_cap, (size_t)std::max<int64_t>(n, 1)));
    Req r{ctx->d_pairs, n, t_num, t_den, ctx->d_out, n, ctx->d_count, SSJ_SIM_JACCARD};
    if ((rc = enqueue_launch(ctx, coll, ctx->def, &r, 1, st, ctx->plan)) != SSJ_OK) return rc;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_count, ctx->d_count, sizeof(long long), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    const long long k = *ctx->h_count;
    if (k < 0) return set_error(SSJ_EDEVICE, "id error in generated candidates");
    const int64_t take = std::min<int64_t>(k, out_cap);
    if (take > 0) {
        HIP_OR_FAIL(ctx, hipMemcpyAsync(out, ctx->d_out, (size_t)take * 8, hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    }
    *out_n = k;
    if (k > out_cap) return set_error(SSJ_ETRUNC, "result larger than out_cap");
    return SSJ_OK;
}

int ssj_verify_device(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand, int64_t n_cand,
                      int64_t t_num, int64_t t_den, ssj_pair* d_out, int64_t out_cap,
                      int64_t* d_count, void* hip_stream) {
    return ssj_verify_device_sim(ctx, coll, d_cand, n_cand, SSJ_SIM_JACCARD, t_num, t_den, d_out,
                                 out_cap, d_count, hip_stream);
}

int ssj_verify_device_noalloc(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand, int64_t n_cand,
                              int64_t t_num, int64_t t_den, ssj_pair* d_out, int64_t out_cap, int64_t* d_count,
                              void* hip_stream) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    Req r{reinterpret_cast<const int2*>(d_cand), n_cand, t_num, t_den, reinterpret_cast<int2*>(d_out),
          out_cap, reinterpret_cast<long long*>(d_count), SSJ_SIM_JACCARD};
    if ((rc = check_req(r)) != SSJ_OK) return rc;
    if (n_cand > SSJ_NOALLOC_MAX_PAIRS)
        return set_error(SSJ_EINVAL, "ssj_verify_device_noalloc takes at most SSJ_NOALLOC_MAX_PAIRS (2^20) "
                                     "candidates per call");
    if (!ctx->noalloc.d_ctr) return set_error(SSJ_EDEVICE, "no scratch on this device");
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    // no graph (building one allocates) and no timing sample (event creation)
    return enqueue_launch(ctx, coll, ctx->noalloc, &r, 1, (hipStream_t)hip_stream, ctx->plan, false, nullptr,
                          false);
}

namespace {

// Host-buffer verification of flat pairs, r ids in coll, s ids in coll_s, in
// chunks that fit the HBM budget.
// Copies bytes from pageable to pinned host memory, in up to four threads
// for large copies (one thread copies at a fraction of what PCIe takes).
void host_copy(void* dst, const void* src, size_t bytes) {
    constexpr size_t kSplit = (size_t)4 << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned T = bytes >= kSplit ? std::min(4u, hw) : 1u;
    if (T <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t part = ((bytes + T - 1) / T + 63) & ~(size_t)63;
    auto copy_part = [=](unsigned t) {
        const size_t b = (size_t)t * part;
        if (b < bytes) std::memcpy((char*)dst + b, (const char*)src + b, std::min(bytes - b, part));
    };
    std::vector<std::thread> th;
    unsigned t = 1;
    try {
        for (; t < T; ++t) th.emplace_back(copy_part, t);
    } catch (...) {  // no thread: the rest in this one
        for (; t < T; ++t) copy_part(t);
    }
    copy_part(0);
    for (auto& x : th) x.join();
}

// The pinned ring and per-piece counts of the host-buffer path (ctx->mu held).
hipError_t ring_init(ssj_ctx* ctx) {
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        if (!ctx->h_ring[k])
            e = hipHostMalloc((void**)&ctx->h_ring[k], (size_t)kRingPiece * sizeof(int2), hipHostMallocDefault);
        if (e == hipSuccess && !ctx->ring_ev[k]) e = hipEventCreateWithFlags(&ctx->ring_ev[k], hipEventDisableTiming);
    }
    if (e == hipSuccess && !ctx->copy_stream) e = hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess && !ctx->d_counts) e = hipMalloc((void**)&ctx->d_counts, sizeof(long long) * kMaxPieces);
    if (e == hipSuccess && !ctx->h_counts)
        e = hipHostMalloc((void**)&ctx->h_counts, sizeof(long long) * kMaxPieces, hipHostMallocDefault);
    return e;
}

// Host-buffer verification.  Each device batch (bounded by the HBM budget)
// of more than kRingPiece pairs is sent in pieces of kRingPiece pairs through
// two pinned buffers: the host fills one buffer with piece k + 1 while piece k
// is copied to the device on the copy stream and piece k - 1 is verified on
// the launch stream (one launch per piece, its own count slot, started once
// its piece's copy is done), so copies and kernels overlap.  A batch of one
// piece is copied straight from the caller's buffer.  The counts of a batch
// come back in one copy, then each piece's passing pairs.
int verify_host(ssj_ctx* ctx, const ssj_coll* coll, const ssj_coll* coll_s, const ssj_pair* cand,
                int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap,
                int64_t* out_n) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_s)) != SSJ_OK) return rc;
    if (!valid_threshold(sim, t_num, t_den)) return set_error(SSJ_EINVAL, kThresholdError);
    if (n_cand < 0 || out_cap < 0) return set_error(SSJ_EINVAL, "negative size");
    if (!out_n || (n_cand > 0 && !cand) || (out_cap > 0 && !out))
        return set_error(SSJ_EINVAL, "null host buffer");
    *out_n = 0;
    if (n_cand == 0) return SSJ_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    HIP_OR_FAIL(ctx, ring_init(ctx));
    hipStream_t st = ctx->stream;
    int64_t chunk = (int64_t)std::max<uint64_t>(1, free_budget(ctx) / kBytesPerPair);
    chunk = std::min<int64_t>({chunk, kMaxLaunchPairs, kRingPiece * kMaxPieces});
    int64_t total = 0, done = 0;
    bool bad_id = false;
    while (done < n_cand && !bad_id) {
        const int64_t n = std::min<int64_t>(chunk, n_cand - done);
        HIP_OR_FAIL(ctx, grow(ctx->d_cand, ctx->cand_cap, (size_t)n));
        HIP_OR_FAIL(ctx, grow(ctx->d_out, ctx->out_cap, (size_t)n));
        const int64_t pieces = (n + kRingPiece - 1) / kRingPiece;  // <= kMaxPieces
        if (pieces == 1) {
            // nothing to overlap: one copy straight from the caller's buffer
            HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->d_cand, cand + done, (size_t)n * sizeof(int2),
                                            hipMemcpyHostToDevice, st));
            Req r{ctx->d_cand, n, t_num, t_den, ctx->d_out, n, ctx->d_counts, sim};
            rc = enqueue_launch(ctx, coll, ctx->def, &r, 1, st, ctx->plan, true, coll_s);
            if (rc != SSJ_OK) return rc;
        }
        for (int64_t k = 0; k < pieces && pieces > 1; ++k) {
            const int64_t off = k * kRingPiece, m = std::min(kRingPiece, n - off);
            const int slot = (int)(ctx->ring_seq++ & 1u);
            // the copy out of this buffer issued two pieces ago has finished
            HIP_OR_FAIL(ctx, hipEventSynchronize(ctx->ring_ev[slot]));
            host_copy(ctx->h_ring[slot], cand + done + off, (size_t)m * sizeof(int2));
            HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->d_cand + off, ctx->h_ring[slot], (size_t)m * sizeof(int2),
                                            hipMemcpyHostToDevice, ctx->copy_stream));
            // the event both releases the pinned buffer to the host (two
            // pieces later) and starts the piece's launch
            HIP_OR_FAIL(ctx, hipEventRecord(ctx->ring_ev[slot], ctx->copy_stream));
            HIP_OR_FAIL(ctx, hipStreamWaitEvent(st, ctx->ring_ev[slot], 0));
            Req r{ctx->d_cand + off, m, t_num, t_den, ctx->d_out + off, m, ctx->d_counts + k, sim};
            rc = enqueue_launch(ctx, coll, ctx->def, &r, 1, st, ctx->plan, true, coll_s);
            if (rc != SSJ_OK) return rc;
        }
        HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_counts, ctx->d_counts, sizeof(long long) * (size_t)pieces,
                                        hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
        for (int64_t k = 0; k < pieces; ++k) bad_id |= ctx->h_counts[k] < 0;
        if (bad_id) break;
        for (int64_t k = 0; k < pieces; ++k) {
            const long long c = ctx->h_counts[k];
            const int64_t take = std::min<int64_t>(std::max<int64_t>(0, out_cap - total), c);
            if (take > 0)
                HIP_OR_FAIL(ctx, hipMemcpyAsync(out + total, ctx->d_out + k * kRingPiece, (size_t)take * sizeof(int2),
                                                hipMemcpyDeviceToHost, st));
            total += c;
        }
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
        done += n;
    }
    if (bad_id) {
        *out_n = 0;
        return set_error(SSJ_EINVAL, "candidate id out of range");
    }
    *out_n = total;
    if (total > out_cap) return set_error(SSJ_ETRUNC, "result larger than out_cap");
    return SSJ_OK;
}

}  // namespace

int ssj_verify_sim(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand, int64_t n_cand,
                   int sim, int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap,
                   int64_t* out_n) {
    return verify_host(ctx, coll, coll, cand, n_cand, sim, t_num, t_den, out, out_cap, out_n);
}

int ssj_verify_rs(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s, const ssj_pair* cand,
                  int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* out,
                  int64_t out_cap, int64_t* out_n) {
    return verify_host(ctx, coll_r, coll_s, cand, n_cand, sim, t_num, t_den, out, out_cap, out_n);
}

int ssj_verify_groups(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                      const ssj_group* groups, int64_t n_groups, const int32_t* cand, int64_t n_cand,
                      int sim, int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap,
                      int64_t* out_n) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_r)) != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll_s)) != SSJ_OK) return rc;
    if (!valid_threshold(sim, t_num, t_den)) return set_error(SSJ_EINVAL, kThresholdError);
    if (n_groups < 0 || n_cand < 0 || out_cap < 0) return set_error(SSJ_EINVAL, "negative size");
    if (!out_n || (n_cand > 0 && !cand) || (n_groups > 0 && !groups) || (out_cap > 0 && !out))
        return set_error(SSJ_EINVAL, "null host buffer");
    // the group list must cover the candidates exactly, in order
    int64_t prev = 0;
    for (int64_t g = 0; g < n_groups; ++g) {
        if (groups[g].end < prev || groups[g].end > n_cand)
            return set_error(SSJ_EINVAL, "group ends must not decrease and must not pass n_cand");
        prev = groups[g].end;
    }
    if (prev != n_cand) return set_error(SSJ_EINVAL, "the last group must end at n_cand");
    *out_n = 0;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // batches of whole groups (a group larger than a batch is split), each
    // copied as its s ids and its groups with ends relative to the batch
    const size_t per_cand = 4 + kBytesPerPair;
    int64_t chunk = (int64_t)std::max<uint64_t>(1, free_budget(ctx) / per_cand);
    chunk = std::min<int64_t>(chunk, kMaxLaunchPairs);
    std::vector<ssj_group> bg;
    int64_t total = 0, c0 = 0, g = 0;
    bool bad_id = false;
    while (c0 < n_cand) {
        const int64_t c1 = std::min<int64_t>(n_cand, c0 + chunk);
        bg.clear();
        while (g < n_groups && groups[g].end <= c0) ++g;  // empty groups before the batch
        for (int64_t h = g; h < n_groups; ++h) {
            const int64_t e = std::min<int64_t>(groups[h].end, c1);
            if (e > c0 || bg.empty()) bg.push_back(ssj_group{groups[h].probe, (int32_t)(e - c0)});
            if (groups[h].end >= c1) break;
        }
        const int64_t n = c1 - c0;
        HIP_OR_FAIL(ctx, grow(ctx->d_sids, ctx->sids_cap, (size_t)n));
        HIP_OR_FAIL(ctx, grow(ctx->d_groups, ctx->groups_cap, bg.size()));
        HIP_OR_FAIL(ctx, grow(ctx->d_out, ctx->out_cap, (size_t)n));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->d_sids, cand + c0, (size_t)n * 4, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->d_groups, bg.data(), bg.size() * sizeof(ssj_group),
                                        hipMemcpyHostToDevice, st));
        rc = enqueue_groups(ctx, coll_r, coll_s, ctx->d_groups, (int64_t)bg.size(), ctx->d_sids, n, sim,
                            t_num, t_den, ctx->d_out, n, ctx->d_count, st);
        if (rc != SSJ_OK) return rc;
        HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_count, ctx->d_count, sizeof(long long), hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
        const long long k = *ctx->h_count;
        if (k < 0) {
            bad_id = true;
            break;
        }
        const int64_t room = std::max<int64_t>(0, out_cap - total);
        const int64_t take = std::min<int64_t>(room, k);
        if (take > 0) {
            HIP_OR_FAIL(ctx, hipMemcpyAsync(out + total, ctx->d_out, (size_t)take * 8, hipMemcpyDeviceToHost, st));
            HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
        }
        total += k;
        c0 = c1;
    }
    if (bad_id) {
        *out_n = 0;
        return set_error(SSJ_EINVAL, "candidate id out of range");
    }
    *out_n = total;
    if (total > out_cap) return set_error(SSJ_ETRUNC, "result larger than out_cap");
    return SSJ_OK;
}

int ssj_verify(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand, int64_t n_cand,
               int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap, int64_t* out_n) {
    return ssj_verify_sim(ctx, coll, cand, n_cand, SSJ_SIM_JACCARD, t_num, t_den, out, out_cap,
                          out_n);
}

}  // extern "C"

namespace {

int64_t gcd64(int64_t a, int64_t b) {
    while (b != 0) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Tuning cache key of a workload on the context's device.
std::string tune_key(const ssj_ctx* ctx, const ssj_coll* coll, int64_t n_cand, int64_t t_num, int64_t t_den) {
    const int64_t g = std::max<int64_t>(1, gcd64(t_num, t_den));
    return ctx->device_key + "|sets=" + std::to_string(coll->n_sets) + ",tokens=" + std::to_string(coll->n_tokens) +
           ",max_len=" + std::to_string(coll->max_len) + "|cand=" + std::to_string(n_cand) + "|t=" +
           std::to_string(t_num / g) + "/" + std::to_string(t_den / g);
}

// The last well-formed entry of key in the cache file.
bool tune_lookup(const std::string& path, const std::string& key, ssj_plan* plan, double* ms) {
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    const std::string want = "{\"key\": \"" + key + "\", ";
    bool found = false;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, want.c_str(), want.size()) != 0) continue;
        ssj_plan p{};
        double t = 0.0;
        const int n = std::sscanf(line + want.size(),
                                  "\"kernel_ms\": %lf, \"plan\": [%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d]}",
                                  &t, &p.inline_lanes, &p.hard_lanes, &p.defer_from, &p.lanes[0], &p.lanes[1],
                                  &p.lanes[2], &p.lanes[3], &p.lanes[4], &p.use_graph, &p.spill_iters,
                                  &p.spill_lanes, &p.wg_per_cu, &p.staged);
        if (n == 14 && plan_valid(p)) {
            *plan = p;
            *ms = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

// Appends an entry (one write of the whole line).
void tune_store(const std::string& path, const std::string& key, const ssj_plan& p, double ms) {
    char buf[1024];
    const int n = std::snprintf(buf, sizeof buf,
                                "{\"key\": \"%s\", \"kernel_ms\": %.6f, \"plan\": [%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d]}\n",
                                key.c_str(), ms, p.inline_lanes, p.hard_lanes, p.defer_from, p.lanes[0], p.lanes[1],
                                p.lanes[2], p.lanes[3], p.lanes[4], p.use_graph, p.spill_iters, p.spill_lanes,
                                p.wg_per_cu, p.staged);
    if (n <= 0 || n >= (int)sizeof buf) return;
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fwrite(buf, 1, (size_t)n, f);
    std::fclose(f);
}

}  // namespace

extern "C" {

int ssj_set_tune_cache(ssj_ctx* ctx, const char* path) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->tune_cache = path ? path : "";
    return SSJ_OK;
}

int ssj_autotune(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand, int64_t n_cand,
                 int64_t t_num, int64_t t_den, int apply, ssj_plan* best, double* best_ms) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    if (!valid_threshold(SSJ_SIM_JACCARD, t_num, t_den)) return set_error(SSJ_EINVAL, kThresholdError);
    if (n_cand <= 0 || n_cand > kMaxLaunchPairs || !d_cand)
        return set_error(SSJ_EINVAL, "autotuning needs 1 .. 2^31-1 device candidates");
    std::lock_guard<std::mutex> g(ctx->mu);
    const std::string key = tune_key(ctx, coll, n_cand, t_num, t_den);
    if (!ctx->tune_cache.empty()) {
        ssj_plan p{};
        double ms = 0.0;
        if (tune_lookup(ctx->tune_cache, key, &p, &ms)) {
            if (best) *best = p;
            if (best_ms) *best_ms = ms;
            if (apply) {
                std::lock_guard<std::mutex> gp(ctx->plan_mu);
                ctx->plan = p;
            }
            return SSJ_CACHED;
        }
    }
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    HIP_OR_FAIL(ctx, grow(ctx->d_out, ctx->out_cap, (size_t)n_cand));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OR_FAIL(ctx, hipEventCreate(&e0));
    HIP_OR_FAIL(ctx, hipEventCreate(&e1));
    const int timing_was = ctx->timing_period.exchange(0);
    auto measure = [&](const ssj_plan& p, double* ms) -> int {
        Req r{reinterpret_cast<const int2*>(d_cand), n_cand, t_num, t_den, ctx->d_out, n_cand,
              ctx->d_count};
        int rc2 = enqueue_launch(ctx, coll, ctx->def, &r, 1, st, p, false);  // warm-up
        if (rc2 != SSJ_OK) return rc2;
        double bestt = 1e30;
        for (int it = 0; it < 3; ++it) {
            HIP_OR_FAIL(ctx, hipEventRecord(e0, st));
            rc2 = enqueue_launch(ctx, coll, ctx->def, &r, 1, st, p, false);
            if (rc2 != SSJ_OK) return rc2;
            HIP_OR_FAIL(ctx, hipEventRecord(e1, st));
            HIP_OR_FAIL(ctx, hipEventSynchronize(e1));
            float t = 0.f;
            HIP_OR_FAIL(ctx, hipEventElapsedTime(&t, e0, e1));
            bestt = std::min(bestt, (double)t);
        }
        *ms = bestt;
        return SSJ_OK;
    };
    // 1) every in-order mapping with every deferral point (deferred classes
    //    start from mappings suited to their lengths)
    static const int kDeferredDefault[ssj::kClasses] = {4, 8, 16, 32, 64};
    ssj_plan cur = ctx->plan;
    double cur_ms = 1e30;
    ssj_plan thread_best = ctx->plan;  // best plan with one thread per pair, no hard lanes
    double thread_ms = 1e30;
    ssj_plan staged_best = ctx->plan;  // best plan with the window ring
    double staged_ms = 1e30;
    for (int k = 0; k < kMappings && rc == SSJ_OK; ++k) {
        for (int d = ssj::kClasses; d >= 1 && rc == SSJ_OK; --d) {
            // each at the resident grid and at twice that (a larger grid
            // evens out wavefronts that start late or issue slowly)
            for (int twice = 0; twice < 2 && rc == SSJ_OK; ++twice) {
                ssj_plan p = ctx->plan;
                p.inline_lanes = kInlineLanes[k];
                p.hard_lanes = kInlineHard[k];
                p.staged = kInlineStaged[k];
                p.defer_from = d;
                p.spill_iters = 0;
                p.wg_per_cu = 0;
                for (int q = 0; q < ssj::kClasses; ++q) p.lanes[q] = kDeferredDefault[q];
                if (twice) p.wg_per_cu = std::min(kMaxWgPerCu, 2 * tiles_occupancy(ctx, p, false));
                double ms = 0;
                if ((rc = measure(p, &ms)) != SSJ_OK) break;
                if (ms < cur_ms) {
                    cur_ms = ms;
                    cur = p;
                }
                if (k == 0 && ms < thread_ms) {
                    thread_ms = ms;
                    thread_best = p;
                }
                if (kInlineStaged[k] && kInlineLanes[k] == 1 && ms < staged_ms) {
                    staged_ms = ms;
                    staged_best = p;
                }
            }
        }
    }
    // 2) thread-per-pair merges cut off after a budget of window steps (the
    //    rest of such a merge goes to the deferred kernel), tried on the best
    //    thread-per-pair plan and the best window-ring plan, each with and
    //    without its deferred classes
    static const int kSpillIters[6] = {4, 8, 12, 16, 24, 32};
    for (const ssj_plan& base : {thread_best, staged_best}) {
        for (int nodefer = 0; nodefer < 2 && rc == SSJ_OK; ++nodefer) {
            if (nodefer && base.defer_from == ssj::kClasses) break;
            for (int it : kSpillIters) {
                ssj_plan p = base;
                if (nodefer) p.defer_from = ssj::kClasses;
                p.spill_iters = it;
                p.spill_lanes = 16;
                double ms = 0;
                if ((rc = measure(p, &ms)) != SSJ_OK) break;
                if (ms < cur_ms * 0.99) {
                    cur_ms = ms;
                    cur = p;
                }
            }
        }
    }
    if (cur.spill_iters > 0 && rc == SSJ_OK) {
        const ssj_plan base = cur;
        for (int o : {4, 8, 32, 64, (int)ssj::kBlock}) {
            ssj_plan p = base;
            p.spill_lanes = o;
            double ms = 0;
            if ((rc = measure(p, &ms)) != SSJ_OK) break;
            if (ms < cur_ms * 0.99) {
                cur_ms = ms;
                cur = p;
            }
        }
    }
    // 3) refine the mapping of each deferred class, one class at a time
    static const int kDeferredOptions[6] = {4, 8, 16, 32, 64, ssj::kBlock};
    for (int q = cur.defer_from; q < ssj::kClasses && rc == SSJ_OK; ++q) {
        const ssj_plan base = cur;
        for (int o : kDeferredOptions) {
            if (o == base.lanes[q]) continue;
            ssj_plan p = base;
            p.lanes[q] = o;
            double ms = 0;
            if ((rc = measure(p, &ms)) != SSJ_OK) break;
            if (ms < cur_ms * 0.99) {
                cur_ms = ms;
                cur = p;
            }
        }
    }
    // 4) the in-order grid: fewer or more workgroups per compute unit than
    //    fit at once
    if (rc == SSJ_OK) {
        const int occ = cur.wg_per_cu > 0 ? cur.wg_per_cu : tiles_occupancy(ctx, cur, false);
        const ssj_plan base = cur;
        for (int wg : {occ - 1, occ + 1, occ + 2, (3 * occ) / 2}) {
            if (wg < 1 || wg > kMaxWgPerCu) continue;
            ssj_plan p = base;
            p.wg_per_cu = wg;
            double ms = 0;
            if ((rc = measure(p, &ms)) != SSJ_OK) break;
            if (ms < cur_ms * 0.99) {
                cur_ms = ms;
                cur = p;
            }
        }
    }
    ctx->timing_period = timing_was;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SSJ_OK) return rc;
    if (!ctx->tune_cache.empty()) tune_store(ctx->tune_cache, key, cur, cur_ms);
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    if (apply) {
        std::lock_guard<std::mutex> gp(ctx->plan_mu);
        ctx->plan = cur;
    }
    return SSJ_OK;
}

int ssj_stream_submit(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand, int64_t n_cand,
                      int64_t t_num, int64_t t_den, int nonblocking, uint64_t* ticket) {
    return ssj_stream_submit_sim(ctx, coll, cand, n_cand, SSJ_SIM_JACCARD, t_num, t_den,
                                 nonblocking, ticket);
}

int ssj_stream_submit_sim(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand,
                          int64_t n_cand, int sim, int64_t t_num, int64_t t_den, int nonblocking,
                          uint64_t* ticket) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_coll(ctx, coll)) != SSJ_OK) return rc;
    if (!ticket) return set_error(SSJ_EINVAL, "null ticket pointer");
    *ticket = 0;
    if (!valid_threshold(sim, t_num, t_den)) return set_error(SSJ_EINVAL, kThresholdError);
    if (n_cand < 0 || (n_cand > 0 && !cand)) return set_error(SSJ_EINVAL, "bad candidate buffer");
    StreamEngine* E = ctx->engine.get();
    if (!E) return set_error(SSJ_EINVAL, "streaming engine not running");
    std::unique_lock<std::mutex> lk(E->mu);
    auto room = [&]() { return (int)E->pending.size() + E->reserved < ctx->queue_depth; };
    if (!room()) {
        if (nonblocking) return set_error(SSJ_EAGAIN, "stream queue full");
        E->cv_space.wait(lk, [&]() { return room() || E->stop || ctx->failed.load(); });
        if (E->stop) return set_error(SSJ_EINVAL, "context is shutting down");
        if (ctx->failed) return set_error(SSJ_EDEVICE, "context failed after a HIP error");
    }
    // the collection list changes only under this lock too: a collection
    // freed since check_coll is refused here, before anything refers to it
    if (std::find(ctx->colls.begin(), ctx->colls.end(), coll) == ctx->colls.end())
        return set_error(SSJ_EINVAL, "unknown collection");
    StreamReq* r = new (std::nothrow) StreamReq();
    if (!r) return set_error(SSJ_ENOMEM, "host allocation failed");
    // the request holds its collection and its queue place from here on: a
    // free of the collection sees it in flight, and concurrent submitters see
    // the place taken while this one copies its candidates
    coll->inflight.fetch_add(1);
    ++E->reserved;
    r->ticket = E->next_ticket++;
    r->coll = coll;
    r->t_num = t_num;
    r->t_den = t_den;
    r->sim = sim;
    r->n = n_cand;
    r->t_submit = now_ns();
    r->h_cand = (int2*)pinned_take(E, (size_t)std::max<int64_t>(n_cand, 1) * 8, &r->h_cand_bytes);
    // a new staging buffer and the copy into staging come outside the lock;
    // the request is not yet visible to the engine
    lk.unlock();
    if (!r->h_cand) {
        void* p = nullptr;
        if (hipHostMalloc(&p, r->h_cand_bytes, hipHostMallocDefault) != hipSuccess || !p) {
            lk.lock();
            --E->reserved;
            coll->inflight.fetch_sub(1);
            lk.unlock();
            E->cv_space.notify_all();
            delete r;
            return set_error(SSJ_ENOMEM, "pinned staging allocation failed");
        }
        r->h_cand = (int2*)p;
    }
    if (n_cand > 0) std::memcpy(r->h_cand, cand, (size_t)n_cand * 8);
    lk.lock();
    --E->reserved;
    E->table.emplace(r->ticket, r);
    E->pending.push_back(r);
    *ticket = r->ticket;
    lk.unlock();
    E->cv_work.notify_all();
    return SSJ_OK;
}

int ssj_stream_pause(ssj_ctx* ctx, int pause) {
    if (!ctx) return set_error(SSJ_EINVAL, "null context");
    StreamEngine* E = ctx->engine.get();
    if (!E) return set_error(SSJ_EINVAL, "streaming engine not running");
    {
        std::lock_guard<std::mutex> g(E->mu);
        E->paused = pause != 0;
    }
    E->cv_work.notify_all();
    return SSJ_OK;
}

int ssj_stream_poll(ssj_ctx* ctx, uint64_t ticket, int wait, ssj_pair* out, int64_t out_cap,
                    int64_t* out_n) {
    if (!ctx) return set_error(SSJ_EINVAL, "null context");
    if (out_n) *out_n = 0;
    StreamEngine* E = ctx->engine.get();
    if (!E) return set_error(SSJ_EINVAL, "streaming engine not running");
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->table.find(ticket);
    if (it == E->table.end()) return set_error(SSJ_ENOTFOUND, "unknown or retired ticket");
    StreamReq* r = it->second;
    if (r->status == SSJ_PENDING) {
        if (!wait) return SSJ_PENDING;
        E->cv_done.wait(lk, [&]() { return r->status != SSJ_PENDING; });
    }
    if (r->status == SSJ_EINVAL || r->status == SSJ_EDEVICE) {
        const int st = r->status;
        E->table.erase(it);
        delete r;
        return set_error(st, st == SSJ_EINVAL ? "candidate id out of range" : "device failure");
    }
    const int64_t k = (int64_t)r->result.size();
    if (out_n) *out_n = k;
    if (k > out_cap) return set_error(SSJ_ETRUNC, "result larger than out_cap");
    if (k > 0) {
        if (!out) return set_error(SSJ_EINVAL, "null output buffer");
        std::memcpy(out, r->result.data(), (size_t)k * 8);
    }
    E->table.erase(it);
    delete r;
    return SSJ_OK;
}

int ssj_stream_stats(ssj_ctx* ctx, ssj_stream_stats_t* out, int reset) {
    if (!ctx) return set_error(SSJ_EINVAL, "null context");
    if (!out) return set_error(SSJ_EINVAL, "null output");
    StreamEngine* E = ctx->engine.get();
    if (!E) return set_error(SSJ_EINVAL, "streaming engine not running");
    std::lock_guard<std::mutex> g(E->mu);
    out->slot_grows = E->slot_grows;
    out->slot_grow_ms = E->slot_grow_ms;
    out->result_grows = E->result_grows;
    out->result_grow_ms = E->result_grow_ms;
    out->longest_pass_ms = E->longest_pass_ms;
    if (reset) {
        E->slot_grows = E->result_grows = 0;
        E->slot_grow_ms = E->result_grow_ms = E->longest_pass_ms = 0.0;
    }
    return SSJ_OK;
}

int ssj_stream_times(ssj_ctx* ctx, uint64_t ticket, int wait, uint64_t* t_submit,
                     uint64_t* t_admit, uint64_t* t_done) {
    if (!ctx) return set_error(SSJ_EINVAL, "null context");
    StreamEngine* E = ctx->engine.get();
    if (!E) return set_error(SSJ_EINVAL, "streaming engine not running");
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->table.find(ticket);
    if (it == E->table.end()) return set_error(SSJ_ENOTFOUND, "unknown or retired ticket");
    StreamReq* r = it->second;
    if (r->status == SSJ_PENDING) {
        if (!wait) return SSJ_PENDING;
        E->cv_done.wait(lk, [&]() { return r->status != SSJ_PENDING; });
    }
    if (t_submit) *t_submit = r->t_submit;
    if (t_admit) *t_admit = r->t_admit;
    if (t_done) *t_done = r->t_done;
    return SSJ_OK;
}

}  // extern "C"
