// Host runtime of libssj: the C ABI, the HBM collection store, scratch and
// launch management, and the streaming request loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ssj.h"
#include "ssj_device.h"

namespace {

thread_local std::string tl_error;

int set_error(int code, const std::string& msg) {
    tl_error = msg;
    return code;
}

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr uint64_t kDefaultBudget = 4ull << 30;
constexpr int64_t kMaxChunk = (int64_t)1 << 30;  // pairs per launch (< 2^31)
constexpr size_t kBytesPerPairBucketed = 8 + 8 + 4 * ssj::kClasses;

bool valid_threshold(int64_t t_num, int64_t t_den) {
    return t_den > 0 && t_den <= INT32_MAX && t_num >= 0 && t_num <= t_den;
}

// Device scratch of one in-flight request.
struct Slot {
    hipStream_t stream = nullptr;
    ssj::Counters* d_ctr = nullptr;
    long long* d_count = nullptr;
    long long* h_count = nullptr;  // pinned
    uint32_t* d_queues = nullptr;
    size_t q_cap = 0;
    int2* d_cand = nullptr;
    size_t cand_cap = 0;
    int2* d_out = nullptr;
    size_t out_cap = 0;
    hipEvent_t ev_done = nullptr;
};

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

}  // namespace

struct ssj_coll {
    ssj_ctx* ctx = nullptr;
    int32_t* d_tok = nullptr;
    uint2* d_desc = nullptr;
    int64_t n_sets = 0;
    int64_t n_tokens = 0;
    int64_t max_len = 0;
    std::atomic<int> inflight{0};
};

struct ssj_ctx {
    int device = 0;
    uint64_t budget = kDefaultBudget;
    int n_slots = 4;
    int queue_depth = 64;
    int n_cu = 0;
    int grid_bucketed = 0;
    int grid_classify = 0;
    int occ_direct[9] = {0};
    ssj_plan plan{};
    std::mutex mu;  // default slot, collections, plan
    Slot def;
    std::atomic<bool> failed{false};
    std::vector<ssj_coll*> colls;
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

int lanes_index(int lanes) {
    switch (lanes) {
        case 1: return 0;
        case 4: return 1;
        case 8: return 2;
        case 16: return 3;
        case 32: return 4;
        case 64: return 5;
        case ssj::kBlock: return 6;
        default: return -1;
    }
}

int slot_init(ssj_ctx* ctx, Slot& s, bool own_stream) {
    if (own_stream) HIP_OR_FAIL(ctx, hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
    HIP_OR_FAIL(ctx, hipMalloc((void**)&s.d_ctr, sizeof(ssj::Counters)));
    HIP_OR_FAIL(ctx, hipMemset(s.d_ctr, 0, sizeof(ssj::Counters)));
    HIP_OR_FAIL(ctx, hipMalloc((void**)&s.d_count, sizeof(long long)));
    HIP_OR_FAIL(ctx, hipHostMalloc((void**)&s.h_count, sizeof(long long), hipHostMallocDefault));
    HIP_OR_FAIL(ctx, hipEventCreateWithFlags(&s.ev_done, hipEventDisableTiming));
    return SSJ_OK;
}

void slot_free(Slot& s) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.d_ctr) (void)hipFree(s.d_ctr);
    if (s.d_count) (void)hipFree(s.d_count);
    if (s.h_count) (void)hipHostFree(s.h_count);
    if (s.d_queues) (void)hipFree(s.d_queues);
    if (s.d_cand) (void)hipFree(s.d_cand);
    if (s.d_out) (void)hipFree(s.d_out);
    if (s.ev_done) (void)hipEventDestroy(s.ev_done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = Slot{};
}

void default_plan(ssj_plan& p) {
    p.mode = SSJ_MODE_BUCKETED;
    const int lanes[ssj::kClasses] = {1, 16, 64, ssj::kBlock, ssj::kBlock};
    for (int q = 0; q < ssj::kClasses; ++q) p.lanes[q] = lanes[q];
    p.use_graph = 0;
}

int grid_direct(const ssj_ctx* ctx, int lanes, int64_t n) {
    const int idx = lanes_index(lanes);
    const int64_t cap = (int64_t)ctx->n_cu * std::max(1, ctx->occ_direct[idx]);
    int64_t want;
    if (lanes == ssj::kBlock) {
        want = n;
    } else {
        const int64_t pairs_per_block = (int64_t)ssj::kBlock / lanes;
        want = (n + pairs_per_block - 1) / pairs_per_block;
    }
    return (int)std::max<int64_t>(1, std::min(want, cap));
}

// Enqueues one verification of n pairs already on the device.
int enqueue_verify(ssj_ctx* ctx, const ssj_coll* coll, Slot& slot, const int2* d_cand, int64_t n,
                   int64_t t_num, int64_t t_den, int2* d_out, int64_t out_cap,
                   long long* d_count, hipStream_t st, const ssj_plan& plan) {
    ssj::VerifyArgs a{};
    a.tok = coll->d_tok;
    a.desc = coll->d_desc;
    a.n_sets = (uint32_t)coll->n_sets;
    a.n = (uint32_t)n;
    a.cand = d_cand;
    a.tn = (unsigned long long)t_num;
    a.tsum = (unsigned long long)(t_num + t_den);
    a.out = d_out;
    a.cap = (unsigned long long)std::max<int64_t>(0, out_cap);
    a.ctr = slot.d_ctr;
    a.d_count = d_count;
    const uint32_t bounds[ssj::kClasses] = SSJ_CLASS_BOUNDS;
    for (int q = 0; q < ssj::kClasses; ++q) {
        a.bounds[q] = bounds[q];
        a.lanes[q] = plan.lanes[q];
        a.order[q] = ssj::kClasses - 1 - q;  // longest class first
    }
    if (plan.mode == SSJ_MODE_DIRECT) {
        HIP_OR_FAIL(ctx, ssj::launch_verify_direct(a, plan.lanes[0],
                                                   grid_direct(ctx, plan.lanes[0], n), st));
        return SSJ_OK;
    }
    HIP_OR_FAIL(ctx, grow(slot.d_queues, slot.q_cap, (size_t)ssj::kClasses * (size_t)std::max<int64_t>(n, 1)));
    a.queues = slot.d_queues;
    a.qcap = (uint32_t)(slot.q_cap / ssj::kClasses);
    const int64_t want_c = (n + ssj::kBlock - 1) / ssj::kBlock;
    const int gc = (int)std::max<int64_t>(1, std::min<int64_t>(want_c, ctx->grid_classify));
    HIP_OR_FAIL(ctx, ssj::launch_classify(a, gc, st));
    HIP_OR_FAIL(ctx, ssj::launch_verify_bucketed(a, ctx->grid_bucketed, st));
    return SSJ_OK;
}

int check_ctx(ssj_ctx* ctx) {
    if (!ctx) return set_error(SSJ_EINVAL, "null context");
    if (ctx->failed) return set_error(SSJ_EDEVICE, "context failed after a HIP error");
    return SSJ_OK;
}

int check_verify_args(const ssj_coll* coll, int64_t n_cand, int64_t t_num, int64_t t_den,
                      int64_t out_cap) {
    if (!coll) return set_error(SSJ_EINVAL, "null collection");
    if (!valid_threshold(t_num, t_den))
        return set_error(SSJ_EINVAL, "threshold must satisfy 0 <= t_num <= t_den, 0 < t_den < 2^31");
    if (n_cand < 0) return set_error(SSJ_EINVAL, "negative candidate count");
    if (out_cap < 0) return set_error(SSJ_EINVAL, "negative output capacity");
    return SSJ_OK;
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
        int occ = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ssj::kernel_verify_bucketed(), ssj::kBlock, 0)) != hipSuccess) {
            rc = hip_fail(ctx, "hipOccupancyMaxActiveBlocksPerMultiprocessor", e);
            break;
        }
        ctx->grid_bucketed = ctx->n_cu * std::max(1, occ);
        ctx->grid_classify = ctx->n_cu * 8;
        const int lanes_list[7] = {1, 4, 8, 16, 32, 64, ssj::kBlock};
        for (int k = 0; k < 7 && rc == SSJ_OK; ++k) {
            occ = 0;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ssj::kernel_verify_direct(lanes_list[k]), ssj::kBlock, 0)) != hipSuccess)
                rc = hip_fail(ctx, "hipOccupancyMaxActiveBlocksPerMultiprocessor", e);
            ctx->occ_direct[k] = occ;
        }
        if (rc != SSJ_OK) break;
        rc = slot_init(ctx, ctx->def, true);
    } while (0);
    if (rc != SSJ_OK) {
        slot_free(ctx->def);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return SSJ_OK;
}

int ssj_shutdown(ssj_ctx* ctx) {
    if (!ctx) return SSJ_OK;
    (void)hipSetDevice(ctx->device);
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        for (ssj_coll* c : ctx->colls) {
            if (c->d_tok) (void)hipFree(c->d_tok);
            if (c->d_desc) (void)hipFree(c->d_desc);
            delete c;
        }
        ctx->colls.clear();
        slot_free(ctx->def);
    }
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
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    ssj_coll* c = new (std::nothrow) ssj_coll();
    if (!c) return set_error(SSJ_ENOMEM, "host allocation failed");
    c->ctx = ctx;
    c->n_sets = n_sets;
    c->n_tokens = n_tokens;
    c->max_len = max_len;
    int64_t* d_off = nullptr;
    hipError_t e = hipSuccess;
    do {
        if ((e = hipMalloc((void**)&c->d_tok, (size_t)std::max<int64_t>(n_tokens, 1) * 4)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&c->d_desc, (size_t)std::max<int64_t>(n_sets, 1) * 8)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&d_off, (size_t)(n_sets + 1) * 8)) != hipSuccess) break;
        if (n_tokens > 0 && (e = hipMemcpyAsync(c->d_tok, tokens, (size_t)n_tokens * 4, hipMemcpyHostToDevice, ctx->def.stream)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(d_off, offsets, (size_t)(n_sets + 1) * 8, hipMemcpyHostToDevice, ctx->def.stream)) != hipSuccess) break;
        if ((e = ssj::launch_build_desc(d_off, c->d_desc, n_sets, ctx->def.stream)) != hipSuccess) break;
        if ((e = hipStreamSynchronize(ctx->def.stream)) != hipSuccess) break;
    } while (0);
    if (d_off) (void)hipFree(d_off);
    if (e != hipSuccess) {
        if (c->d_tok) (void)hipFree(c->d_tok);
        if (c->d_desc) (void)hipFree(c->d_desc);
        delete c;
        if (e == hipErrorOutOfMemory) return set_error(SSJ_ENOMEM, "device allocation failed");
        return hip_fail(ctx, "upload", e);
    }
    ctx->colls.push_back(c);
    *out = c;
    return SSJ_OK;
}

int ssj_free_collection(ssj_ctx* ctx, ssj_coll* coll) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if (!coll || coll->ctx != ctx) return set_error(SSJ_EINVAL, "collection does not belong to this context");
    if (coll->inflight.load() != 0) return set_error(SSJ_EAGAIN, "collection has requests in flight");
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = std::find(ctx->colls.begin(), ctx->colls.end(), coll);
    if (it == ctx->colls.end()) return set_error(SSJ_EINVAL, "unknown collection");
    ctx->colls.erase(it);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->def.stream);
    if (coll->d_tok) (void)hipFree(coll->d_tok);
    if (coll->d_desc) (void)hipFree(coll->d_desc);
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
    if (plan->mode != SSJ_MODE_BUCKETED && plan->mode != SSJ_MODE_DIRECT)
        return set_error(SSJ_EINVAL, "unknown plan mode");
    for (int q = 0; q < ssj::kClasses; ++q)
        if (!ssj::lanes_supported(plan->lanes[q]))
            return set_error(SSJ_EINVAL, "lanes must be one of 1, 4, 8, 16, 32, 64, 256");
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->plan = *plan;
    return SSJ_OK;
}

int ssj_verify_device(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand, int64_t n_cand,
                      int64_t t_num, int64_t t_den, ssj_pair* d_out, int64_t out_cap,
                      int64_t* d_count, void* hip_stream) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_verify_args(coll, n_cand, t_num, t_den, out_cap)) != SSJ_OK) return rc;
    if (coll->ctx != ctx) return set_error(SSJ_EINVAL, "collection does not belong to this context");
    if (n_cand >= INT32_MAX) return set_error(SSJ_EINVAL, "n_cand must be below 2^31 per device call");
    if (!d_count || (n_cand > 0 && !d_cand)) return set_error(SSJ_EINVAL, "null device buffer");
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    return enqueue_verify(ctx, coll, ctx->def, reinterpret_cast<const int2*>(d_cand), n_cand, t_num,
                          t_den, reinterpret_cast<int2*>(d_out), out_cap,
                          reinterpret_cast<long long*>(d_count), (hipStream_t)hip_stream, ctx->plan);
}

int ssj_verify(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand, int64_t n_cand,
               int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap, int64_t* out_n) {
    int rc = check_ctx(ctx);
    if (rc != SSJ_OK) return rc;
    if ((rc = check_verify_args(coll, n_cand, t_num, t_den, out_cap)) != SSJ_OK) return rc;
    if (coll->ctx != ctx) return set_error(SSJ_EINVAL, "collection does not belong to this context");
    if (!out_n || (n_cand > 0 && !cand) || (out_cap > 0 && !out))
        return set_error(SSJ_EINVAL, "null host buffer");
    *out_n = 0;
    std::lock_guard<std::mutex> g(ctx->mu);
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    Slot& s = ctx->def;
    int64_t chunk = (int64_t)std::max<uint64_t>(1, ctx->budget / kBytesPerPairBucketed);
    chunk = std::min<int64_t>(chunk, kMaxChunk);
    int64_t total = 0;
    bool bad_id = false;
    int64_t done = 0;
    do {
        const int64_t n = std::min<int64_t>(chunk, n_cand - done);
        HIP_OR_FAIL(ctx, grow(s.d_cand, s.cand_cap, (size_t)std::max<int64_t>(n, 1)));
        HIP_OR_FAIL(ctx, grow(s.d_out, s.out_cap, (size_t)std::max<int64_t>(n, 1)));
        if (n > 0)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(s.d_cand, cand + done, (size_t)n * 8, hipMemcpyHostToDevice, s.stream));
        rc = enqueue_verify(ctx, coll, s, s.d_cand, n, t_num, t_den, s.d_out, n, s.d_count, s.stream, ctx->plan);
        if (rc != SSJ_OK) return rc;
        HIP_OR_FAIL(ctx, hipMemcpyAsync(s.h_count, s.d_count, sizeof(long long), hipMemcpyDeviceToHost, s.stream));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(s.stream));
        const long long k = *s.h_count;
        if (k < 0) {
            bad_id = true;
            break;
        }
        const int64_t room = std::max<int64_t>(0, out_cap - total);
        const int64_t take = std::min<int64_t>(room, k);
        if (take > 0)
            HIP_OR_FAIL(ctx, hipMemcpy(out + total, s.d_out, (size_t)take * 8, hipMemcpyDeviceToHost));
        total += k;
        done += n;
    } while (done < n_cand);
    if (bad_id) {
        *out_n = 0;
        return set_error(SSJ_EINVAL, "candidate id out of range");
    }
    *out_n = total;
    if (total > out_cap) return set_error(SSJ_ETRUNC, "result larger than out_cap");
    return SSJ_OK;
}

int ssj_stream_submit(ssj_ctx* ctx, const ssj_coll*, const ssj_pair*, int64_t, int64_t, int64_t,
                      int, uint64_t* ticket) {
    if (ticket) *ticket = 0;
    (void)ctx;
    return set_error(SSJ_EINVAL, "streaming is not available in this build");
}

int ssj_stream_poll(ssj_ctx*, uint64_t, int, ssj_pair*, int64_t, int64_t* out_n) {
    if (out_n) *out_n = 0;
    return set_error(SSJ_ENOTFOUND, "streaming is not available in this build");
}

int ssj_stream_times(ssj_ctx*, uint64_t, uint64_t*, uint64_t*, uint64_t*) {
    return set_error(SSJ_ENOTFOUND, "streaming is not available in this build");
}

}  // extern "C"
