/*
 * libssj -- verification phase of exact set-similarity joins on MI355X (gfx950).
 *
 * The library verifies candidate pairs (r, s) of token sets held in an HBM
 * resident collection: a pair is in the result iff its similarity is at
 * least t = t_num / t_den (paper Sec. 3, Definition 1).  The similarity is
 * Jaccard |r & s| / |r | s| unless a call names another function of Table 1
 * (SSJ_SIM_*).  Each function is turned into the equivalent overlap of
 * Table 1, the least |r & s| that reaches t, computed exactly in integers;  no
 * floating point decides a pair.  The overlap comes from an intersection that
 * stops as soon as the required overlap is met or can no longer be reached
 * (paper Sec. 3.1), so only candidates whose outcome is undecided cost more
 * work.
 *
 * Collections follow the paper's preprocessing contract (Sec. 2.2, "Data
 * layout"): every set is non-empty, its tokens are unique non-negative int32
 * ids in strictly increasing order.  (The frequency ordering of token ids and
 * the size ordering of sets help the candidate filter; verification does not
 * depend on them and does not check them.)  Set ids are positions in the
 * uploaded collection.
 *
 * Status: every function returns an int; SSJ_OK (0) on success, a positive
 * value for a non-error state (SSJ_PENDING), a negative value for an error.
 * No C++ exception crosses this interface.
 */
#ifndef SSJ_H
#define SSJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SSJ_OK = 0,
    SSJ_PENDING = 1,     /* stream request not finished yet */
    SSJ_CACHED = 2,      /* ssj_autotune: the plan came from the tuning cache */
    SSJ_EINVAL = -1,     /* bad argument, malformed collection, id out of range */
    SSJ_ENOMEM = -2,     /* device or host allocation failed / over the HBM budget */
    SSJ_ETRUNC = -3,     /* result larger than out_cap; *out_n holds the size needed */
    SSJ_EAGAIN = -4,     /* non-blocking submit found the queue full; or object busy */
    SSJ_EDEVICE = -5,    /* a HIP runtime call failed; the context stays failed */
    SSJ_ENOTFOUND = -6   /* unknown or already retired ticket */
};

typedef struct ssj_ctx ssj_ctx;   /* one per GPU; opaque */
typedef struct ssj_coll ssj_coll; /* an HBM-resident collection; opaque */

/* One candidate pair: two set ids (paper Table 2, C) -- of the same
 * collection in a self-join, r of R and s of S in an R-S join. */
typedef struct {
    int32_t r;
    int32_t s;
} ssj_pair;

/* One group of grouped candidates, an entry of the paper's interleaved
 * C_O (Sec. 3.3.1): the probe set id and the exclusive end of its candidates
 * in the array of s ids (the group starts where the previous one ends; the
 * first at 0). */
typedef struct {
    int32_t probe;
    int32_t end;
} ssj_group;

typedef struct {
    int device;           /* HIP device ordinal */
    uint64_t hbm_budget;  /* device bytes for the uploaded collections plus
                             the candidate chunks of each call and their
                             worst-case output (the paper's M_c, Sec. 3.3.1):
                             collections must fit it together, and what they
                             leave bounds the chunks; 0 selects 4 GiB */
    int n_slots;          /* concurrent stream requests on the device (0 -> 4) */
    int queue_depth;      /* stream requests accepted but not yet admitted (0 -> 64) */
} ssj_opts;

/* Creates a context on opts->device (opts may be NULL for defaults).
 * Allocates small device scratch and streams (candidate buffers are sized on
 * first use, within the budget).  SSJ_EINVAL for a bad device or option,
 * SSJ_EDEVICE if HIP fails. */
int ssj_init(const ssj_opts* opts, ssj_ctx** out);

/* Waits for in-flight stream work, releases everything the context owns
 * (collections included).  NULL is accepted. */
int ssj_shutdown(ssj_ctx* ctx);

/* Message of the last failure on the calling thread (never NULL). */
const char* ssj_last_error(ssj_ctx* ctx);

/*
 * Uploads a CSR collection: set i owns tokens[offsets[i] .. offsets[i+1]).
 * offsets: host, n_sets + 1 entries, offsets[0] == 0, non-decreasing.
 * tokens:  host, n_tokens entries (== offsets[n_sets]).
 * Checks on the host: every set non-empty, tokens strictly increasing inside
 * a set, 0 <= token < 2^31, n_sets < 2^31, n_tokens < 2^32  (else
 * SSJ_EINVAL).  The library copies both arrays; the caller keeps ownership.
 * The device copy is the token array (each set padded to a multiple of 4
 * tokens) plus a 32-byte record per set.  SSJ_ENOMEM when that copy and the
 * context's resident collections together exceed hbm_budget (nothing is
 * uploaded then).  The handle is valid until ssj_free_collection /
 * ssj_shutdown.  (The paper transfers each collection once, Sec. 3.3.1.)
 */
int ssj_upload_collection(ssj_ctx* ctx, const int64_t* offsets, int64_t n_sets,
                          const int32_t* tokens, int64_t n_tokens, ssj_coll** out);

/* Frees a collection.  SSJ_EAGAIN if stream requests on it are in flight. */
int ssj_free_collection(ssj_ctx* ctx, ssj_coll* coll);

/*
 * Similarity functions (paper Table 1) and the decision each one takes, with
 * o = |r & s|:
 *   SSJ_SIM_JACCARD  o / |r | s| >= t        o * (t_num + t_den) >= t_num * (|r| + |s|)
 *   SSJ_SIM_COSINE   o / sqrt(|r||s|) >= t   o^2 * t_den^2 >= t_num^2 * |r| * |s|
 *   SSJ_SIM_DICE     2o / (|r| + |s|) >= t   2 * o * t_den >= t_num * (|r| + |s|)
 *   SSJ_SIM_OVERLAP  o >= t                  o * t_den >= t_num
 * Thresholds: 0 < t_den < 2^31 and 0 <= t_num < 2^31; t_num <= t_den except
 * for SSJ_SIM_OVERLAP, whose threshold is a count.
 */
#define SSJ_SIM_JACCARD 0
#define SSJ_SIM_COSINE 1
#define SSJ_SIM_DICE 2
#define SSJ_SIM_OVERLAP 3

/*
 * Synchronous verification of host-resident candidates.
 * cand:   host, n_cand pairs (ids must lie in [0, n_sets)).
 * t:      0 <= t_num <= t_den, 0 < t_den < 2^31.
 * out:    host, room for out_cap pairs; receives the passing candidates,
 *         with multiplicity and orientation kept, in unspecified order.
 * *out_n: number of passing candidates.  out_cap >= n_cand always suffices.
 * Requests bigger than the HBM budget are split into chunks (paper Sec.
 * 3.3.1, M_c).  Returns SSJ_ETRUNC when the result exceeds out_cap (out then
 * holds out_cap of the pairs, *out_n the full count), SSJ_EINVAL for a bad
 * threshold or an id out of range (*out_n = 0).  cand may be reused as soon
 * as the call returns.
 */
int ssj_verify(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand, int64_t n_cand,
               int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap, int64_t* out_n);

/* ssj_verify with the similarity function sim (SSJ_SIM_*, paper Table 1);
 * SSJ_EINVAL for an unknown function or a threshold outside its range. */
int ssj_verify_sim(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand, int64_t n_cand,
                   int sim, int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap,
                   int64_t* out_n);

/*
 * Device-pointer variant: no host copies, no synchronisation.  d_cand and
 * d_out are device buffers owned by the caller; d_count is a device int64.
 * Output-count mode (the paper's aggregation on top of the join, Sec. 3.3.2
 * and Sec. 5.1): d_out = NULL and out_cap = 0 produce only the count, with no
 * pair writes.
 * The work is enqueued on hip_stream (a hipStream_t; NULL = the legacy
 * default stream).  When the stream reaches the end of the call, *d_count
 * holds the number of passing candidates (which may exceed out_cap: then
 * only out_cap pairs were written), or -1 if an id was out of range.
 * Synchronous argument errors (bad threshold, negative sizes, n_cand >= 2^31)
 * return SSJ_EINVAL without enqueuing anything.  Calls that share a context
 * share its device scratch: they must be ordered on one stream (or
 * otherwise serialised) by the caller.
 */
int ssj_verify_device(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand,
                      int64_t n_cand, int64_t t_num, int64_t t_den, ssj_pair* d_out,
                      int64_t out_cap, int64_t* d_count, void* hip_stream);

/*
 * ssj_verify_device for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * verification, arguments, ordering and results, but the call allocates
 * nothing -- no hipMalloc / hipFree, no graph, no timing events.  Its
 * counters and deferral queues live in a fixed device array that the library
 * holds on each device from ssj_init until the process ends
 * (SSJ_NOALLOC_SCRATCH_BYTES: a 256-byte counter block plus 6 queue words per
 * pair for SSJ_NOALLOC_MAX_PAIRS pairs, about 24 MiB).
 * n_cand above SSJ_NOALLOC_MAX_PAIRS returns SSJ_EINVAL without enqueuing
 * anything (split larger inputs into several calls).  Every call on one
 * device, from any context, shares that array: calls that overlap on one
 * device race and must be ordered by the caller (one stream, or events).
 * Each launch leaves the counters zeroed for the next.
 */
#define SSJ_NOALLOC_MAX_PAIRS (1 << 20)
#define SSJ_NOALLOC_SCRATCH_BYTES (256 + 6 * 4 * SSJ_NOALLOC_MAX_PAIRS)
int ssj_verify_device_noalloc(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand,
                              int64_t n_cand, int64_t t_num, int64_t t_den, ssj_pair* d_out,
                              int64_t out_cap, int64_t* d_count, void* hip_stream);

/* ssj_verify_device with the similarity function sim (SSJ_SIM_*, paper
 * Table 1). */
int ssj_verify_device_sim(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand,
                          int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* d_out,
                          int64_t out_cap, int64_t* d_count, void* hip_stream);

/*
 * R-S join (Definition 1 with two collections R and S; Sec. 3.3.1 keeps
 * R_T/R_O and S_T/S_O on the device): each pair's r indexes coll_r and its s
 * indexes coll_s, both uploaded to ctx (they may be the same collection,
 * which is the self-join).  Otherwise as ssj_verify_sim / ssj_verify_device_sim:
 * an r outside coll_r or an s outside coll_s is an id error.
 */
int ssj_verify_rs(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s, const ssj_pair* cand,
                  int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* out,
                  int64_t out_cap, int64_t* out_n);
int ssj_verify_rs_device(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                         const ssj_pair* d_cand, int64_t n_cand, int sim, int64_t t_num,
                         int64_t t_den, ssj_pair* d_out, int64_t out_cap, int64_t* d_count,
                         void* hip_stream);

/*
 * Grouped candidates (the C / C_O layout of Sec. 3.3.1: every probe's
 * candidates stored once as s ids after a group entry, 4 bytes per candidate
 * instead of 8): n_groups entries {probe id in coll_r, exclusive end into
 * cand} and n_cand s ids of coll_s.  The result is the same as for the flat
 * pairs (probe, s) in the same order (pass coll_r = coll_s for a self-join).
 * ssj_verify_groups takes host buffers (groups must cover cand exactly:
 * ends not decreasing, the last one n_cand, else SSJ_EINVAL; large inputs are
 * split into batches, a group across a batch border in two);
 * ssj_verify_groups_device takes device buffers on hip_stream, with the
 * rules of ssj_verify_device: ends that decrease, are negative, exceed n_cand
 * or stop short of it (the last one must be n_cand), and candidates no group
 * covers, make *d_count -1, like an id out of range (checked on the device
 * over every group; with n_cand = 0 the ends are not checked and *d_count
 * is 0).
 * The verification kernels read the groups in place (a pre-pass kernel
 * first notes the group of every 64th candidate in the context's scratch),
 * so no expanded pairs are written.  Device calls on one context must not
 * overlap.
 */
int ssj_verify_groups(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                      const ssj_group* groups, int64_t n_groups, const int32_t* cand, int64_t n_cand,
                      int sim, int64_t t_num, int64_t t_den, ssj_pair* out, int64_t out_cap,
                      int64_t* out_n);
int ssj_verify_groups_device(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                             const ssj_group* d_groups, int64_t n_groups, const int32_t* d_cand,
                             int64_t n_cand, int sim, int64_t t_num, int64_t t_den, ssj_pair* d_out,
                             int64_t out_cap, int64_t* d_count, void* hip_stream);

/* One request of a batched grouped launch: device buffers owned by the
 * caller, with the meaning of the ssj_verify_groups_device arguments of the
 * same names (sim = 0 is SSJ_SIM_JACCARD). */
typedef struct {
    const ssj_group* d_groups;
    int64_t n_groups;
    const int32_t* d_cand;
    int64_t n_cand;
    int64_t t_num;
    int64_t t_den;
    ssj_pair* d_out;
    int64_t out_cap;
    int64_t* d_count;
    int32_t sim;
} ssj_group_request;

/*
 * Batched grouped verification (Sec. 3.3.1 C / C_O per request): up to
 * SSJ_MAX_BATCH requests over one pair of collections, verified together by
 * one launch on hip_stream (as ssj_verify_batch_device) after one pre-pass
 * kernel over the groups of all requests.  Each d_count receives its
 * request's count, or -1 when that request's groups are malformed (the
 * rules of ssj_verify_groups_device) or an id is out of range; the other
 * requests are unaffected.  The candidates of all requests together must
 * stay below 2^31.  Device calls on one context must not overlap.
 */
int ssj_verify_groups_batch_device(ssj_ctx* ctx, const ssj_coll* coll_r, const ssj_coll* coll_s,
                                   const ssj_group_request* reqs, int n_reqs, void* hip_stream);

/*
 * The whole self-join on the GPU: candidate generation by the prefix filter
 * with the length filter (Sec. 2.2 "Filters"; Sec. 3.1 AllPairs) and, with
 * positional != 0, PPJoin's positional filter -- the filtering phase the
 * paper leaves on the CPU and names as future work for the GPU -- followed by
 * the verification of ssj_verify_device (Jaccard t = t_num / t_den, which
 * must be above 0).  Each similar pair {x, y} (x != y) is found once, as
 * (r, s) with r the larger set id.  The candidates are the same set as those
 * of the CPU prefix filter at the same threshold (with the positional filter:
 * of the CPU PPJoin filter), produced in probe order.
 * ssj_candidates_device writes the candidates themselves (*d_count: their
 * number, possibly above out_cap; then out_cap of them are written);
 * ssj_join_device verifies them into d_out / d_count like
 * ssj_verify_device; ssj_join does the same with host output buffers.  All
 * three synchronise the stream three times to size their buffers (the
 * prefix index, the probe work items and the candidate count) and share the
 * context's device scratch.
 */
int ssj_candidates_device(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den,
                          int positional, ssj_pair* d_out, int64_t out_cap, int64_t* d_count,
                          void* hip_stream);
int ssj_join_device(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den, int positional,
                    ssj_pair* d_out, int64_t out_cap, int64_t* d_count, void* hip_stream);
int ssj_join(ssj_ctx* ctx, const ssj_coll* coll, int64_t t_num, int64_t t_den, int positional,
             ssj_pair* out, int64_t out_cap, int64_t* out_n);

/*
 * Streaming (continuous batching) -- the paper's host/device pipeline
 * (Sec. 3.2, threads H0/H1/H2; Sec. 4.1.2) as a request loop.
 * submit copies cand into library-owned pinned staging and returns a ticket
 * at once; an admission thread starts requests as slots and HBM budget free
 * up, several at a time on separate streams.  Thread-safe.
 * nonblocking != 0: SSJ_EAGAIN when the queue is full; otherwise the call
 * waits for room.  Same argument rules as ssj_verify.
 */
int ssj_stream_submit(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand, int64_t n_cand,
                      int64_t t_num, int64_t t_den, int nonblocking, uint64_t* ticket);

/* ssj_stream_submit with the similarity function sim (SSJ_SIM_*, paper
 * Table 1). */
int ssj_stream_submit_sim(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* cand,
                          int64_t n_cand, int sim, int64_t t_num, int64_t t_den, int nonblocking,
                          uint64_t* ticket);

/*
 * Collects a request.  wait != 0 blocks until it is done.  SSJ_PENDING if
 * not done (and wait == 0).  On SSJ_OK the passing pairs are copied to out
 * (host, out_cap pairs), *out_n is set and the ticket is retired.  On
 * SSJ_ETRUNC *out_n holds the size needed and the ticket stays valid for a
 * retry.  SSJ_EINVAL if the request had an id out of range (ticket
 * retired), SSJ_ENOTFOUND for an unknown or retired ticket.
 */
int ssj_stream_poll(ssj_ctx* ctx, uint64_t ticket, int wait, ssj_pair* out, int64_t out_cap,
                    int64_t* out_n);

/* Timing of a finished stream request, in nanoseconds of CLOCK_MONOTONIC:
 * submit (entry of ssj_stream_submit), admission (its first copy to the
 * device was enqueued), completion (its results were on the host).  wait != 0
 * blocks until the request is done; otherwise SSJ_PENDING while it runs.
 * Does not retire the ticket.  SSJ_ENOTFOUND for an unknown ticket. */
int ssj_stream_times(ssj_ctx* ctx, uint64_t ticket, int wait, uint64_t* t_submit,
                     uint64_t* t_admit, uint64_t* t_done);

/* Holds (pause != 0) or resumes (pause == 0) admission of stream requests:
 * while held, requests already on the device finish and submits still queue
 * up to queue_depth (then block, or SSJ_EAGAIN when non-blocking), but no
 * queued request is admitted.  For draining a device (and for tests of the
 * queue limits).  ssj_shutdown resumes admission first.  SSJ_EINVAL for a
 * context without a stream engine. */
int ssj_stream_pause(ssj_ctx* ctx, int pause);

/*
 * Statistics of the streaming engine since it started (or the last reset):
 * how often slots regrew their device buffers (stream-ordered reallocations
 * on the slot's idle stream) and their pinned result buffers, the host time
 * spent doing so, and the longest pass of the engine loop over its slots
 * (host time, with the engine lock held: a long pass delays every request's
 * admission and completion).  reset != 0 zeroes them after reading.
 * SSJ_EINVAL without a running engine.
 */
typedef struct {
    uint64_t slot_grows;
    double slot_grow_ms;
    uint64_t result_grows;
    double result_grow_ms;
    double longest_pass_ms;
} ssj_stream_stats_t;
int ssj_stream_stats(ssj_ctx* ctx, ssj_stream_stats_t* out, int reset);

/*
 * Execution plan.  Verification runs as one or two kernels per launch:
 *  1. an in-order kernel in which every wavefront walks chunks of 64
 *     consecutive pairs and verifies each pair with inline_lanes lanes (1 =
 *     one thread per pair, an early-exit merge that starts from the six
 *     tokens kept in each set's record; 4..64 = a group of lanes of one
 *     wavefront per pair, intersecting tile by tile).  With one thread per
 *     pair and hard_lanes > 0, a merge that outruns the six record tokens is
 *     handed, with its state, to groups of hard_lanes lanes of the same
 *     wavefront (0: the thread continues on the token array);
 *  2. pairs whose length class (by |r| + |s|, inclusive upper bounds
 *     SSJ_CLASS_BOUNDS) is defer_from or higher are not verified by (1) but
 *     queued per class; a persistent kernel then drains each class with
 *     lanes[class] lanes per pair (256 = one workgroup per pair, handed out
 *     by work stealing).  defer_from = SSJ_N_CLASSES defers nothing and runs
 *     the in-order kernel alone.
 *  3. with one thread per pair and no hard lanes, spill_iters > 0 bounds the
 *     merge of each pair in (1) to that many steps over 4-token windows: a
 *     pair still undecided then is queued and finished by the kernel of (2),
 *     with spill_lanes lanes per pair, from the merge state where it stopped
 *     (from its start in the calls of the stream engine and in
 *     ssj_verify_device_noalloc, which keep no per-pair state).  This keeps
 *     a few long merges from holding up their wavefronts.  0: no bound.
 *  4. staged != 0 (with one thread per pair and no hard lanes) stages the
 *     4-token windows of the thread-per-pair merges of (1) in a ring of LDS
 *     slots per lane, so that each window is requested two merge steps
 *     before it is needed instead of one (for long sets, whose merges wait
 *     on their window loads); spill_iters counts window steps as in (3).
 *     Grouped launches (ssj_verify_groups*) ignore it: their merges take the
 *     plain windows of (1), which run faster there.
 * use_graph != 0 replays the launch through a captured hipGraph whose kernel
 * parameters are updated per call.  wg_per_cu sizes the in-order kernel's
 * grid (its wavefronts split the chunks evenly; more workgroups than fit at
 * once start as earlier ones finish).
 */
#define SSJ_N_CLASSES 5
#define SSJ_CLASS_BOUNDS {32, 128, 512, 2048, 0x7fffffff}
#define SSJ_MAX_BATCH 16

typedef struct {
    int inline_lanes;            /* 1, 4, 8, 16, 32 or 64 */
    int hard_lanes;              /* 0, 8 or 16 with inline_lanes == 1, else 0 */
    int defer_from;              /* 0 .. SSJ_N_CLASSES */
    int lanes[SSJ_N_CLASSES];    /* per deferred class: 1, 4, 8, 16, 32, 64 or 256 */
    int use_graph;
    int spill_iters;             /* 0 .. 2^20; > 0 only with inline_lanes 1, hard_lanes 0 */
    int spill_lanes;             /* lanes per spilled pair: 1, 4, 8, 16, 32, 64 or 256 */
    int wg_per_cu;               /* in-order kernel workgroups per compute unit, 0 .. 64
                                    (0: as many as the device holds at once) */
    int staged;                  /* 0 or 1 (1 only with inline_lanes 1, hard_lanes 0) */
} ssj_plan;

/* Reads / replaces the context's plan.  SSJ_EINVAL for an unsupported
 * value.  Not thread-safe against in-flight calls on the same context. */
int ssj_get_plan(ssj_ctx* ctx, ssj_plan* plan);
int ssj_set_plan(ssj_ctx* ctx, const ssj_plan* plan);

/* One request of a batched launch: device buffers owned by the caller, with
 * the meaning of the ssj_verify_device_sim arguments of the same names
 * (sim = 0 is SSJ_SIM_JACCARD, so a zero-filled field keeps Jaccard). */
typedef struct {
    const ssj_pair* d_cand;
    int64_t n_cand;
    int64_t t_num;
    int64_t t_den;
    ssj_pair* d_out;
    int64_t out_cap;
    int64_t* d_count;
    int32_t sim;
} ssj_request;

/*
 * Batched verification: up to SSJ_MAX_BATCH requests (each with its own
 * candidates, threshold and output) verified by one launch on hip_stream.
 * Each d_count receives its request's result count (or -1 on an id out of
 * range).  The pairs of all requests together must stay below 2^31.  Same
 * ordering rule as ssj_verify_device.  SSJ_EINVAL for bad arguments.
 */
int ssj_verify_batch_device(ssj_ctx* ctx, const ssj_coll* coll, const ssj_request* reqs,
                            int n_reqs, void* hip_stream);

/*
 * Autotuner: times candidate plans on the given device candidates (which
 * should be representative of the workload; a few million pairs suffice) and
 * returns the fastest in *best (its kernel time per launch in *best_ms).
 * apply != 0 also makes it the context's plan.  The search times every
 * in-order mapping with every deferral point (deferred classes starting from
 * mappings suited to their lengths), then step budgets (spill_iters) on the
 * best thread-per-pair plan, then refines the mapping of each deferred class
 * of the best plan, one class at a time, and last the in-order grid size.
 * Synchronous.  With a tuning cache (ssj_set_tune_cache) it first looks the
 * workload up there and, on a hit, returns the stored plan and time without
 * measuring anything (SSJ_CACHED instead of SSJ_OK); a tuned result is
 * appended to the cache.
 */
int ssj_autotune(ssj_ctx* ctx, const ssj_coll* coll, const ssj_pair* d_cand, int64_t n_cand,
                 int64_t t_num, int64_t t_den, int apply, ssj_plan* best, double* best_ms);

/*
 * Tuning cache of ssj_autotune: a text file of one JSON object per line,
 * {"key": ..., "kernel_ms": ..., "plan": [inline_lanes, hard_lanes,
 * defer_from, lanes[0..4], use_graph, spill_iters, spill_lanes, wg_per_cu,
 * staged]}, keyed by the device (architecture and compute units) and the
 * workload (the collection's set count, token count and longest set, the
 * candidate count and the threshold in lowest terms).  The last entry of a
 * key wins; lines that do not parse, and plans the library no longer
 * supports, are ignored.  path NULL or "" turns the cache off (the default).
 * The file is read and appended to by ssj_autotune only, under the
 * context's lock; appends are single writes, so several processes may share
 * one file.
 */
int ssj_set_tune_cache(ssj_ctx* ctx, const char* path);

/*
 * Kernel timing, for measurement.  With period > 0, every period-th launch
 * that the library enqueues from ssj_verify, ssj_verify_device and
 * ssj_verify_batch_device has its verification kernels bracketed by HIP
 * events recorded on the launch stream (period = 1: every launch; event
 * records slow a launch down slightly, so sampling keeps a timed run close
 * to an untimed one).  period = 0 turns timing off.
 * ssj_timing_read waits for the recorded events and returns the summed
 * elapsed milliseconds of the in-order kernels and of the deferred-class
 * kernels (0 for launches that defer nothing), and the number of timed
 * launches; reset != 0 clears the sums.  Do not enable it while the calls
 * are being captured into a graph.
 */
int ssj_timing_enable(ssj_ctx* ctx, int period);
int ssj_timing_read(ssj_ctx* ctx, int reset, double* inorder_ms, double* deferred_ms,
                    int64_t* launches);

/* Collection facts: number of sets, tokens, and the largest set size. */
int ssj_collection_info(const ssj_coll* coll, int64_t* n_sets, int64_t* n_tokens,
                        int64_t* max_len);

#ifdef __cplusplus
}
#endif

#endif /* SSJ_H */
