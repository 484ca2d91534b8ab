// Verification kernels for gfx950 (CDNA4, wave64).
//
// A candidate pair (r, s) is similar iff its overlap o = |r & s| reaches the
// required overlap alpha of its similarity function (paper Sec. 3, Definition
// 1; the equivalent overlaps of Table 1 in integers): for Jaccard
//     alpha = ceil(t_num * (|r| + |s|) / (t_num + t_den)),
// for Dice ceil(t_num (|r| + |s|) / (2 t_den)), for Cosine the least o with
// o^2 t_den^2 >= t_num^2 |r| |s|, for Overlap ceil(t_num / t_den).  The r side
// of a pair reads one collection, the s side another in an R-S join (the same
// one in a self-join).
// The overlap is found by walking the two sorted token lists and stopping as
// soon as o >= alpha (accept) or o + min(tokens left in r, tokens left in s)
// < alpha (reject: alpha is out of reach) -- the early-terminating merge of
// paper Sec. 3.1.  Any sound stopping rule yields the same decisions.
//
// Mappings of pairs onto lanes (the paper's alternatives A/B/C of Sec. 3.3.2
// give a probe set to a thread or a block; here the unit is one pair):
//   * one thread per pair: the merge of the first six tokens of both sets,
//     kept in their 32-byte set records, in straight-line code, then, for a
//     pair still undecided, a merge over 16-byte windows of the token arrays
//     (every set starts on a 16-byte boundary) with the next window in
//     flight; optionally cut off after a budget of window steps, the pair
//     then being queued for the second kernel;
//   * a group of G lanes (G = 4..64) of one wavefront per pair: tile merge;
//   * one 256-thread workgroup per pair: the same tile merge over LDS.
// The tile merge advances in rounds.  A round loads the next G tokens of r
// (one per lane) and of s, counts the r tokens found in the s tile by a
// binary search over the tile (cross-lane permutes or LDS), and then
// consumes every token that can have no partner beyond the two tiles: if
// max(r tile) < max(s tile) the whole r tile plus the s tokens <= max(r tile)
// are consumed (and symmetrically; both tiles when the maxima are equal).
// Every equal pair of tokens lies in the consumed part of both sides in the
// round that finds it and in no later round, so each match is counted
// exactly once; the stopping rule is checked before every round.
//
// Scheduling.  One launch carries up to kMaxReq requests (candidate arrays
// with their own threshold and output).  In the in-order kernel every
// wavefront walks chunks of kWave consecutive pairs of one request (a static
// grid-stride split: with early termination the cost of a pair depends on its
// first few tokens, not on its length, so in-order chunks are balanced), with
// the loads of the next chunks in flight.  Optionally, pairs whose length
// class |r| + |s| is at or above defer_from are not verified there but queued
// per class (collected in LDS, one global atomic per flush); a second,
// persistent kernel drains those queues with the class's own mapping --
// workgroup-per-pair classes by work stealing, the others by a static split.
// Passing pairs are compacted in LDS (a ballot of the pass flags and each
// lane's rank among the passing lanes) and moved to the request's output
// with one global atomic per flush.  The in-order kernel keeps all of this
// per wavefront, so it has no workgroup barrier, and each wavefront lowers
// its priority as it works through its share, so that the youngest
// wavefronts of a SIMD do not finish long after the rest.
#include <algorithm>

#include "ssj_device.h"

namespace ssj {
namespace {

// Required overlap of a pair with sizes na, nb under the request's rule
// (paper Table 1, in integers).
__device__ __forceinline__ uint32_t cosine_overlap(uint32_t na, uint32_t nb, unsigned long long tn,
                                                   unsigned long long td) {
    // least o with (o td)^2 >= tn^2 na nb; both sides stay below 2^124.  A
    // double estimate lands within one of it and exact steps finish the job.
    const unsigned __int128 x = (unsigned __int128)(tn * tn) * ((unsigned long long)na * nb);
    unsigned long long o = (unsigned long long)ceil((double)tn * sqrt((double)na * (double)nb) / (double)td);
    auto sq = [&](unsigned long long v) { return (unsigned __int128)(v * td) * (v * td); };
    while (o > 0 && sq(o - 1) >= x) --o;
    while (sq(o) < x) ++o;
    return (uint32_t)o;
}

// C: whether the instance handles the Cosine rule (its 128-bit arithmetic
// costs registers in every kernel that contains it, so only launches with a
// Cosine request use such an instance).
template <bool C>
__device__ __forceinline__ uint32_t required_overlap(uint32_t na, uint32_t nb, const Request& R) {
    if constexpr (C) {
        if (R.rule == kCosine) return cosine_overlap(na, nb, R.num, R.den);
    }
    if (R.rule == kConstant) return (uint32_t)R.num;
    const unsigned long long L = (unsigned long long)na + nb;
    const unsigned long long x = R.num * L + R.den - 1ull;
    if ((x >> 32) == 0ull) {
        // ceil(num L / den) = floor(x / den) by a multiply with the request's
        // precomputed magic number (the round-up method for unsigned division
        // by an invariant integer of Granlund and Montgomery, PLDI 1994)
        const uint32_t n = (uint32_t)x;
        const uint32_t t = __umulhi(R.dmagic, n);
        return (t + ((n - t) >> (R.dshift & 0xffu))) >> (R.dshift >> 8);
    }
    return (uint32_t)(x / R.den);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// Value of v held by lane src of the same wavefront.
__device__ __forceinline__ int bperm(int v, int src) {
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

// Orders one wavefront's LDS accesses: writes by some lanes before reads by
// others (the LDS serves a wavefront's operations in issue order; the fences
// keep the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of set bits of m below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Set record: {start, len, first kHeadTokens tokens} in two 16-byte words
// (slots past the end of a shorter set hold -1).
__device__ __forceinline__ uint2 set_desc(const LaunchArgs& a, int id) {
    const uint4 v = a.heads[2 * id];
    return make_uint2(v.x, v.y);
}

// The same for a set of the s-side collection.
__device__ __forceinline__ uint2 set_desc_s(const LaunchArgs& a, int id) {
    const uint4 v = a.heads_s[2 * id];
    return make_uint2(v.x, v.y);
}

// Candidate pair k of a request.
__device__ __forceinline__ int2 load_pair(const int2* __restrict__ cand, uint32_t k) {
    return cand[k];
}

__device__ __forceinline__ uint32_t load_relaxed(const unsigned int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread: sequential early-terminating merge.
__device__ __forceinline__ bool merge_thread(const int32_t* __restrict__ A, uint32_t na,
                                             const int32_t* __restrict__ B, uint32_t nb,
                                             uint32_t alpha) {
    uint32_t i = 0, j = 0, o = 0;
    for (;;) {
        if (o >= alpha) return true;
        const uint32_t rem = min(na - i, nb - j);
        if (o + rem < alpha) return false;
        const int32_t x = A[i], y = B[j];
        i += (x <= y);
        j += (y <= x);
        o += (x == y);
    }
}

// One round of the tile merge of G lanes of one wavefront (lanes gbase ..
// gbase+G-1, g = lane - gbase) at merge position (i, j): lane g holds a = A[i+g]
// if g < ka and b = B[j+g] if g < kb.  Each lane finds its a-token in the
// s tile by binary search over the lanes; the side whose tile ends lower is
// consumed whole, the other up to that end, so an equal pair on the seam is
// counted exactly once.  Control flow is uniform inside the group, so the
// cross-lane permutes only read lanes that are active.
template <int G>
__device__ __forceinline__ void group_round(int32_t a, int32_t b, int ka, int kb, int g, int gbase,
                                            uint32_t& i, uint32_t& j, uint32_t& o) {
    const unsigned long long gmask =
        (G == kWave) ? ~0ull : (((1ull << (G % kWave)) - 1ull) << gbase);
    const bool va = g < ka, vb = g < kb;
    const int32_t amax = bperm(a, gbase + ka - 1);
    const int32_t bmax = bperm(b, gbase + kb - 1);
    // pos = number of s-tile tokens below a (capped at G-1)
    int pos = 0;
#pragma unroll
    for (int step = G / 2; step >= 1; step >>= 1) {
        const int k = pos + step - 1;
        const int32_t v = bperm(b, gbase + k);
        if (k < kb && v < a) pos += step;
    }
    const int32_t at = bperm(b, gbase + pos);
    const bool hit = va && pos < kb && at == a;
    const uint32_t nh = (uint32_t)__popcll(ballot(hit) & gmask);
    const uint32_t na_le = (uint32_t)__popcll(ballot(va && a <= bmax) & gmask);
    const uint32_t nb_le = (uint32_t)__popcll(ballot(vb && b <= amax) & gmask);
    // value selects (branches that update i or j by reference end up as a
    // select of addresses, which puts i and j in scratch memory)
    const bool a_low = amax < bmax, b_low = bmax < amax;
    i += b_low ? na_le : (uint32_t)ka;
    j += a_low ? nb_le : (uint32_t)kb;
    o += nh;
}

// Tile merge of G lanes from merge state (i, j, o), loading each tile.
template <int G>
__device__ __forceinline__ bool merge_group(const int32_t* __restrict__ A, uint32_t na,
                                            const int32_t* __restrict__ B, uint32_t nb,
                                            uint32_t alpha, int g, int gbase, uint32_t i = 0,
                                            uint32_t j = 0, uint32_t o = 0) {
    for (;;) {
        if (o >= alpha) return true;
        const uint32_t ra = na - i, rb = nb - j;
        if (o + min(ra, rb) < alpha) return false;
        const int ka = (int)min(ra, (uint32_t)G), kb = (int)min(rb, (uint32_t)G);
        const int32_t a = g < ka ? A[i + g] : 0;
        const int32_t b = g < kb ? B[j + g] : 0;
        group_round<G>(a, b, ka, kb, g, gbase, i, j, o);
    }
}

// The same merge from the start, with the first tiles already loaded by the
// caller: a0 = A[min(g, na-1)], b0 = B[min(g, nb-1)] (a software pipeline
// issues them one pair ahead, so a pair decided within its first tiles waits
// for no load).
template <int G>
__device__ __forceinline__ bool merge_group_first(const int32_t* __restrict__ A, uint32_t na,
                                                  const int32_t* __restrict__ B, uint32_t nb,
                                                  uint32_t alpha, int g, int gbase, int32_t a0,
                                                  int32_t b0) {
    if (alpha == 0u) return true;
    if (min(na, nb) < alpha) return false;
    const int ka = (int)min(na, (uint32_t)G), kb = (int)min(nb, (uint32_t)G);
    uint32_t i = 0, j = 0, o = 0;
    group_round<G>(g < ka ? a0 : 0, g < kb ? b0 : 0, ka, kb, g, gbase, i, j, o);
    return merge_group<G>(A, na, B, nb, alpha, g, gbase, i, j, o);
}

// Token min(g, n-1) of a set with descriptor d = (start, n), n >= 1: the
// lane's token of the set's first tile (clamped, so the load is unconditional).
__device__ __forceinline__ int32_t first_tile_token(const int32_t* __restrict__ tok, uint2 d, int g) {
    return tok[d.x + min((uint32_t)g, d.y - 1u)];
}

// Whole workgroup: the tile merge with kBlock-token tiles, the s tile in LDS.
// Must be called by all threads of the workgroup with the same arguments.
__device__ bool merge_block(const int32_t* __restrict__ A, uint32_t na,
                            const int32_t* __restrict__ B, uint32_t nb, uint32_t alpha,
                            int32_t* sb, uint32_t* red) {
    const int t = (int)threadIdx.x, w = t >> 6, lane = lane_id();
    uint32_t i = 0, j = 0, o = 0;
    for (;;) {
        if (o >= alpha) return true;
        const uint32_t ra = na - i, rb = nb - j;
        if (o + min(ra, rb) < alpha) return false;
        const int ka = (int)min(ra, (uint32_t)kBlock), kb = (int)min(rb, (uint32_t)kBlock);
        const bool va = t < ka, vb = t < kb;
        const int32_t a = va ? A[i + t] : 0;
        const int32_t b = vb ? B[j + t] : 0;
        const int32_t amax = A[i + ka - 1];
        const int32_t bmax = B[j + kb - 1];
        sb[t] = b;
        __syncthreads();
        int pos = 0;
#pragma unroll
        for (int step = kBlock / 2; step >= 1; step >>= 1) {
            const int k = pos + step - 1;
            if (k < kb && sb[k] < a) pos += step;
        }
        const bool hit = va && pos < kb && sb[pos] == a;
        const uint32_t c0 = (uint32_t)__popcll(ballot(hit));
        const uint32_t c1 = (uint32_t)__popcll(ballot(va && a <= bmax));
        const uint32_t c2 = (uint32_t)__popcll(ballot(vb && b <= amax));
        if (lane == 0) {
            red[w * 3 + 0] = c0;
            red[w * 3 + 1] = c1;
            red[w * 3 + 2] = c2;
        }
        __syncthreads();
        uint32_t nh = 0, na_le = 0, nb_le = 0;
#pragma unroll
        for (int q = 0; q < kBlock / kWave; ++q) {
            nh += red[q * 3 + 0];
            na_le += red[q * 3 + 1];
            nb_le += red[q * 3 + 2];
        }
        __syncthreads();  // sb and red are rewritten by the next round
        i += bmax < amax ? na_le : (uint32_t)ka;
        j += amax < bmax ? nb_le : (uint32_t)kb;
        o += nh;
    }
}

__device__ __forceinline__ void append_one(int2 pr, const Request& R, unsigned long long* counter) {
    const unsigned long long k = atomicAdd(counter, 1ull);
    if (k < R.cap) R.out[k] = pr;
}

// Whether r indexes the r-side collection and s the s-side one.
__device__ __forceinline__ bool ids_ok(int2 pr, const LaunchArgs& a) {
    return (uint32_t)pr.x < a.n_sets && (uint32_t)pr.y < a.n_sets_s;
}

__device__ __forceinline__ int class_of(uint32_t L, const LaunchArgs& a) {
    int cls = kClasses - 1;
#pragma unroll
    for (int q = kClasses - 2; q >= 0; --q)
        if (L <= a.bounds[q]) cls = q;
    return cls;
}

// Request holding global pair index gi (prefix sums in pair_off).
__device__ __forceinline__ int request_of_pair(uint32_t gi, const LaunchArgs& a) {
    int r = 0;
    for (int q = 1; q < a.n_req; ++q) r += (gi >= a.pair_off[q]) ? 1 : 0;
    return r;
}

// ---------------------------------------------------------------------------
// Wavefront-private buffers of the in-order kernel.  Every wavefront works on
// its own chunks of kWave consecutive pairs and keeps its own LDS buffers
// (staged output pairs, deferred pairs, hard pairs).  Their fill counts are
// wave-uniform values held in registers, so the kernel needs no workgroup
// barrier: a wavefront slowed by a long merge holds up no other.


// Lane 0's value of v (all lanes active).
__device__ __forceinline__ unsigned long long lane0_u64(unsigned long long v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Appends the pairs of the lanes with pass set to the wavefront's staged
// output (ocnt entries so far, wave-uniform).  A request without an output
// buffer only counts.
__device__ __forceinline__ void stage_pass(bool pass, int2 pr, int2* w_out, uint32_t& ocnt,
                                           bool count_only) {
    const unsigned long long m = ballot(pass);
    if (!count_only && pass) w_out[ocnt + mbcnt(m)] = pr;
    ocnt += (uint32_t)__popcll(m);
}

// Moves the wavefront's c staged pairs of request r to the request's output
// with one global atomic.  Called by the whole wavefront.
__device__ void wave_flush_out(const LaunchArgs& a, int r, uint32_t c, const int2* w_out) {
    wave_sync();
    const int lane = lane_id();
    unsigned long long base = 0ull;
    if (lane == 0) base = atomicAdd(&a.ctr->out_count[r], (unsigned long long)c);
    base = lane0_u64(base);
    const Request& R = a.req[r];
    if (R.cap != 0) {
        for (uint32_t i = (uint32_t)lane; i < c; i += kWave) {
            const unsigned long long k = base + i;
            if (k < R.cap) R.out[k] = w_out[i];
        }
    }
    wave_sync();
}

// Entries of class q in the wavefront's deferred queues: 8 bits per class
// in one wave-uniform word (a queue never holds more than defer_cap <= 255).
__device__ __forceinline__ uint32_t dcount(unsigned long long dc, int q) {
    return (uint32_t)(dc >> (8 * q)) & 0xffu;
}

// Appends the pairs (global pair index gi) of the lanes with mine set to
// the wavefront's LDS queue q.
__device__ __forceinline__ void queue_lanes(const LaunchArgs& a, bool mine, int q, uint32_t gi,
                                            uint32_t* w_defer, unsigned long long& dc) {
    const unsigned long long m = ballot(mine);
    if (mine) w_defer[(uint32_t)(q - a.defer_from) * a.defer_cap + dcount(dc, q) + mbcnt(m)] = gi;
    dc += (unsigned long long)__popcll(m) << (8 * q);
}

// Queues deferred pairs in the wavefront's LDS queue of their class, and
// spilled merges in its spill queue (after the class queues).
__device__ __forceinline__ void defer_pass(const LaunchArgs& a, bool defer, int cls, bool spill,
                                           uint32_t gi, uint32_t* w_defer, unsigned long long& dc) {
    for (int q = a.defer_from; q < kClasses; ++q) queue_lanes(a, defer && cls == q, q, gi, w_defer, dc);
    if (spilling(a)) queue_lanes(a, spill, kSpillQ, gi, w_defer, dc);
}

// One past the last LDS queue of the in-order kernel's wavefronts.
__device__ __forceinline__ int queue_end(const LaunchArgs& a) {
    return spilling(a) ? kQueues : kClasses;
}

// Moves the wavefront's c queued pairs of class q to the global queue.
__device__ void wave_flush_deferred(const LaunchArgs& a, int q, uint32_t c, const uint32_t* w_defer) {
    wave_sync();
    const int lane = lane_id();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->tail[q], c);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
    const uint32_t* src = w_defer + (uint32_t)(q - a.defer_from) * a.defer_cap;
    uint32_t* dst = a.queues + (size_t)q * a.qcap + base;
    for (uint32_t i = (uint32_t)lane; i < c; i += kWave) dst[i] = src[i];
    wave_sync();
}

// Wavefront priority from progress: 3 before the first quarter of its
// chunks is done, down to 0 in the last quarter.  The SIMD's arbiter favours
// the oldest wavefronts among those of equal priority, so with equal shares
// of chunks the youngest ones would otherwise finish long after the rest and
// leave the end of the launch to a few wavefronts; a wavefront that is ahead
// now yields to one that is behind.  quarter[k - 1] = ceil(k share / 4) for
// k = 1, 2, 3 (share: the wavefront's chunk count), so that done chunks are
// past the k-th quarter when done >= quarter[k - 1], without a division per
// chunk.  done, quarter and level are wave-uniform.
__device__ __forceinline__ void progress_priority(uint32_t done, const uint32_t (&quarter)[3], uint32_t& level) {
    const uint32_t l = 3u - (done >= quarter[0] ? 1u : 0u) - (done >= quarter[1] ? 1u : 0u) -
                       (done >= quarter[2] ? 1u : 0u);
    if (l == level) return;
    level = l;
    switch (l) {
        case 0: __builtin_amdgcn_s_setprio(0); break;
        case 1: __builtin_amdgcn_s_setprio(1); break;
        case 2: __builtin_amdgcn_s_setprio(2); break;
        default: __builtin_amdgcn_s_setprio(3); break;
    }
}

// Request and first pair index of chunk T (prefix sums in tile_off, in
// chunks of kWave pairs).
__device__ __forceinline__ void chunk_origin(const LaunchArgs& a, uint32_t T, int* r, uint32_t* kb) {
    if (a.n_req == 1) {  // the common launch of one request: no search
        *r = 0;
        *kb = T * (uint32_t)kWave;
        return;
    }
    int q = 0;
    while (q + 1 < a.n_req && a.tile_off[q + 1] <= T) ++q;
    *r = q;
    *kb = (T - a.tile_off[q]) * (uint32_t)kWave;
}

// ---------------------------------------------------------------------------
// Candidates of a chunk of a flat or a grouped request.  Loading and finding
// the pair are separate steps, so that a pipeline can issue a chunk's loads
// one iteration before it needs its pairs.  A grouped chunk's lanes load
// their s ids and a window of 64 consecutive groups from the chunk's first
// group (chunk_g); each lane then finds its group among them.

// The loads of a lane's candidate: the pair (flat), or the s id in p.y and
// the lane's entry of the chunk's group window, groups[g0 + lane] (clamped
// to the last group), in gw (grouped).
struct CandLoad {
    int2 p;
    int2 gw;
    uint32_t g0;  // the window's first group (wave-uniform)
};

// First groups of a wavefront's upcoming chunks, one per lane: lane L holds
// chunk_g of the wavefront's chunk with ordinal base + L (its chunk
// first + (base + L) * nw, clamped to the last chunk as the pipelines clamp
// their chunks), so that a grouped chunk's first group is in a register
// before its loads are issued (one vector load per 64 chunks of a wavefront).
template <bool GR>
__device__ __forceinline__ uint32_t load_chunk_groups(const LaunchArgs& a, uint32_t first, uint32_t nw,
                                                      uint32_t n_chunks, uint32_t base, int lane) {
    if constexpr (!GR) return 0u;
    const unsigned long long c = (unsigned long long)first + (unsigned long long)(base + (uint32_t)lane) * nw;
    return a.chunk_g[c < n_chunks ? (uint32_t)c : n_chunks - 1u];
}

// Issues the loads of the lane's candidate of the chunk at candidate kb of
// request R, whose first group is g0 (chunk_g; unused for a flat request).
// chunk_g entries of a request with malformed groups may be stale (that
// request reports an error): g0 is clamped, so every load stays inside the
// request's buffers.
template <bool GR>
__device__ __forceinline__ CandLoad issue_cand(const LaunchArgs& a, const Request& R, uint32_t kb, int lane,
                                               uint32_t g0) {
    CandLoad c;
    const uint32_t k = kb + (uint32_t)lane;
    const uint32_t kc = k < R.n ? k : R.n - 1u;
    if constexpr (!GR) {
        c.p = load_pair(R.cand, kc);
        c.gw = make_int2(0, 0);
        c.g0 = 0u;
        return c;
    }
    c.g0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)min(g0, R.n_groups));
    c.p = make_int2(0, R.sids[kc]);
    c.gw = R.n_groups != 0u ? R.groups[min(c.g0 + (uint32_t)lane, R.n_groups - 1u)] : make_int2(-1, -1);
    return c;
}

// Maximum of v over lanes 0 .. lane of the wavefront (v >= 0): within each
// row of 16 lanes by shifted maxima (DPP row shifts), then across rows from
// the rows' last lanes.
__device__ __forceinline__ uint32_t wave_max_scan(uint32_t v, int lane) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    const int row = lane >> 4;
    const uint32_t below = row == 0 ? 0u : row == 1 ? r0 : row == 2 ? max(r0, r1) : max(max(r0, r1), r2);
    return max(v, below);
}

// The lane's pair from its loads (all lanes of the wavefront call it
// together: cross-lane operations); marks is the wavefront's 64-word LDS
// scratch.  The group of candidate kb + k is the first one whose end exceeds
// it, so its index in a window of ends that do not decrease is the number of
// window groups ending at or before kb + k.  Each window group marks the
// chunk position its end falls on (the largest group index + 1 per
// position, by an LDS maximum), and a running maximum over the positions
// gives every lane that number at once.  A lane past all 64 ends searches
// the next window; a candidate no group covers gets probe id -1 (an id
// error).
template <bool GR>
__device__ __forceinline__ int2 resolve_cand(const LaunchArgs& a, const Request& R, uint32_t kb, int lane,
                                             const CandLoad& c, uint32_t* marks) {
    if constexpr (!GR) return c.p;
    const uint32_t k = kb + (uint32_t)lane;
    const bool valid = k < R.n;
    uint32_t w0 = c.g0;
    int2 e = c.gw;
    int32_t probe = -1;
    bool found = false;
    while (w0 < R.n_groups) {
        const uint32_t ek = w0 + (uint32_t)lane < R.n_groups ? (uint32_t)e.y : 0xffffffffu;
        // chunk candidates before the end of the lane's window group (0 .. 64)
        const uint32_t cpos = ek <= kb ? 0u : min(ek - kb, (uint32_t)kWave);
        marks[lane] = 0u;
        wave_sync();
        if (cpos < (uint32_t)kWave) atomicMax(&marks[cpos], (uint32_t)lane + 1u);
        wave_sync();
        const uint32_t cnt = wave_max_scan(marks[lane], lane);
        wave_sync();  // the marks are cleared again by the next use
        const int32_t pp = bperm(e.x, (int)min(cnt, (uint32_t)kWave - 1u));
        if (!found && cnt < (uint32_t)kWave && w0 + cnt < R.n_groups) {
            probe = pp;
            found = true;
        }
        if (ballot(valid && !found) == 0ull) break;
        w0 += (uint32_t)kWave;
        if (w0 < R.n_groups) e = R.groups[min(w0 + (uint32_t)lane, R.n_groups - 1u)];
    }
    return make_int2(probe, c.p.y);
}

// A queued pair (global pair index gi of request r) in the deferred kernel:
// from the request's pairs, or for a grouped launch its s id and the probe id
// that the in-order kernel stored when it queued the pair.
template <bool GR>
__device__ __forceinline__ int2 queued_pair(const LaunchArgs& a, uint32_t gi, int r) {
    const Request& R = a.req[r];
    const uint32_t k = gi - a.pair_off[r];
    if constexpr (GR) return make_int2((int32_t)a.probes[gi], R.sids[k]);
    return load_pair(R.cand, k);
}

// Records the probe id of a pair that the in-order kernel queues (grouped
// launches only; the deferred kernel reads it back by global pair index).
template <bool GR>
__device__ __forceinline__ void note_queued(const LaunchArgs& a, bool queued, int2 pr, uint32_t gi) {
    if constexpr (GR) {
        if (queued) a.probes[gi] = (uint32_t)pr.x;
    }
}

// Set records of a lane's pair: four 16-byte loads (first and second word of
// both sides), issued back to back.  A pair with an invalid id reads record 0
// and is ignored later.
struct LaneRecords {
    uint4 ra0, ra1, rb0, rb1;
};

__device__ __forceinline__ void issue_records(const LaunchArgs& a, int2 pr, LaneRecords& rec) {
    const bool ok = ids_ok(pr, a);
    const int ir = ok ? pr.x : 0, is = ok ? pr.y : 0;
    rec.ra0 = a.heads[2 * ir];
    rec.ra1 = a.heads[2 * ir + 1];
    rec.rb0 = a.heads_s[2 * is];
    rec.rb1 = a.heads_s[2 * is + 1];
}

// Merge state after the first tile of one side is consumed, with the first
// H record tokens of each side as the tiles (the tile merge of merge_group,
// done by one lane in straight-line code): with m the smaller of the two
// tile ends, the merge has consumed every token <= m of both tiles, and the
// overlap so far is the number of equal tokens in the two tiles (all of them
// are <= m).  Record slots past the end of a set hold -1; tokens are >= 0, so
// unsigned comparisons with m >= 0 leave those slots out of both counts (sets
// are not empty, so m >= 0).  A larger H gives a state at least as far along
// the same merge.
template <int H>
__device__ __forceinline__ void head_tiles(uint4 a0, uint4 a1, uint4 b0, uint4 b1, uint32_t* i,
                                           uint32_t* j, uint32_t* o) {
    static_assert(H >= 1 && H <= kHeadTokens, "head tiles come from the record tokens");
    const int32_t A[kHeadTokens] = {(int32_t)a0.z, (int32_t)a0.w, (int32_t)a1.x,
                                    (int32_t)a1.y, (int32_t)a1.z, (int32_t)a1.w};
    const int32_t B[kHeadTokens] = {(int32_t)b0.z, (int32_t)b0.w, (int32_t)b1.x,
                                    (int32_t)b1.y, (int32_t)b1.z, (int32_t)b1.w};
    int32_t am = A[0], bm = B[0];
#pragma unroll
    for (int x = 1; x < H; ++x) {
        am = max(am, A[x]);
        bm = max(bm, B[x]);
    }
    const uint32_t m = (uint32_t)min(am, bm);
    uint32_t ci = 0, cj = 0, co = 0;
#pragma unroll
    for (int x = 0; x < H; ++x) {
        ci += ((uint32_t)A[x] <= m) ? 1u : 0u;
        cj += ((uint32_t)B[x] <= m) ? 1u : 0u;
        bool hit = false;
#pragma unroll
        for (int y = 0; y < H; ++y) hit |= A[x] == B[y];
        co += (hit && A[x] >= 0) ? 1u : 0u;
    }
    *i = ci;
    *j = cj;
    *o = co;
}

// One window step on the current 4-token windows a (set positions ba ..
// ba + 3 of A) and b (bb .. bb + 3 of B), with i and j tokens consumed
// (ba <= i < min(ba + 4, na), the same for j): the window with the lower
// last token is consumed whole, the other up to that token (both on equal
// ones), and o counts the matches among the unconsumed tokens.  Consumed
// tokens are exactly those up to the last consumption point, and slots past
// a set's end hold -1 (the smallest signed, the largest unsigned value), so:
// a window's largest token is the largest of its four slots; an unconsumed
// real token of A is one at a position >= i that is <= bmax as unsigned
// (larger ones cannot match and are not consumed); and such a token can only
// equal an unconsumed token of B, so its matches need no test on b's side.
__device__ __forceinline__ void step_windows(const int32_t (&a)[4], const int32_t (&b)[4], uint32_t ba,
                                             uint32_t bb, uint32_t na, uint32_t nb, uint32_t& i, uint32_t& j,
                                             uint32_t& o) {
    const int32_t amax = max(max(a[0], a[1]), max(a[2], a[3]));
    const int32_t bmax = max(max(b[0], b[1]), max(b[2], b[3]));
    uint32_t hits = 0, na_le = 0, nb_le = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool va = ba + k >= i && (uint32_t)a[k] <= (uint32_t)bmax;
        const bool vb = bb + k >= j && (uint32_t)b[k] <= (uint32_t)amax;
        bool hit = false;
#pragma unroll
        for (int t = 0; t < 4; ++t) hit |= a[k] == b[t];
        hits += (va && hit) ? 1u : 0u;
        na_le += va ? 1u : 0u;
        nb_le += vb ? 1u : 0u;
    }
    i = bmax < amax ? i + na_le : min(ba + 4u, na);
    j = amax < bmax ? j + nb_le : min(bb + 4u, nb);
    o += hits;
}

// One lane's merge continued from state (i, j, o) over 16-byte windows of
// the two token lists (A from slot sa of tok_a, B from slot sb of tok_b;
// every set starts on a 16-byte boundary of its token array): window w of a
// side holds its tokens 4w .. 4w+3.  A step merges the
// unconsumed tokens of the current windows of both sides (up to 4 x 4
// comparisons) and consumes, as in the tile merge, every token that can have
// no partner beyond the two windows: all of the window with the lower end,
// and the tokens of the other window up to that end (both windows when the
// ends are equal).  The window after the current one of each side is always
// one step in flight: a step takes it over where the current window is used
// up, and then requests the next one unconditionally (a side that did not
// advance requests the window it already holds, a cache hit; a conditional
// load ends up in a temporary register plus a copy that waits for it).  The
// scheduling barrier keeps those loads after the selects that read the
// registers they refill, for the same reason.  The pair must be undecided at (i, j, o), so
// i < na and j < nb; (i, j, o) hold the state where the merge stopped.  After
// budget steps a merge still undecided stops with *spilled set (all lanes
// enter together, so the step count is the same in every lane and the cut is
// a wave-uniform branch).
__device__ __forceinline__ bool merge_windows(const int32_t* __restrict__ tok_a, uint32_t sa,
                                              uint32_t na, const int32_t* __restrict__ tok_b,
                                              uint32_t sb, uint32_t nb, uint32_t alpha, uint32_t& i,
                                              uint32_t& j, uint32_t& o, uint32_t budget, bool* spilled) {
    const uint4* __restrict__ t4a = reinterpret_cast<const uint4*>(tok_a);
    const uint4* __restrict__ t4b = reinterpret_cast<const uint4*>(tok_b);
    const uint32_t qa = sa >> 2, qb = sb >> 2;              // first window of each set
    const uint32_t la = (na - 1u) >> 2, lb = (nb - 1u) >> 2;  // last window index
    uint32_t wa = i >> 2, wb = j >> 2;
    // the windows as separate 32-bit values (selects on whole vectors become
    // address selects into scratch memory)
    int32_t a[4], b[4], an[4], bn[4];
    auto unpack = [](uint4 v, int32_t (&d)[4]) {
        d[0] = (int32_t)v.x;
        d[1] = (int32_t)v.y;
        d[2] = (int32_t)v.z;
        d[3] = (int32_t)v.w;
    };
    unpack(t4a[qa + wa], a);
    unpack(t4b[qb + wb], b);
    unpack(t4a[qa + min(wa + 1u, la)], an);
    unpack(t4b[qb + min(wb + 1u, lb)], bn);
    for (uint32_t step = 1;; ++step) {
        const uint32_t ba = wa << 2, bb = wb << 2;
        step_windows(a, b, ba, bb, na, nb, i, j, o);
        if (o >= alpha) return true;
        if (o + min(na - i, nb - j) < alpha) return false;
        if (step >= budget) {
            *spilled = true;
            return false;
        }
        const bool adv_a = i >= ba + 4u, adv_b = j >= bb + 4u;
        wa += adv_a ? 1u : 0u;
        wb += adv_b ? 1u : 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = adv_a ? an[k] : a[k];
            b[k] = adv_b ? bn[k] : b[k];
        }
        __builtin_amdgcn_sched_barrier(0);
        unpack(t4a[qa + min(wa + 1u, la)], an);
        unpack(t4b[qb + min(wb + 1u, lb)], bn);
    }
}

// One window step of the tile merge on the current 4-token windows va (of
// the r side, tokens 4*(i/4).. of a set of na tokens) and vb (s side): the
// side whose window ends lower is consumed whole, the other up to that end
// (both on equal ends); equal tokens inside the unconsumed parts are matches.
// Same rule as the steps of merge_windows.
__device__ __forceinline__ void window_step(uint4 va, uint4 vb, uint32_t na, uint32_t nb, uint32_t& i,
                                            uint32_t& j, uint32_t& o) {
    const int32_t a[4] = {(int32_t)va.x, (int32_t)va.y, (int32_t)va.z, (int32_t)va.w};
    const int32_t b[4] = {(int32_t)vb.x, (int32_t)vb.y, (int32_t)vb.z, (int32_t)vb.w};
    step_windows(a, b, i & ~3u, j & ~3u, na, nb, i, j, o);
}

// Entries of the wavefront's window ring (merge_ring): three 16-byte slots per
// side and lane, slot s of side d of lane l at ring[(3 d + s) * kWave + l]
// (so that a wavefront's accesses to one slot are consecutive).
constexpr uint32_t kRingSlots = 6u * (uint32_t)kWave;

// The merge of merge_windows (same steps, same step budget) with the loads
// two steps ahead instead of one.  Each side's windows pass through a ring of
// three LDS slots of the lane (window w in slot w % 3).  After every step the
// lane requests the window two past its new current one of each side into
// one of two register sets, which is written to the ring two steps later; a
// step reads its two windows from the ring.  The current window of a side
// moves by at most one per step, so every window a step can need has been
// written, and no written window is still needed when its slot is reused; a
// load has two steps to arrive before anything waits for it.  Windows past a
// set's last one are loaded clamped (and never read).
__device__ __forceinline__ bool merge_ring(const int32_t* __restrict__ tok_a, uint32_t sa, uint32_t na,
                                           const int32_t* __restrict__ tok_b, uint32_t sb, uint32_t nb,
                                           uint32_t alpha, uint32_t& i, uint32_t& j, uint32_t& o, uint32_t budget,
                                           bool* spilled, uint4* ring, int lane) {
    const uint4* __restrict__ t4a = reinterpret_cast<const uint4*>(tok_a);
    const uint4* __restrict__ t4b = reinterpret_cast<const uint4*>(tok_b);
    const uint32_t qa = sa >> 2, qb = sb >> 2;              // first window of each set
    const uint32_t la = (na - 1u) >> 2, lb = (nb - 1u) >> 2;  // last window index
    uint4* ra = ring + lane;
    uint4* rb = ring + 3 * kWave + lane;
    auto slot = [](uint32_t w) { return (w % 3u) * (uint32_t)kWave; };
    uint32_t wa = i >> 2, wb = j >> 2;
    ra[slot(wa)] = t4a[qa + wa];
    ra[slot(wa + 1u)] = t4a[qa + min(wa + 1u, la)];
    rb[slot(wb)] = t4b[qb + wb];
    rb[slot(wb + 1u)] = t4b[qb + min(wb + 1u, lb)];
    // set x: the windows two past the first step's (written before step 3)
    uint32_t xwa = wa + 2u, xwb = wb + 2u;
    uint4 xa = t4a[qa + min(xwa, la)], xb = t4b[qb + min(xwb, lb)];
    uint32_t ywa, ywb;
    uint4 ya, yb;
    uint32_t step = 0;
    // one step on the ring: 0 undecided, 1 similar, 2 not similar, 3 cut off
    auto merge_step = [&]() -> int {
        ++step;
        wave_sync();
        const uint4 va = ra[slot(i >> 2)], vb = rb[slot(j >> 2)];
        window_step(va, vb, na, nb, i, j, o);
        if (o >= alpha) return 1;
        if (o + min(na - i, nb - j) < alpha) return 2;
        if (step >= budget) return 3;
        return 0;
    };
    auto finish = [&](int st) {
        if (st == 3) *spilled = true;
        return st == 1;
    };
    int st = merge_step();
    if (st != 0) return finish(st);
    ywa = (i >> 2) + 2u;
    ywb = (j >> 2) + 2u;
    ya = t4a[qa + min(ywa, la)];
    yb = t4b[qb + min(ywb, lb)];
    st = merge_step();
    if (st != 0) return finish(st);
    for (;;) {
        ra[slot(xwa)] = xa;
        rb[slot(xwb)] = xb;
        xwa = (i >> 2) + 2u;
        xwb = (j >> 2) + 2u;
        xa = t4a[qa + min(xwa, la)];
        xb = t4b[qb + min(xwb, lb)];
        st = merge_step();
        if (st != 0) return finish(st);
        ra[slot(ywa)] = ya;
        rb[slot(ywb)] = yb;
        ywa = (i >> 2) + 2u;
        ywb = (j >> 2) + 2u;
        ya = t4a[qa + min(ywa, la)];
        yb = t4b[qb + min(ywb, lb)];
        st = merge_step();
        if (st != 0) return finish(st);
    }
}

// Thread-per-pair verification of the lane's pair (chunk index kb + lane)
// from its records: first the head tiles (head_tiles), which decide most
// pairs (with try4, four tokens per side first: see the caller); a pair
// still undecided continues from that merge state.  F == 0: it
// continues in the same lane over 16-byte windows of the token array
// (merge_windows, or with S merge_ring, its loads two steps ahead through
// the wavefront's window ring).  F > 0: it is appended, with
// its merge state, to the wavefront's list of hard pairs (hcnt entries), which
// groups of F lanes finish (finish_hard), so that no lane walks the token
// array alone while the rest of its wavefront waits.
template <int F, bool C, bool S, bool GR>
__device__ __forceinline__ void chunk_thread_pairs(const LaunchArgs& a, const Request& R, int r,
                                                   uint32_t kb, int2 pr, const LaneRecords& rec,
                                                   bool deferring, uint32_t* w_defer,
                                                   unsigned long long& dc, int2* w_out, uint32_t& ocnt,
                                                   int2* w_hpr, uint32_t* w_hst, uint32_t& hcnt, uint4* ring,
                                                   bool try4, bool& need6) {
    const int lane = lane_id();
    const uint32_t k = kb + (uint32_t)lane;
    const bool valid = k < R.n;
    const bool ok = valid && ids_ok(pr, a);
    const uint32_t na = rec.ra0.y, nb = rec.rb0.y;
    const uint32_t L = na + nb;
    const int cls = deferring ? class_of(L, a) : 0;
    const bool defer = ok && deferring && cls >= a.defer_from;
    const bool run = ok && !defer;
    const uint32_t alpha = run ? required_overlap<C>(na, nb, R) : 0u;
    uint32_t i = 0, j = 0, o = 0;
    bool pass = false, act = false;
    auto decide = [&]() {
        pass = run && o >= alpha;
        act = run && !pass && o + min(na - i, nb - j) >= alpha;
    };
    // with try4 (wave-uniform) the head step first takes four record tokens
    // per side, and the six only when that left some lane of the chunk
    // undecided (need6); the six-token state supersedes the four-token one
    bool full = true;
    if (try4) {
        head_tiles<4>(rec.ra0, rec.ra1, rec.rb0, rec.rb1, &i, &j, &o);
        decide();
        full = ballot(act) != 0ull;
        need6 = full;
    }
    if (full) {
        head_tiles<kHeadTokens>(rec.ra0, rec.ra1, rec.rb0, rec.rb1, &i, &j, &o);
        decide();
    }
    bool spill = false;
    if constexpr (F == 0) {
        const uint32_t budget = deferring ? a.spill_iters : 0xffffffffu;
        if constexpr (S) {
            if (act)
                pass = merge_ring(a.tok, rec.ra0.x, na, a.tok_s, rec.rb0.x, nb, alpha, i, j, o, budget, &spill,
                                  ring, lane);
        } else {
            if (act) pass = merge_windows(a.tok, rec.ra0.x, na, a.tok_s, rec.rb0.x, nb, alpha, i, j, o, budget, &spill);
        }
    }
    // a spilled merge leaves its state (i, j, o) for the deferred kernel
    if (deferring && spill && a.spill_state != nullptr)
        a.spill_state[a.pair_off[r] + k] = make_uint4(i, j, o, 0u);
    // (after the merges: atomics count with loads, so none sits between the
    // record loads in flight and their use)
    if (ballot(valid && !ok) != 0ull && lane == 0) atomicOr(&a.ctr->err[r], 1u);
    if constexpr (F > 0) {
        const unsigned long long m = ballot(act);
        if (act) {
            const uint32_t pos = hcnt + mbcnt(m);
            w_hpr[pos] = pr;
            w_hst[pos] = i | (j << 8) | (o << 16);  // each <= kHeadTokens
        }
        hcnt += (uint32_t)__popcll(m);
    }
    stage_pass(pass, pr, w_out, ocnt, R.cap == 0);
    if (deferring) {
        defer_pass(a, defer, cls, spill, a.pair_off[r] + k, w_defer, dc);
        note_queued<GR>(a, defer || spill, pr, a.pair_off[r] + k);
    }
}

// Finishes the wavefront's h hard pairs: groups of G lanes resume their
// merges from the saved state with the tile merge.  The loop over the list
// is wave-uniform, so the staging after each step runs with all lanes.
template <int G, bool C>
__device__ __forceinline__ void finish_hard(const LaunchArgs& a, const Request& R, uint32_t h,
                                            const int2* w_hpr, const uint32_t* w_hst, int2* w_out,
                                            uint32_t& ocnt) {
    constexpr uint32_t kGroups = kWave / G;
    const int lane = lane_id();
    const int g = lane % G, gbase = (lane / G) * G;
    const uint32_t grp = (uint32_t)(lane / G);
    wave_sync();
    for (uint32_t e0 = 0; e0 < h; e0 += kGroups) {
        const uint32_t e = e0 + grp;
        bool pass = false;
        int2 pq = make_int2(0, 0);
        if (e < h) {
            pq = w_hpr[e];
            const uint32_t st = w_hst[e];
            const uint2 dr = set_desc(a, pq.x);
            const uint2 ds = set_desc_s(a, pq.y);
            const uint32_t alpha = required_overlap<C>(dr.y, ds.y, R);
            pass = merge_group<G>(a.tok + dr.x, dr.y, a.tok_s + ds.x, ds.y, alpha, g, gbase,
                                  st & 0xffu, (st >> 8) & 0xffu, st >> 16);
        }
        stage_pass(pass && g == 0, pq, w_out, ocnt, R.cap == 0);
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// In-order kernel.  Every wavefront takes chunks of kWave consecutive pairs
// of one request, grid-stride over all wavefronts of the grid.  G == 1: a
// lane per pair.  G > 1: 64/G pairs at a time, G lanes each.  D: whether
// the instance can defer length classes (an instance without that code needs
// fewer registers).  S (G == 1, F == 0): merges through the window ring
// (merge_ring).  GR: a grouped launch (every request's candidates read in
// place from its groups and s ids).
template <int G, int F, bool D, bool C, bool S, bool GR>
__global__ __launch_bounds__(kBlock) void k_verify_tiles(LaunchArgs a) {
    constexpr int GPW = kWave / G;
    constexpr uint32_t kWaves = (uint32_t)(kBlock / kWave);
    // staged output pairs per wavefront: every flush is one atomic on the
    // request's counter, and same-address atomics from all wavefronts are
    // serialised, so flushes carry at least kWStage - kWave pairs
    constexpr uint32_t kWStage = kWaveStage;
    // the wavefront index is uniform in the wavefront: taken through a scalar
    // register for the chunk walk (which then stays scalar); the LDS
    // addresses use the per-lane copy (vector registers are the cheaper ones)
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t wl = threadIdx.x >> 6;
    const int lane = lane_id();
    const int grp = lane / G, g = lane % G, gbase = grp * G;
    // dynamic LDS, per wavefront: kWStage staged output pairs, then defer_cap
    // entries per queue: the deferred classes q >= defer_from, then the spill
    // queue when merges are cut off (defer_cap >= 2 * kWave)
    extern __shared__ uint4 s_dyn[];
    const bool deferring = D && (a.defer_from < kClasses || spilling(a));
    const uint32_t wave_words =
        (kWStage * 8u +
         (deferring ? (uint32_t)wave_queues(a.defer_from, spilling(a)) * a.defer_cap * 4u : 0u)) / 16u;
    int2* w_out = reinterpret_cast<int2*>(s_dyn + wl * wave_words);
    uint32_t* w_defer = reinterpret_cast<uint32_t*>(w_out + kWStage);
    // hard pairs of the current chunk (thread-per-pair mapping with F > 0)
    __shared__ int2 s_hpr[F > 0 ? kWaves * kWave : 1];
    __shared__ uint32_t s_hst[F > 0 ? kWaves * kWave : 1];
    int2* w_hpr = s_hpr + (F > 0 ? wl * kWave : 0u);
    uint32_t* w_hst = s_hst + (F > 0 ? wl * kWave : 0u);
    // group search scratch of grouped launches (resolve_cand)
    __shared__ uint32_t s_marks[GR ? kWaves * kWave : 1];
    uint32_t* w_marks = s_marks + (GR ? wl * kWave : 0u);
    // the window rings of merge_ring
    __shared__ uint4 s_ring[S ? kWaves * kRingSlots : 1];
    uint4* w_ring = s_ring + (S ? wl * kRingSlots : 0u);
    uint32_t ocnt = 0, hcnt = 0;
    unsigned long long dc = 0ull;  // deferred queue fill counts (dcount)
    const uint32_t n_chunks = a.tile_off[a.n_req];
    const uint32_t nw = gridDim.x * kWaves;
    const uint32_t first = blockIdx.x * kWaves + (uint32_t)w;
    // G == 1: a two-stage pipeline.  While chunk T is verified, the records of
    // chunk T + nw and the pairs of chunk T + 2 nw are in flight (memory
    // operations complete in issue order, so the records of T, issued one
    // iteration earlier, are waited for without draining the newer loads).
    int2 p0 = make_int2(0, 0);
    CandLoad c1{};
    LaneRecords rec0{}, rec1{};
    int r_cur = 0, r1 = 0;
    uint32_t kb_cur = 0, kb1 = 0;
    // grouped: first groups of this wavefront's chunks with ordinals
    // vbase .. vbase + 63, one per lane
    uint32_t vbase = 0, vg = 0;
    auto group_of_ord = [&](uint32_t q) -> uint32_t {
        if constexpr (!GR) return 0u;
        if (q - vbase >= (uint32_t)kWave) {
            vbase = q;
            vg = load_chunk_groups<GR>(a, first, nw, n_chunks, vbase, lane);
        }
        return (uint32_t)__builtin_amdgcn_readlane((int)vg, (int)(q - vbase));
    };
    if (first < n_chunks) {
        chunk_origin(a, first, &r_cur, &kb_cur);
        if constexpr (G == 1) {
            // loads beyond the last chunk are clamped to it (results unused),
            // so every iteration issues the same loads in the same order
            vg = load_chunk_groups<GR>(a, first, nw, n_chunks, 0u, lane);
            p0 = resolve_cand<GR>(a, a.req[r_cur], kb_cur, lane,
                                  issue_cand<GR>(a, a.req[r_cur], kb_cur, lane, group_of_ord(0u)), w_marks);
            issue_records(a, p0, rec0);
            chunk_origin(a, min(first + nw, n_chunks - 1), &r1, &kb1);
            c1 = issue_cand<GR>(a, a.req[r1], kb1, lane, group_of_ord(1u));
        }
    }
    const uint32_t share = first < n_chunks ? (n_chunks - 1u - first) / nw + 1u : 1u;
    const uint32_t quarter[3] = {(uint32_t)__builtin_amdgcn_readfirstlane((int)((share + 3u) / 4u)),
                                 (uint32_t)__builtin_amdgcn_readfirstlane((int)((2u * share + 3u) / 4u)),
                                 (uint32_t)__builtin_amdgcn_readfirstlane((int)((3u * share + 3u) / 4u))};
    uint32_t done = 0, level = 3;
    // thread-per-pair head step: four tokens per side first while that
    // decides whole chunks often enough.  h4est tracks 256 times the share of
    // recent tries that still needed the six-token step; the four-token step
    // costs about 60% of the six-token one, so trying it first pays while
    // that share stays below about 3/8, and it is tried again on every
    // eighth chunk
    uint32_t h4est = 96u;
    __builtin_amdgcn_s_setprio(3);
    for (uint32_t T = first; T < n_chunks; T += nw) {
        progress_priority(done++, quarter, level);
        const int r = r_cur;
        const uint32_t kb = kb_cur;
        const uint32_t Tn = T + nw;
        const Request& R = a.req[r];
        if constexpr (G == 1) {
            const int2 p1 = resolve_cand<GR>(a, a.req[r1], kb1, lane, c1, w_marks);
            issue_records(a, p1, rec1);
            int r2 = 0;
            uint32_t kb2 = 0;
            chunk_origin(a, min(Tn + nw, n_chunks - 1), &r2, &kb2);
            const CandLoad c2 = issue_cand<GR>(a, a.req[r2], kb2, lane, group_of_ord(done + 1u));
            // (only in the plain thread-per-pair instances: with the deferral
            // code it spills scalar registers, with the window ring it costs
            // a wavefront per SIMD)
            const bool try4 = !D && !S && (h4est < 96u || ((done - 1u) & 7u) == 0u);
            bool need6 = false;
            chunk_thread_pairs<F, C, S, GR>(a, R, r, kb, p0, rec0, deferring, w_defer, dc, w_out, ocnt,
                                            w_hpr, w_hst, hcnt, w_ring, try4, need6);
            if (try4) h4est = h4est - (h4est >> 3) + (need6 ? 32u : 0u);
            if constexpr (F > 0) {
                if (hcnt > 0) {
                    finish_hard<F, C>(a, R, hcnt, w_hpr, w_hst, w_out, ocnt);
                    hcnt = 0;
                }
            }
            // rotate the pipeline
            p0 = p1;
            c1 = c2;
            rec0 = rec1;
            r_cur = r1;
            kb_cur = kb1;
            r1 = r2;
            kb1 = kb2;
        } else {
            if (Tn < n_chunks) chunk_origin(a, Tn, &r_cur, &kb_cur);
            // sub-rounds of 64/G pairs, software-pipelined: while sub-round s
            // is merged, the first tiles of s + 1, the set descriptors of s + 2
            // and the pair of s + 3 are in flight (clamped, unconditional loads
            // keep the issue order fixed)
            // a grouped chunk's pairs are found once, lane k holding pair
            // kb + k, and handed to the groups by permutes
            int2 cp = make_int2(0, 0);
            if constexpr (GR) cp = resolve_cand<GR>(a, R, kb, lane, issue_cand<GR>(a, R, kb, lane, a.chunk_g[T]), w_marks);
            auto pair_at = [&](int sub) -> int2 {
                const int src = min(sub, G - 1) * GPW + grp;
                if constexpr (GR) return make_int2(bperm(cp.x, src), bperm(cp.y, src));
                const uint32_t k = kb + (uint32_t)src;
                return load_pair(R.cand, k < R.n ? k : R.n - 1);
            };
            auto desc_of = [&](int2 pq, uint2* dr, uint2* ds) {
                const bool ok = ids_ok(pq, a);
                *dr = set_desc(a, ok ? pq.x : 0);
                *ds = set_desc_s(a, ok ? pq.y : 0);
            };
            int2 pq0 = pair_at(0), pq1 = pair_at(1), pq2 = pair_at(2);
            uint2 dr0, ds0, dr1, ds1;
            desc_of(pq0, &dr0, &ds0);
            desc_of(pq1, &dr1, &ds1);
            int32_t wa0 = first_tile_token(a.tok, dr0, g), wb0 = first_tile_token(a.tok_s, ds0, g);
            bool bad = false;
            for (int sub = 0; sub < G; ++sub) {
                const int2 pq3 = pair_at(sub + 3);
                uint2 dr2, ds2;
                desc_of(pq2, &dr2, &ds2);
                const int32_t wa1 = first_tile_token(a.tok, dr1, g);
                const int32_t wb1 = first_tile_token(a.tok_s, ds1, g);
                const uint32_t k = kb + (uint32_t)(sub * GPW + grp);
                bool pass = false, defer = false;
                int cls = 0;
                const int2 pq = pq0;
                if (k < R.n) {
                    if (ids_ok(pq, a)) {
                        const uint32_t L = dr0.y + ds0.y;
                        if (deferring) {
                            cls = class_of(L, a);
                            defer = cls >= a.defer_from;
                        }
                        if (!defer)
                            pass = merge_group_first<G>(a.tok + dr0.x, dr0.y, a.tok_s + ds0.x, ds0.y,
                                                        required_overlap<C>(dr0.y, ds0.y, R), g, gbase,
                                                        wa0, wb0);
                    } else {
                        bad = true;
                    }
                }
                stage_pass(pass && g == 0, pq, w_out, ocnt, R.cap == 0);
                if (deferring) {
                    defer_pass(a, defer && g == 0, cls, false, a.pair_off[r] + k, w_defer, dc);
                    note_queued<GR>(a, defer && g == 0, pq, a.pair_off[r] + k);
                }
                pq0 = pq1;
                pq1 = pq2;
                pq2 = pq3;
                dr0 = dr1;
                ds0 = ds1;
                dr1 = dr2;
                ds1 = ds2;
                wa0 = wa1;
                wb0 = wb1;
            }
            if (ballot(bad) != 0ull && lane == 0) atomicOr(&a.ctr->err[r], 1u);
        }
        // at most kWave pairs are staged per chunk: flush when fewer than that
        // fit, or when the next chunk belongs to another request
        const bool same_next = Tn < n_chunks && r_cur == r;
        if (ocnt > 0 && ((R.cap != 0 && ocnt > kWStage - kWave) || !same_next)) {
            wave_flush_out(a, r, ocnt, w_out);
            ocnt = 0;
        }
        if (deferring) {
            // the same bound holds for each queue
            for (int q = a.defer_from; q < queue_end(a); ++q) {
                const uint32_t c = dcount(dc, q);
                if (c > a.defer_cap - kWave) {
                    wave_flush_deferred(a, q, c, w_defer);
                    dc &= ~(0xffull << (8 * q));
                }
            }
        }
    }
    if (deferring) {
        for (int q = a.defer_from; q < queue_end(a); ++q) {
            if (dcount(dc, q) > 0) wave_flush_deferred(a, q, dcount(dc, q), w_defer);
        }
    }
}

// Publishes each request's count (-1 after an id error) and returns the
// counters to zero for the next launch.  One workgroup, after the verify
// kernels of the launch (the kernel boundary makes their atomics visible).
__global__ void k_finalize(LaunchArgs a) {
    const int t = (int)threadIdx.x;
    if (t < a.n_req) {
        const unsigned long long cnt = a.ctr->out_count[t];
        const unsigned err = a.ctr->err[t];
        *a.req[t].d_count = err ? -1ll : (long long)cnt;
        a.ctr->out_count[t] = 0ull;
        a.ctr->err[t] = 0u;
    }
    if (t < kQueues) {
        a.ctr->head[t] = 0u;
        a.ctr->tail[t] = 0u;
    }
}

// ---------------------------------------------------------------------------
// Deferred classes.  Workgroup-mapped classes (lanes == kBlock) are taken one
// pair per workgroup by work stealing; the others are split statically over
// all wavefronts of the grid.
template <int G, bool C, bool GR>
__device__ void drain_static(const LaunchArgs& a, int q, uint32_t cnt) {
    constexpr int GPW = kWave / G;
    const int lane = lane_id();
    const int grp = lane / G, g = lane % G, gbase = grp * G;
    const uint32_t* queue = a.queues + (size_t)q * a.qcap;
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t stride = (gridDim.x * kBlock) / kWave * GPW;
    const uint32_t t0 = wave * GPW;
    // Item s of the group is queue entry t0 + s * stride + grp.  Software
    // pipeline: while item s is merged, the first tiles of s + 1, the set
    // descriptors of s + 2, the pair of s + 3 and the queue entry of s + 4
    // are in flight (loads clamped to the last entry, so every iteration
    // issues the same loads in the same order).
    auto entry_at = [&](uint32_t s) -> uint32_t {
        const uint32_t k = t0 + s * stride + (uint32_t)grp;
        return queue[min(k, cnt - 1u)];
    };
    // spilled merges resume from the state the in-order kernel left (the
    // merge of the unconsumed suffixes against alpha - o decides the pair the
    // same way: no consumed token matches an unconsumed one)
    const bool resume = q == kSpillQ && a.spill_state != nullptr;
    auto pair_of = [&](uint32_t gi, int* r, uint4* st) -> int2 {
        *r = request_of_pair(gi, a);
        *st = resume ? a.spill_state[gi] : make_uint4(0u, 0u, 0u, 0u);
        return queued_pair<GR>(a, gi, *r);
    };
    // a set's descriptor without its first c tokens
    auto suffix = [](uint2 d, uint32_t c) { return make_uint2(d.x + c, d.y - c); };
    uint32_t e3;
    int2 p0, p1, p2;
    int r0, r1, r2;
    uint4 st0, st1, st2;
    uint2 dr0, ds0, dr1, ds1;
    int32_t wa0, wb0;
    {
        const uint32_t e0 = entry_at(0), e1 = entry_at(1), e2 = entry_at(2);
        e3 = entry_at(3);
        p0 = pair_of(e0, &r0, &st0);
        p1 = pair_of(e1, &r1, &st1);
        p2 = pair_of(e2, &r2, &st2);
        dr0 = set_desc(a, p0.x);
        ds0 = set_desc_s(a, p0.y);
        dr1 = set_desc(a, p1.x);
        ds1 = set_desc_s(a, p1.y);
        wa0 = first_tile_token(a.tok, suffix(dr0, st0.x), g);
        wb0 = first_tile_token(a.tok_s, suffix(ds0, st0.y), g);
    }
    for (uint32_t t = t0, s = 0; t < cnt; t += stride, ++s) {
        const uint32_t e4 = entry_at(s + 4);
        int r3;
        uint4 st3;
        const int2 p3 = pair_of(e3, &r3, &st3);
        const uint2 dr2 = set_desc(a, p2.x);
        const uint2 ds2 = set_desc_s(a, p2.y);
        const int32_t wa1 = first_tile_token(a.tok, suffix(dr1, st1.x), g);
        const int32_t wb1 = first_tile_token(a.tok_s, suffix(ds1, st1.y), g);
        if (t + (uint32_t)grp < cnt) {
            const Request& R = a.req[r0];
            const uint32_t alpha = required_overlap<C>(dr0.y, ds0.y, R) - st0.z;
            const uint2 ar = suffix(dr0, st0.x), as = suffix(ds0, st0.y);
            bool pass;
            if constexpr (G == 1)
                pass = merge_thread(a.tok + ar.x, ar.y, a.tok_s + as.x, as.y, alpha);
            else
                pass = merge_group_first<G>(a.tok + ar.x, ar.y, a.tok_s + as.x, as.y, alpha, g, gbase, wa0,
                                            wb0);
            if (pass && g == 0) append_one(p0, R, &a.ctr->out_count[r0]);
        }
        e3 = e4;
        p0 = p1;
        r0 = r1;
        st0 = st1;
        p1 = p2;
        r1 = r2;
        st1 = st2;
        p2 = p3;
        r2 = r3;
        st2 = st3;
        dr0 = dr1;
        ds0 = ds1;
        dr1 = dr2;
        ds1 = ds2;
        wa0 = wa1;
        wb0 = wb1;
    }
}

// Lanes per pair of queue q.
__device__ __forceinline__ int lanes_of_queue(const LaunchArgs& a, int q) {
    return q == kSpillQ ? a.spill_lanes : a.lanes[q];
}

// Queues are drained from the spill queue (the longest merges) down to the
// first deferred class.
template <bool C, bool GR>
__global__ __launch_bounds__(kBlock) void k_verify_deferred(LaunchArgs a) {
    __shared__ int32_t sb[kBlock];
    __shared__ uint32_t red[16];
    __shared__ uint32_t s_tile;
    for (int q = kQueues - 1; q >= 0; --q) {
        if (q < a.defer_from && q != kSpillQ) break;
        if (lanes_of_queue(a, q) != kBlock) continue;
        const uint32_t cnt = load_relaxed(&a.ctr->tail[q]);
        const uint32_t* queue = a.queues + (size_t)q * a.qcap;
        for (;;) {
            if (threadIdx.x == 0) {
                // a plain read first: no atomic traffic once the queue is drained
                s_tile = load_relaxed(&a.ctr->head[q]) >= cnt ? cnt : atomicAdd(&a.ctr->head[q], 1u);
            }
            __syncthreads();
            const uint32_t t = s_tile;
            __syncthreads();
            if (t >= cnt) break;
            const uint32_t gi = queue[t];
            const int r = request_of_pair(gi, a);
            const Request& R = a.req[r];
            const int2 pr = queued_pair<GR>(a, gi, r);
            const uint2 dr = set_desc(a, pr.x);
            const uint2 ds = set_desc_s(a, pr.y);
            // a spilled merge resumes from its state (as in drain_static)
            const uint4 st = q == kSpillQ && a.spill_state != nullptr ? a.spill_state[gi]
                                                                       : make_uint4(0u, 0u, 0u, 0u);
            const bool pass = merge_block(a.tok + dr.x + st.x, dr.y - st.x, a.tok_s + ds.x + st.y, ds.y - st.y,
                                          required_overlap<C>(dr.y, ds.y, R) - st.z, sb, red);
            if (threadIdx.x == 0 && pass) append_one(pr, R, &a.ctr->out_count[r]);
        }
    }
    for (int q = kQueues - 1; q >= 0; --q) {
        if (q < a.defer_from && q != kSpillQ) break;
        const uint32_t cnt = load_relaxed(&a.ctr->tail[q]);
        if (cnt == 0) continue;
        switch (lanes_of_queue(a, q)) {
            case 1: drain_static<1, C, GR>(a, q, cnt); break;
            case 4: drain_static<4, C, GR>(a, q, cnt); break;
            case 8: drain_static<8, C, GR>(a, q, cnt); break;
            case 16: drain_static<16, C, GR>(a, q, cnt); break;
            case 32: drain_static<32, C, GR>(a, q, cnt); break;
            case 64: drain_static<64, C, GR>(a, q, cnt); break;
            default: break;
        }
    }
}

// ---------------------------------------------------------------------------
// Grouped candidates (the interleaved C_O / C form of Sec. 3.3.1): group g is
// {probe id, exclusive end}, and its candidates are the s ids
// sids[end(g-1) .. end(g)) with end(-1) = 0.  The verification kernels read
// them in place (issue_cand / resolve_cand); this pre-pass gives each chunk
// of kWave candidates its first group.

__device__ __forceinline__ int32_t group_end(const int2* groups, uint32_t g) {
    return reinterpret_cast<const int32_t*>(groups)[2u * g + 1u];
}

// One thread per group of all requests of the launch (requests located by
// the prefix sums group_off): checks the group's end against its
// predecessor's and the request's size, and writes chunk_g[t] = g for every
// chunk start t * kWave inside the group's candidates.  With ends that do not
// decrease, end above n or a last end other than n, the request's error flag
// is set; only in-range entries of chunk_g are ever written.
__global__ void k_group_chunks(LaunchArgs a) {
    const uint32_t total = a.group_off[a.n_req];
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < total; x += gridDim.x * blockDim.x) {
        int r = 0;
        for (int q = 1; q < a.n_req; ++q) r += (x >= a.group_off[q]) ? 1 : 0;
        const Request& R = a.req[r];
        const uint32_t g = x - a.group_off[r];
        const int32_t e = group_end(R.groups, g);
        const int32_t pv = g > 0u ? group_end(R.groups, g - 1u) : 0;
        const bool bad = e < pv || (uint32_t)e > R.n || (g + 1u == R.n_groups && (uint32_t)e != R.n);
        if (bad) {
            atomicOr(&a.ctr->err[r], 1u);
            continue;
        }
        // 0 <= max(pv, 0) <= e <= n: every t written is below the request's chunk count
        const uint32_t lo = (uint32_t)max(pv, 0), hi = (uint32_t)e;
        for (uint32_t t = (lo + (uint32_t)kWave - 1u) / (uint32_t)kWave; t * (uint32_t)kWave < hi; ++t)
            R.chunk_g[t] = g;
    }
}

// Zeroes n 32-bit words (a fill kernel: usable where a memset node is not).
__global__ void k_clear_words(uint32_t* __restrict__ p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Set records from the set lengths (CSR offsets of the caller's layout) and
// the start of each set in the device token array (16-byte aligned).
__global__ void k_build_heads(const int64_t* __restrict__ off, const uint32_t* __restrict__ start,
                              const int32_t* __restrict__ tok, uint4* __restrict__ heads, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = start[i];
        const uint32_t len = (uint32_t)(off[i + 1] - off[i]);
        int32_t h[kHeadTokens];
#pragma unroll
        for (int k = 0; k < kHeadTokens; ++k) h[k] = ((uint32_t)k < len) ? tok[b + k] : -1;
        heads[2 * i] = make_uint4(b, len, (uint32_t)h[0], (uint32_t)h[1]);
        heads[2 * i + 1] = make_uint4((uint32_t)h[2], (uint32_t)h[3], (uint32_t)h[4], (uint32_t)h[5]);
    }
}

}  // namespace

bool lanes_supported(int lanes) {
    switch (lanes) {
        case 1: case 4: case 8: case 16: case 32: case 64: case kBlock: return true;
        default: return false;
    }
}

bool inline_supported(int lanes, int hard_lanes, bool staged) {
    return kernel_verify_tiles(lanes, hard_lanes, staged, false, false, false) != nullptr;
}

template <bool D, bool C, bool GR>
const void* verify_tiles_instance(int lanes, int hard_lanes, bool staged) {
    if (lanes == 1) {
        if constexpr (!GR) {
            if (staged) return hard_lanes == 0 ? (const void*)&k_verify_tiles<1, 0, D, C, true, GR> : nullptr;
        }
        switch (hard_lanes) {
            case 0: return (const void*)&k_verify_tiles<1, 0, D, C, false, GR>;
            case 8: return (const void*)&k_verify_tiles<1, 8, D, C, false, GR>;
            case 16: return (const void*)&k_verify_tiles<1, 16, D, C, false, GR>;
            default: return nullptr;
        }
    }
    if (hard_lanes != 0 || staged) return nullptr;
    switch (lanes) {
        case 4: return (const void*)&k_verify_tiles<4, 0, D, C, false, GR>;
        case 8: return (const void*)&k_verify_tiles<8, 0, D, C, false, GR>;
        case 16: return (const void*)&k_verify_tiles<16, 0, D, C, false, GR>;
        case 32: return (const void*)&k_verify_tiles<32, 0, D, C, false, GR>;
        case 64: return (const void*)&k_verify_tiles<64, 0, D, C, false, GR>;
        default: return nullptr;
    }
}

template <bool GR>
const void* verify_tiles_by_flags(int lanes, int hard_lanes, bool staged, bool deferring, bool cosine) {
    if (cosine)
        return deferring ? verify_tiles_instance<true, true, GR>(lanes, hard_lanes, staged)
                         : verify_tiles_instance<false, true, GR>(lanes, hard_lanes, staged);
    return deferring ? verify_tiles_instance<true, false, GR>(lanes, hard_lanes, staged)
                     : verify_tiles_instance<false, false, GR>(lanes, hard_lanes, staged);
}

// Grouped launches run the plain window merge whatever staged says: their
// instances hold about ten more registers than the flat ones, and with the
// window ring that costs a wavefront per SIMD (on the offline grouped step
// the plain instance runs 12-14% faster).
const void* kernel_verify_tiles(int lanes, int hard_lanes, bool staged, bool deferring, bool cosine, bool grouped) {
    return grouped ? verify_tiles_by_flags<true>(lanes, hard_lanes, false, deferring, cosine)
                   : verify_tiles_by_flags<false>(lanes, hard_lanes, staged, deferring, cosine);
}

const void* kernel_verify_deferred(bool cosine, bool grouped) {
    if (grouped)
        return cosine ? (const void*)&k_verify_deferred<true, true> : (const void*)&k_verify_deferred<false, true>;
    return cosine ? (const void*)&k_verify_deferred<true, false> : (const void*)&k_verify_deferred<false, false>;
}

hipError_t launch_group_chunks(const LaunchArgs& a, hipStream_t st) {
    const uint32_t total = a.group_off[a.n_req];
    if (total == 0) return hipSuccess;
    const uint32_t b = std::min<uint32_t>((total + kBlock - 1) / kBlock, 65536u);
    hipLaunchKernelGGL(k_group_chunks, dim3(b), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_build_heads(const int64_t* d_offsets, const uint32_t* d_start, const int32_t* d_tok,
                              uint4* d_heads, int64_t n_sets, hipStream_t st) {
    if (n_sets <= 0) return hipSuccess;
    int64_t blocks = (n_sets + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_build_heads, dim3((unsigned)blocks), dim3(kBlock), 0, st, d_offsets, d_start,
                       d_tok, d_heads, n_sets);
    return hipGetLastError();
}

size_t tiles_lds_bytes(const LaunchArgs& a) {
    // per wavefront: kWaveStage staged output pairs, then defer_cap entries
    // per queue (a multiple of 16 bytes)
    const size_t stage = (size_t)kWaveStage * sizeof(int2);
    const size_t defer = (size_t)wave_queues(a.defer_from, spilling(a)) * a.defer_cap * 4u;
    return (size_t)(kBlock / kWave) * (stage + defer);
}

hipError_t launch_verify_tiles(const LaunchArgs& a, int grid, hipStream_t st) {
    const void* f = kernel_verify_tiles(a.inline_lanes, a.hard_lanes, a.staged != 0,
                                        a.defer_from < kClasses || spilling(a), a.cosine != 0, a.grouped != 0);
    if (!f) return hipErrorInvalidValue;
    LaunchArgs args = a;
    void* params[] = {&args};
    return hipLaunchKernel(f, dim3((unsigned)grid), dim3(kBlock), params, tiles_lds_bytes(a), st);
}

hipError_t launch_clear_words(uint32_t* d_words, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t b = std::min<size_t>((n + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_clear_words, dim3((unsigned)b), dim3(kBlock), 0, st, d_words, (uint32_t)n);
    return hipGetLastError();
}

hipError_t launch_finalize(const LaunchArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kWave), 0, st, a);
    return hipGetLastError();
}

const void* kernel_finalize() { return (const void*)&k_finalize; }

hipError_t launch_verify_deferred(const LaunchArgs& a, int grid, hipStream_t st) {
    const void* f = kernel_verify_deferred(a.cosine != 0, a.grouped != 0);
    LaunchArgs args = a;
    void* params[] = {&args};
    return hipLaunchKernel(f, dim3((unsigned)grid), dim3(kBlock), params, 0, st);
}

}  // namespace ssj
