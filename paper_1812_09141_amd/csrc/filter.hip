// Candidate generation on the GPU: the prefix filter of a self-join, with the
// length filter and, optionally, PPJoin's positional filter (paper Sec. 2.2
// "Filters" and "Algorithm outline"; Sec. 3.1 AllPairs and PPJoin).  The
// paper keeps filtering on the CPU and names moving it to the GPU as future
// work; this is that step, built from the same definitions as the CPU
// filters of the candidate generator.
//
// For t = num / den > 0 a set x of |x| tokens has prefix length
// p(x) = |x| - ceil(t |x|) + 1.  Two sets with Jaccard similarity >= t share a
// token within their prefixes (prefix-filter lemma).  The index holds every
// prefix token as a 64-bit key (token << 32 | set id) with its position,
// sorted, so the list of a token is a contiguous range ordered by set id.
// Every prefix position (r, i) of every set r is one probe: it walks the list
// of its token up to set r (each unordered pair is found from its larger id)
// and meets each set s there at the token's position j in s.
//
//  * A pair is emitted once, at its first meeting: when the prefixes hold no
//    common token before positions i and j.
//  * The length filter drops pairs with |s| < ceil(t |r|) or
//    |r| < ceil(t |s|).
//  * With the positional filter, every meeting of the two prefixes from the
//    first one on is checked in token order: at a meeting with A earlier
//    meetings at positions (x, y) the overlap is at most
//    A + 1 + min(|r| - x - 1, |s| - y - 1), and a pair whose bound falls
//    below the overlap it needs, ceil(num (|r| + |s|) / (num + den)), is
//    dropped.  This is the candidate set of the CPU PPJoin filter.
//
// Work items: a probe position whose list holds more than kPiece sets below
// the probe is split into pieces of kPiece list entries, one thread each, so a
// long list does not hold up its wavefront; every other position is one item.
// Items are numbered in (probe position, piece) order by a scan over the
// pieces per position, and two passes over them (count, then fill at the
// exclusive prefix sum of the counts) write the candidates in probe order --
// the order of the CPU filters -- with no atomics.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "ssj_device.h"
#include "filter.h"

namespace ssj {
namespace {

struct Thr {
    unsigned long long num, den;
};

__device__ __forceinline__ uint32_t need_of(uint32_t len, Thr t) {
    return (uint32_t)((t.num * len + t.den - 1ull) / t.den);
}

__device__ __forceinline__ uint32_t prefix_of(uint32_t len, Thr t) {
    const uint32_t need = need_of(len, t);
    return need > len ? 0u : len - need + 1u;
}

__global__ void k_prefix_len(const uint4* __restrict__ heads, uint32_t n, Thr t,
                             uint32_t* __restrict__ plen) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x)
        plen[x] = prefix_of(heads[2 * x].y, t);
}

// Index entries of set x at pre[x] .. pre[x] + plen[x]: sort key (token << 32
// | x) and position; the probe arrays hold (x, position) in the same order.
__global__ void k_prefix_entries(const uint4* __restrict__ heads, const int32_t* __restrict__ tok,
                                 uint32_t n, const uint32_t* __restrict__ plen,
                                 const uint32_t* __restrict__ pre, unsigned long long* __restrict__ keys,
                                 uint32_t* __restrict__ pos, uint2* __restrict__ probes) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        const uint32_t start = heads[2 * x].x, p = plen[x], base = pre[x];
        for (uint32_t j = 0; j < p; ++j) {
            keys[base + j] = ((unsigned long long)(uint32_t)tok[start + j] << 32) | x;
            pos[base + j] = j;
            probes[base + j] = make_uint2(x, j);
        }
    }
}

// First index in keys[0, m) not below v.
__device__ __forceinline__ uint32_t lower_bound64(const unsigned long long* __restrict__ keys,
                                                  uint32_t m, unsigned long long v) {
    uint32_t lo = 0, hi = m;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2u;
        if (keys[mid] < v)
            lo = mid + 1u;
        else
            hi = mid;
    }
    return lo;
}

// Whether the meeting of r and s at prefix positions (i, j) is their first
// and, with POS, whether every meeting of their prefixes passes the
// positional bound.
template <bool POS>
__device__ bool keep_pair(const int32_t* __restrict__ R, uint32_t lr, uint32_t pr,
                          const int32_t* __restrict__ S, uint32_t ls, uint32_t ps, uint32_t i,
                          uint32_t j, Thr t) {
    // first meeting: no common token in R[0, i) and S[0, j)
    uint32_t x = 0, y = 0;
    while (x < i && y < j) {
        const int32_t a = R[x], b = S[y];
        if (a == b) return false;
        x += a < b ? 1u : 0u;
        y += b < a ? 1u : 0u;
    }
    if constexpr (POS) {
        const uint32_t alpha = (uint32_t)((t.num * ((unsigned long long)lr + ls) + t.num + t.den - 1ull) /
                                          (t.num + t.den));
        uint32_t A = 0;
        x = i;
        y = j;
        while (x < pr && y < ps) {
            const int32_t a = R[x], b = S[y];
            if (a == b) {
                if (A + 1u + min(lr - x - 1u, ls - y - 1u) < alpha) return false;
                ++A;
                ++x;
                ++y;
            } else {
                x += a < b ? 1u : 0u;
                y += b < a ? 1u : 0u;
            }
        }
    }
    return true;
}

constexpr uint32_t kPiece = 64;  // list entries per work item of a split list

// List range of each probe position (the entries of its token for sets below
// the probe) and its number of work items.
__global__ void k_probe_ranges(const uint4* __restrict__ heads, const int32_t* __restrict__ tok,
                               const uint2* __restrict__ probes, uint32_t m,
                               const unsigned long long* __restrict__ keys, uint2* __restrict__ range,
                               unsigned long long* __restrict__ items) {
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
        const uint2 pe = probes[e];
        const uint32_t r = pe.x;
        const unsigned long long w = (unsigned long long)(uint32_t)tok[heads[2 * r].x + pe.y] << 32;
        const uint32_t lo = lower_bound64(keys, m, w);
        const uint32_t hi = lower_bound64(keys, m, w | r);
        range[e] = make_uint2(lo, hi);
        items[e] = max(1ull, ((unsigned long long)(hi - lo) + kPiece - 1ull) / kPiece);
    }
}

// Item i belongs to the last probe position e with istart[e] <= i; every
// position has at least one item, so e <= i: galloping down from i.
__device__ __forceinline__ uint32_t item_owner(const unsigned long long* __restrict__ istart, uint32_t m,
                                               uint32_t i) {
    uint32_t hi = min(i, m - 1u);  // istart[hi] may exceed i
    if (istart[hi] <= i) return hi;
    uint32_t step = 1, lo = hi;
    while (true) {  // find lo with istart[lo] <= i (istart[0] = 0 <= i ends it)
        lo = hi >= step ? hi - step : 0u;
        if (istart[lo] <= i) break;
        hi = lo;
        step *= 2u;
    }
    while (hi - lo > 1u) {  // istart[lo] <= i < istart[hi]
        const uint32_t mid = lo + (hi - lo) / 2u;
        if (istart[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <bool FILL, bool POS>
__global__ void k_probe(const uint4* __restrict__ heads, const int32_t* __restrict__ tok,
                        const uint2* __restrict__ probes, uint32_t m, uint32_t n_items,
                        const unsigned long long* __restrict__ keys, const uint32_t* __restrict__ pos,
                        const uint32_t* __restrict__ plen, const uint2* __restrict__ range,
                        const unsigned long long* __restrict__ istart, Thr t,
                        unsigned long long* __restrict__ counts, const unsigned long long* __restrict__ off,
                        int2* __restrict__ out, unsigned long long cap) {
    for (uint32_t it = blockIdx.x * blockDim.x + threadIdx.x; it < n_items; it += gridDim.x * blockDim.x) {
        const uint32_t e = item_owner(istart, m, it);
        const uint32_t piece = (uint32_t)(it - istart[e]);
        const uint2 pe = probes[e];
        const uint32_t r = pe.x, i = pe.y;
        const uint4 hr = heads[2 * r];
        const uint32_t lr = hr.y, pr = plen[r];
        const int32_t* R = tok + hr.x;
        const uint2 rg = range[e];
        const uint32_t lo = rg.x + piece * kPiece, hi = min(rg.y, lo + kPiece);
        const uint32_t need_r = need_of(lr, t);
        uint32_t c = 0;
        const unsigned long long base = FILL ? off[it] : 0ull;
        for (uint32_t q = lo; q < hi; ++q) {
            const uint32_t s = (uint32_t)keys[q];
            const uint4 hs = heads[2 * s];
            const uint32_t ls = hs.y;
            if (ls < need_r || lr < need_of(ls, t)) continue;
            if (!keep_pair<POS>(R, lr, pr, tok + hs.x, ls, plen[s], i, pos[q], t)) continue;
            if constexpr (FILL) {
                if (base + c < cap) out[base + c] = make_int2((int)r, (int)s);
            }
            ++c;
        }
        if constexpr (!FILL) counts[it] = c;
    }
}

// Exclusive prefix sum of n values (rocPRIM's device scan; a null d_temp
// only reports the scratch size in *temp_bytes).
template <class T>
hipError_t scan_exclusive(void* d_temp, size_t* temp_bytes, const T* d_in, T* d_out, uint64_t n,
                          hipStream_t st) {
    return rocprim::exclusive_scan(d_temp, *temp_bytes, d_in, d_out, T(0), (size_t)n, rocprim::plus<T>(), st);
}

// Index entries sorted by their 64-bit key (token << 32 | set), positions
// moved with them (rocPRIM's device radix sort over all 64 key bits).
hipError_t sort_entries(void* d_temp, size_t* temp_bytes, const unsigned long long* d_keys,
                        unsigned long long* d_keys_out, const uint32_t* d_pos, uint32_t* d_pos_out, uint32_t m,
                        hipStream_t st) {
    return rocprim::radix_sort_pairs(d_temp, *temp_bytes, d_keys, d_keys_out, d_pos, d_pos_out, (size_t)m, 0u,
                                     64u, st);
}

int blocks_for(uint64_t n) {
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((n + kBlock - 1) / kBlock, 65536));
}

}  // namespace

hipError_t filter_prefix_lengths(const uint4* d_heads, uint32_t n, uint64_t num, uint64_t den,
                                 uint32_t* d_plen, uint32_t* d_pre, void* d_temp, size_t* temp_bytes,
                                 hipStream_t st) {
    if (!d_temp) return scan_exclusive(nullptr, temp_bytes, d_plen, d_pre, n + 1, st);
    hipLaunchKernelGGL(k_prefix_len, dim3(blocks_for(n)), dim3(kBlock), 0, st, d_heads, n, Thr{num, den},
                       d_plen);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // d_plen[n] is 0, so d_pre[n] is the number of index entries
    e = hipMemsetAsync(d_plen + n, 0, sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
    return scan_exclusive(d_temp, temp_bytes, d_plen, d_pre, n + 1, st);
}

hipError_t filter_build_index(const uint4* d_heads, const int32_t* d_tok, uint32_t n, uint32_t m,
                              const uint32_t* d_plen, const uint32_t* d_pre, unsigned long long* d_keys,
                              uint32_t* d_pos, unsigned long long* d_keys2, uint32_t* d_pos2, uint2* d_probes,
                              void* d_temp, size_t* temp_bytes, hipStream_t st) {
    if (!d_temp)
        return sort_entries(nullptr, temp_bytes, d_keys, d_keys2, d_pos, d_pos2, m, st);
    hipLaunchKernelGGL(k_prefix_entries, dim3(blocks_for(n)), dim3(kBlock), 0, st, d_heads, d_tok, n, d_plen,
                       d_pre, d_keys, d_pos, d_probes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sort_entries(d_temp, temp_bytes, d_keys, d_keys2, d_pos, d_pos2, m, st);
}

hipError_t filter_probe_items(const uint4* d_heads, const int32_t* d_tok, const uint2* d_probes, uint32_t m,
                              const unsigned long long* d_keys, uint2* d_range, unsigned long long* d_items,
                              unsigned long long* d_istart, void* d_temp, size_t* temp_bytes, hipStream_t st) {
    // d_items[m] is 0, so d_istart[m] is the number of work items
    if (!d_temp) return scan_exclusive(nullptr, temp_bytes, d_items, d_istart, m + 1, st);
    hipLaunchKernelGGL(k_probe_ranges, dim3(blocks_for(m)), dim3(kBlock), 0, st, d_heads, d_tok, d_probes, m,
                       d_keys, d_range, d_items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(d_items + m, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    return scan_exclusive(d_temp, temp_bytes, d_items, d_istart, m + 1, st);
}

hipError_t filter_probe(const uint4* d_heads, const int32_t* d_tok, const uint2* d_probes, uint32_t m,
                        uint32_t n_items, const unsigned long long* d_keys, const uint32_t* d_pos,
                        const uint32_t* d_plen, const uint2* d_range, const unsigned long long* d_istart,
                        uint64_t num, uint64_t den, bool positional, unsigned long long* d_counts,
                        const unsigned long long* d_off, int2* d_out, uint64_t cap, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    const Thr t{num, den};
    const dim3 g(blocks_for(n_items)), b(kBlock);
    if (!d_off) {
        if (positional)
            hipLaunchKernelGGL((k_probe<false, true>), g, b, 0, st, d_heads, d_tok, d_probes, m, n_items, d_keys,
                               d_pos, d_plen, d_range, d_istart, t, d_counts, nullptr, nullptr, 0ull);
        else
            hipLaunchKernelGGL((k_probe<false, false>), g, b, 0, st, d_heads, d_tok, d_probes, m, n_items,
                               d_keys, d_pos, d_plen, d_range, d_istart, t, d_counts, nullptr, nullptr, 0ull);
    } else {
        if (positional)
            hipLaunchKernelGGL((k_probe<true, true>), g, b, 0, st, d_heads, d_tok, d_probes, m, n_items, d_keys,
                               d_pos, d_plen, d_range, d_istart, t, nullptr, d_off, d_out, (unsigned long long)cap);
        else
            hipLaunchKernelGGL((k_probe<true, false>), g, b, 0, st, d_heads, d_tok, d_probes, m, n_items, d_keys,
                               d_pos, d_plen, d_range, d_istart, t, nullptr, d_off, d_out, (unsigned long long)cap);
    }
    return hipGetLastError();
}

hipError_t filter_scan_counts(unsigned long long* d_counts, unsigned long long* d_off, uint32_t n, void* d_temp,
                              size_t* temp_bytes, hipStream_t st) {
    // d_counts[n] is 0, so d_off[n] is the number of candidates
    if (!d_temp) return scan_exclusive(nullptr, temp_bytes, d_counts, d_off, n + 1, st);
    hipError_t e = hipMemsetAsync(d_counts + n, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    return scan_exclusive(d_temp, temp_bytes, d_counts, d_off, n + 1, st);
}

}  // namespace ssj
