// Host-side launch helpers of the GPU candidate generation (filter.hip):
// the prefix and length filters of a self-join and PPJoin's positional filter
// (paper Sec. 2.2 "Filters"; Sec. 3.1).  Used by the runtime's
// ssj_candidates_device / ssj_join entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssj {

// GPU candidate generation (filter.hip).  Each call with d_temp null only
// sets *temp_bytes to the temporary storage it needs.
// Prefix lengths of the n sets in d_plen[0, n) and their exclusive prefix sum
// in d_pre[0, n] (d_pre[n]: index entries).  d_plen needs n + 1 words.
hipError_t filter_prefix_lengths(const uint4* d_heads, uint32_t n, uint64_t num, uint64_t den,
                                 uint32_t* d_plen, uint32_t* d_pre, void* d_temp, size_t* temp_bytes,
                                 hipStream_t st);
// The m index entries, sorted into d_keys2 / d_pos2 (d_keys / d_pos are
// overwritten), and the probes (set, position) in set order.
hipError_t filter_build_index(const uint4* d_heads, const int32_t* d_tok, uint32_t n, uint32_t m,
                              const uint32_t* d_plen, const uint32_t* d_pre, unsigned long long* d_keys,
                              uint32_t* d_pos, unsigned long long* d_keys2, uint32_t* d_pos2, uint2* d_probes,
                              void* d_temp, size_t* temp_bytes, hipStream_t st);
// The list range of each probe position in d_range, its work items in
// d_items (m + 1 words) and their exclusive prefix sum in d_istart[0, m]
// (d_istart[m]: work items).
hipError_t filter_probe_items(const uint4* d_heads, const int32_t* d_tok, const uint2* d_probes, uint32_t m,
                              const unsigned long long* d_keys, uint2* d_range, unsigned long long* d_items,
                              unsigned long long* d_istart, void* d_temp, size_t* temp_bytes, hipStream_t st);
// Count pass (d_off null: candidates per work item into d_counts) or fill
// pass (candidates written at d_off, at most cap).
hipError_t filter_probe(const uint4* d_heads, const int32_t* d_tok, const uint2* d_probes, uint32_t m,
                        uint32_t n_items, const unsigned long long* d_keys, const uint32_t* d_pos,
                        const uint32_t* d_plen, const uint2* d_range, const unsigned long long* d_istart,
                        uint64_t num, uint64_t den, bool positional, unsigned long long* d_counts,
                        const unsigned long long* d_off, int2* d_out, uint64_t cap, hipStream_t st);
// Exclusive prefix sum of d_counts[0, n) into d_off[0, n] (d_counts needs n + 1 words).
hipError_t filter_scan_counts(unsigned long long* d_counts, unsigned long long* d_off, uint32_t n, void* d_temp,
                              size_t* temp_bytes, hipStream_t st);

}  // namespace ssj
