// CPU candidate generators: the AllPairs prefix + length filter, and the
// same with PPJoin's positional filter.
//
// This is the filtering phase that feeds verification (paper Sec. 2.2,
// "Filters" and "Algorithm outline"; Sec. 3.1, AllPairs and PPJoin).  It is
// input generation for the verification path, not part of it.
//
// Self-join over a collection whose sets are sorted by size (set id order ==
// non-decreasing size).  For a threshold t = t_num / t_den > 0:
//   need(x)   = ceil(t * |x|)            (J >= t implies |x & y| >= t |x|)
//   prefix(x) = |x| - need(x) + 1        (prefix-filter lemma)
// A set r probes, for every token w of its prefix, the prefix inverted list
// of w restricted to earlier sets s (s < r, so |s| <= |r|) whose size passes
// the length filter |s| >= need(r).  Each distinct s found becomes the
// candidate (r, s), in order of first discovery.  The index holds every set's
// prefix; restricting a list to ids below r is the same as building it
// incrementally (probe, then insert), as the paper's self-join does.
//
// Positional filter (PPJoin; Sec. 2.2 "Filters"): the index also keeps the
// position j of each prefix token w in s.  When probe r meets s through w at
// its position i, every token the two sets share below w lies in both
// prefixes and was met earlier in this probe, so the count A(s) of earlier
// meetings is exactly that shared part, and the overlap is at most
// A(s) + 1 + min(|r| - i - 1, |s| - j - 1).  If that is below the overlap
// Jaccard t requires of the pair, ceil(t / (1 + t) * (|r| + |s|)) (Sec. 2.2,
// the equivalent overlap), s is dropped for the rest of the probe.  The
// remaining partners are emitted after the probe, in order of first meeting.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

struct Index {
    int64_t n_sets = 0;
    int64_t t_num = 0, t_den = 1;
    std::vector<int64_t> offsets;   // set CSR
    std::vector<int32_t> tokens;
    std::vector<int64_t> list_off;  // token -> [list_off[w], list_off[w+1]) in list_ids
    std::vector<int32_t> list_ids;  // ascending set ids
    std::vector<int32_t> list_pos;  // position of the token in that set (positional filter)
    bool positional = false;
    uint64_t serial = 0;
};

std::atomic<uint64_t> g_serial{1};

inline int64_t need_of(const Index& ix, int64_t len) {
    return (ix.t_num * len + ix.t_den - 1) / ix.t_den;
}

// Overlap Jaccard t requires of sets of sizes a and b:
// ceil(t_num (a + b) / (t_num + t_den)).
inline int64_t pair_need(const Index& ix, int64_t a, int64_t b) {
    const int64_t d = ix.t_num + ix.t_den;
    return (ix.t_num * (a + b) + d - 1) / d;
}

inline int64_t prefix_of(const Index& ix, int64_t len) {
    int64_t p = len - need_of(ix, len) + 1;
    return p < 0 ? 0 : (p > len ? len : p);
}

// Per-thread dedupe marks: every probe takes a fresh stamp, so no clearing is
// needed between probes or between calls.
struct Stamps {
    uint64_t serial = 0;
    uint32_t cur = 0;
    std::vector<uint32_t> mark;
    std::vector<int32_t> acc;       // positional filter: meetings so far, -1 once dropped
    std::vector<int32_t> found;     // positional filter: partners in order of first meeting
    uint32_t next() {
        if (++cur == 0) {
            std::fill(mark.begin(), mark.end(), 0u);
            cur = 1;
        }
        return cur;
    }
};

thread_local Stamps tl_stamps;

Stamps& stamps_for(const Index& ix) {
    if (tl_stamps.serial != ix.serial || (int64_t)tl_stamps.mark.size() != ix.n_sets) {
        tl_stamps.mark.assign((size_t)ix.n_sets, 0u);
        tl_stamps.acc.assign(ix.positional ? (size_t)ix.n_sets : 0u, 0);
        tl_stamps.cur = 0;
        tl_stamps.serial = ix.serial;
    }
    return tl_stamps;
}

// Calls emit(s) for every candidate partner s of probe r; returns the count.
template <class Emit>
int64_t probe_one(const Index& ix, int64_t r, Stamps& st, Emit emit) {
    const uint32_t stamp = st.next();
    uint32_t* mark = st.mark.data();
    const int64_t rb = ix.offsets[r], len = ix.offsets[r + 1] - rb;
    const int64_t need = need_of(ix, len);
    const int64_t p = prefix_of(ix, len);
    int64_t n = 0;
    for (int64_t k = 0; k < p; ++k) {
        const int32_t w = ix.tokens[rb + k];
        const int32_t* lb = ix.list_ids.data() + ix.list_off[w];
        const int32_t* le = ix.list_ids.data() + ix.list_off[w + 1];
        // length filter: first s with |s| >= need (sizes ascend with id)
        const int32_t* a = std::partition_point(lb, le, [&](int32_t s) {
            return ix.offsets[s + 1] - ix.offsets[s] < need;
        });
        // only sets indexed before r
        const int32_t* b = std::lower_bound(a, le, (int32_t)r);
        if (!ix.positional) {
            for (const int32_t* q = a; q < b; ++q) {
                const int32_t s = *q;
                if (mark[s] != stamp) {
                    mark[s] = stamp;
                    emit(s);
                    ++n;
                }
            }
            continue;
        }
        const int32_t* pos = ix.list_pos.data() + (a - ix.list_ids.data());
        for (const int32_t* q = a; q < b; ++q, ++pos) {
            const int32_t s = *q;
            if (mark[s] != stamp) {
                mark[s] = stamp;
                st.acc[s] = 0;
                st.found.push_back(s);
            }
            if (st.acc[s] < 0) continue;
            const int64_t ls = ix.offsets[s + 1] - ix.offsets[s];
            const int64_t bound = st.acc[s] + 1 + std::min(len - k - 1, ls - *pos - 1);
            if (bound < pair_need(ix, len, ls))
                st.acc[s] = -1;
            else
                ++st.acc[s];
        }
    }
    if (ix.positional) {
        for (const int32_t s : st.found) {
            if (st.acc[s] > 0) {
                emit(s);
                ++n;
            }
        }
        st.found.clear();
    }
    return n;
}

template <class Fn>
void parallel_chunks(int64_t n, int n_threads, Fn fn) {
    if (n_threads < 1) n_threads = 1;
    const int64_t chunk = 256;
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (;;) {
            int64_t b = next.fetch_add(chunk);
            if (b >= n) break;
            fn(b, std::min(n, b + chunk));
        }
    };
    if (n_threads == 1) {
        worker();
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) th.emplace_back(worker);
    for (auto& t : th) t.join();
}

}  // namespace

extern "C" {

struct ssjf_index;

// Builds the prefix index (positional != 0: with the positional filter).
// Returns 0, or -1 on invalid arguments/no memory.
int ssjf_build2(const int64_t* offsets, int64_t n_sets, const int32_t* tokens, int64_t t_num,
                int64_t t_den, int positional, ssjf_index** out) {
    if (!out || !offsets || n_sets < 0 || n_sets >= INT32_MAX || t_den <= 0 || t_num <= 0 ||
        t_num > t_den)
        return -1;
    *out = nullptr;
    try {
        Index* ix = new Index();
        ix->n_sets = n_sets;
        ix->t_num = t_num;
        ix->t_den = t_den;
        ix->positional = positional != 0;
        ix->serial = g_serial.fetch_add(1);
        ix->offsets.assign(offsets, offsets + n_sets + 1);
        const int64_t nnz = offsets[n_sets] - offsets[0];
        if (offsets[0] != 0 || nnz < 0 || (nnz > 0 && !tokens)) {
            delete ix;
            return -1;
        }
        ix->tokens.assign(tokens, tokens + nnz);
        int64_t max_tok = -1;
        for (int64_t i = 0; i < n_sets; ++i) {
            if (offsets[i + 1] < offsets[i]) {
                delete ix;
                return -1;
            }
            if (i > 0 && offsets[i + 1] - offsets[i] < offsets[i] - offsets[i - 1]) {
                delete ix;  // sets must be ordered by size
                return -1;
            }
        }
        for (int64_t k = 0; k < nnz; ++k) {
            if (tokens[k] < 0) {
                delete ix;
                return -1;
            }
            max_tok = std::max<int64_t>(max_tok, tokens[k]);
        }
        const int64_t n_tok = max_tok + 1;
        ix->list_off.assign((size_t)n_tok + 1, 0);
        for (int64_t i = 0; i < n_sets; ++i) {
            const int64_t b = offsets[i], p = prefix_of(*ix, offsets[i + 1] - b);
            for (int64_t k = 0; k < p; ++k) ix->list_off[(size_t)tokens[b + k] + 1]++;
        }
        for (int64_t w = 0; w < n_tok; ++w) ix->list_off[w + 1] += ix->list_off[w];
        ix->list_ids.resize((size_t)ix->list_off[n_tok]);
        if (ix->positional) ix->list_pos.resize((size_t)ix->list_off[n_tok]);
        std::vector<int64_t> fill(ix->list_off.begin(), ix->list_off.end() - 1);
        for (int64_t i = 0; i < n_sets; ++i) {
            const int64_t b = offsets[i], p = prefix_of(*ix, offsets[i + 1] - b);
            for (int64_t k = 0; k < p; ++k) {
                const int64_t at = fill[tokens[b + k]]++;
                ix->list_ids[(size_t)at] = (int32_t)i;
                if (ix->positional) ix->list_pos[(size_t)at] = (int32_t)k;
            }
        }
        *out = reinterpret_cast<ssjf_index*>(ix);
        return 0;
    } catch (const std::bad_alloc&) {
        return -1;
    }
}

// The AllPairs index (no positional filter).
int ssjf_build(const int64_t* offsets, int64_t n_sets, const int32_t* tokens, int64_t t_num,
               int64_t t_den, ssjf_index** out) {
    return ssjf_build2(offsets, n_sets, tokens, t_num, t_den, 0, out);
}

void ssjf_free(ssjf_index* h) { delete reinterpret_cast<Index*>(h); }

// Candidates of probes r_begin, r_begin+1, ... written as (r, s) int32 pairs
// into out (capacity cap pairs).  Stops before a probe whose candidates do not
// fit; *next_r receives the first probe not emitted.  Returns pairs written,
// or -1 on bad arguments.  Thread-safe for concurrent calls on one index.
int64_t ssjf_probe(ssjf_index* h, int64_t r_begin, int64_t r_end, int32_t* out, int64_t cap,
                   int64_t* next_r) {
    const Index* ix = reinterpret_cast<const Index*>(h);
    if (!ix || r_begin < 0 || r_end > ix->n_sets || r_begin > r_end || cap < 0) return -1;
    auto& mark = stamps_for(*ix);
    int64_t n = 0, r = r_begin;
    std::vector<int32_t> tmp;
    for (; r < r_end; ++r) {
        tmp.clear();
        probe_one(*ix, r, mark, [&](int32_t s) { tmp.push_back(s); });
        if (n + (int64_t)tmp.size() > cap) break;
        for (int32_t s : tmp) {
            out[2 * n] = (int32_t)r;
            out[2 * n + 1] = s;
            ++n;
        }
    }
    if (next_r) *next_r = r;
    return n;
}

// Per-probe candidate counts (counts may be null).  Returns the total.
int64_t ssjf_count(ssjf_index* h, int n_threads, int64_t* counts) {
    const Index* ix = reinterpret_cast<const Index*>(h);
    if (!ix) return -1;
    std::atomic<int64_t> total{0};
    parallel_chunks(ix->n_sets, n_threads, [&](int64_t b, int64_t e) {
        auto& mark = stamps_for(*ix);
        int64_t loc = 0;
        for (int64_t r = b; r < e; ++r) {
            int64_t c = probe_one(*ix, r, mark, [](int32_t) {});
            if (counts) counts[r] = c;
            loc += c;
        }
        total.fetch_add(loc);
    });
    return total.load();
}

// Writes every candidate; probe r's candidates start at pair index starts[r]
// (the exclusive prefix sum of ssjf_count's counts).
int ssjf_fill(ssjf_index* h, int n_threads, const int64_t* starts, int32_t* out) {
    const Index* ix = reinterpret_cast<const Index*>(h);
    if (!ix || !starts || !out) return -1;
    parallel_chunks(ix->n_sets, n_threads, [&](int64_t b, int64_t e) {
        auto& mark = stamps_for(*ix);
        for (int64_t r = b; r < e; ++r) {
            int64_t k = starts[r];
            probe_one(*ix, r, mark, [&](int32_t s) {
                out[2 * k] = (int32_t)r;
                out[2 * k + 1] = s;
                ++k;
            });
        }
    });
    return 0;
}

}  // extern "C"
