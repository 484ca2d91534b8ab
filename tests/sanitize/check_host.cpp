// Host-code sanitizer harness (test infrastructure only): drives the C oracle
// (oracle/verify_ref.c) and the CPU candidate filter (ssj_inputs/csrc/
// allpairs.cpp) over small random collections so that an AddressSanitizer /
// UndefinedBehaviorSanitizer build of both sees every code path: all four
// similarity functions, the merge trace, both filter modes, probe ranges that
// do not fit their buffer, and the argument errors.  Consistency checks
// against a plain set intersection make a wrong result fail here too, but the
// point of this program is the sanitizers' reports; it exits non-zero on the
// first mismatch and the sanitizers abort on the first error.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

extern "C" {
int ssjref_verify_sim(const int64_t*, int64_t, const int32_t*, const int32_t*, int64_t, int, int64_t, int64_t,
                      uint8_t*, int32_t*, int);
int64_t ssjref_select_sim(const int64_t*, int64_t, const int32_t*, const int32_t*, int64_t, int, int64_t,
                          int64_t, uint8_t*, int32_t*, int);
int ssjref_merge_trace(const int64_t*, int64_t, const int32_t*, const int32_t*, int64_t, int64_t, int64_t,
                       int32_t*, int32_t*, uint8_t*, int);
struct ssjf_index;
int ssjf_build2(const int64_t*, int64_t, const int32_t*, int64_t, int64_t, int, ssjf_index**);
void ssjf_free(ssjf_index*);
int64_t ssjf_probe(ssjf_index*, int64_t, int64_t, int32_t*, int64_t, int64_t*);
int64_t ssjf_count(ssjf_index*, int, int64_t*);
int ssjf_fill(ssjf_index*, int, const int64_t*, int32_t*);
}

namespace {

int g_fail = 0;

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            g_fail = 1;                                                      \
            return;                                                          \
        }                                                                    \
    } while (0)

struct Coll {
    std::vector<int64_t> off;
    std::vector<int32_t> tok;
    int64_t n() const { return (int64_t)off.size() - 1; }
    int64_t len(int64_t i) const { return off[i + 1] - off[i]; }
};

// Sets of sizes in [lo, hi], sorted by size, tokens strictly increasing and
// drawn from a small universe so that many pairs overlap.
Coll make_coll(std::mt19937_64& g, int n, int lo, int hi, int universe) {
    std::vector<std::vector<int32_t>> sets(n);
    std::uniform_int_distribution<int> sz(lo, hi), tk(0, universe - 1);
    for (auto& s : sets) {
        std::set<int32_t> u;
        const int want = std::min(sz(g), universe);
        while ((int)u.size() < want) u.insert(tk(g));
        s.assign(u.begin(), u.end());
    }
    std::sort(sets.begin(), sets.end(), [](const auto& a, const auto& b) {
        return a.size() != b.size() ? a.size() < b.size() : a < b;
    });
    Coll c;
    c.off.push_back(0);
    for (auto& s : sets) {
        c.tok.insert(c.tok.end(), s.begin(), s.end());
        c.off.push_back((int64_t)c.tok.size());
    }
    return c;
}

int64_t overlap(const Coll& c, int32_t r, int32_t s) {
    std::vector<int32_t> out;
    std::set_intersection(c.tok.begin() + c.off[r], c.tok.begin() + c.off[r + 1], c.tok.begin() + c.off[s],
                          c.tok.begin() + c.off[s + 1], std::back_inserter(out));
    return (int64_t)out.size();
}

void run_case(std::mt19937_64& g, int n, int lo, int hi, int universe, int64_t tn, int64_t td) {
    const Coll c = make_coll(g, n, lo, hi, universe);
    for (int positional = 0; positional < 2; ++positional) {
        ssjf_index* ix = nullptr;
        CHECK(ssjf_build2(c.off.data(), c.n(), c.tok.data(), tn, td, positional, &ix) == 0);
        std::vector<int64_t> counts((size_t)c.n());
        const int64_t total = ssjf_count(ix, 3, counts.data());
        CHECK(total >= 0);
        std::vector<int64_t> starts((size_t)c.n() + 1, 0);
        for (int64_t r = 0; r < c.n(); ++r) starts[r + 1] = starts[r] + counts[r];
        CHECK(starts[c.n()] == total);
        std::vector<int32_t> cand((size_t)(2 * total + 2));
        CHECK(ssjf_fill(ix, 3, starts.data(), cand.data()) == 0);
        // probe in pieces whose buffer holds about a tenth of the candidates
        const int64_t cap = std::max<int64_t>(1, total / 10);
        std::vector<int32_t> piece((size_t)(2 * cap));
        int64_t r = 0, at = 0;
        while (r < c.n()) {
            int64_t next = -1;
            const int64_t got = ssjf_probe(ix, r, c.n(), piece.data(), cap, &next);
            CHECK(got >= 0 && next >= r);
            if (next == r) {  // one probe larger than the piece: take it alone
                std::vector<int32_t> big((size_t)(2 * counts[r] + 2));
                CHECK(ssjf_probe(ix, r, r + 1, big.data(), counts[r], &next) == counts[r] && next == r + 1);
                CHECK(std::equal(big.begin(), big.begin() + 2 * counts[r], cand.begin() + 2 * at));
                at += counts[r];
                r = next;
                continue;
            }
            CHECK(std::equal(piece.begin(), piece.begin() + 2 * got, cand.begin() + 2 * at));
            at += got;
            r = next;
        }
        CHECK(at == total);
        // every pair whose Jaccard similarity reaches t is a candidate
        std::set<std::pair<int32_t, int32_t>> cs;
        for (int64_t k = 0; k < total; ++k) cs.insert({cand[2 * k], cand[2 * k + 1]});
        for (int32_t a = 0; a < c.n(); ++a)
            for (int32_t b = 0; b < a; ++b) {
                const int64_t o = overlap(c, a, b);
                if (o * td >= tn * (c.len(a) + c.len(b) - o)) CHECK(cs.count({a, b}) == 1);
            }
        ssjf_free(ix);
        // the oracle over these candidates, every function
        const int64_t m = total;
        std::vector<uint8_t> pass((size_t)m + 1);
        std::vector<int32_t> ov((size_t)m + 1), sel((size_t)(2 * m + 2));
        for (int sim = 0; sim < 4; ++sim) {
            const int64_t sn = sim == 3 ? 3 : tn, sd = sim == 3 ? 1 : td;
            CHECK(ssjref_verify_sim(c.off.data(), c.n(), c.tok.data(), cand.data(), m, sim, sn, sd, pass.data(),
                                    ov.data(), 2) == 0);
            int64_t npass = 0;
            for (int64_t k = 0; k < m; ++k) {
                CHECK(ov[k] == overlap(c, cand[2 * k], cand[2 * k + 1]));
                npass += pass[k];
            }
            CHECK(ssjref_select_sim(c.off.data(), c.n(), c.tok.data(), cand.data(), m, sim, sn, sd, pass.data(),
                                    sel.data(), 2) == npass);
        }
        std::vector<int32_t> cr((size_t)m + 1), cs2((size_t)m + 1);
        std::vector<uint8_t> dec((size_t)m + 1);
        CHECK(ssjref_merge_trace(c.off.data(), c.n(), c.tok.data(), cand.data(), m, tn, td, cr.data(), cs2.data(),
                                 dec.data(), 2) == 0);
        CHECK(ssjref_verify_sim(c.off.data(), c.n(), c.tok.data(), cand.data(), m, 0, tn, td, pass.data(),
                                nullptr, 1) == 0);
        for (int64_t k = 0; k < m; ++k) {
            CHECK(dec[k] == pass[k]);
            CHECK(cr[k] >= 0 && cr[k] <= c.len(cand[2 * k]) && cs2[k] >= 0 && cs2[k] <= c.len(cand[2 * k + 1]));
        }
    }
    // argument errors: ids out of range, bad thresholds, unsorted sizes
    const int32_t bad[4] = {0, (int32_t)c.n(), -1, 0};
    uint8_t p2[2];
    CHECK(ssjref_verify_sim(c.off.data(), c.n(), c.tok.data(), bad, 2, 0, tn, td, p2, nullptr, 1) < 0);
    CHECK(ssjref_verify_sim(c.off.data(), c.n(), c.tok.data(), bad, 0, 0, 1, 0, p2, nullptr, 1) < 0);
    CHECK(ssjref_verify_sim(c.off.data(), c.n(), c.tok.data(), bad, 0, 0, 3, 2, p2, nullptr, 1) < 0);
    ssjf_index* ix = nullptr;
    CHECK(ssjf_build2(c.off.data(), c.n(), c.tok.data(), 0, 1, 0, &ix) < 0);
    if (c.n() >= 2 && c.len(c.n() - 1) > c.len(0)) {
        std::vector<int64_t> rev(c.off.size(), 0);  // largest set first: refused
        rev[1] = c.len(c.n() - 1);
        for (int64_t i = 1; i < c.n(); ++i) rev[i + 1] = rev[i] + c.len(i - 1);
        std::vector<int32_t> rtok(c.tok.begin() + c.off[c.n() - 1], c.tok.end());
        rtok.insert(rtok.end(), c.tok.begin(), c.tok.begin() + c.off[c.n() - 1]);
        CHECK(ssjf_build2(rev.data(), c.n(), rtok.data(), 1, 2, 0, &ix) < 0);
    }
}

}  // namespace

int main() {
    std::mt19937_64 g(20181221);
    const int64_t ts[][2] = {{1, 2}, {3, 5}, {7, 10}, {4, 5}, {9, 10}, {1, 1}};
    for (int rep = 0; rep < 3 && !g_fail; ++rep)
        for (const auto& t : ts) {
            run_case(g, 120, 1, 12, 40, t[0], t[1]);
            run_case(g, 60, 5, 60, 120, t[0], t[1]);
            if (g_fail) break;
        }
    if (!g_fail) run_case(g, 1, 3, 3, 10, 1, 2);  // one set: no candidates
    std::printf(g_fail ? "FAILED\n" : "sanitized host checks passed\n");
    return g_fail;
}
