/*
 * Verification oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU reference for the verification phase of
 * an exact set-similarity join.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * constant with the GPU library and includes nothing from it.
 *
 * What it computes (paper Sec. 3, Definition 1, with the similarity
 * functions of Table 1): a candidate pair (r, s) is in the result iff
 * sim(r, s) >= t = t_num / t_den, evaluated exactly in integers with
 * o = |r & s|:
 *     Jaccard  o / |r | s| >= t        o * t_den >= t_num * (|r| + |s| - o)
 *     Cosine   o / sqrt(|r||s|) >= t   o^2 * t_den^2 >= t_num^2 * |r| * |s|
 *     Dice     2o / (|r| + |s|) >= t   2 * o * t_den >= t_num * (|r| + |s|)
 *     Overlap  o >= t                  o * t_den >= t_num
 * (the Cosine form squares both non-negative sides; its right side needs 128
 * bits).  The overlap is a full two-pointer merge of the two sorted token
 * lists (no early exit), so the result is the plain definition, not the
 * paper's early-terminating procedure.
 *
 * A second routine replays the paper's early-terminating merge (Sec. 3.1:
 * the merge-like loop stops once the required overlap is met or can no
 * longer be reached) only to count the tokens it consumes; those counts are
 * a reporting quantity for the benchmark's byte accounting.
 */
#include <stdint.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Status codes of this oracle. */
#define REF_OK 0
#define REF_EINVAL -1

/* |a & b| for two strictly increasing token lists, by a full merge. */
static int64_t overlap_full(const int32_t *a, int64_t na, const int32_t *b, int64_t nb)
{
    int64_t i = 0, j = 0, o = 0;
    while (i < na && j < nb) {
        if (a[i] == b[j]) {
            o++;
            i++;
            j++;
        } else if (a[i] < b[j]) {
            i++;
        } else {
            j++;
        }
    }
    return o;
}

/* Similarity functions of Table 1. */
#define REF_JACCARD 0
#define REF_COSINE 1
#define REF_DICE 2
#define REF_OVERLAP 3

/* sim(r, s) >= t_num / t_den, given the overlap o and the two sizes. */
static int sim_at_least(int sim, int64_t o, int64_t nr, int64_t ns, int64_t t_num, int64_t t_den)
{
    switch (sim) {
    case REF_JACCARD:
        return o * t_den >= t_num * (nr + ns - o);
    case REF_COSINE: {
        unsigned __int128 lhs = (unsigned __int128)(uint64_t)(o * t_den) * (uint64_t)(o * t_den);
        unsigned __int128 rhs = (unsigned __int128)(uint64_t)(t_num * t_num) *
                                (unsigned __int128)((uint64_t)nr * (uint64_t)ns);
        return lhs >= rhs;
    }
    case REF_DICE:
        return 2 * o * t_den >= t_num * (nr + ns);
    case REF_OVERLAP:
        return o * t_den >= t_num;
    }
    return 0;
}

/* 0 < t_den < 2^31 and 0 <= t_num; t <= 1 for the normalised functions. */
static int valid_sim_threshold(int sim, int64_t t_num, int64_t t_den)
{
    if (sim < REF_JACCARD || sim > REF_OVERLAP)
        return 0;
    if (t_den <= 0 || t_den > INT32_MAX || t_num < 0 || t_num > INT32_MAX)
        return 0;
    return sim == REF_OVERLAP || t_num <= t_den;
}

static int valid_threshold(int64_t t_num, int64_t t_den)
{
    return valid_sim_threshold(REF_JACCARD, t_num, t_den);
}

static int pair_ok(const int64_t *offsets, int64_t n_sets, int32_t r, int32_t s)
{
    if (r < 0 || s < 0 || r >= n_sets || s >= n_sets)
        return 0;
    if (offsets[r + 1] <= offsets[r] || offsets[s + 1] <= offsets[s])
        return 0; /* empty sets are outside the problem (0/0) */
    return 1;
}

/*
 * For each pair k (pairs[2k] = r, pairs[2k+1] = s): pass[k] = 1 iff
 * sim(r, s) >= t_num / t_den for the similarity function sim (REF_*);
 * overlap[k] = |r & s| (overlap may be NULL).  Returns REF_EINVAL (and writes
 * nothing useful) for an invalid function or threshold or any id out of
 * range / empty set.
 */
int ssjref_verify_sim(const int64_t *offsets, int64_t n_sets, const int32_t *tokens,
                      const int32_t *pairs, int64_t n_pairs, int sim, int64_t t_num,
                      int64_t t_den, uint8_t *pass, int32_t *overlap, int n_threads)
{
    int64_t k;
    int bad = 0;
    if (!valid_sim_threshold(sim, t_num, t_den) || n_pairs < 0)
        return REF_EINVAL;
    for (k = 0; k < n_pairs; k++)
        if (!pair_ok(offsets, n_sets, pairs[2 * k], pairs[2 * k + 1]))
            bad = 1;
    if (bad)
        return REF_EINVAL;
#ifdef _OPENMP
    if (n_threads < 1)
        n_threads = 1;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(n_threads)
#endif
    for (k = 0; k < n_pairs; k++) {
        int32_t r = pairs[2 * k], s = pairs[2 * k + 1];
        int64_t nr = offsets[r + 1] - offsets[r];
        int64_t ns = offsets[s + 1] - offsets[s];
        int64_t o = overlap_full(tokens + offsets[r], nr, tokens + offsets[s], ns);
        pass[k] = (uint8_t)sim_at_least(sim, o, nr, ns, t_num, t_den);
        if (overlap)
            overlap[k] = (int32_t)o;
    }
    (void)n_threads;
    return REF_OK;
}

/* ssjref_verify_sim with the Jaccard similarity. */
int ssjref_verify(const int64_t *offsets, int64_t n_sets, const int32_t *tokens,
                  const int32_t *pairs, int64_t n_pairs, int64_t t_num, int64_t t_den,
                  uint8_t *pass, int32_t *overlap, int n_threads)
{
    return ssjref_verify_sim(offsets, n_sets, tokens, pairs, n_pairs, REF_JACCARD, t_num, t_den,
                             pass, overlap, n_threads);
}

/*
 * Copies the passing pairs, in input order, to out (2 ints per pair) and
 * returns their number (or REF_EINVAL).  out must hold n_pairs pairs.
 */
int64_t ssjref_select_sim(const int64_t *offsets, int64_t n_sets, const int32_t *tokens,
                          const int32_t *pairs, int64_t n_pairs, int sim, int64_t t_num,
                          int64_t t_den, uint8_t *scratch_pass, int32_t *out, int n_threads)
{
    int64_t k, n = 0;
    int rc = ssjref_verify_sim(offsets, n_sets, tokens, pairs, n_pairs, sim, t_num, t_den,
                               scratch_pass, NULL, n_threads);
    if (rc != REF_OK)
        return rc;
    for (k = 0; k < n_pairs; k++) {
        if (scratch_pass[k]) {
            out[2 * n] = pairs[2 * k];
            out[2 * n + 1] = pairs[2 * k + 1];
            n++;
        }
    }
    return n;
}

/* ssjref_select_sim with the Jaccard similarity. */
int64_t ssjref_select(const int64_t *offsets, int64_t n_sets, const int32_t *tokens,
                      const int32_t *pairs, int64_t n_pairs, int64_t t_num, int64_t t_den,
                      uint8_t *scratch_pass, int32_t *out, int n_threads)
{
    return ssjref_select_sim(offsets, n_sets, tokens, pairs, n_pairs, REF_JACCARD, t_num, t_den,
                             scratch_pass, out, n_threads);
}

/*
 * Early-terminating merge, replayed for accounting only.
 *
 * The required overlap is the Jaccard row of Table 1,
 *     alpha = ceil(t / (1 + t) * (|r| + |s|)) = ceil(t_num (|r|+|s|) / (t_num + t_den)),
 * taken in integers.  Two cursors i (into r) and j (into s) walk the merge;
 * before each step the loop stops with "accept" if o >= alpha, or with
 * "reject" if o + min(|r| - i, |s| - j) < alpha (the overlap can no longer
 * be reached).  Otherwise the smaller current token is consumed (both on a
 * match, which adds one to o).  On exit c_r = i and c_s = j are the tokens
 * consumed from each side, and decided[k] is the decision reached.
 */
int ssjref_merge_trace(const int64_t *offsets, int64_t n_sets, const int32_t *tokens,
                       const int32_t *pairs, int64_t n_pairs, int64_t t_num, int64_t t_den,
                       int32_t *c_r, int32_t *c_s, uint8_t *decided, int n_threads)
{
    int64_t k;
    int bad = 0;
    if (!valid_threshold(t_num, t_den) || n_pairs < 0)
        return REF_EINVAL;
    for (k = 0; k < n_pairs; k++)
        if (!pair_ok(offsets, n_sets, pairs[2 * k], pairs[2 * k + 1]))
            bad = 1;
    if (bad)
        return REF_EINVAL;
#ifdef _OPENMP
    if (n_threads < 1)
        n_threads = 1;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(n_threads)
#endif
    for (k = 0; k < n_pairs; k++) {
        int32_t r = pairs[2 * k], s = pairs[2 * k + 1];
        const int32_t *a = tokens + offsets[r];
        const int32_t *b = tokens + offsets[s];
        int64_t na = offsets[r + 1] - offsets[r];
        int64_t nb = offsets[s + 1] - offsets[s];
        int64_t alpha = (t_num * (na + nb) + (t_num + t_den) - 1) / (t_num + t_den);
        int64_t i = 0, j = 0, o = 0;
        int acc;
        for (;;) {
            int64_t rem_a = na - i, rem_b = nb - j;
            int64_t rem = rem_a < rem_b ? rem_a : rem_b;
            if (o >= alpha) {
                acc = 1;
                break;
            }
            if (o + rem < alpha) {
                acc = 0;
                break;
            }
            if (a[i] == b[j]) {
                o++;
                i++;
                j++;
            } else if (a[i] < b[j]) {
                i++;
            } else {
                j++;
            }
        }
        c_r[k] = (int32_t)i;
        c_s[k] = (int32_t)j;
        decided[k] = (uint8_t)acc;
    }
    (void)n_threads;
    return REF_OK;
}

/* Number of OpenMP threads a call with n_threads <= 0 would use. */
int ssjref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
