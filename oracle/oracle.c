/*
 * oracle.c -- plain CPU oracle for the joins of "GPU-based Efficient Join Algorithms on Hadoop".
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
 * leg may load this library.  It shares no code, header, table or constant with the GPU library
 * (paper_1904_11201_amd/csrc): its operator codes below are its own, and callers map operator
 * names to them.
 *
 * What it computes (Section 2.3 of the paper, "Join Operation"):
 *   equi join   EQ(R,S)    = multiset { (R.rid[i], S.rid[j]) : R.key[i] == S.key[j] }
 *   theta join  THETA(R,S) = multiset { (R.rid[i], S.rid[j]) : op_a(R.a[i],S.a[j]) and
 *                                                              op_c(R.c[i],S.c[j]) }
 * with the operators =, !=, <, <=, >, >= of Section 2.3 and Section 4.1 (figures "greena",
 * "greenb", "greenc"), plus a band |R.a - S.a| <= w evaluated in exact 64-bit arithmetic (a
 * reading: the paper has no band operator; it is the band-join workload's predicate).
 * Output pairs are positions (m, n) when a rid column is absent (Section 3.2.2).
 *
 * Every function returns the exact count (uint64) and, when `out` is not NULL and `cap` is at
 * least the count, writes the pairs as interleaved int32 (rid_R, rid_S) sorted ascending by
 * (rid_R, rid_S) -- the canonical order used for comparison.  When cap < count nothing is
 * written.
 *
 *   oracle_theta_nlj      brute-force nested loop over all |R|*|S| pairs: the definition itself
 *                          (Section 2.3, "Nested loop join").
 *   oracle_equi_sortmerge  sort both sides by key, emit the cross product of each equal-key run
 *                          (Section 2.3, "Sort merge join"); the stand-in where |R|*|S| is too
 *                          large for brute force.
 *   oracle_band_window     sort S by a; for each R row scan the S rows with a in [a-w, a+w] and
 *                          test the c predicate.  Stand-in for large band joins.
 *   oracle_count_equi      sum over keys of cntR[k] * cntS[k] (sorted runs).
 *   oracle_count_lt        sum over R of |{ j : S.a[j] > R.a[i] }| by binary search.
 *   oracle_sort_pairs      canonical sort of an interleaved pair array.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Operator codes of this oracle (private to it). */
#define ORC_NONE 0
#define ORC_EQ 1
#define ORC_NE 2
#define ORC_LT 3
#define ORC_LE 4
#define ORC_GT 5
#define ORC_GE 6
#define ORC_BAND 7

/* One comparison of the predicate, as the paper's operators define it on the int32 values. */
static int orc_holds(int op, int32_t r, int32_t s, int64_t w)
{
    switch (op) {
    case ORC_NONE: return 1;
    case ORC_EQ: return r == s;
    case ORC_NE: return r != s;
    case ORC_LT: return r < s;
    case ORC_LE: return r <= s;
    case ORC_GT: return r > s;
    case ORC_GE: return r >= s;
    case ORC_BAND: {
        int64_t d = (int64_t)r - (int64_t)s;
        if (d < 0) d = -d;
        return d <= w;
    }
    default: return 0;
    }
}

static int32_t rid_of(const int32_t* rid, int64_t i) { return rid ? rid[i] : (int32_t)i; }

static int cmp_pair(const void* a, const void* b)
{
    const int32_t* x = (const int32_t*)a;
    const int32_t* y = (const int32_t*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

void oracle_sort_pairs(int32_t* pairs, uint64_t n)
{
    if (n > 1) qsort(pairs, (size_t)n, 2 * sizeof(int32_t), cmp_pair);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Brute-force nested loop: for every (i, j) evaluate op_a and op_c.  Parallel over R rows: a
 * first pass counts matches per R row, an exclusive prefix over R rows places each row's
 * matches, a second pass writes them, and a final sort makes the order canonical. */
uint64_t oracle_theta_nlj(int64_t nR, const int32_t* Ra, const int32_t* Rc, const int32_t* Rrid,
                          int64_t nS, const int32_t* Sa, const int32_t* Sc, const int32_t* Srid,
                          int op_a, int64_t w, int op_c, int32_t* out, uint64_t cap)
{
    if (nR <= 0 || nS <= 0) return 0;
    uint64_t* per_row = (uint64_t*)calloc((size_t)nR + 1, sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nR; ++i) {
        uint64_t c = 0;
        for (int64_t j = 0; j < nS; ++j) {
            int ok = orc_holds(op_a, Ra[i], Sa[j], w);
            if (ok && op_c != ORC_NONE) ok = orc_holds(op_c, Rc[i], Sc[j], w);
            c += (uint64_t)ok;
        }
        per_row[i] = c;
    }
    uint64_t total = 0;
    for (int64_t i = 0; i < nR; ++i) {
        uint64_t c = per_row[i];
        per_row[i] = total;
        total += c;
    }
    if (out && cap >= total) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < nR; ++i) {
            uint64_t k = per_row[i];
            for (int64_t j = 0; j < nS; ++j) {
                int ok = orc_holds(op_a, Ra[i], Sa[j], w);
                if (ok && op_c != ORC_NONE) ok = orc_holds(op_c, Rc[i], Sc[j], w);
                if (ok) {
                    out[2 * k] = rid_of(Rrid, i);
                    out[2 * k + 1] = rid_of(Srid, j);
                    ++k;
                }
            }
        }
        oracle_sort_pairs(out, total);
    }
    free(per_row);
    return total;
}

/* (key, rid) record used by the sort-based oracles. */
typedef struct {
    int32_t key;
    int32_t aux;
    int32_t rid;
} orc_rec;

static int cmp_rec_key(const void* a, const void* b)
{
    const orc_rec* x = (const orc_rec*)a;
    const orc_rec* y = (const orc_rec*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->rid != y->rid) return x->rid < y->rid ? -1 : 1;
    return 0;
}

static orc_rec* to_recs(int64_t n, const int32_t* key, const int32_t* aux, const int32_t* rid)
{
    orc_rec* v = (orc_rec*)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_rec));
    for (int64_t i = 0; i < n; ++i) {
        v[i].key = key[i];
        v[i].aux = aux ? aux[i] : 0;
        v[i].rid = rid_of(rid, i);
    }
    qsort(v, (size_t)n, sizeof(orc_rec), cmp_rec_key);
    return v;
}

/* Sort-merge equi join: after sorting both sides by key, walk the two sorted lists; for every
 * key present in both, every R record of that key pairs with every S record of that key. */
uint64_t oracle_equi_sortmerge(int64_t nR, const int32_t* Rk, const int32_t* Rrid, int64_t nS,
                               const int32_t* Sk, const int32_t* Srid, int32_t* out, uint64_t cap)
{
    if (nR <= 0 || nS <= 0) return 0;
    orc_rec* r = to_recs(nR, Rk, NULL, Rrid);
    orc_rec* s = to_recs(nS, Sk, NULL, Srid);
    uint64_t total = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1 && !(out && cap >= total)) break;
        int64_t i = 0, j = 0;
        uint64_t k = 0;
        while (i < nR && j < nS) {
            if (r[i].key < s[j].key) { ++i; continue; }
            if (r[i].key > s[j].key) { ++j; continue; }
            int64_t i2 = i, j2 = j;
            while (i2 < nR && r[i2].key == r[i].key) ++i2;
            while (j2 < nS && s[j2].key == s[j].key) ++j2;
            if (pass == 0) {
                total += (uint64_t)(i2 - i) * (uint64_t)(j2 - j);
            } else {
                for (int64_t a = i; a < i2; ++a)
                    for (int64_t b = j; b < j2; ++b) {
                        out[2 * k] = r[a].rid;
                        out[2 * k + 1] = s[b].rid;
                        ++k;
                    }
            }
            i = i2;
            j = j2;
        }
        if (pass == 1) oracle_sort_pairs(out, total);
    }
    free(r);
    free(s);
    return total;
}

/* First index in sorted s[0..n) whose key is >= v (lower bound), computed in 64-bit. */
static int64_t lower_idx(const orc_rec* s, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)s[mid].key < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Band join |R.a - S.a| <= w (and op_c on column c): S sorted by a; for each R row only the S
 * rows whose a lies in [R.a - w, R.a + w] (64-bit bounds) are examined. */
uint64_t oracle_band_window(int64_t nR, const int32_t* Ra, const int32_t* Rc, const int32_t* Rrid,
                            int64_t nS, const int32_t* Sa, const int32_t* Sc, const int32_t* Srid,
                            int64_t w, int op_c, int32_t* out, uint64_t cap)
{
    if (nR <= 0 || nS <= 0 || w < 0) return 0;
    orc_rec* s = to_recs(nS, Sa, Sc, Srid);
    uint64_t* per_row = (uint64_t*)calloc((size_t)nR + 1, sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nR; ++i) {
        int64_t lo = (int64_t)Ra[i] - w, hi = (int64_t)Ra[i] + w;
        uint64_t c = 0;
        for (int64_t j = lower_idx(s, nS, lo); j < nS && (int64_t)s[j].key <= hi; ++j)
            c += (uint64_t)(op_c == ORC_NONE || orc_holds(op_c, Rc[i], s[j].aux, 0));
        per_row[i] = c;
    }
    uint64_t total = 0;
    for (int64_t i = 0; i < nR; ++i) {
        uint64_t c = per_row[i];
        per_row[i] = total;
        total += c;
    }
    if (out && cap >= total) {
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < nR; ++i) {
            int64_t lo = (int64_t)Ra[i] - w, hi = (int64_t)Ra[i] + w;
            uint64_t k = per_row[i];
            for (int64_t j = lower_idx(s, nS, lo); j < nS && (int64_t)s[j].key <= hi; ++j)
                if (op_c == ORC_NONE || orc_holds(op_c, Rc[i], s[j].aux, 0)) {
                    out[2 * k] = rid_of(Rrid, i);
                    out[2 * k + 1] = s[j].rid;
                    ++k;
                }
        }
        oracle_sort_pairs(out, total);
    }
    free(per_row);
    free(s);
    return total;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return x < y ? -1 : (x > y);
}

static int32_t* sorted_copy(int64_t n, const int32_t* v)
{
    int32_t* c = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (n > 0) memcpy(c, v, (size_t)n * sizeof(int32_t));
    qsort(c, (size_t)n, sizeof(int32_t), cmp_i32);
    return c;
}

/* Equi-join count as a sum over distinct keys of (multiplicity in R) * (multiplicity in S). */
uint64_t oracle_count_equi(int64_t nR, const int32_t* Rk, int64_t nS, const int32_t* Sk)
{
    if (nR <= 0 || nS <= 0) return 0;
    int32_t* r = sorted_copy(nR, Rk);
    int32_t* s = sorted_copy(nS, Sk);
    uint64_t total = 0;
    int64_t i = 0, j = 0;
    while (i < nR && j < nS) {
        if (r[i] < s[j]) { ++i; continue; }
        if (r[i] > s[j]) { ++j; continue; }
        int64_t i2 = i, j2 = j;
        while (i2 < nR && r[i2] == r[i]) ++i2;
        while (j2 < nS && s[j2] == s[j]) ++j2;
        total += (uint64_t)(i2 - i) * (uint64_t)(j2 - j);
        i = i2;
        j = j2;
    }
    free(r);
    free(s);
    return total;
}

/* Count of pairs with R.a < S.a: for each R value, the S values strictly above it, found by
 * binary search in sorted S. */
uint64_t oracle_count_lt(int64_t nR, const int32_t* Ra, int64_t nS, const int32_t* Sa)
{
    if (nR <= 0 || nS <= 0) return 0;
    int32_t* s = sorted_copy(nS, Sa);
    uint64_t total = 0;
#pragma omp parallel for reduction(+ : total)
    for (int64_t i = 0; i < nR; ++i) {
        int64_t lo = 0, hi = nS; /* first index with s[idx] > Ra[i] */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (s[mid] <= Ra[i]) lo = mid + 1; else hi = mid;
        }
        total += (uint64_t)(nS - lo);
    }
    free(s);
    return total;
}
