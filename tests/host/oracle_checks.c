/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built
 * together with oracle/fclsh_oracle.c, OpenMP on): every function on small
 * random inputs, including the edges (an empty row, a point in every bucket,
 * ragged d), with the consistency the pins rely on: Strategy 2 equals the
 * linear scan, the sparse keys and scan equal the dense ones on the same
 * points.  A sanitizer report aborts; a failed check exits with status 1. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_derive_params(int d, int r, uint64_t seed, int override_t, uint64_t P, int skip_col0, int32_t *t_out,
                      int32_t *rpart_out, int32_t *part, int32_t *col, uint64_t *b);
void orc_masks(int d, int t, int rp, const int32_t *part, const int32_t *col, uint8_t *mask);
void orc_keys(const uint64_t *points, int d, const int64_t *which, int64_t npick, int ntab, const uint8_t *mask,
              const uint64_t *b, uint64_t P, uint32_t *keys);
void orc_tables(const uint32_t *keys, int64_t n, int ntab, uint32_t *tkeys, uint32_t *tids);
void orc_query_batch(const uint64_t *points, int64_t n, int d, const uint32_t *tkeys, const uint32_t *tids, int ntab,
                     const uint64_t *queries, int64_t nq, const uint32_t *qkeys, int rq, int64_t cap, uint32_t *out,
                     int64_t *counts, int64_t *collisions, int64_t *candidates);
void orc_brute_force(const uint64_t *points, int64_t n, int d, const uint64_t *queries, int64_t nq, int rq,
                     int64_t cap, uint32_t *out, int64_t *counts);
void orc_keys_sparse(const int64_t *ptr, const int32_t *cols, int64_t m, int t, int rp, const int32_t *part,
                     const int32_t *col, const uint64_t *b, uint64_t P, uint32_t *keys);
void orc_brute_force_sparse(const int64_t *ptr, const int32_t *cols, int64_t n, const int64_t *qptr,
                            const int32_t *qcols, int64_t nq, int d, int rq, int64_t cap, uint32_t *out,
                            int64_t *counts);

static int g_fail = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            printf("check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                              \
        }                                                          \
    } while (0)

static uint64_t rng_state = 88172645463325252ULL;
static uint64_t next_u64(void) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static void run_case(int n, int d, int r, int t, int density_pct) {
    const uint64_t P = 2147483647ULL;
    const int W = (d + 63) / 64;
    int32_t tt = 0, rp = 0;
    int32_t *part = calloc((size_t)d, 4), *col = calloc((size_t)d, 4);
    uint64_t *b = calloc((size_t)d, 8);
    CHECK(orc_derive_params(d, r, 1234u + (unsigned)d, t, P, 0, &tt, &rp, part, col, b) == 0);
    const int D = 1 << (rp + 1), L = tt * (D - 1);
    /* points as bit vectors and as rows; point 0 empty, point 1 all ones,
     * the queries are points 2..5 */
    uint64_t *pts = calloc((size_t)n * W, 8);
    int64_t *ptr = calloc((size_t)n + 1, 8);
    int32_t *cols = calloc((size_t)n * d + 1, 4);
    int64_t e = 0;
    for (int i = 0; i < n; ++i) {
        ptr[i] = e;
        for (int c = 0; c < d; ++c) {
            const int on = i == 0 ? 0 : i == 1 ? 1 : (int)(next_u64() % 100) < density_pct;
            if (on) {
                pts[(size_t)i * W + c / 64] |= 1ULL << (c % 64);
                cols[e++] = c;
            }
        }
    }
    ptr[n] = e;
    uint8_t *mask = calloc((size_t)L * d, 1);
    orc_masks(d, tt, rp, part, col, mask);
    uint32_t *keys = calloc((size_t)L * n, 4), *skeys = calloc((size_t)L * n, 4);
    orc_keys(pts, d, NULL, n, L, mask, b, P, keys);
    orc_keys_sparse(ptr, cols, n, tt, rp, part, col, b, P, skeys);
    CHECK(memcmp(keys, skeys, (size_t)L * n * 4) == 0);
    for (int T = 0; T < L; ++T) CHECK(keys[(size_t)T * n] == 0); /* the empty point */
    uint32_t *tk = calloc((size_t)L * n, 4), *ti = calloc((size_t)L * n, 4);
    orc_tables(keys, n, L, tk, ti);
    const int nq = 4;
    uint32_t *qkeys = calloc((size_t)L * nq, 4);
    for (int T = 0; T < L; ++T)
        for (int q = 0; q < nq; ++q) qkeys[(size_t)T * nq + q] = keys[(size_t)T * n + 2 + q];
    uint32_t *out = calloc((size_t)nq * n, 4), *bout = calloc((size_t)nq * n, 4), *sout = calloc((size_t)nq * n, 4);
    int64_t cnt[4], bcnt[4], scnt[4], coll[4], cand[4];
    for (int rq = 0; rq <= r; rq += (r > 4 ? r / 4 : 1)) {
        orc_query_batch(pts, n, d, tk, ti, L, pts + 2 * (size_t)W, nq, qkeys, rq, n, out, cnt, coll, cand);
        orc_brute_force(pts, n, d, pts + 2 * (size_t)W, nq, rq, n, bout, bcnt);
        orc_brute_force_sparse(ptr, cols, n, ptr + 2, cols, nq, d, rq, n, sout, scnt);
        for (int q = 0; q < nq; ++q) {
            CHECK(cnt[q] == bcnt[q] && scnt[q] == bcnt[q] && cnt[q] >= 1);
            CHECK(memcmp(out + (size_t)q * n, bout + (size_t)q * n, (size_t)cnt[q] * 4) == 0);
            CHECK(memcmp(sout + (size_t)q * n, bout + (size_t)q * n, (size_t)cnt[q] * 4) == 0);
            CHECK(coll[q] >= cand[q] && cand[q] >= cnt[q]);
        }
    }
    free(part); free(col); free(b); free(pts); free(ptr); free(cols); free(mask); free(keys); free(skeys);
    free(tk); free(ti); free(qkeys); free(out); free(bout); free(sout);
}

int main(void) {
    run_case(200, 64, 4, 0, 50);
    run_case(150, 100, 6, 0, 10);    /* ragged d, sparse-ish */
    run_case(120, 300, 12, 0, 3);    /* two parts, general construction */
    run_case(90, 70, 9, 3, 40);      /* three parts */
    run_case(60, 5, 2, 0, 50);       /* specific construction with padding */
    if (g_fail) {
        printf("%d checks failed\n", g_fail);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
