/*
 * Plain CPU oracle for Fast CoveringLSH (Pham & Pagh, "Scalability and Total
 * Recall with Fast CoveringLSH", arXiv:1602.02620).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes is the plain definition that Fast CoveringLSH reaches
 * exactly (Lemma 3): the basic CoveringLSH masks g_v of Eq. (2) / Eq. (5),
 * turned into integer bucket keys by the universal hash of Eq. (1), O(d L)
 * work per point.  On top of that: hash tables of non-empty buckets
 * (Sec. 2.2), the Strategy-2 query with an n-bit bitmap for duplicate
 * removal (Sec. 2.2 and Steps S1-S3 of Sec. 4.1), and a linear scan
 * (Sec. 4.2) as ground truth; for points given by their nonzero
 * coordinates, the keys and the linear scan over the nonzeros.  No blocking, fusion or reordering beyond what
 * those definitions state.
 *
 * Conventions (the paper is silent on them; each is a stated reading):
 *  - A point of d bits is W = ceil(d/64) uint64 words, coordinate c being
 *    bit (c & 63) of word (c >> 6).  The paper's 1-indexed string position k
 *    is coordinate k-1.
 *  - Hadamard code convention of Eq. (3): with a(j) the binary representation
 *    of the integer j, C[v][j] = <a(j), v> mod 2 = popcount(v & j) mod 2.
 *    This reproduces the printed matrix C_{7,8} of Sec. 3.1.1.
 *  - A coordinate c belongs to part part[c] (Alg. 1 partitioning; a single
 *    part when no partitioning is done) and is mapped to Hadamard column
 *    col[c] in [0, D), D = 2^(r'+1).  Table (p, v), v = 1..D-1, has index
 *    T = p*(D-1) + (v-1).  Row v = 0 is the all-zero codeword and is never a
 *    table (Alg. 2 removes the first hash value).
 *  - Random draws (the permutation of Alg. 1, the mapping or permutation m of
 *    Alg. 2, the seed vector b) come from SplitMix64 (Steele, Lea and Flood,
 *    "Fast splittable pseudorandom number generators", OOPSLA 2014) used as a
 *    counter-based generator, with unbiased bounded draws by rejection.  The
 *    paper fixes no generator, so this part has no pin beyond agreement with
 *    an independent implementation ("parity unpinned").
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Random draws                                                              */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output number k (k = 0, 1, ...) for a generator whose state
 * starts at `seed`: the state after k+1 steps of adding the golden-gamma
 * constant, passed through the published finaliser. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t seed;
    uint64_t k;
} orc_rng;

/* A uniform integer in [0, s), s >= 1: draws below 2^64 mod s are rejected so
 * that every residue is equally likely. */
static uint64_t orc_bounded(orc_rng *g, uint64_t s)
{
    uint64_t threshold = (0 - s) % s;
    for (;;) {
        uint64_t u = orc_splitmix64(g->seed, g->k++);
        if (u >= threshold)
            return u % s;
    }
}

/* Uniform random permutation of [0, len) in `perm` (Fisher-Yates, swapping
 * position i with a uniform position in [0, i], for i from len-1 down to 1). */
static void orc_shuffle(orc_rng *g, int32_t *perm, int32_t len)
{
    for (int32_t i = 0; i < len; i++)
        perm[i] = i;
    for (int32_t i = len - 1; i >= 1; i--) {
        int32_t j = (int32_t)orc_bounded(g, (uint64_t)i + 1);
        int32_t tmp = perm[i];
        perm[i] = perm[j];
        perm[j] = tmp;
    }
}

/* ------------------------------------------------------------------------ */
/* Parameters (Alg. 1 pre-processing; the random draws of Alg. 2)            */
/* ------------------------------------------------------------------------ */

/* Number of parts t.  The experiments (Sec. 4.1 parameter settings and
 * Sec. 4.3) use no pre-processing for r < 10 and 2 partitions for r >= 10;
 * an explicit positive override wins. */
int orc_parts_for_radius(int r, int override_t)
{
    if (override_t > 0)
        return override_t;
    return r < 10 ? 1 : 2;
}

/* Draws the index parameters from `seed`.
 *
 *  t       : number of parts (orc_parts_for_radius).
 *  r'      : floor(r / t), the per-part radius (pigeonhole, Sec. 3.1.2).
 *  D       : 2^(r'+1) Hadamard columns, L' = D - 1 tables per part.
 *  pi      : with t > 1 a uniform permutation of the d coordinates (Alg. 1
 *            "randomly permute"), else the identity (no draws).
 *  parts   : part p holds the coordinates at positions
 *            [p*floor(d/t), (p+1)*floor(d/t)) of pi; the last part also
 *            takes the remainder up to d (Alg. 1, contiguous split).
 *  col     : per part, in pi order.  If the part has d_p <= D coordinates
 *            (specific construction of Alg. 2) its coordinates take the
 *            first d_p entries of a uniform permutation of [0, D); otherwise
 *            (general construction, Eq. (5), Alg. 2) each coordinate
 *            takes an independent uniform column in [0, D).
 *  b       : b[c] uniform in [0, P) for c = 0..d-1 (the seed vector of Eq. (1)).
 *
 * Draw order: pi, then the columns part by part, then b.
 * Returns 0, or -1 on bad arguments (r' + 1 > 20 is refused). */
int orc_derive_params(int d, int r, uint64_t seed, int override_t, uint64_t P,
                      int skip_col0, int32_t *t_out, int32_t *rpart_out,
                      int32_t *part, int32_t *col, uint64_t *b)
{
    if (d <= 0 || r < 0 || P < 2)
        return -1;
    int t = orc_parts_for_radius(r, override_t);
    if (t > d)
        return -1;
    int rp = r / t;
    if (rp + 1 > 20)
        return -1;
    int32_t D = 1 << (rp + 1);
    /* Sec. 3.3 variant: the map m takes values in the columns other than
     * column 0, so there are D - 1 of them, numbered from 1 */
    int32_t ncol = skip_col0 ? D - 1 : D;
    int32_t first = skip_col0 ? 1 : 0;
    orc_rng g = {seed, 0};

    int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)d);
    if (t > 1) {
        orc_shuffle(&g, pi, d);
    } else {
        for (int c = 0; c < d; c++)
            pi[c] = c;
    }
    int32_t block = d / t;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    for (int p = 0; p < t; p++) {
        int32_t lo = p * block;
        int32_t hi = (p == t - 1) ? d : (p + 1) * block;
        int32_t dp = hi - lo;
        if (dp <= ncol) {
            orc_shuffle(&g, perm, ncol);
            for (int32_t k = 0; k < dp; k++) {
                part[pi[lo + k]] = p;
                col[pi[lo + k]] = first + perm[k];
            }
        } else {
            for (int32_t k = 0; k < dp; k++) {
                part[pi[lo + k]] = p;
                col[pi[lo + k]] = first + (int32_t)orc_bounded(&g, (uint64_t)ncol);
            }
        }
    }
    for (int c = 0; c < d; c++)
        b[c] = orc_bounded(&g, P);
    free(perm);
    free(pi);
    *t_out = t;
    *rpart_out = rp;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Basic CoveringLSH masks (Eq. (2), Eq. (5))                                */
/* ------------------------------------------------------------------------ */

static int orc_parity(uint32_t x)
{
    return __builtin_popcount(x) & 1;
}

/* mask[T*d + c] = 1 iff coordinate c is in part p and <m(c), v> = 1, i.e.
 * the Hadamard codeword of v has a one in column col[c]; T = p*(D-1)+(v-1). */
void orc_masks(int d, int t, int rp, const int32_t *part, const int32_t *col,
               uint8_t *mask)
{
    int32_t D = 1 << (rp + 1);
    for (int p = 0; p < t; p++)
        for (int32_t v = 1; v < D; v++) {
            int64_t T = (int64_t)p * (D - 1) + (v - 1);
            for (int c = 0; c < d; c++)
                mask[T * d + c] =
                    (part[c] == p) && orc_parity((uint32_t)v & (uint32_t)col[c]);
        }
}

/* ------------------------------------------------------------------------ */
/* Integer bucket keys (Eq. (1) applied to g_v(x) = g_v AND x)               */
/* ------------------------------------------------------------------------ */

static int orc_bit(const uint64_t *x, int c)
{
    return (int)((x[c >> 6] >> (c & 63)) & 1ULL);
}

/* key = sum over coordinates c with x_c = 1 and mask bit 1 of b_c, mod P. */
static uint64_t orc_key_one(const uint64_t *x, int d, const uint8_t *mask_row,
                            const uint64_t *b, uint64_t P)
{
    uint64_t s = 0;
    for (int c = 0; c < d; c++)
        if (orc_bit(x, c) && mask_row[c])
            s = (s + b[c]) % P;
    return s;
}

/* Keys of the points listed in `which` (npick entries) for all ntab tables:
 * keys[T*npick + i] = key of point which[i] in table T.  `which` may be NULL,
 * meaning points 0..npick-1. */
void orc_keys(const uint64_t *points, int d, const int64_t *which, int64_t npick,
              int ntab, const uint8_t *mask, const uint64_t *b, uint64_t P,
              uint32_t *keys)
{
    int W = (d + 63) / 64;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < npick; i++) {
        int64_t id = which ? which[i] : i;
        const uint64_t *x = points + id * W;
        for (int T = 0; T < ntab; T++)
            keys[(int64_t)T * npick + i] =
                (uint32_t)orc_key_one(x, d, mask + (int64_t)T * d, b, P);
    }
}

/* The same keys for points given by their nonzero coordinates (Sec. 3.2's
 * sparse setting): point i has the coordinates cols[ptr[i] .. ptr[i+1]) set
 * and no others.  The key of table T = p*(D-1)+(v-1) sums b_c over the set
 * coordinates c of part p whose Hadamard column has <col[c], v> = 1, i.e.
 * over the set coordinates under the mask g_v, mod P: Eq. (1) restricted to
 * the nonzeros, O(nnz L) per point.  keys[T*m + i] for the m points. */
void orc_keys_sparse(const int64_t *ptr, const int32_t *cols, int64_t m,
                     int t, int rp, const int32_t *part, const int32_t *col,
                     const uint64_t *b, uint64_t P, uint32_t *keys)
{
    int32_t D = 1 << (rp + 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; i++) {
        for (int p = 0; p < t; p++)
            for (int32_t v = 1; v < D; v++) {
                uint64_t s = 0;
                for (int64_t e = ptr[i]; e < ptr[i + 1]; e++) {
                    int32_t c = cols[e];
                    if (part[c] == p && orc_parity((uint32_t)v & (uint32_t)col[c]))
                        s = (s + b[c]) % P;
                }
                int64_t T = (int64_t)p * (D - 1) + (v - 1);
                keys[T * m + i] = (uint32_t)s;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Hash tables of non-empty buckets (Sec. 2.2)                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t key;
    uint32_t id;
} orc_pair;

static int orc_pair_cmp(const void *a, const void *b)
{
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    if (x->id != y->id)
        return x->id < y->id ? -1 : 1;
    return 0;
}

/* Each table T becomes the n pairs (key, id) sorted by key, then id.  A
 * bucket is the run of equal keys.  Output: tkeys[T*n+i], tids[T*n+i]. */
void orc_tables(const uint32_t *keys, int64_t n, int ntab, uint32_t *tkeys,
                uint32_t *tids)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int T = 0; T < ntab; T++) {
        orc_pair *pr = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
        for (int64_t i = 0; i < n; i++) {
            pr[i].key = keys[(int64_t)T * n + i];
            pr[i].id = (uint32_t)i;
        }
        qsort(pr, (size_t)n, sizeof(orc_pair), orc_pair_cmp);
        for (int64_t i = 0; i < n; i++) {
            tkeys[(int64_t)T * n + i] = pr[i].key;
            tids[(int64_t)T * n + i] = pr[i].id;
        }
        free(pr);
    }
}

/* ------------------------------------------------------------------------ */
/* Queries                                                                   */
/* ------------------------------------------------------------------------ */

/* Hamming distance over the d coordinates (bits of the last word beyond d
 * are not coordinates and are ignored). */
static int orc_hamming(const uint64_t *x, const uint64_t *y, int d)
{
    int s = 0;
    for (int w = 0; w < d / 64; w++)
        s += __builtin_popcountll(x[w] ^ y[w]);
    if (d & 63) {
        uint64_t keep = (1ULL << (d & 63)) - 1;
        s += __builtin_popcountll((x[d / 64] ^ y[d / 64]) & keep);
    }
    return s;
}

/* First index in the sorted array a[0..n) whose value is >= key. */
static int64_t orc_lower_bound(const uint32_t *a, int64_t n, uint32_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

static int orc_u32_cmp(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y);
}

/* Strategy 2 for one query (Sec. 2.2), as the three steps of Sec. 4.1:
 *  S1  the query's key in every table (qkeys[T], computed by the caller);
 *  S2  every point in the query's bucket of each table, T in increasing
 *      order, is a collision; a bitmap of n bits keeps the first sighting of
 *      each point, which makes it a distinct candidate;
 *  S3  a distinct candidate at Hamming distance <= rq is reported.
 * Reported ids are returned ascending in out (capacity n).  Returns |out|. */
static int64_t orc_query_one(const uint64_t *points, int64_t n, int d,
                             const uint32_t *tkeys, const uint32_t *tids,
                             int ntab, const uint32_t *qkeys,
                             const uint64_t *q, int rq, uint8_t *bitmap,
                             uint32_t *out, int64_t *collisions,
                             int64_t *candidates)
{
    int W = (d + 63) / 64;
    int64_t nout = 0, ncoll = 0, ncand = 0;
    memset(bitmap, 0, (size_t)((n + 7) / 8));
    for (int T = 0; T < ntab; T++) {
        const uint32_t *tk = tkeys + (int64_t)T * n;
        const uint32_t *ti = tids + (int64_t)T * n;
        for (int64_t j = orc_lower_bound(tk, n, qkeys[T]); j < n && tk[j] == qkeys[T]; j++) {
            uint32_t id = ti[j];
            ncoll++;
            if (bitmap[id >> 3] & (1u << (id & 7)))
                continue;
            bitmap[id >> 3] |= (uint8_t)(1u << (id & 7));
            ncand++;
            if (orc_hamming(points + (int64_t)id * W, q, d) <= rq)
                out[nout++] = id;
        }
    }
    qsort(out, (size_t)nout, sizeof(uint32_t), orc_u32_cmp);
    *collisions = ncoll;
    *candidates = ncand;
    return nout;
}

/* Strategy-2 queries for a batch.  qkeys[T*nq + i] are the S1 keys of query
 * i.  Results: counts[i] reported ids of query i, written ascending at
 * out + i*cap (cap >= the largest possible answer, at most n).
 * collisions[i] / candidates[i] are the #Collisions / #Candidates counters of
 * Sec. 4.1. */
void orc_query_batch(const uint64_t *points, int64_t n, int d,
                     const uint32_t *tkeys, const uint32_t *tids, int ntab,
                     const uint64_t *queries, int64_t nq, const uint32_t *qkeys,
                     int rq, int64_t cap, uint32_t *out, int64_t *counts,
                     int64_t *collisions, int64_t *candidates)
{
    int W = (d + 63) / 64;
#pragma omp parallel
    {
        uint8_t *bitmap = (uint8_t *)malloc((size_t)((n + 7) / 8 + 1));
        uint32_t *qk = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(ntab > 0 ? ntab : 1));
        uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < nq; i++) {
            for (int T = 0; T < ntab; T++)
                qk[T] = qkeys[(int64_t)T * nq + i];
            int64_t c = orc_query_one(points, n, d, tkeys, tids, ntab, qk,
                                      queries + i * W, rq, bitmap, tmp,
                                      &collisions[i], &candidates[i]);
            counts[i] = c;
            memcpy(out + i * cap, tmp, sizeof(uint32_t) * (size_t)(c < cap ? c : cap));
        }
        free(tmp);
        free(qk);
        free(bitmap);
    }
}

/* Linear scan (Sec. 4.2 ground truth): ids of all points at Hamming distance
 * <= rq from each query, ascending, with the same output layout as
 * orc_query_batch. */
void orc_brute_force(const uint64_t *points, int64_t n, int d,
                     const uint64_t *queries, int64_t nq, int rq, int64_t cap,
                     uint32_t *out, int64_t *counts)
{
    int W = (d + 63) / 64;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nq; i++) {
        int64_t c = 0;
        for (int64_t id = 0; id < n; id++)
            if (orc_hamming(points + id * W, queries + i * W, d) <= rq) {
                if (c < cap)
                    out[i * cap + c] = (uint32_t)id;
                c++;
            }
        counts[i] = c;
    }
}

/* Linear scan over points given by their nonzero coordinates (as in
 * orc_keys_sparse; d coordinates): the Hamming distance of two such points is
 * the size of the symmetric difference of their coordinate sets,
 * |X| + |Q| - 2 |X and Q|, the intersection counted with a d-entry marker of
 * the query's coordinates.  Same output layout as orc_brute_force. */
void orc_brute_force_sparse(const int64_t *ptr, const int32_t *cols, int64_t n,
                            const int64_t *qptr, const int32_t *qcols, int64_t nq,
                            int d, int rq, int64_t cap, uint32_t *out, int64_t *counts)
{
#pragma omp parallel
    {
        uint8_t *mark = (uint8_t *)calloc((size_t)(d > 0 ? d : 1), 1);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < nq; i++) {
            int64_t nqi = qptr[i + 1] - qptr[i];
            for (int64_t e = qptr[i]; e < qptr[i + 1]; e++)
                mark[qcols[e]] = 1;
            int64_t c = 0;
            for (int64_t id = 0; id < n; id++) {
                int64_t both = 0;
                for (int64_t e = ptr[id]; e < ptr[id + 1]; e++)
                    both += mark[cols[e]];
                int64_t dist = (ptr[id + 1] - ptr[id]) + nqi - 2 * both;
                if (dist <= rq) {
                    if (c < cap)
                        out[i * cap + c] = (uint32_t)id;
                    c++;
                }
            }
            counts[i] = c;
            for (int64_t e = qptr[i]; e < qptr[i + 1]; e++)
                mark[qcols[e]] = 0;
        }
        free(mark);
    }
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0)
        omp_set_num_threads(k);
#else
    (void)k;
#endif
}
