/*
 * fclsh.h -- C ABI of the MI355X (gfx950) Fast CoveringLSH library.
 *
 * Fast CoveringLSH (Pham & Pagh, "Scalability and Total Recall with Fast
 * CoveringLSH", arXiv:1602.02620) answers r-near-neighbour *reporting* in
 * Hamming space exactly (Def. 2 with delta = 0): a query returns every data
 * point within Hamming distance r, with no false negatives.  The index holds
 * L = t * (2^(r'+1) - 1) hash tables; a point's L bucket keys are computed in
 * O(d + L log L) with the fast Hadamard transform (Alg. 2) instead of the
 * O(d L) of the basic CoveringLSH masks (Eq. (2), Eq. (1)).
 *
 * Conventions shared by every call:
 *  - Points and queries are bit vectors of d coordinates, packed row-major as
 *    W = ceil(d/64) uint64 words per vector; coordinate c is bit (c & 63) of
 *    word (c >> 6).  Bits beyond d in the last word are ignored.
 *  - A sparse index (fclsh_build_index_sparse) takes its points and queries
 *    as rows of nonzero coordinates instead (the "_sparse" calls, layout
 *    given there); every call on bit vectors rejects it with FCLSH_EINVAL,
 *    and every "_sparse" call rejects a dense index.
 *  - Pointers named d_* are DEVICE pointers (HIP device memory of the current
 *    device); all others are host pointers.  Input buffers stay owned by the
 *    caller and are only read during the call (and, for asynchronous calls,
 *    until the work on `stream` has finished).  The index copies what it
 *    keeps.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    enqueue their kernels on it and return; a call that must read a size
 *    back to the host (query result sizes, oversize-bucket detection in the
 *    build) synchronises that stream.
 *  - Every call returns FCLSH_OK (0) or a negative status; the thread-local
 *    fclsh_last_error() then describes the failure.  On failure no output is
 *    valid and no index is created.
 *  - The keys use the Mersenne prime P = 2^31 - 1 (a reading of the paper's
 *    "sufficiently large prime"; P affects only false bucket merges, never
 *    recall).
 */
#ifndef FCLSH_H
#define FCLSH_H

#include <stdint.h>

/* The library is built with hidden visibility; only these calls are exported. */
#define FCLSH_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fclsh_status;

#define FCLSH_OK 0
#define FCLSH_EINVAL (-1)      /* bad argument (size, radius, pointer)          */
#define FCLSH_ERADIUS (-2)     /* query radius larger than the index radius    */
#define FCLSH_ENOMEM (-3)      /* device allocation failed or over the budget  */
#define FCLSH_ECAPACITY (-4)   /* output buffer too small; *total_out is set   */
#define FCLSH_EDEVICE (-5)     /* HIP runtime error                            */
#define FCLSH_EUNSUPPORTED (-6)/* parameters the GPU kernels do not cover      */

/* Opaque, immutable once built; may be queried from several streams. */
typedef struct fclsh_index_s *fclsh_index;

/* An instantiated HIP graph of one batched query (fclsh_query_graph_create). */
typedef struct fclsh_graph_s *fclsh_graph;

/* Build options.  struct_size must be sizeof(fclsh_build_opts) as the caller
 * was compiled with it (FCLSH_BUILD_OPTS_INIT sets it): the library reads
 * only the fields that lie inside struct_size and gives the others their
 * defaults, so a caller built against an older, shorter struct keeps working.
 * struct_size 0, or larger than the library's struct, is FCLSH_EINVAL.  With
 * every other field zero the options are the paper's defaults. */
typedef struct {
    uint32_t struct_size;      /* sizeof(fclsh_build_opts)                         */
    int32_t partitions;        /* t; 0 = the experiments' rule: 1 if r < 10 else 2
                                  (Sec. 4.1 parameter settings, Sec. 4.3)          */
    int32_t replicate;         /* Alg. 1's first branch: 0 or 1 = none; k > 1 builds
                                  the family on k copies of every point (the
                                  replicated point has k*d coordinates, k*d <= 4096,
                                  and distances grow k-fold, so the radius becomes
                                  k*r with one part; partitions must be 0 or 1)   */
    int32_t exclude_column0;   /* nonzero: the coordinate map never targets column 0
                                  (the all-zero column), the variant of Sec. 3.3
                                  with the sharper bound on expected collisions;
                                  a part is then specific when it has at most
                                  D - 1 coordinates                               */
    uint64_t prime;            /* 0 or 2^31-1 (the only prime the kernels support) */
    uint64_t mem_budget_bytes; /* 0 = no limit; else the build fails with
                                  FCLSH_ENOMEM if the index and its build scratch
                                  would exceed it                                  */
    int32_t keep_build_scratch;/* nonzero: keep the build's scratch (3 uint32 per
                                  table entry plus histograms) resident after the
                                  build, for rebuilds; 0 = release it when the
                                  build ends (a later rebuild allocates it again
                                  and keeps it)                                    */
    int32_t test_flags;        /* 0; for tests only, bit 0 (FCLSH_TEST_P2_FALLBACK):
                                  the table build treats the id-order check of
                                  every pass-2 group as failed, so that its
                                  fallbacks run; other bits are FCLSH_EINVAL      */
} fclsh_build_opts;

#define FCLSH_TEST_P2_FALLBACK 1

#define FCLSH_BUILD_OPTS_INIT {(uint32_t)sizeof(fclsh_build_opts), 0, 0, 0, 0, 0, 0, 0}

/* ---------------------------------------------------------------------------
 * Index parameters (host only, no device work).
 *
 * Alg. 1 (pre-processing) with the experiments' choice of t, and the random
 * draws of Alg. 2: per part a mapping m into the 2^(r'+1) Hadamard columns
 * (general construction, Eq. (5), when the part has more than 2^(r'+1)
 * coordinates) or a random permutation of the columns (specific construction,
 * 0-padded), and the seed vector b in [P]^d of Eq. (1).  r' = floor(r/t).
 *
 * Draws come from SplitMix64 seeded with `seed` (counter-based: output k is
 * the finaliser applied to seed + (k+1) * 0x9E3779B97F4A7C15), unbiased
 * bounded draws by rejection, in the order: the coordinate permutation
 * (only if t > 1; Fisher-Yates from the last position down), then per part
 * its column permutation (Fisher-Yates of [0, 2^(r'+1))) or its i.i.d.
 * columns in permuted-coordinate order, then b[0..d).  Part p is positions
 * [p*floor(d/t), (p+1)*floor(d/t)) of the permutation, the last part taking
 * the remainder.
 *
 * With opts->replicate = k > 1 (Alg. 1, first branch) the draws are those
 * of d' = k*d coordinates and radius k*r with t = 1: coordinate c' of the
 * replicated point is copy c' / d of coordinate c' mod d.
 *
 * Outputs (host arrays of d' entries, d' = d without replication): part[c]
 * in [0,t), col[c] in [0, 2^(r'+1)), b[c] in [0, P).  *t_out and
 * *r_part_out receive t and r'.  d up to 4096 (replicated: d' up to 4096)
 * for indexes on bit vectors, up to 2^19 for sparse indexes (whose draws are
 * the same; replication is not offered for them).
 * Errors: FCLSH_EINVAL (d <= 0, r < 0, null pointer), FCLSH_EUNSUPPORTED
 * (r' > 11, t > 64 or t > d, prime other than 2^31-1).
 * ------------------------------------------------------------------------- */
/* Alg. 1's choice of pre-processing for n points, radius r and
 * approximation ratio c, with log taken base 2 (the keys' bits): when
 * c*r < log n the points are replicated k = floor(log n / (c*r)) times
 * (*replicate = k, *partitions = 1); when c*r > log n they are split into
 * t = ceil(c*r / log n) parts (*replicate = 1, *partitions = t); when c*r
 * equals log n neither (1, 1).  The results go into fclsh_build_opts.
 * Errors: FCLSH_EINVAL (n < 2, r <= 0, c <= 1 or not a number, null
 * pointer). */
FCLSH_API fclsh_status fclsh_preprocessing(int64_t n, int32_t r, double c,
                                           int32_t *replicate, int32_t *partitions);

FCLSH_API fclsh_status fclsh_derive_params(int32_t d, int32_t r, uint64_t seed,
                                 const fclsh_build_opts *opts, int32_t *t_out,
                                 int32_t *r_part_out, int32_t *part, int32_t *col,
                                 uint64_t *b);

/* ---------------------------------------------------------------------------
 * Build an index over n points (Def. 2: the data structure over S).
 *
 * d_points: device, n*W uint64 (layout above).  n in [1, 2^31-1].
 * d in [1, 4096], r >= 0; parameters from fclsh_derive_params(d, r, seed);
 * at most 65535 tables.
 * The build hashes every point into its L keys (Alg. 2), then buckets each
 * table (hash tables of non-empty buckets, Sec. 2.2): every table is stored
 * as its n (key, id) pairs grouped by directory bin (the top dir_bits bits of
 * the 31-bit key), ids ascending within a bin, with the directory of bin
 * starts.  A bucket (equal keys) lies inside one bin; keys within a bin are
 * not sorted.  The index keeps a copy of the points for the distance
 * checks of queries.  Index memory is allocated by the library on the current
 * device and released by fclsh_index_free.
 * Errors: FCLSH_EINVAL, FCLSH_EUNSUPPORTED, FCLSH_ENOMEM, FCLSH_EDEVICE.
 * ------------------------------------------------------------------------- */
FCLSH_API fclsh_status fclsh_build_index(const uint64_t *d_points, int64_t n, int32_t d,
                               int32_t r, uint64_t seed,
                               const fclsh_build_opts *opts, void *stream,
                               fclsh_index *out);

/* Same, with explicit parameters instead of a seed: t parts, per-part radius
 * r_part, host arrays part[d] (every part non-empty), col[d] < 2^(r_part+1)
 * and b[d] < prime.  Covering (Theorem 1) holds for every mapping and Lemma 3
 * for every b, so any such arrays index radius r as long as the pigeonhole
 * split of Sec. 3.1.2 leaves some part with at most r_part differences:
 * floor(r/t) <= r_part (else FCLSH_EINVAL).  prime must be 0 or 2^31-1.
 * Errors as fclsh_build_index. */
FCLSH_API fclsh_status fclsh_build_index_with_params(const uint64_t *d_points, int64_t n,
                                           int32_t d, int32_t r, int32_t t,
                                           int32_t r_part, const int32_t *part,
                                           const int32_t *col, const uint64_t *b,
                                           uint64_t prime, void *stream,
                                           fclsh_index *out);

/* ---------------------------------------------------------------------------
 * Sparse high-dimensional points (the bag-of-words and rating data of
 * Sec. 4, where Alg. 2 costs O(nnz + L log L) per point: its sketch only
 * sums over the nonzero coordinates).
 *
 * Rows: d_ptr (device, m+1 int64) and d_cols (device, nnz int32); row i is
 * the point whose coordinates d_cols[d_ptr[i] .. d_ptr[i+1]) are 1 and all
 * others 0.  d_ptr[0] = 0, d_ptr[m] = nnz, non-decreasing; each row's columns
 * strictly ascending and in [0, d).  nnz < 2^31.  d in [1, 2^19] (so a
 * point's sketch stays below 2^51 and the FHT exact in fp64).
 *
 * fclsh_build_index_sparse: as fclsh_build_index (same parameters for the
 * same d, r, seed and opts; opts->replicate must be 0 or 1).  The rows are
 * checked first (one device pass and a synchronisation); malformed rows give
 * FCLSH_EINVAL.  The index keeps its own copy of the rows (8 (n+1) + 4 nnz
 * bytes in place of the bit vectors).
 * Errors: FCLSH_EINVAL, FCLSH_EUNSUPPORTED, FCLSH_ENOMEM, FCLSH_EDEVICE.
 * ------------------------------------------------------------------------- */
FCLSH_API fclsh_status fclsh_build_index_sparse(const int64_t *d_ptr, const int32_t *d_cols,
                                                int64_t n, int64_t nnz, int32_t d, int32_t r,
                                                uint64_t seed, const fclsh_build_opts *opts,
                                                void *stream, fclsh_index *out);

/* Alg. 2 on m rows: their L keys under the index's family, laid out as in
 * fclsh_hash (d_keys: device [L][m] uint32), equal to the keys of the same
 * points given as bit vectors.  Asynchronous; rows are not checked (a row is
 * clamped to [0, nnz) and columns outside [0, d) are skipped, so malformed
 * rows give meaningless keys, never stray memory accesses).  Sparse index
 * only. */
FCLSH_API fclsh_status fclsh_hash_sparse(fclsh_index idx, const int64_t *d_ptr,
                                         const int32_t *d_cols, int64_t m, int64_t nnz,
                                         uint32_t *d_keys, void *stream);

/* fclsh_query_batch for nq queries given as rows (sparse index only): the
 * same outputs, ids ascending per query, and the same FCLSH_ECAPACITY
 * protocol (fclsh_query_batch_finish applies).  The rows are checked on the
 * device within the batch; malformed rows give FCLSH_EINVAL.  The stream's
 * workspace also holds the queries as bit vectors (nq * ceil(d/64) words). */
FCLSH_API fclsh_status fclsh_query_batch_sparse(fclsh_index idx, const int64_t *d_ptr,
                                                const int32_t *d_cols, int64_t nq, int64_t nnz,
                                                int32_t r_query, void *stream,
                                                uint64_t *d_offsets, uint32_t *d_ids,
                                                int64_t ids_capacity, int64_t *total_out);

/* fclsh_query_cost for nq query rows (sparse index only): Sec. 4.1's
 * #Collisions and #Candidates per query, the measures of the paper's sparse
 * experiments.  The rows are checked first (FCLSH_EINVAL if malformed).
 * Synchronises `stream`. */
FCLSH_API fclsh_status fclsh_query_cost_sparse(fclsh_index idx, const int64_t *d_ptr,
                                               const int32_t *d_cols, int64_t nq, int64_t nnz,
                                               void *stream, uint64_t *d_collisions,
                                               uint64_t *d_candidates);

/* ---------------------------------------------------------------------------
 * Exact r-NN reporting for a batch of queries (Def. 2, Strategy 2 of
 * Sec. 2.2 with Steps S1-S3 of Sec. 4.1): for each query, every data point id
 * at Hamming distance <= r_query, ids ascending.
 *
 * d_queries: device, nq*W uint64.  nq >= 0 with nq * L < 2^32 (else
 * FCLSH_EINVAL; split larger batches).  0 <= r_query <= the index's r (an
 * r-covering family covers every smaller radius); larger r_query gives
 * FCLSH_ERADIUS.
 * Output (device, caller-owned): d_offsets[nq+1] uint64 CSR offsets and
 * d_ids[ids_capacity] uint32; query i's neighbours are
 * d_ids[d_offsets[i] .. d_offsets[i+1]).  *total_out (host) receives the
 * total number of reported ids.  If it exceeds ids_capacity the call returns
 * FCLSH_ECAPACITY with *total_out set and d_ids untouched (d_offsets is
 * written); fclsh_query_batch_finish then writes the ids into a larger
 * buffer without recomputing them.
 * The call synchronises `stream` once, to read the result size.
 * Duplicate elimination: a verified near point is reported only from the
 * first table (in (part, v) order) whose mask it shares with the query;
 * covering guarantees that table exists and that the point lies in the
 * query's bucket there, so each neighbour is reported exactly once.
 * ------------------------------------------------------------------------- */
FCLSH_API fclsh_status fclsh_query_batch(fclsh_index idx, const uint64_t *d_queries,
                               int64_t nq, int32_t r_query, void *stream,
                               uint64_t *d_offsets, uint32_t *d_ids,
                               int64_t ids_capacity, int64_t *total_out);

/* Release an index (NULL is ignored).  The caller must make sure no work using
 * it is still queued.  A graph captured on the index (fclsh_query_graph_create)
 * keeps the index's memory alive: with graphs still alive the index only
 * becomes unusable (every later call on it fails with FCLSH_EINVAL) and its
 * memory is released when the last of its graphs is freed. */
FCLSH_API void fclsh_index_free(fclsh_index idx);

/* Thread-local description of the last failure ("" if none). */
FCLSH_API const char *fclsh_last_error(void);

/* ---------------------------------------------------------------------------
 * Hot-path pieces, exported for tests and measurement.
 * ------------------------------------------------------------------------- */

/* Shape of a built index. Any output pointer may be NULL.  dir_bits: the
 * directory's bin width B (bins = top B key bits); group_bits: the key bits
 * that form the groups of the table build's last pass (8; more for large n,
 * where a middle pass splits the 256 super-bins further; fewer for small n,
 * where the last pass merges neighbouring super-bins). */
FCLSH_API fclsh_status fclsh_index_info(fclsh_index idx, int32_t *d, int32_t *r,
                              int32_t *t, int32_t *r_part, int64_t *n,
                              int32_t *L, int32_t *dir_bits, int32_t *group_bits);

/* Device memory held by an index, in bytes (any output pointer may be NULL):
 * *index_bytes = what answering queries needs (the point copy, the tables,
 * the directory and the hash parameters); *build_scratch_bytes = the table
 * build's scratch, held only when the index keeps it (keep_build_scratch, or
 * after a rebuild); *workspace_bytes = the query workspaces of every stream
 * that has queried the index, and of its live graphs.  Host only. */
FCLSH_API fclsh_status fclsh_index_memory(fclsh_index idx, uint64_t *index_bytes,
                                          uint64_t *build_scratch_bytes, uint64_t *workspace_bytes);

/* The parameters an index was built with (host arrays of d' entries: d
 * times the replication, see fclsh_derive_params). */
FCLSH_API fclsh_status fclsh_index_params(fclsh_index idx, int32_t *part, int32_t *col,
                                uint64_t *b);

/* Alg. 2 on a batch: the L keys of m points under the index's hash family.
 * d_pts: device m*W uint64; d_keys: device [L][m] uint32, key of point i in
 * table T = p*(2^(r'+1)-1) + (v-1) at d_keys[T*m + i] (v = 1..2^(r'+1)-1:
 * the all-zero first Hadamard row is dropped).  Asynchronous on `stream`. */
FCLSH_API fclsh_status fclsh_hash(fclsh_index idx, const uint64_t *d_pts, int64_t m,
                        uint32_t *d_keys, void *stream);

/* Device pointers of the index's tables: keys [L][n] of *key_bytes bytes
 * each and ids [L][n] uint32 (table T at offset T*n, grouped by directory
 * bin, ids ascending within a bin; see fclsh_build_index), directory
 * [L][2^dir_bits + 1] uint32 (start of the entries whose key has the given
 * top dir_bits bits of 31) and the point copy [n][W] uint64 (NULL for a
 * sparse index).  A key is stored whole (key_bytes 4) or, when the 31 -
 * dir_bits key bits below the bin fit 16 bits (dir_bits >= 15, n >= 2^17),
 * as its low 16 bits (key_bytes 2): the bin supplies the rest
 * (fclsh_index_table_keys writes whole keys).  Owned by the index; read
 * only.  Any output pointer may be NULL. */
FCLSH_API fclsh_status fclsh_index_tables(fclsh_index idx, const void **d_tkeys,
                                int32_t *key_bytes, const uint32_t **d_tids,
                                const uint32_t **d_dir, const uint64_t **d_points);

/* Whole 31-bit keys of tables [T0, T1) into d_keys (device, [T1-T0][n]
 * uint32), in the tables' order; asynchronous on `stream`.  Errors:
 * FCLSH_EINVAL (released index, range outside [0, L], null output). */
FCLSH_API fclsh_status fclsh_index_table_keys(fclsh_index idx, int32_t T0, int32_t T1,
                                              uint32_t *d_keys, void *stream);

/* Rebuild the tables of an existing index from its own points (the bucketing
 * step alone: hash + table build), for timing.  Synchronises `stream`. */
FCLSH_API fclsh_status fclsh_index_rebuild(fclsh_index idx, void *stream);

/* The same rebuild, enqueued on `stream` without waiting for it: later work
 * on `stream` (queries, table reads) sees the new tables.  It may wait for
 * the previous build of the index to finish (it reads that build's pass-2
 * counters, see fclsh_index_rebuild_timed).  The index must not be used on
 * another stream until `stream` has passed this point.  Errors as
 * fclsh_index_rebuild. */
FCLSH_API fclsh_status fclsh_index_rebuild_async(fclsh_index idx, void *stream);

/* The same rebuild with HIP events recorded on `stream` around each kernel.
 * phase_ms[0..6] (host, nphase >= 7) receive the durations in ms of: the key
 * computation of Alg. 2 for all points and tables, the pass-1 histogram, the
 * pass-1 scan, the pass-1 scatter, the pass-1b split (0 when n is small
 * enough not to need it), the pass-2 group kernel (every group of the
 * table of at most 4608 entries) and the pass-2 kernel for larger groups.
 * The group kernel has a full form and a slot-only form (faster, but it
 * leaves groups with a bin over 48 entries to the second kernel) and a
 * slot-all form; fclsh_index_build_mode tells which the rebuild takes.  All
 * give identical tables.
 * Errors: FCLSH_EINVAL for a short phase_ms, FCLSH_EDEVICE for HIP errors.
 * Synchronises `stream`. */
FCLSH_API fclsh_status fclsh_index_rebuild_timed(fclsh_index idx, void *stream, float *phase_ms,
                                                 int32_t nphase);

/* The form of pass 2's group kernel that the index's next rebuild takes,
 * written to *mode (host):
 *   0  full: slot and ballot branches (every index's first build);
 *   1  slot-only: groups with a bin over 48 entries go to the second kernel;
 *   2  slot-all: the slot branch for every group up to 4608 entries, bin
 *      sizes not checked (its ranking is right for any bin, slow on large
 *      ones).
 * A rebuild hashes the same points with the same functions as the last
 * build, whose pass-2 counters decide: slot-all when no group left the slot
 * branch, slot-only when at most 1 % did, else full.  Every form gives the
 * same tables.  Waits for the last build's counters if an asynchronous
 * rebuild is still running.  Errors: FCLSH_EINVAL (null argument),
 * FCLSH_EDEVICE. */
FCLSH_API fclsh_status fclsh_index_build_mode(fclsh_index idx, int32_t *mode);

/* Per-query diagnostics of Sec. 4.1: #Collisions (summed sizes of the query's
 * L buckets) for each query, written to device d_collisions[nq] (uint64).
 * Asynchronous. */
FCLSH_API fclsh_status fclsh_query_collisions(fclsh_index idx, const uint64_t *d_queries,
                                    int64_t nq, void *stream,
                                    uint64_t *d_collisions);

/* Both cost measures of Sec. 4.1 per query (device uint64 outputs of nq
 * entries): d_collisions[i] = #Collisions, the summed sizes of query i's L
 * buckets (what C_lookup is proportional to); d_candidates[i] = #Candidates,
 * the number of distinct points among them (what C_check is proportional
 * to).  Duplicates are removed as the paper does, with an n-bit bitmap per
 * query (queries are processed in chunks whose bitmaps fit 256 MB).  A
 * diagnostic pass next to fclsh_query_batch, which needs neither counter.
 * Allocates the bitmaps; synchronises `stream`.  Errors: FCLSH_EINVAL,
 * FCLSH_ENOMEM, FCLSH_EDEVICE. */
FCLSH_API fclsh_status fclsh_query_cost(fclsh_index idx, const uint64_t *d_queries, int64_t nq,
                                        void *stream, uint64_t *d_collisions, uint64_t *d_candidates);

/* Linear scan, the baseline of the paper's evaluation (Sec. 4) and the
 * ground truth its recall is measured against: for each query, every point
 * at Hamming distance <= r, ids ascending, without any index.  d_points:
 * device n*W uint64 (n in [1, 2^31-1]); d_queries: device nq*W uint64, nq in
 * [0, 65535].  Outputs and FCLSH_ECAPACITY as fclsh_query_batch.  Allocates
 * per-call tile counts (16 bytes per query and 4096 points); synchronises
 * `stream`.  Errors: FCLSH_EINVAL, FCLSH_ENOMEM, FCLSH_ECAPACITY,
 * FCLSH_EDEVICE. */
FCLSH_API fclsh_status fclsh_linear_scan(const uint64_t *d_points, int64_t n, int32_t d,
                                         const uint64_t *d_queries, int64_t nq, int32_t r, void *stream,
                                         uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                                         int64_t *total_out);

/* The plain path: one query at a time, each answered by its own launch
 * sequence (hash, lookup and verify, compaction) and a synchronisation; the
 * baseline the batched path is measured against.  Same outputs and errors as
 * fclsh_query_batch. */
FCLSH_API fclsh_status fclsh_query_plain(fclsh_index idx, const uint64_t *d_queries,
                               int64_t nq, int32_t r_query, void *stream,
                               uint64_t *d_offsets, uint32_t *d_ids,
                               int64_t ids_capacity, int64_t *total_out);

/* Completes the last fclsh_query_batch or fclsh_query_batch_radii call on
 * `stream` that returned FCLSH_ECAPACITY: the pairs it found stay in the
 * stream's workspace, and this call scatters and sorts them into d_ids
 * (device, ids_capacity uint32) with no new verification.  d_offsets must be
 * the offsets array that call wrote (its contents are used as written).
 * *total_out (host) receives the total.  Errors: FCLSH_EINVAL if no such call
 * is pending on `stream` (any other query call, reserve or collision count on
 * the stream in between discards it) or d_offsets differs; FCLSH_ECAPACITY if
 * ids_capacity is still too small (the batch stays pending).  Synchronises
 * `stream`. */
FCLSH_API fclsh_status fclsh_query_batch_finish(fclsh_index idx, void *stream, const uint64_t *d_offsets,
                                                uint32_t *d_ids, int64_t ids_capacity, int64_t *total_out);

/* ---------------------------------------------------------------------------
 * Batching and serving (batched execution of Strategy 2 for many queries).
 * ------------------------------------------------------------------------- */

/* As fclsh_query_batch, with one radius per query: d_radii (device, nq int32,
 * each in [0, max_radius]) and max_radius <= the index's r (else
 * FCLSH_ERADIUS).  Queries of different radii share one launch sequence. */
FCLSH_API fclsh_status fclsh_query_batch_radii(fclsh_index idx, const uint64_t *d_queries, int64_t nq,
                                               const int32_t *d_radii, int32_t max_radius, void *stream,
                                               uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                                               int64_t *total_out);

/* Sizes the query workspace of `stream` for up to max_nq queries per batch,
 * pair_capacity reported (query, id) pairs and spill_capacity chunks of large
 * buckets (see fclsh_query_batch_async).  Allocates; synchronises `stream`.
 * Call before fclsh_query_batch_async or graph capture. */
FCLSH_API fclsh_status fclsh_query_reserve(fclsh_index idx, int64_t max_nq, int64_t pair_capacity,
                                           int64_t spill_capacity, void *stream);

/* The batched pipeline without any host synchronisation or allocation:
 * hash, bucket lookup, verification by persistent waves that stride over the
 * (query, table) items and then over a device queue of chunks of the larger
 * buckets (a bucket larger than the tuned tile is split into tile-sized
 * chunks), CSR offsets and per-query sorting, all enqueued on
 * `stream`.  The workspace of `stream` must have been reserved for nq
 * queries.  r_query applies to all queries unless d_radii (device, nq int32)
 * is given.  Outputs as fclsh_query_batch, plus d_result (device, 2 uint64):
 * [0] = total reported ids, [1] = status bits: 1 pair buffer overflow,
 * 2 spill queue overflow (reserve more and rerun), 4 ids_capacity too small
 * (d_offsets valid, d_ids not written).  Capturable in a HIP graph. */
FCLSH_API fclsh_status fclsh_query_batch_async(fclsh_index idx, const uint64_t *d_queries, int64_t nq,
                                               int32_t r_query, const int32_t *d_radii, void *stream,
                                               uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                                               uint64_t *d_result);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fclsh_query_batch_async with the same arguments, outputs and status bits,
 * but its workspace (query keys, per-query counters, scan partials, control
 * block, spill queue, result pairs) is laid out in one fixed array of 64 MiB
 * that the library holds in static device memory on each GPU it runs on,
 * until the process ends.  The call allocates and frees nothing.  The query
 * keys and per-query counters take 4*L + 16 bytes per query (plus alignment);
 * a quarter of the rest holds spill chunks (16 B each) and the remainder
 * result pairs (12 B each).  A batch whose fixed part does not fit is
 * rejected with FCLSH_ENOMEM before anything is enqueued; one whose pairs or
 * spill chunks overflow what is left reports it in d_result's status bits
 * (1 pairs, 2 spill), as fclsh_query_batch_async does.  Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents (the
 * counters are cleared by the call's own kernels): calls whose work overlaps
 * on one GPU, on any streams, race and must be serialised by the caller.
 * The first call on a device looks up the array's address there. */
FCLSH_API fclsh_status fclsh_query_batch_noalloc(fclsh_index idx, const uint64_t *d_queries, int64_t nq,
                                                 int32_t r_query, const int32_t *d_radii, void *stream,
                                                 uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                                                 uint64_t *d_result);

/* Captures fclsh_query_batch_async with these fixed buffers into a HIP graph
 * on `stream` (which must not be the null stream) and instantiates it.
 * Replaying it (fclsh_graph_launch) answers whatever queries d_queries holds
 * at that time.  The stream's workspace must be reserved first (for at least
 * nq queries); the graph gets a private copy of that workspace of the same
 * capacities, so later calls on the stream (which may grow its workspace)
 * never touch the graph's buffers.  The graph keeps the index alive (see
 * fclsh_index_free).  Allocates; synchronises `stream`. */
FCLSH_API fclsh_status fclsh_query_graph_create(fclsh_index idx, const uint64_t *d_queries, int64_t nq,
                                                int32_t r_query, const int32_t *d_radii, uint64_t *d_offsets,
                                                uint32_t *d_ids, int64_t ids_capacity, uint64_t *d_result,
                                                void *stream, fclsh_graph *out);
FCLSH_API fclsh_status fclsh_graph_launch(fclsh_graph graph, void *stream);
FCLSH_API void fclsh_graph_free(fclsh_graph graph);

/* Launch shape of the batched verification: tile = bucket entries per work
 * item and per spill chunk (64 .. 2^20), blocks_per_cu = persistent
 * workgroups per compute unit (1 .. 64). */
FCLSH_API fclsh_status fclsh_index_set_tuning(fclsh_index idx, int32_t tile, int32_t blocks_per_cu);
FCLSH_API fclsh_status fclsh_index_get_tuning(fclsh_index idx, int32_t *tile, int32_t *blocks_per_cu);

/* How the persistent verification waves share a batch's work (an
 * implementation choice, no passage of the paper): 0 = a fixed stride (wave
 * g of G takes rounds of 64 items g, g + G, ... and spill chunks likewise),
 * 1 = claims from counters in the batch's control block (2 rounds of items,
 * or 4 spill chunks, per atomic), which evens out uneven bucket sizes at the
 * price of the atomics.  Both give identical answers.  Errors: FCLSH_EINVAL
 * (released index, schedule not 0 or 1, null pointer). */
FCLSH_API fclsh_status fclsh_index_set_schedule(fclsh_index idx, int32_t schedule);
FCLSH_API fclsh_status fclsh_index_get_schedule(fclsh_index idx, int32_t *schedule);

/* Autotuner: times the batched pipeline on a sample batch (device queries)
 * for a grid of (tile, blocks_per_cu, schedule) and keeps the fastest on the
 * index (the schedule chosen is read with fclsh_index_get_schedule); the
 * choice is also cached for later indexes of the same shape (d, t, r',
 * ceil(log2 n)) on the same device.  Each shape first runs once through the
 * synchronous path, which grows the stream's workspace until the run is
 * complete; a timed run that still reports an overflow is not a candidate.
 * Outputs (optional): the chosen values and its time per batch in ms.
 * Errors: FCLSH_EDEVICE if no shape completes or a HIP call fails (the
 * index keeps its previous shape).  Synchronises `stream`. */
FCLSH_API fclsh_status fclsh_autotune(fclsh_index idx, const uint64_t *d_queries, int64_t nq,
                                      int32_t r_query, void *stream, int32_t *tile_out,
                                      int32_t *blocks_out, float *best_ms_out);

#ifdef __cplusplus
}
#endif

#endif /* FCLSH_H */
