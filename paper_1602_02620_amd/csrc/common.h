// Shared definitions of the gfx950 Fast CoveringLSH library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fclsh.h"

namespace fclsh {

// Mersenne prime 2^31 - 1: the modulus of the Eq. (1) universal hash.
constexpr uint32_t kPrime = 0x7FFFFFFFu;
// Largest per-part Hadamard order handled by the kernels: D = 2^(r'+1) <= 4096.
constexpr int kMaxLogD = 12;
constexpr int kMaxParts = 64;
constexpr int kMaxDims = 4096;
// Coordinates of points given by their nonzeros.  The sketch of such a point
// sums at most d even representatives b'' < 2^32, so S'' < 2^51 and every
// FHT value and S'' - F''_v (< 2^52) stay exact integers in fp64, with the
// key extraction's exponent fixed at 2^52.
constexpr int kMaxSparseDims = 1 << 19;

void set_error(const char *fmt, ...);
fclsh_status fail(fclsh_status st, const char *fmt, ...);

#define FCLSH_HIP(expr)                                                        \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::fclsh::fail(FCLSH_EDEVICE, "%s failed: %s (%s:%d)", #expr, \
                                 hipGetErrorString(e_), __FILE__, __LINE__);   \
    } while (0)

#define FCLSH_TRY(expr)                                                        \
    do {                                                                       \
        fclsh_status s_ = (expr);                                              \
        if (s_ != FCLSH_OK)                                                    \
            return s_;                                                         \
    } while (0)

inline int words_of(int d) { return (d + 63) / 64; }

inline int ilog2_ceil(uint64_t x) {
    int k = 0;
    while ((uint64_t(1) << k) < x) ++k;
    return k;
}

// Host-side parameters of one index (Alg. 1 + Alg. 2 draws).
// d: dimensions of the points; rep: copies of every point the family is
// built on (Alg. 1's replication; 1 = none), so the family's coordinates
// are the dd() = rep * d bits of the replicated point, coordinate c' reading
// bit c' mod d.  part, col and b have dd() entries.
struct Params {
    int d = 0, r = 0, t = 1, rp = 0, rep = 1;
    bool sparse = false;  // points given by their nonzero coordinates (d up to kMaxSparseDims)
    std::vector<int32_t> part, col;
    std::vector<uint64_t> b;
    int dd() const { return rep * d; }
    int D() const { return 1 << (rp + 1); }
    int Lp() const { return D() - 1; }
    int L() const { return t * Lp(); }
};

fclsh_status derive_params(int d, int r, uint64_t seed, const fclsh_build_opts *opts,
                           Params *out, bool sparse = false);
fclsh_status check_params(const Params &p);

// ----------------------------------------------------------------------------
// Device allocation with a byte budget.
// ----------------------------------------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Per-part gather plan of the hash kernel (see hash.hip).
struct HashPlan {
    int logD = 1, logV = 1, G = 1, V = 2, U = 64, t = 1, E = 0, W = 1;
    bool specific = true;        // at most one coordinate per Hadamard column
    int32_t *seg = nullptr;      // [t][V+1] entry ranges per in-lane column k
    uint2 *gtab = nullptr;       // [t][E][G] (even representative of b mod P, coordinate)
    uint2 *coord = nullptr;      // sparse points: [d] (even representative, part << 16 | column)
};

// Points given by their nonzero coordinates: row i holds cols[ptr[i] ..
// ptr[i+1]), ascending and distinct, each below d; ptr[0] = 0 and
// ptr[m] = nnz.  Kernels clamp every row to [0, nnz) and skip columns
// outside [0, d), so malformed rows give wrong answers, never stray accesses;
// csr_check reports them.
struct CsrRows {
    const int64_t *ptr = nullptr;
    const int32_t *cols = nullptr;
    int64_t nnz = 0;
};

// Launch shape of the batched verify kernels, chosen by the autotuner.
struct QueryTuning {
    int tile = 256;          // bucket entries per work item / spill chunk
    int blocks_per_cu = 8;   // persistent workgroups per CU
    int schedule = 0;        // kScheduleStatic or kScheduleClaim
};
// How the persistent verification waves share the work: a fixed stride
// (wave g takes rounds g, g + G, ...) or claims from a counter in the batch's
// control block (a wave takes kClaimRounds rounds of items, or kClaimChunks
// spill chunks, per atomic).
constexpr int kScheduleStatic = 0;
constexpr int kScheduleClaim = 1;
constexpr int kClaimRounds = 2;
constexpr int kClaimChunks = 4;

// Pass 2's group kernel form of a build (identical tables in every one):
//   kFull      slot and ballot branches (every index's first build);
//   kSlotOnly  slot branch, groups with a bin over kMaxFastBin entries left
//              to the second kernel;
//   kSlotAll   slot branch for every group up to the tile, bin sizes not
//              checked (right for any bin, slow on large ones).
enum class BuildMode { kFull, kSlotOnly, kSlotAll };

struct Index {
    Params prm;
    QueryTuning tuning;
    int num_cus = 256;
    BuildMode build_mode = BuildMode::kFull;  // for the next build (see build_tables_2pass)
    int W = 1;
    int64_t n = 0;
    int dir_bits = 1;
    int device = 0;
    uint64_t budget = 0;
    HashPlan plan;
    uint64_t *pts = nullptr;   // [n][W]
    void *tkeys = nullptr;     // [L][n] of key_bytes each (the low 16 bits, or the whole key)
    int key_bytes = 4;
    bool p2_fallback = false;  // tests: pass 2 takes its fallbacks (FCLSH_TEST_P2_FALLBACK)
    uint32_t *tids = nullptr;  // [L][n]
    uint32_t *dir = nullptr;   // [L][2^dir_bits + 1]
    // per-index device copies of part/col for the duplicate-elimination rule
    uint32_t *dpc = nullptr;  // part(c) << 16 | column(c) per coordinate
    // sparse points (prm.sparse): the index's copy of the rows, pts unused
    int64_t *sptr = nullptr;   // [n+1]
    int32_t *scols = nullptr;  // [nnz]
    int64_t nnz = 0;
    std::vector<DevBuf> owned;
    size_t bytes_owned = 0;
};

fclsh_status dev_alloc(Index *ix, void **p, size_t bytes, const char *what);
void dev_free_all(Index *ix);

// ----------------------------------------------------------------------------
// Kernels (launchers)
// ----------------------------------------------------------------------------
fclsh_status build_hash_plan(Index *ix);
fclsh_status launch_hash(const Index &ix, const uint64_t *pts, int64_t m, uint32_t *keys,
                         int64_t key_stride, hipStream_t st);
// The same keys for m points given by their nonzeros (a sparse index).
fclsh_status launch_hash_sparse(const Index &ix, const CsrRows &rows, int64_t m, uint32_t *keys, int64_t key_stride,
                                hipStream_t st);
// Checks m CSR rows over d coordinates on the device: ORs the kCsrBad* bits
// found, shifted left by `shift`, into *flag (device word, not cleared here).
constexpr uint32_t kCsrBadPtr = 1u;     // ptr[0] != 0, ptr[m] != nnz or a row ends before it starts
constexpr uint32_t kCsrBadCol = 2u;     // a column outside [0, d)
constexpr uint32_t kCsrBadOrder = 4u;   // a row's columns not strictly ascending
fclsh_status csr_check(const CsrRows &rows, int64_t m, int d, uint32_t *flag, int shift, hipStream_t st);
// The m rows as bit vectors of words_of(d) words each (out: m * words_of(d)
// words, overwritten).
fclsh_status csr_densify(const CsrRows &rows, int64_t m, int d, uint64_t *out, hipStream_t st);

// Workgroups are handed to the 8 XCDs (each with its own L2) in turn.  The
// streaming kernels map workgroup b of a 1-D grid (a multiple of kXcds) to
// work item (b % 8) * (grid / 8) + b / 8, so each XCD takes a contiguous range
// of items in order: writes of neighbouring items that share cache lines (the
// runs of one digit from neighbouring pass-1 tiles, the boundaries of
// neighbouring super-bins, the row segments of neighbouring point groups)
// meet in the same L2, which merges them before they go to HBM.
constexpr int kXcds = 8;

__device__ inline int64_t xcd_contiguous_item(unsigned b, unsigned grid) {
    return int64_t(b % kXcds) * (grid / kXcds) + b / kXcds;
}

inline int64_t xcd_grid(int64_t nitems) { return (nitems + kXcds - 1) / kXcds * kXcds; }

// Table build (tables.hip): keys [L][n] -> tables grouped by the top dir_bits
// key bits, ids ascending per bin, plus the directory [L][2^dir_bits + 1].
// keys is consumed (reused as a buffer).  marks (optional, 6 events) are
// recorded on st after each of: pass-1 histogram, pass-1 scan, pass-1
// scatter, pass-1b split (recorded also when the split is not needed),
// pass-2 group kernel, pass-2 kernel for large groups.
int table_dir_bits(int64_t n);
int table_split_bits(int64_t n, int dir_bits);
int table_merge_bits(int64_t n, int dir_bits);
size_t table_build_scratch_bytes(int64_t L, int64_t n, int dir_bits);
fclsh_status build_tables_2pass(uint32_t *keys, int64_t L, int64_t n, int dir_bits, uint32_t *tmpk, uint32_t *tmpv,
                                uint32_t *scratch, void *tkeys, uint32_t *tids, uint32_t *dir, BuildMode mode,
                                bool p2_fallback, hipStream_t st, hipEvent_t *marks = nullptr);
// Bytes per stored table key: 2 when the key bits below the directory bin
// (31 - dir_bits) fit 16 bits, so that a bin's keys are told apart by their
// low 16 bits, else 4.
int table_key_bytes(int dir_bits);
// Whether the passes hand on 6-byte entries (16-bit stored keys, no merged
// pass-2 groups, ids below 2^25) instead of 8-byte ones.
bool table_packed_pass1(int64_t n, int dir_bits);
// Whole 31-bit keys of tables [T0, T1) into out [T1-T0][n] (the bin bits
// from the directory), on st.
fclsh_status expand_table_keys(const void *tkeys, int key_bytes, const uint32_t *dir, int64_t n, int dir_bits, int T0,
                               int T1, uint32_t *out, hipStream_t st);
// Pass 2's counters in the scratch after a build: [0] groups listed for the
// second kernel, [1] groups that took the ballot branch.
const uint32_t *table_build_counts(const uint32_t *scratch, int64_t L, int64_t n, int dir_bits);

// Device-side control block of one query batch.
struct QueryCtrl {
    unsigned long long spills;      // spill chunks recorded
    unsigned long long pairs;       // reported (query, id) pairs
    unsigned long long total;       // pairs, as published with the offsets
    uint32_t status;                // kQuery*Overflow bits
    uint32_t nlong;                 // segments the sort hands to its long-segment kernel
    unsigned long long claim_items; // claimed item rounds x 64 (claim schedule)
    unsigned long long claim_spill; // claimed spill chunks (claim schedule)
};
constexpr uint32_t kQueryPairOverflow = 1u;
constexpr uint32_t kQuerySpillOverflow = 2u;
constexpr uint32_t kQueryIdsOverflow = 4u;
// the sparse queries failed csr_check (its bits shifted by kQueryBadShift)
constexpr int kQueryBadShift = 3;
constexpr uint32_t kQueryBadRows = (kCsrBadPtr | kCsrBadCol | kCsrBadOrder) << kQueryBadShift;

// Scratch of the query path for one index and stream, grown on demand.
struct QueryWorkspace {
    uint32_t *qkeys = nullptr, *rstart = nullptr, *rlen = nullptr, *rmatch = nullptr;
    uint32_t *qcount = nullptr, *qfill = nullptr;
    uint64_t *qcount64 = nullptr, *scan_part = nullptr, *offs1 = nullptr;
    QueryCtrl *ctrl = nullptr;
    uint32_t *pq = nullptr, *pid = nullptr, *sorttmp = nullptr;
    uint4 *spill = nullptr;
    uint64_t *qdense = nullptr;  // sparse queries as bit vectors
    uint32_t *seen = nullptr;    // sparse queries: an n-bit bitmap per query (points already checked)
    int64_t cap_items = 0, cap_q = 0, cap_pairs = 0, cap_spill = 0, cap_qdense = 0, cap_seen = 0;
    // a synchronous batch whose ids did not fit the caller's buffer: its
    // pairs stay here until the next query call on the stream
    int64_t pending_nq = -1, pending_total = 0;
    const uint64_t *pending_offsets = nullptr;
};

fclsh_status ws_reserve(QueryWorkspace &ws, int64_t nq, int L, int64_t pairs, int64_t spills,
                        int64_t dense_words = 0, int64_t seen_words = 0);
void ws_release(QueryWorkspace &ws);
// A workspace laid out in one caller-owned device buffer (no allocation).
fclsh_status ws_carve(QueryWorkspace &ws, void *base, size_t bytes, int64_t nq, int L);
// Device bytes the workspace holds.
uint64_t ws_bytes(const QueryWorkspace &ws);
// queries: dense [nq][W] words, or null with sq the queries' rows (sparse
// index).
fclsh_status query_batch_async(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, int rq,
                               const int32_t *rq_vec, hipStream_t st, uint64_t *offsets, uint32_t *ids,
                               int64_t ids_cap, const CsrRows *sq = nullptr);
fclsh_status query_batch(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, int rq,
                         const int32_t *rq_vec, hipStream_t st, uint64_t *offsets, uint32_t *ids, int64_t ids_cap,
                         int64_t *total_out, const CsrRows *sq = nullptr);
fclsh_status query_finish(Index &ix, QueryWorkspace &ws, hipStream_t st, const uint64_t *offsets, uint32_t *ids,
                          int64_t ids_cap, int64_t *total_out);
fclsh_status query_plain(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, int rq,
                         hipStream_t st, uint64_t *offsets, uint32_t *ids, int64_t ids_cap, int64_t *total_out);
fclsh_status query_collisions(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq,
                              uint64_t *coll, hipStream_t st);
fclsh_status query_cost(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, uint64_t *coll,
                        uint64_t *cand, hipStream_t st, const CsrRows *sq = nullptr);
// Exclusive scan of n uint64 (in place allowed) using caller-provided
// partials (scan_partials_needed(n) entries): no allocation, graph-safe.
int64_t scan_partials_needed(int64_t n);
fclsh_status exclusive_scan_u64_ws(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *partials,
                                   hipStream_t st);
const char *last_error_cstr();
// Linear scan (linear.hip): CSR of every point within r of each query, ids
// ascending; synchronises st once for the result size.
fclsh_status linear_scan(const uint64_t *pts, int64_t n, int d, const uint64_t *qs, int64_t nq, int r,
                         hipStream_t st, uint64_t *offsets, uint32_t *ids, int64_t ids_cap, int64_t *total_out);

}  // namespace fclsh
