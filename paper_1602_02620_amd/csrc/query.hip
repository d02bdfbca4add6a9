// Queries: Strategy 2 of Sec. 2.2 as the three steps of Sec. 4.1.
//
//   S1  the query's L keys, by the same Alg. 2 kernel as the build
//   S2  per table, the query's directory bin; the entries of the bin whose
//       key equals the query's form its bucket (#Collisions = their count)
//   S3  every colliding point is checked by popcount(x XOR q) <= r_query
//
// Duplicate elimination without per-query state.  The paper removes
// duplicates with an n-bit bitmap per query; a batch of thousands of queries
// in flight cannot afford that.  Instead a verified near point x is reported
// only from one table: the first table (part p, row v) in which x and q agree
// on all masked coordinates, i.e. v is orthogonal over GF(2) to the column
// m_p(c) of every coordinate c of part p where x and q differ.  Such a table
// exists whenever d(x, q) <= r (covering, Theorem 1, with the pigeonhole
// split of Alg. 1), equal masked values give equal keys, so x lies in q's
// bucket of that table and is reported there and nowhere else.  The set of
// such v within a part is a linear subspace; its smallest non-zero element
// is found by keeping a basis with distinct leading bits while the
// constraints are added, then taking the basis vector with the lowest
// leading bit.
//
// The batched pipeline runs on the device without a host round trip, so a
// whole batch can be captured in a HIP graph:
//   hash -> verify (each lane takes one (query, table) item: it probes the
//   directory and, when the bin holds at most kLaneBin entries, scans it and
//   verifies the bucket itself; a larger bin is cut into `tile`-sized chunks
//   on a spill queue) -> spill (persistent waves verify one chunk at a time,
//   a lane per entry) -> CSR offsets -> scatter into per-query segments ->
//   per-query sort (ids ascending).  Small buckets thus cost one lane, not one
//   wave, and skewed buckets (1 to 1e5 candidates) spread over all CUs.
//   Counters are cleared by fill kernels, never by memset nodes, so graph
//   replays start clean.
#include <algorithm>

#include "common.h"

namespace fclsh {

namespace {

// First table (in (part, v) order) where x and q share the masked value, or
// -1 if there is none (then d(x, q) exceeds what the family covers).
// pc[c] = part(c) << 16 | column(c) (the verification kernels stage it in
// LDS).
// With replication (rep copies of every point, Alg. 1), the family's
// coordinates are the rep * d0 bits of the replicated point: a differing bit
// c differs in every copy, and each copy i constrains by its own column
// pc[i * d0 + c].
// Restricts the basis B (distinct leading bits) to the v with <v, uc> = 0:
// the odd vector with the lowest leading bit is dropped and XORed into the
// other odd ones (their leading bits are higher, so they stay distinct).
__device__ inline void constrain_basis(uint32_t (&B)[kMaxLogD], uint32_t uc) {
    int star = -1;
    uint32_t bs = 0;
#pragma unroll
    for (int l = 0; l < kMaxLogD; ++l) {
        if (B[l] && (__popc(B[l] & uc) & 1)) {
            if (star < 0) {
                star = l;
                bs = B[l];
                B[l] = 0u;
            } else {
                B[l] ^= bs;
            }
        }
    }
}

__device__ int first_shared_table(const uint64_t *__restrict__ x, const uint64_t *__restrict__ q, int W,
                                  const uint32_t *__restrict__ pc, int t, int mbits, int Lp, uint64_t last_mask,
                                  int d0, int rep) {
    for (int p = 0; p < t; ++p) {
        uint32_t B[kMaxLogD];
#pragma unroll
        for (int l = 0; l < kMaxLogD; ++l) B[l] = l < mbits ? (1u << l) : 0u;
        for (int w0 = 0; w0 < W; w0 += 4) {
            // four words per round trip (clamped indexes, as in the Hamming
            // test), one when the vectors have one word
            uint64_t dw[4];
            if (W == 1) {
                dw[0] = x[0] ^ q[0];
                dw[1] = dw[2] = dw[3] = 0ull;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int w = min(w0 + j, W - 1);
                    dw[j] = x[w] ^ q[w];
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int w = w0 + j;
                uint64_t diff = w < W ? dw[j] : 0ull;
                if (w == W - 1) diff &= last_mask;
                while (diff) {
                    const int c0 = w * 64 + __builtin_ctzll(diff);
                    diff &= diff - 1;
                    for (int i = 0, c = c0; i < rep; ++i, c += d0) {
                        const uint32_t pcc = pc[c];
                        if (int(pcc >> 16) == p) constrain_basis(B, pcc & 0xFFFFu);
                    }
                }
            }
        }
#pragma unroll
        for (int l = 0; l < kMaxLogD; ++l)
            if (B[l]) return p * Lp + int(B[l]) - 1;
    }
    return -1;
}

// The same for a point x and a query q given by their ascending coordinate
// lists: the coordinates where they differ are those in exactly one list
// (one merge per part).  Query columns outside [0, d) are skipped.
__device__ int first_shared_table_sparse(const int32_t *__restrict__ xs, int nx, const int32_t *__restrict__ qs,
                                         int nq, const uint32_t *__restrict__ pc, int t, int mbits, int Lp, int d) {
    for (int p = 0; p < t; ++p) {
        uint32_t B[kMaxLogD];
#pragma unroll
        for (int l = 0; l < kMaxLogD; ++l) B[l] = l < mbits ? (1u << l) : 0u;
        int i = 0, j = 0;
        while (i < nx || j < nq) {
            const int32_t a = i < nx ? xs[i] : 0x7FFFFFFF;
            const int32_t b = j < nq ? qs[j] : 0x7FFFFFFF;
            int32_t c;
            if (a == b) {
                ++i;
                ++j;
                continue;
            }
            if (a < b) {
                c = a;
                ++i;
            } else {
                c = b;
                ++j;
            }
            if (uint32_t(c) >= uint32_t(d)) continue;
            const uint32_t pcc = pc[c];
            if (int(pcc >> 16) == p) constrain_basis(B, pcc & 0xFFFFu);
        }
#pragma unroll
        for (int l = 0; l < kMaxLogD; ++l)
            if (B[l]) return p * Lp + int(B[l]) - 1;
    }
    return -1;
}

struct VerifyArgs {
    const uint64_t *pts;
    int W, d, t, mbits, Lp, L;
    int d0, rep;  // dimensions of a point and copies per point (d = rep * d0 staged words)
    uint64_t last_mask;
    const uint32_t *pc;  // part << 16 | column per coordinate (global; staged in LDS per workgroup)
    const uint64_t *queries;  // [nq][W] bit vectors (sparse queries: densified)
    int64_t nq;
    // sparse index: the points' rows and the queries' rows (pts unused)
    const int64_t *xptr, *qptr;
    const int32_t *xcols, *qcols;
    int64_t qnnz;
    // the paper's duplicate elimination (an n-bit bitmap per query, seen_wpq
    // words each), or null: the first-shared-table rule
    uint32_t *seen;
    int64_t seen_wpq;
    const int32_t *rq_vec;  // per-query radius, or null: rq for all
    int rq;
    const void *tkeys;  // [L][n] KT: the low 16 bits of the keys, or the keys (key_bytes 2 or 4)
    const uint32_t *tids, *dir;
    int64_t n;
    int dir_bits;
    const uint32_t *qkeys;  // [L][nq]
    QueryCtrl *ctrl;
    uint4 *spill;  // (item, begin, end, 0): absolute positions in the item's table
    int64_t spill_cap;
    uint32_t *out_q, *out_id;
    int64_t pair_cap;
    uint32_t *qcount;
    uint32_t tile;
    int table_major;  // item numbering, see item_coords
    int schedule;     // kScheduleStatic or kScheduleClaim
};

// (query, table) of a verification item.  Large batches number the items
// table-major (it = T * nq + qi), so that neighbouring lanes read
// neighbouring query keys of one table ([L][nq] layout); small batches
// number them query-major (it = qi * L + T), which touches fewer distinct
// directory lines per wave when the query keys are few anyway.  nq * L < 2^32.
__device__ inline void item_coords(const VerifyArgs &a, uint32_t it, int64_t &qi, int &T) {
    if (a.table_major) {
        const uint32_t t = it / uint32_t(a.nq);
        T = int(t);
        qi = int64_t(it - t * uint32_t(a.nq));
    } else {
        const uint32_t q = it / uint32_t(a.L);
        qi = int64_t(q);
        T = int(it - q * uint32_t(a.L));
    }
}

// Bins of at most this many entries are scanned by one lane.
constexpr uint32_t kLaneBin = 32;
static_assert(kLaneBin <= 32, "a lane keeps the matches of its bin in a 32-bit mask");
// Batches of more queries number their items table-major.
constexpr int64_t kTableMajorBatch = 2048;

__device__ inline int query_radius(const VerifyArgs &a, int64_t qi) { return a.rq_vec ? a.rq_vec[qi] : a.rq; }

// popcount(x XOR q) over the W words (pad bits masked).  The words are
// loaded four at a time (indexes clamped to the last word, which is then
// masked out), so a candidate costs one round trip per four words rather
// than one per word.
__device__ inline int hamming(const uint64_t *x, const uint64_t *q, int W, uint64_t last_mask) {
    if (W == 1) return __popcll((x[0] ^ q[0]) & last_mask);
    int dist = 0;
    for (int w0 = 0; w0 < W; w0 += 4) {
        uint64_t xw[4], qw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int w = min(w0 + j, W - 1);
            xw[j] = x[w];
            qw[j] = q[w];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint64_t df = xw[j] ^ qw[j];
            if (w0 + j == W - 1) df &= last_mask;
            dist += w0 + j < W ? __popcll(df) : 0;
        }
    }
    return dist;
}

// Reported pairs are staged per wave in LDS (kPairBuf of them) and copied to
// the pair buffer when the stage is full and when the wave ends, each copy
// reserving exactly its slots with one atomic.  A batch reports up to millions
// of pairs, and one counter shared by every emitting wave round serialised
// that many atomics on one address.  The stage count is read and written with
// wavefront-scope atomics: lanes that skipped an earlier emission must still
// see its count.
constexpr uint32_t kPairBuf = 256;
constexpr int kVerifyWaves = 4;  // waves per verification workgroup

struct PairStage {
    uint32_t *q, *id, *count;  // this wave's slice of the workgroup's LDS
};

__device__ inline uint32_t stage_count(const PairStage &ps) {
    return __hip_atomic_load(ps.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Copies the c staged pairs out; called by the active lanes of the wave.
__device__ inline void flush_pairs(const VerifyArgs &a, const PairStage &ps, uint32_t c) {
    const int lane = threadIdx.x & 63;
    const uint64_t act = __ballot(1);
    const int leader = __builtin_ctzll(act);
    const uint32_t k = uint32_t(__popcll(act));
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned long long base = 0;
    if (lane == leader && c) base = atomicAdd(&a.ctrl->pairs, (unsigned long long)c);
    base = __shfl(base, leader, 64);
    for (uint32_t j = uint32_t(__popcll(act & lt)); j < c; j += k) {
        const unsigned long long slot = base + j;
        if (slot < (unsigned long long)a.pair_cap) {
            a.out_q[slot] = ps.q[j];
            a.out_id[slot] = ps.id[j];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
}

// Records (qi, id) for the lanes of the wave that call it together, plus one
// count atomic per distinct query among them (the calling lanes mostly share
// one or two queries).
__device__ inline void emit_pair(const VerifyArgs &a, const PairStage &ps, int64_t qi, uint32_t id) {
    const int lane = threadIdx.x & 63;
    const uint64_t act = __ballot(1);
    const uint32_t n = uint32_t(__popcll(act));
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint32_t c = stage_count(ps);
    if (c + n > kPairBuf) {
        flush_pairs(a, ps, c);
        c = 0;
    }
    const uint32_t j = c + uint32_t(__popcll(act & lt));
    const uint32_t q32 = uint32_t(qi);  // nq * L < 2^32
    ps.q[j] = q32;
    ps.id[j] = id;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __hip_atomic_store(ps.count, c + n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    for (uint64_t rem = act; rem;) {
        const int l = __builtin_ctzll(rem);
        const uint32_t q0 = uint32_t(__shfl(int(q32), l, 64));
        const uint64_t same = __ballot(q32 == q0) & rem;
        if (lane == l) atomicAdd(&a.qcount[q0], uint32_t(__popcll(same)));
        rem &= ~same;
    }
}

// Sparse index: |x| + |q| - 2 |x and q| <= rq, the common coordinates
// counted by testing x's coordinates against q's bit vector (independent
// loads, four at a time), after the length filter ||x| - |q|| <= rq.  After
// j of x's coordinates with c common, the distance is at least (j - c) (x's
// misses so far) + max(0, |q| - c - (|x| - j)) (q's coordinates that x can no
// longer match): the test stops as soon as that exceeds rq.
__device__ inline bool within_sparse(const VerifyArgs &a, int64_t qi, int rq, uint32_t id, int64_t &xb, int &nx,
                                     int64_t &qb, int &nqi) {
    xb = a.xptr[id];
    nx = int(a.xptr[int64_t(id) + 1] - xb);  // the index's own rows, checked at build
    qb = min(max(a.qptr[qi], int64_t(0)), a.qnnz);
    nqi = int(min(max(a.qptr[qi + 1], qb), a.qnnz) - qb);
    if (abs(nx - nqi) > rq) return false;
    const uint64_t *qw = a.queries + qi * a.W;
    const int32_t *xs = a.xcols + xb;
    int common = 0;
    for (int e0 = 0; e0 < nx; e0 += 4) {
        int32_t c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = xs[min(e0 + k, nx - 1)];
        uint64_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = qw[c[k] >> 6];
#pragma unroll
        for (int k = 0; k < 4; ++k) common += (e0 + k < nx) ? int((w[k] >> (c[k] & 63)) & 1ull) : 0;
        const int j = min(e0 + 4, nx);
        if ((j - common) + max(0, nqi - common - (nx - j)) > rq) return false;
    }
    return nx + nqi - 2 * common <= rq;
}

// First sighting of point id by query qi in the per-query bitmap (the
// paper's duplicate elimination): true exactly once per (query, point), for
// whichever table reaches it first.
__device__ inline bool first_sighting(const VerifyArgs &a, int64_t qi, uint32_t id) {
    const uint32_t bit = 1u << (id & 31);
    return !(atomicOr(a.seen + qi * a.seen_wpq + (id >> 5), bit) & bit);
}

// Checks one bin entry j of table T against query qi: same key, within the
// query's radius, and T is the first table the two share (dedupe).
template <bool SPARSE>
__device__ inline bool near_in_table(const VerifyArgs &a, const uint32_t *spc, int64_t qi, int T, uint32_t qkey,
                                     int rq, uint32_t key, uint32_t id) {
    if (key != qkey) return false;
    if constexpr (SPARSE) {
        if (a.seen) {
            if (!first_sighting(a, qi, id)) return false;  // checked in an earlier table
            int64_t xb, qb;
            int nx, nqi;
            return within_sparse(a, qi, rq, id, xb, nx, qb, nqi);
        }
        int64_t xb, qb;
        int nx, nqi;
        if (!within_sparse(a, qi, rq, id, xb, nx, qb, nqi)) return false;
        return first_shared_table_sparse(a.xcols + xb, nx, a.qcols + qb, nqi, spc, a.t, a.mbits, a.Lp, a.d) == T;
    } else {
        const uint64_t *xp = a.pts + int64_t(id) * a.W;
        const uint64_t *qp = a.queries + qi * a.W;
        if (a.seen) return first_sighting(a, qi, id) && hamming(xp, qp, a.W, a.last_mask) <= rq;
        if (hamming(xp, qp, a.W, a.last_mask) > rq) return false;
        return first_shared_table(xp, qp, a.W, spc, a.t, a.mbits, a.Lp, a.last_mask, a.d0, a.rep) == T;
    }
}

// Stages the per-coordinate (part, column) words in the workgroup's LDS
// (dense points, at most 4096 coordinates); a sparse index reads them from
// global memory.
template <bool SPARSE>
__device__ inline const uint32_t *stage_pc(const VerifyArgs &a, uint32_t *spc) {
    if constexpr (SPARSE) {
        return a.pc;
    } else {
        for (int i = threadIdx.x; i < a.d; i += blockDim.x) spc[i] = a.pc[i];
        __syncthreads();
        return spc;
    }
}

// Whole wave, uniform arguments: entries [j0, j1) of table T (absolute
// positions), a lane per entry.
template <bool SPARSE, typename KT>
__device__ inline void verify_range(const VerifyArgs &a, const PairStage &ps, const uint32_t *spc, int64_t qi,
                                    int T, uint32_t j0, uint32_t j1) {
    const int lane = threadIdx.x & 63;
    const uint32_t qkey = a.qkeys[int64_t(T) * a.nq + qi];
    const uint32_t qk = uint32_t(KT(qkey));  // the stored part of the key (the bin holds the rest)
    const uint32_t *ids = a.tids + int64_t(T) * a.n;
    const KT *bk = static_cast<const KT *>(a.tkeys) + int64_t(T) * a.n;
    const int rq = query_radius(a, qi);
    // four rounds of 64 entries at a time: their keys and ids are loaded
    // together (independent loads), then the matches are verified
    constexpr int R4 = 4;
    for (uint32_t b0 = j0; b0 < j1; b0 += 64 * R4) {
        uint32_t key[R4], id[R4];
#pragma unroll
        for (int k = 0; k < R4; ++k) {
            const uint32_t j = b0 + uint32_t(k) * 64u + uint32_t(lane);
            key[k] = uint32_t(bk[min(j, j1 - 1)]);  // clamped, so the loads need no branch
            id[k] = ids[min(j, j1 - 1)];
        }
        // the lane's matches among its R4 entries, verified one per round
        // (as in the item pass)
        uint32_t mm = 0;
#pragma unroll
        for (int k = 0; k < R4; ++k)
            mm |= uint32_t(key[k] == qk && b0 + uint32_t(k) * 64u + uint32_t(lane) < j1) << k;
        while (mm) {
            const int k = __builtin_ctz(mm);
            mm &= mm - 1;
            uint32_t idk = id[0];
#pragma unroll
            for (int h = 1; h < R4; ++h) idk = k == h ? id[h] : idk;
            if (near_in_table<SPARSE>(a, spc, qi, T, qkey, rq, qkey, idk)) emit_pair(a, ps, qi, idk);
        }
    }
}

// S2: per (query, table) the query's directory bin [start, start+len) in
// table T and the number of entries in it whose key equals the query's key
// (the bucket size, i.e. this table's share of #Collisions).
template <typename KT>
__global__ void lookup_kernel(const uint32_t *__restrict__ qkeys, int64_t nq, int L,
                              const KT *__restrict__ tkeys, const uint32_t *__restrict__ dir, int64_t n,
                              int dir_bits, uint32_t *__restrict__ rstart, uint32_t *__restrict__ rlen,
                              uint32_t *__restrict__ rmatch) {
    const int64_t total = nq * L;
    const int64_t nb = int64_t(1) << dir_bits;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += int64_t(gridDim.x) * blockDim.x) {
        const int T = int(g / nq);
        const int64_t qi = g - int64_t(T) * nq;
        const uint32_t key = qkeys[g];
        const KT *tk = tkeys + int64_t(T) * n;
        const uint32_t *dr = dir + int64_t(T) * (nb + 1);
        const uint32_t bin = key >> (31 - dir_bits);
        const uint32_t lo = dr[bin], hi = dr[bin + 1];
        uint32_t m = 0;
        for (uint32_t j = lo; j < hi; ++j) m += tk[j] == KT(key);
        rstart[qi * L + T] = lo;
        rlen[qi * L + T] = hi - lo;
        rmatch[qi * L + T] = m;
    }
}

__global__ void collisions_kernel(const uint32_t *__restrict__ rmatch, int64_t nq, int L,
                                  uint64_t *__restrict__ coll) {
    const int64_t qi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    uint64_t s = 0;
    for (int T = 0; T < L; ++T) s += rmatch[qi * L + T];
    coll[qi] = s;
}

__global__ void zero_u32_kernel(uint32_t *__restrict__ p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

// Clears the per-batch counters (a kernel, not a memset: graph-safe).
__global__ void reset_kernel(QueryCtrl *ctrl, uint32_t *qcount, uint32_t *qfill, int64_t nq) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) *ctrl = QueryCtrl{};
    for (int64_t k = i; k < nq; k += int64_t(gridDim.x) * blockDim.x) {
        qcount[k] = 0;
        qfill[k] = 0;
    }
}

// S2 + S3, pass 1: a lane per (query, table) item; wave g takes the rounds
// of 64 items g, g + G, g + 2G, ... (G waves in the grid; no claim counter,
// which would serialise one atomic per round on one address).  The lane
// probes the directory; a bin of at most kLaneBin entries is scanned and
// verified by the lane alone, a larger one is cut into `tile`-entry chunks on
// the spill queue.
template <bool SPARSE, typename KT>
__global__ __launch_bounds__(64 * kVerifyWaves) void verify_items_kernel(VerifyArgs a) {
    __shared__ uint32_t stq[kVerifyWaves][kPairBuf], sti[kVerifyWaves][kPairBuf], stc[kVerifyWaves];
    extern __shared__ uint32_t dyn_pc[];
    const uint32_t *spc = stage_pc<SPARSE>(a, dyn_pc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const PairStage ps{stq[wave], sti[wave], &stc[wave]};
    if (lane == 0) __hip_atomic_store(ps.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const unsigned long long items = (unsigned long long)(a.nq * a.L);
    const int64_t nb = int64_t(1) << a.dir_bits;
    const unsigned long long nw = (unsigned long long)gridDim.x * kVerifyWaves;
    // static: wave g takes rounds g, g + nw, ...; claim: a wave takes
    // kClaimRounds consecutive rounds per atomic on the control block
    const bool claim = a.schedule == kScheduleClaim;
    unsigned long long it0 = 0, claim_end = 0;
    if (!claim) it0 = ((unsigned long long)blockIdx.x * kVerifyWaves + wave) * 64;
    for (;;) {
        if (claim) {
            if (it0 >= claim_end) {
                unsigned long long at = 0;
                if (lane == 0) at = atomicAdd(&a.ctrl->claim_items, (unsigned long long)(kClaimRounds * 64));
                it0 = __shfl(at, 0, 64);
                claim_end = it0 + kClaimRounds * 64;
            }
        }
        if (it0 >= items) break;  // wave-uniform
        const unsigned long long it = it0 + lane;
        it0 += claim ? 64 : nw * 64;
        const bool valid = it < items;
        int64_t qi = 0;
        int T = 0;
        if (valid) item_coords(a, uint32_t(it), qi, T);
        uint32_t qkey = 0, lo = 0, hi = 0;
        if (valid) {
            qkey = a.qkeys[int64_t(T) * a.nq + qi];
            const uint32_t *dr = a.dir + int64_t(T) * (nb + 1);
            const uint32_t bin = qkey >> (31 - a.dir_bits);
            lo = dr[bin];
            hi = dr[bin + 1];
        }
        // bins over kLaneBin entries go to the spill queue: the wave's
        // chunk counts are summed (exclusive prefix across lanes) and
        // reserved with one atomic
        const uint32_t nch = (valid && hi - lo > kLaneBin) ? (hi - lo + a.tile - 1) / a.tile : 0u;
        uint32_t pre = nch;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = uint32_t(__shfl_up(int(pre), o, 64));
            if (lane >= o) pre += y;
        }
        const uint32_t wtot = uint32_t(__shfl(int(pre), 63, 64));
        pre -= nch;
        if (wtot) {
            unsigned long long at = 0;
            if (lane == 0) at = atomicAdd(&a.ctrl->spills, (unsigned long long)wtot);
            at = __shfl(at, 0, 64) + pre;
            for (uint32_t c = 0; c < nch; ++c)
                if (at + c < (unsigned long long)a.spill_cap) {
                    const uint32_t b = lo + c * a.tile;
                    a.spill[at + c] = make_uint4(uint32_t(it), b, min(hi, b + a.tile), 0u);
                }
        }
        if (!valid || nch) continue;
        const KT *bk = static_cast<const KT *>(a.tkeys) + int64_t(T) * a.n;
        const uint32_t qk = uint32_t(KT(qkey));  // the stored part of the key (the bin holds the rest)
        const uint32_t *ids = a.tids + int64_t(T) * a.n;
        const int rq = query_radius(a, qi);
        // the bin's keys in chunks of 8 independent loads, giving the mask of
        // matching positions (a bin here holds at most kLaneBin = 32)
        uint32_t mm = 0;
        for (uint32_t j0 = lo; j0 < hi; j0 += 8) {
            // unconditional loads (index clamped to the bin's last entry) so
            // that all 8 are in flight together; positions past the bin are
            // masked below
            uint32_t kk[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) kk[c] = uint32_t(bk[min(j0 + uint32_t(c), hi - 1)]);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                mm |= uint32_t(kk[c] == qk && j0 + uint32_t(c) < hi) << (j0 - lo + uint32_t(c));
        }
        // then the matches, one per lane at a time: the lanes verify their
        // k-th matches together, so the wave runs as many rounds of the
        // dependent loads (id, then point) as its busiest lane has matches,
        // not one per matching position
        while (mm) {
            const uint32_t c = uint32_t(__builtin_ctz(mm));
            mm &= mm - 1;
            const uint32_t id = ids[lo + c];
            if (near_in_table<SPARSE>(a, spc, qi, T, qkey, rq, qkey, id)) emit_pair(a, ps, qi, id);
        }
    }
    flush_pairs(a, ps, stage_count(ps));
}

// S3, pass 2: persistent waves verify the recorded chunks, wave g taking
// chunks g, g + G, g + 2G, ... (G waves in the grid).  The chunks of one
// batch number up to the hundreds of thousands: a shared claim counter would
// serialise that many atomics on one address, while the fixed stride spreads
// the chunks' uneven costs over tens of chunks per wave.
template <bool SPARSE, typename KT>
__global__ __launch_bounds__(64 * kVerifyWaves) void verify_spill_kernel(VerifyArgs a) {
    __shared__ uint32_t stq[kVerifyWaves][kPairBuf], sti[kVerifyWaves][kPairBuf], stc[kVerifyWaves];
    extern __shared__ uint32_t dyn_pc[];
    const uint32_t *spc = stage_pc<SPARSE>(a, dyn_pc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const PairStage ps{stq[wave], sti[wave], &stc[wave]};
    if (lane == 0) __hip_atomic_store(ps.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const unsigned long long nsp = min((unsigned long long)a.spill_cap, a.ctrl->spills);
    const unsigned long long nw = (unsigned long long)gridDim.x * kVerifyWaves;
    if (a.schedule == kScheduleClaim) {
        // kClaimChunks chunks per atomic on the control block
        for (;;) {
            unsigned long long at = 0;
            if (lane == 0) at = atomicAdd(&a.ctrl->claim_spill, (unsigned long long)kClaimChunks);
            const unsigned long long k0 = __shfl(at, 0, 64);
            if (k0 >= nsp) break;  // wave-uniform
            for (unsigned long long k = k0; k < k0 + kClaimChunks && k < nsp; ++k) {
                const uint4 r = a.spill[k];
                int64_t qi;
                int T;
                item_coords(a, r.x, qi, T);
                verify_range<SPARSE, KT>(a, ps, spc, qi, T, r.y, r.z);
            }
        }
    } else {
        for (unsigned long long k = (unsigned long long)blockIdx.x * kVerifyWaves + wave; k < nsp; k += nw) {
            const uint4 r = a.spill[k];
            int64_t qi;
            int T;
            item_coords(a, r.x, qi, T);
            verify_range<SPARSE, KT>(a, ps, spc, qi, T, r.y, r.z);
        }
    }
    flush_pairs(a, ps, stage_count(ps));
}

__global__ void widen_counts_kernel(const uint32_t *__restrict__ c32, int64_t nq, uint64_t *__restrict__ c64) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nq) c64[i] = c32[i];
}

// offsets[nq] = number of reported pairs; flags overflow of the internal
// pair buffer, the spill queue or the caller's id buffer.
__global__ void finish_offsets_kernel(uint64_t *offsets, int64_t nq, QueryCtrl *ctrl, int64_t pair_cap,
                                      int64_t spill_cap, int64_t ids_cap) {
    const unsigned long long tot = ctrl->pairs;
    offsets[nq] = tot;
    ctrl->total = tot;
    uint32_t st = 0;
    if (tot > (unsigned long long)pair_cap) st |= kQueryPairOverflow;
    if (ctrl->spills > (unsigned long long)spill_cap) st |= kQuerySpillOverflow;
    if (tot > (unsigned long long)ids_cap) st |= kQueryIdsOverflow;
    ctrl->status = st | (ctrl->status & kQueryBadRows);
}

// Conditions under which the scatter and sort leave the id buffer alone.
constexpr uint32_t kAnyOverflow = kQueryPairOverflow | kQuerySpillOverflow | kQueryIdsOverflow | kQueryBadRows;

// Pairs into per-query segments (order inside a segment fixed by the sort).
// Pairs arrive in runs of one query, and a query with tens of thousands of
// answers would serialise that many atomics on its fill counter: the lanes
// of a wave that hold pairs of the same query reserve their slots with one
// atomic.  Block 0 also clears the long-segment count of the sort.
__global__ void scatter_pairs_kernel(const uint32_t *__restrict__ pq, const uint32_t *__restrict__ pid,
                                     QueryCtrl *__restrict__ ctrl, int64_t pair_cap,
                                     const uint64_t *__restrict__ offsets, uint32_t *__restrict__ qfill,
                                     uint32_t *__restrict__ ids, int64_t ids_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->nlong = 0;
    if (ctrl->status & kAnyOverflow) return;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t tot = int64_t(min((unsigned long long)pair_cap, ctrl->pairs));
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    // whole waves step together, so that every lane takes part in the
    // ballots.  A run of lanes with the same query takes one fill atomic,
    // issued by its first lane; all runs of a wave issue theirs together.
    for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63); i0 < tot; i0 += stride) {
        const int64_t i = i0 + lane;
        const bool valid = i < tot;  // the valid lanes are a prefix of the wave
        const uint32_t q = valid ? pq[i] : 0u;
        const uint32_t id = valid ? pid[i] : 0u;
        const uint32_t qprev = uint32_t(__shfl_up(int(q), 1, 64));
        const bool head = valid && (lane == 0 || qprev != q);
        const uint64_t heads = __ballot(head);
        const int nvalid = __popcll(__ballot(valid));
        const uint64_t upto = heads & (lt | (1ull << lane));  // heads at or below this lane
        const int h = upto ? 63 - __builtin_clzll(upto) : 0;  // this lane's run head
        uint32_t base = 0;
        if (head) {
            const uint64_t above = heads & ~(lt | (1ull << lane));
            const int next = above ? __builtin_ctzll(above) : nvalid;
            base = atomicAdd(&qfill[q], uint32_t(next - lane));
        }
        base = uint32_t(__shfl(int(base), h, 64));
        if (valid) {
            const uint64_t slot = offsets[q] + base + uint32_t(lane - h);
            if (slot < uint64_t(ids_cap)) ids[slot] = id;
        }
    }
}

// Sorts each query's segment of ids ascending.  Segments up to kSortCap ids:
// a bitonic sort in LDS, a workgroup per query.  Longer ones are listed
// (list[k], k < ctrl->nlong) for segment_sort_long_kernel.
constexpr int kSortNT = 256;
constexpr int kSortCap = 4096;

__global__ __launch_bounds__(kSortNT) void segment_sort_kernel(const uint64_t *__restrict__ offsets,
                                                               QueryCtrl *__restrict__ ctrl,
                                                               uint32_t *__restrict__ ids, int64_t q0,
                                                               uint32_t *__restrict__ list) {
    __shared__ uint32_t s[kSortCap];
    if (ctrl->status & kAnyOverflow) return;
    const int64_t q = blockIdx.x;
    const uint64_t b = offsets[q], e = offsets[q + 1];
    const uint32_t m = uint32_t(e - b);
    if (m <= 1) return;
    uint32_t *seg = ids + b;
    if (m > uint32_t(kSortCap)) {
        if (threadIdx.x == 0) list[atomicAdd(&ctrl->nlong, 1u)] = uint32_t(q0 + q);
        return;
    }
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += kSortNT) s[i] = i < m ? seg[i] : 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kSortNT) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t x = s[i], y = s[l];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        s[i] = y;
                        s[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < m; i += kSortNT) seg[i] = s[i];
}

// Long segments (listed by segment_sort_kernel), a workgroup at a time each:
// a segment's ids are distinct (the first-shared-table rule reports a point
// once) and below n, so they are marked in an LDS bitmap of the id universe,
// kLongBits ids per pass, and read back in ascending order into tmp (thread
// t reads a run of `per` consecutive words, per odd so that the 64 lanes of
// a wave hit 64 different banks, and a block scan of the runs' popcounts
// places its ids); then tmp is copied over the segment.  O(m + n/32) per
// pass over the universe, instead of a sort's O(m log m) passes over global
// memory.
constexpr int64_t kLongBits = int64_t(1) << 20;  // 128 KB of LDS

__global__ __launch_bounds__(kSortNT) void segment_sort_long_kernel(const uint64_t *__restrict__ offsets,
                                                                    const QueryCtrl *__restrict__ ctrl,
                                                                    const uint32_t *__restrict__ list,
                                                                    uint32_t *__restrict__ ids,
                                                                    uint32_t *__restrict__ tmp, int64_t n) {
    extern __shared__ uint32_t bm[];
    __shared__ uint32_t wsum[kSortNT / 64];
    if (ctrl->status & kAnyOverflow) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t nlong = ctrl->nlong;
    for (uint32_t k = blockIdx.x; k < nlong; k += gridDim.x) {
        const uint32_t q = list[k];
        const uint64_t b = offsets[q];
        const uint32_t m = uint32_t(offsets[q + 1] - b);
        uint32_t *seg = ids + b;
        uint32_t *out = tmp + b;
        uint32_t written = 0;
        for (int64_t base = 0; base < n; base += kLongBits) {
            const uint32_t span = uint32_t(min(kLongBits, n - base));
            const uint32_t words = (span + 31) / 32;
            for (uint32_t w = threadIdx.x; w < words; w += kSortNT) bm[w] = 0u;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < m; i += kSortNT) {
                const int64_t off = int64_t(seg[i]) - base;
                if (off >= 0 && off < int64_t(span)) atomicOr(&bm[off >> 5], 1u << (off & 31));
            }
            __syncthreads();
            const uint32_t per = ((words + kSortNT - 1) / kSortNT) | 1u;
            const uint32_t w0 = min(words, threadIdx.x * per), w1 = min(words, w0 + per);
            uint32_t c = 0;
            for (uint32_t w = w0; w < w1; ++w) c += uint32_t(__popc(bm[w]));
            uint32_t x = c;  // inclusive scan over the wave
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = uint32_t(__shfl_up(int(x), o, 64));
                if (lane >= o) x += y;
            }
            if (lane == 63) wsum[wave] = x;
            __syncthreads();
            uint32_t before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < kSortNT / 64; ++w) {
                before += w < wave ? wsum[w] : 0u;
                total += wsum[w];
            }
            uint32_t pos = written + before + x - c;
            for (uint32_t w = w0; w < w1; ++w) {
                for (uint32_t bits = bm[w]; bits; bits &= bits - 1)
                    if (pos < m) out[pos++] = uint32_t(base) + w * 32u + uint32_t(__builtin_ctz(bits));
            }
            written += total;
            __syncthreads();  // bm and wsum are reused by the next pass
        }
        for (uint32_t i = threadIdx.x; i < m; i += kSortNT) seg[i] = out[i];
        __syncthreads();
    }
}

unsigned grid_for(int64_t work, int per_block, unsigned cap = 1u << 20) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

uint64_t last_word_mask(int d) { return (d % 64) ? ((uint64_t(1) << (d % 64)) - 1) : ~uint64_t(0); }

}  // namespace

// Grows the workspace to hold nq queries of L tables, `pairs` reported pairs
// and `spills` spill chunks.  All-or-nothing: every buffer that must grow is
// allocated first, and only when all of them succeed are the old ones
// released and the new ones and their capacities installed.  A failed
// allocation leaves the workspace exactly as it was (old buffers, old
// capacities), so a later call never runs on a half-grown workspace.
fclsh_status ws_reserve(QueryWorkspace &ws, int64_t nq, int L, int64_t pairs, int64_t spills, int64_t dense_words,
                        int64_t seen_words) {
    ws.pending_nq = -1;  // buffers may be replaced: nothing pending survives
    const int64_t items = nq * L;
    struct Grow {
        void **slot;
        size_t bytes;
        const char *what;
    };
    std::vector<Grow> grow;
    auto want = [&](auto **slot, int64_t count, const char *what) {
        grow.push_back({reinterpret_cast<void **>(slot),
                        size_t(std::max<int64_t>(count, 1)) * sizeof(**slot), what});
    };
    const bool g_items = items > ws.cap_items || !ws.qkeys;
    const bool g_q = nq + 1 > ws.cap_q || !ws.qcount;
    const bool g_pairs = pairs > ws.cap_pairs || !ws.pq;
    const bool g_spill = spills > ws.cap_spill || !ws.spill;
    const bool g_dense = dense_words > ws.cap_qdense;
    const bool g_seen = seen_words > ws.cap_seen;
    if (g_items) {
        want(&ws.qkeys, items, "query keys");
        want(&ws.rstart, items, "query ranges");
        want(&ws.rlen, items, "query ranges");
        want(&ws.rmatch, items, "query ranges");
    }
    if (g_q) {
        want(&ws.qcount, nq + 1, "query counts");
        want(&ws.qfill, nq + 1, "query counts");
        want(&ws.qcount64, nq + 1, "query counts");
        want(&ws.scan_part, scan_partials_needed(nq + 1), "scan partials");
    }
    if (!ws.ctrl) want(&ws.ctrl, 1, "query control");
    if (!ws.offs1) want(&ws.offs1, 2, "plain offsets");
    if (g_pairs) {
        want(&ws.pq, pairs, "result pairs");
        want(&ws.pid, pairs, "result pairs");
        want(&ws.sorttmp, pairs, "result sort");
    }
    if (g_spill) want(&ws.spill, spills, "spill queue");
    if (g_dense) want(&ws.qdense, dense_words, "query bit vectors");
    if (g_seen) want(&ws.seen, seen_words, "per-query point bitmaps");
    std::vector<void *> fresh(grow.size(), nullptr);
    for (size_t i = 0; i < grow.size(); ++i) {
        if (hipMalloc(&fresh[i], grow[i].bytes) != hipSuccess) {
            (void)hipGetLastError();
            for (size_t j = 0; j < i; ++j) (void)hipFree(fresh[j]);
            return fail(FCLSH_ENOMEM, "device allocation of %zu bytes for %s failed", grow[i].bytes, grow[i].what);
        }
    }
    for (size_t i = 0; i < grow.size(); ++i) {
        if (*grow[i].slot) (void)hipFree(*grow[i].slot);
        *grow[i].slot = fresh[i];
    }
    if (g_items) ws.cap_items = items;
    if (g_q) ws.cap_q = nq + 1;
    if (g_pairs) ws.cap_pairs = pairs;
    if (g_spill) ws.cap_spill = spills;
    if (g_dense) ws.cap_qdense = dense_words;
    if (g_seen) ws.cap_seen = seen_words;
    return FCLSH_OK;
}

// Lays a workspace for nq queries of L tables out in one caller-owned device
// buffer of `bytes` bytes (256-byte aligned pieces): query keys, per-query
// counters, scan partials and the control block first, then the spill queue
// and the pair buffers share what is left, a quarter of it for spill chunks
// (16 B each) and the rest for pairs (12 B each: query, id and the sort's
// second buffer).  The lookup ranges of the collision count are not laid out.
// Nothing is allocated.  Returns FCLSH_ENOMEM when the fixed part, at least
// one pair and one spill chunk do not fit.
fclsh_status ws_carve(QueryWorkspace &ws, void *base, size_t bytes, int64_t nq, int L) {
    ws = QueryWorkspace{};
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    const int64_t items = nq * L;
    // offsets of the fixed pieces, computed before any pointer is formed
    const size_t sz_fixed[] = {size_t(std::max<int64_t>(items, 1)) * 4, size_t(nq + 1) * 4, size_t(nq + 1) * 4,
                               size_t(nq + 1) * 8, size_t(scan_partials_needed(nq + 1)) * 8, sizeof(QueryCtrl)};
    size_t off_fixed[6], at = 0;
    for (int i = 0; i < 6; ++i) {
        off_fixed[i] = up(at);
        at = off_fixed[i] + sz_fixed[i];
    }
    at = up(at);
    if (at + 3 * 256 + 16 + 12 > bytes)
        return fail(FCLSH_ENOMEM, "%lld queries x %d tables need more than the %zu scratch bytes", (long long)nq, L,
                    bytes);
    const size_t rest = bytes - at - 3 * 256;  // room for the alignment of the last pieces
    const int64_t spills = std::max<int64_t>(1, int64_t(rest / 4 / 16));
    const int64_t pairs = int64_t((rest - size_t(spills) * 16) / 12);
    const size_t off_spill = at;
    const size_t off_pq = up(off_spill + size_t(spills) * 16);
    const size_t off_pid = up(off_pq + size_t(pairs) * 4);
    const size_t off_tmp = up(off_pid + size_t(pairs) * 4);
    if (pairs < 1 || off_tmp + size_t(pairs) * 4 > bytes)
        return fail(FCLSH_ENOMEM, "%lld queries x %d tables leave no room for results in %zu scratch bytes",
                    (long long)nq, L, bytes);
    char *const b0 = static_cast<char *>(base);
    ws.qkeys = reinterpret_cast<uint32_t *>(b0 + off_fixed[0]);
    ws.qcount = reinterpret_cast<uint32_t *>(b0 + off_fixed[1]);
    ws.qfill = reinterpret_cast<uint32_t *>(b0 + off_fixed[2]);
    ws.qcount64 = reinterpret_cast<uint64_t *>(b0 + off_fixed[3]);
    ws.scan_part = reinterpret_cast<uint64_t *>(b0 + off_fixed[4]);
    ws.ctrl = reinterpret_cast<QueryCtrl *>(b0 + off_fixed[5]);
    ws.spill = reinterpret_cast<uint4 *>(b0 + off_spill);
    ws.pq = reinterpret_cast<uint32_t *>(b0 + off_pq);
    ws.pid = reinterpret_cast<uint32_t *>(b0 + off_pid);
    ws.sorttmp = reinterpret_cast<uint32_t *>(b0 + off_tmp);
    ws.cap_items = items;
    ws.cap_q = nq + 1;
    ws.cap_pairs = pairs;
    ws.cap_spill = spills;
    return FCLSH_OK;
}

uint64_t ws_bytes(const QueryWorkspace &ws) {
    if (!ws.ctrl) return 0;
    return uint64_t(ws.cap_items) * 16 + uint64_t(ws.cap_q) * 16 +
           uint64_t(scan_partials_needed(ws.cap_q)) * 8 + sizeof(QueryCtrl) + 16 + uint64_t(ws.cap_pairs) * 12 +
           uint64_t(ws.cap_spill) * 16 + uint64_t(ws.cap_qdense) * 8 +
           uint64_t(ws.cap_seen) * 4;
}

void ws_release(QueryWorkspace &ws) {
    void *ps[] = {ws.qkeys, ws.rstart, ws.rlen, ws.rmatch, ws.qcount, ws.qfill, ws.qcount64, ws.scan_part,
                  ws.offs1, ws.ctrl, ws.pq, ws.pid, ws.sorttmp, ws.spill, ws.qdense, ws.seen};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    ws = QueryWorkspace{};
}

// S1 + S2 for a batch; leaves keys and ranges in the workspace.
fclsh_status query_lookup(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, hipStream_t st) {
    const int L = ix.prm.L();
    FCLSH_TRY(launch_hash(ix, queries, nq, ws.qkeys, nq, st));
    if (ix.key_bytes == 2)
        hipLaunchKernelGGL(lookup_kernel<uint16_t>, dim3(grid_for(nq * L, 256)), dim3(256), 0, st, ws.qkeys, nq, L,
                           static_cast<const uint16_t *>(ix.tkeys), ix.dir, ix.n, ix.dir_bits, ws.rstart, ws.rlen,
                           ws.rmatch);
    else
        hipLaunchKernelGGL(lookup_kernel<uint32_t>, dim3(grid_for(nq * L, 256)), dim3(256), 0, st, ws.qkeys, nq, L,
                           static_cast<const uint32_t *>(ix.tkeys), ix.dir, ix.n, ix.dir_bits, ws.rstart, ws.rlen,
                           ws.rmatch);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

fclsh_status query_collisions(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq,
                              uint64_t *coll, hipStream_t st) {
    FCLSH_TRY(ws_reserve(ws, nq, ix.prm.L(), std::max<int64_t>(ws.cap_pairs, 1), std::max<int64_t>(ws.cap_spill, 1)));
    FCLSH_TRY(query_lookup(ix, ws, queries, nq, st));
    hipLaunchKernelGGL(collisions_kernel, dim3(grid_for(nq, 256)), dim3(256), 0, st, ws.rmatch, nq, ix.prm.L(),
                       coll);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

namespace {

// Sec. 4.1's two cost measures per query, with the paper's own duplicate
// elimination: an n-bit bitmap per query.  Every entry of the query's L
// buckets is a collision; its id's bit is set with one atomic OR, and a bit
// found clear is a new distinct candidate.  One wave per (query, table) item
// (query-major, so a query's tables share its bitmap in cache); the lanes
// stride over the item's directory bin and keep the entries whose key equals
// the query's.  Wave totals go to the per-query counters with one atomic each.
template <typename KT>
__global__ __launch_bounds__(256) void cost_kernel(const uint32_t *__restrict__ qkeys, int64_t qn, int L,
                                                   const KT *__restrict__ tkeys,
                                                   const uint32_t *__restrict__ tids,
                                                   const uint32_t *__restrict__ dir, int64_t n, int dir_bits,
                                                   uint32_t *__restrict__ bitmap, int64_t bm_words,
                                                   unsigned long long *__restrict__ coll,
                                                   unsigned long long *__restrict__ cand) {
    const int lane = threadIdx.x & 63;
    const int64_t nb = int64_t(1) << dir_bits;
    const int64_t items = qn * L;
    const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x / 64);
    for (int64_t it = int64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6); it < items; it += nwaves) {
        const int64_t ql = it / L;
        const int T = int(it - ql * L);
        const uint32_t key = qkeys[int64_t(T) * qn + ql];
        const uint32_t *dr = dir + int64_t(T) * (nb + 1);
        const uint32_t bin = key >> (31 - dir_bits);
        const uint32_t lo = dr[bin], hi = dr[bin + 1];
        const KT *tk = tkeys + int64_t(T) * n;
        const uint32_t *ti = tids + int64_t(T) * n;
        uint32_t *bm = bitmap + ql * bm_words;
        uint32_t nc = 0, nd = 0;
        for (uint32_t j = lo + uint32_t(lane); j < hi; j += 64) {
            if (tk[j] != KT(key)) continue;
            const uint32_t id = ti[j];
            const uint32_t bit = 1u << (id & 31u);
            ++nc;
            nd += (atomicOr(&bm[id >> 5], bit) & bit) ? 0u : 1u;
        }
        for (int o = 32; o > 0; o >>= 1) {
            nc += uint32_t(__shfl_xor(int(nc), o, 64));
            nd += uint32_t(__shfl_xor(int(nd), o, 64));
        }
        if (lane == 0 && nc) {
            atomicAdd(&coll[ql], (unsigned long long)nc);
            atomicAdd(&cand[ql], (unsigned long long)nd);
        }
    }
}

// Clears a chunk's bitmaps and counters (a kernel, not a memset).
__global__ void cost_clear_kernel(uint32_t *__restrict__ bitmap, int64_t words, unsigned long long *__restrict__ coll,
                                  unsigned long long *__restrict__ cand, int64_t qn) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < words; i += stride) bitmap[i] = 0u;
    for (int64_t i = i0; i < qn; i += stride) {
        coll[i] = 0ull;
        cand[i] = 0ull;
    }
}

}  // namespace

// #Collisions and #Candidates of Sec. 4.1 for a batch, in chunks of queries
// whose bitmaps fit a fixed budget.
fclsh_status query_cost(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, uint64_t *coll,
                        uint64_t *cand, hipStream_t st, const CsrRows *sq) {
    const int L = ix.prm.L();
    const int64_t bm_words = (ix.n + 31) / 32;
    constexpr int64_t kBitmapBudget = int64_t(256) << 20;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nq, kBitmapBudget / (bm_words * 4)));
    FCLSH_TRY(ws_reserve(ws, chunk, L, std::max<int64_t>(ws.cap_pairs, 1), std::max<int64_t>(ws.cap_spill, 1)));
    uint32_t *bitmap = nullptr;
    if (hipMalloc(&bitmap, size_t(chunk * bm_words) * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FCLSH_ENOMEM, "device allocation of the candidate bitmaps failed");
    }
    fclsh_status s = FCLSH_OK;
    for (int64_t q0 = 0; q0 < nq && s == FCLSH_OK; q0 += chunk) {
        const int64_t qn = std::min(chunk, nq - q0);
        auto *c0 = reinterpret_cast<unsigned long long *>(coll + q0);
        auto *d0 = reinterpret_cast<unsigned long long *>(cand + q0);
        hipLaunchKernelGGL(cost_clear_kernel, dim3(grid_for(qn * bm_words, 256, 4096)), dim3(256), 0, st, bitmap,
                           qn * bm_words, c0, d0, qn);
        s = sq ? launch_hash_sparse(ix, CsrRows{sq->ptr + q0, sq->cols, sq->nnz}, qn, ws.qkeys, qn, st)
               : launch_hash(ix, queries + q0 * ix.W, qn, ws.qkeys, qn, st);
        if (s != FCLSH_OK) break;
        if (ix.key_bytes == 2)
            hipLaunchKernelGGL(cost_kernel<uint16_t>, dim3(grid_for(qn * L, 4, 1u << 16)), dim3(256), 0, st, ws.qkeys,
                               qn, L, static_cast<const uint16_t *>(ix.tkeys), ix.tids, ix.dir, ix.n, ix.dir_bits,
                               bitmap, bm_words, c0, d0);
        else
            hipLaunchKernelGGL(cost_kernel<uint32_t>, dim3(grid_for(qn * L, 4, 1u << 16)), dim3(256), 0, st, ws.qkeys,
                               qn, L, static_cast<const uint32_t *>(ix.tkeys), ix.tids, ix.dir, ix.n, ix.dir_bits,
                               bitmap, bm_words, c0, d0);
        if (hipGetLastError() != hipSuccess) s = fail(FCLSH_EDEVICE, "cost kernel launch failed");
    }
    const hipError_t e = hipStreamSynchronize(st);
    (void)hipFree(bitmap);
    if (s == FCLSH_OK && e != hipSuccess)
        s = fail(FCLSH_EDEVICE, "query cost counters failed: %s", hipGetErrorString(e));
    return s;
}

// The batched pipeline, entirely on the stream: no allocation, no host
// synchronisation (the workspace must already hold nq queries, ws.cap_pairs
// pairs and ws.cap_spill spill chunks).  Outputs: offsets[nq+1], ids (up to
// ids_cap), and ws.ctrl->{total, status}.
namespace {

// Clears the id-buffer overflow flag and the per-query fill counters, so that
// the pairs of the last batch can be scattered into a new id buffer.
__global__ void rearm_scatter_kernel(QueryCtrl *ctrl, uint32_t *qfill, int64_t nq) {
    const int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i0 == 0) ctrl->status &= ~kQueryIdsOverflow;
    for (int64_t i = i0; i < nq; i += int64_t(gridDim.x) * blockDim.x) qfill[i] = 0;
}

// The two verification passes of a batch.
template <bool SPARSE, typename KT>
fclsh_status launch_verify(const VerifyArgs &a, unsigned iblocks, unsigned vblocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(verify_items_kernel<SPARSE, KT>), dim3(iblocks), dim3(64 * kVerifyWaves), lds,
                       st, a);
    FCLSH_HIP(hipGetLastError());
    hipLaunchKernelGGL(HIP_KERNEL_NAME(verify_spill_kernel<SPARSE, KT>), dim3(vblocks), dim3(64 * kVerifyWaves), lds,
                       st, a);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

// Pairs into the per-query segments of ids, then each segment sorted (the
// long segments listed in ws.qcount, free once the offsets are scanned).
fclsh_status launch_scatter_sort(Index &ix, QueryWorkspace &ws, int64_t nq, const uint64_t *offsets, uint32_t *ids,
                                 int64_t ids_cap, hipStream_t st) {
    hipLaunchKernelGGL(scatter_pairs_kernel, dim3(grid_for(ws.cap_pairs, 256, 4096)), dim3(256), 0, st, ws.pq,
                       ws.pid, ws.ctrl, ws.cap_pairs, offsets, ws.qfill, ids, ids_cap);
    FCLSH_HIP(hipGetLastError());
    for (int64_t q0 = 0; q0 < nq; q0 += 65535) {
        const int64_t qn = std::min<int64_t>(65535, nq - q0);
        hipLaunchKernelGGL(segment_sort_kernel, dim3(unsigned(qn)), dim3(kSortNT), 0, st, offsets + q0, ws.ctrl, ids,
                           q0, ws.qcount);
        FCLSH_HIP(hipGetLastError());
    }
    // a segment over kSortCap ids holds at least that many distinct points
    if (ix.n > kSortCap) {
        const size_t lds = size_t(std::min<int64_t>(kLongBits, ix.n) + 31) / 32 * 4;
        const unsigned grid = unsigned(std::min<int64_t>(std::max(1, ix.num_cus), nq));
        hipLaunchKernelGGL(segment_sort_long_kernel, dim3(grid), dim3(kSortNT), lds, st, offsets, ws.ctrl, ws.qcount,
                           ids, ws.sorttmp, ix.n);
        FCLSH_HIP(hipGetLastError());
    }
    return FCLSH_OK;
}

}  // namespace

fclsh_status query_batch_async(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, int rq,
                               const int32_t *rq_vec, hipStream_t st, uint64_t *offsets, uint32_t *ids,
                               int64_t ids_cap, const CsrRows *sq) {
    const int L = ix.prm.L();
    ws.pending_nq = -1;
    const QueryTuning &tu = ix.tuning;
    const bool sparse = ix.prm.sparse;
    if (sparse != (sq != nullptr)) return fail(FCLSH_EINVAL, "query rows do not match the index's point format");
    if (nq * L > ws.cap_items || nq + 1 > ws.cap_q || !ws.ctrl || !ws.pq || !ws.spill)
        return fail(FCLSH_EINVAL, "query workspace not reserved for %lld queries", (long long)nq);
    if (sparse && nq * ix.W > ws.cap_qdense)
        return fail(FCLSH_EINVAL, "query workspace not reserved for %lld sparse queries", (long long)nq);
    if (nq * L > int64_t(0xFFFFFFFF))  // spill chunks name their item in 32 bits
        return fail(FCLSH_EINVAL, "%lld queries x %d tables exceed 2^32 items per batch", (long long)nq, L);
    hipLaunchKernelGGL(reset_kernel, dim3(grid_for(nq, 256, 1024)), dim3(256), 0, st, ws.ctrl, ws.qcount, ws.qfill,
                       nq);
    FCLSH_HIP(hipGetLastError());
    if (sparse && nq > 0) {
        // the rows are checked (any fault is reported in the status word and
        // the ids are left alone), then hashed from their nonzeros and
        // densified for the distance tests
        FCLSH_TRY(csr_check(*sq, nq, ix.prm.d, &ws.ctrl->status, kQueryBadShift, st));
        FCLSH_TRY(csr_densify(*sq, nq, ix.prm.d, ws.qdense, st));
        FCLSH_TRY(launch_hash_sparse(ix, *sq, nq, ws.qkeys, nq, st));
        queries = ws.qdense;
    } else if (nq > 0) {
        FCLSH_TRY(launch_hash(ix, queries, nq, ws.qkeys, nq, st));
    }
    VerifyArgs a{};
    a.pts = ix.pts;
    a.W = ix.W;
    a.t = ix.prm.t;
    a.mbits = ix.prm.rp + 1;
    a.Lp = ix.prm.Lp();
    a.L = L;
    a.last_mask = last_word_mask(ix.prm.d);
    a.pc = ix.dpc;
    a.d = ix.prm.dd();
    a.d0 = ix.prm.d;
    a.rep = ix.prm.rep;
    a.queries = queries;
    a.nq = nq;
    a.rq_vec = rq_vec;
    a.rq = rq;
    a.tkeys = ix.tkeys;
    a.tids = ix.tids;
    a.dir = ix.dir;
    a.n = ix.n;
    a.dir_bits = ix.dir_bits;
    a.qkeys = ws.qkeys;
    a.ctrl = ws.ctrl;
    a.spill = ws.spill;
    a.spill_cap = ws.cap_spill;
    a.out_q = ws.pq;
    a.out_id = ws.pid;
    a.pair_cap = ws.cap_pairs;
    a.qcount = ws.qcount;
    a.tile = uint32_t(tu.tile);
    a.table_major = nq > kTableMajorBatch ? 1 : 0;
    a.schedule = tu.schedule;
    if (sparse) {
        a.xptr = ix.sptr;
        a.xcols = ix.scols;
        a.qptr = sq->ptr;
        a.qcols = sq->cols;
        a.qnnz = sq->nnz;
    }
    {
        // the paper's bitmap dedupe when the workspace holds one bitmap per
        // query: a point is checked once per query, not once per table it
        // collides in
        const int64_t wpq = (ix.n + 31) / 32;
        if (nq > 0 && ws.cap_seen >= nq * wpq) {
            a.seen = ws.seen;
            a.seen_wpq = wpq;
            hipLaunchKernelGGL(zero_u32_kernel, dim3(grid_for(nq * wpq, 256, 8192)), dim3(256), 0, st, ws.seen,
                               nq * wpq);
            FCLSH_HIP(hipGetLastError());
        }
    }
    const unsigned vblocks = unsigned(std::max(1, tu.blocks_per_cu * ix.num_cus));
    if (nq > 0) {
        // the item pass needs no more waves than rounds of 64 items
        const unsigned iblocks = std::min<unsigned>(vblocks, grid_for(nq * L, 64 * kVerifyWaves));
        if (sparse && ix.key_bytes == 2)
            FCLSH_TRY((launch_verify<true, uint16_t>(a, iblocks, vblocks, 0, st)));
        else if (sparse)
            FCLSH_TRY((launch_verify<true, uint32_t>(a, iblocks, vblocks, 0, st)));
        else if (ix.key_bytes == 2)  // staged (part, column) words, at most 4096
            FCLSH_TRY((launch_verify<false, uint16_t>(a, iblocks, vblocks, size_t(ix.prm.dd()) * 4, st)));
        else
            FCLSH_TRY((launch_verify<false, uint32_t>(a, iblocks, vblocks, size_t(ix.prm.dd()) * 4, st)));
    }
    hipLaunchKernelGGL(widen_counts_kernel, dim3(grid_for(nq, 256)), dim3(256), 0, st, ws.qcount, nq, ws.qcount64);
    FCLSH_HIP(hipGetLastError());
    FCLSH_TRY(exclusive_scan_u64_ws(ws.qcount64, offsets, nq, ws.scan_part, st));
    hipLaunchKernelGGL(finish_offsets_kernel, dim3(1), dim3(1), 0, st, offsets, nq, ws.ctrl, ws.cap_pairs,
                       ws.cap_spill, ids_cap);
    FCLSH_HIP(hipGetLastError());
    if (nq > 0 && ids_cap > 0) FCLSH_TRY(launch_scatter_sort(ix, ws, nq, offsets, ids, ids_cap, st));
    return FCLSH_OK;
}

// Finishes the pending synchronous batch of the workspace into a larger id
// buffer: the stored pairs are scattered and sorted again, with no
// recomputation.
fclsh_status query_finish(Index &ix, QueryWorkspace &ws, hipStream_t st, const uint64_t *offsets, uint32_t *ids,
                          int64_t ids_cap, int64_t *total_out) {
    if (ws.pending_nq < 0) return fail(FCLSH_EINVAL, "no batch on this stream is waiting for a larger id buffer");
    if (offsets != ws.pending_offsets) return fail(FCLSH_EINVAL, "offsets differ from those of the pending batch");
    *total_out = ws.pending_total;
    if (ids_cap < ws.pending_total)
        return fail(FCLSH_ECAPACITY, "%lld ids do not fit the output capacity %lld", (long long)ws.pending_total,
                    (long long)ids_cap);
    const int64_t nq = ws.pending_nq;
    ws.pending_nq = -1;
    hipLaunchKernelGGL(rearm_scatter_kernel, dim3(grid_for(nq, 256, 1024)), dim3(256), 0, st, ws.ctrl, ws.qfill, nq);
    FCLSH_HIP(hipGetLastError());
    if (nq > 0 && ids_cap > 0) FCLSH_TRY(launch_scatter_sort(ix, ws, nq, offsets, ids, ids_cap, st));
    FCLSH_HIP(hipStreamSynchronize(st));
    return FCLSH_OK;
}

constexpr int64_t kSeenBudget = int64_t(1) << 30;

// Whether a synchronous batch dedupes with per-query bitmaps.
bool use_seen(const Index &ix, int64_t nq) {
    return ix.prm.sparse && nq * ((ix.n + 31) / 32) * 4 <= kSeenBudget;
}

// Synchronous form (fclsh_query_batch): sizes the workspace, runs the device
// pipeline, reads the result size back once and grows and reruns if an
// internal buffer overflowed.
fclsh_status query_batch(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, int rq,
                         const int32_t *rq_vec, hipStream_t st, uint64_t *offsets, uint32_t *ids, int64_t ids_cap,
                         int64_t *total_out, const CsrRows *sq) {
    const int L = ix.prm.L();
    int64_t pairs = std::max<int64_t>(ws.cap_pairs, std::max<int64_t>(1 << 16, nq * 16));
    int64_t spills = std::max<int64_t>(ws.cap_spill, 1 << 16);
    const int64_t dense_words = ix.prm.sparse ? nq * ix.W : 0;
    // sparse queries take a bitmap per query when all of them fit in
    // kSeenBudget bytes (else the first-shared-table rule)
    const int64_t seen_words = use_seen(ix, nq) ? nq * ((ix.n + 31) / 32) : 0;
    QueryCtrl h{};
    for (int attempt = 0; attempt < 3; ++attempt) {
        FCLSH_TRY(ws_reserve(ws, nq, L, pairs, spills, dense_words, seen_words));
        FCLSH_TRY(query_batch_async(ix, ws, queries, nq, rq, rq_vec, st, offsets, ids, ids_cap, sq));
        FCLSH_HIP(hipMemcpyAsync(&h, ws.ctrl, sizeof h, hipMemcpyDeviceToHost, st));
        FCLSH_HIP(hipStreamSynchronize(st));
        if (h.status & kQueryBadRows)
            return fail(FCLSH_EINVAL, "malformed query rows:%s%s%s",
                        (h.status >> kQueryBadShift) & kCsrBadPtr ? " bad row bounds" : "",
                        (h.status >> kQueryBadShift) & kCsrBadCol ? " column outside [0, d)" : "",
                        (h.status >> kQueryBadShift) & kCsrBadOrder ? " columns not strictly ascending" : "");
        if (!(h.status & (kQueryPairOverflow | kQuerySpillOverflow))) break;
        if (h.status & kQueryPairOverflow) pairs = int64_t(h.pairs) + int64_t(h.pairs >> 3) + 1;
        if (h.status & kQuerySpillOverflow) spills = int64_t(h.spills) + int64_t(h.spills >> 3) + 1;
    }
    if (h.status & (kQueryPairOverflow | kQuerySpillOverflow))
        return fail(FCLSH_ENOMEM, "query buffers kept overflowing");
    *total_out = int64_t(h.total);
    if (h.status & kQueryIdsOverflow) {
        ws.pending_nq = nq;
        ws.pending_total = int64_t(h.total);
        ws.pending_offsets = offsets;
        return fail(FCLSH_ECAPACITY, "%lld ids do not fit the output capacity %lld", (long long)h.total,
                    (long long)ids_cap);
    }
    return FCLSH_OK;
}

// The plain path: every query gets its own launch sequence and
// synchronisation (hash, lookup, verify, compaction), with no batching.
fclsh_status query_plain(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, int rq,
                         hipStream_t st, uint64_t *offsets, uint32_t *ids, int64_t ids_cap, int64_t *total_out) {
    std::vector<uint64_t> off(size_t(nq) + 1, 0);
    int64_t run = 0;
    bool over = false;
    for (int64_t i = 0; i < nq; ++i) {
        int64_t got = 0;
        const int64_t room = over ? 0 : ids_cap - run;
        fclsh_status s = query_batch(ix, ws, queries + i * ix.W, 1, rq, nullptr, st, ws.offs1,
                                     room > 0 ? ids + run : nullptr, room > 0 ? room : 0, &got);
        if (s == FCLSH_ECAPACITY) {
            over = true;
        } else if (s != FCLSH_OK) {
            return s;
        }
        run += got;
        off[size_t(i) + 1] = uint64_t(run);
    }
    ws.pending_nq = -1;  // per-query batches above; nothing to finish for the whole
    FCLSH_HIP(hipMemcpyAsync(offsets, off.data(), off.size() * 8, hipMemcpyHostToDevice, st));
    FCLSH_HIP(hipStreamSynchronize(st));
    *total_out = run;
    if (over)
        return fail(FCLSH_ECAPACITY, "%lld ids do not fit the output capacity %lld", (long long)run,
                    (long long)ids_cap);
    return FCLSH_OK;
}

}  // namespace fclsh
