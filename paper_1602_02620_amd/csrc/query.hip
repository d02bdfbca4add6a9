// Queries: Strategy 2 of Sec. 2.2 as the three steps of Sec. 4.1.
//
//   S1  the query's L keys, by the same Alg. 2 kernel as the build
//   S2  per table, the query's bucket (directory bin + binary search in the
//       sorted keys); #Collisions is the sum of the bucket sizes
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
#include <algorithm>

#include "common.h"

namespace fclsh {

namespace {

// First table (in (part, v) order) where x and q share the masked value, or
// -1 if there is none (then d(x, q) exceeds what the family covers).
__device__ int first_shared_table(const uint64_t *__restrict__ x, const uint64_t *__restrict__ q, int W,
                                  int d, const int32_t *__restrict__ part, const int32_t *__restrict__ col,
                                  int t, int mbits, int Lp, uint64_t last_mask) {
    for (int p = 0; p < t; ++p) {
        uint32_t B[kMaxLogD];
#pragma unroll
        for (int l = 0; l < kMaxLogD; ++l) B[l] = l < mbits ? (1u << l) : 0u;
        for (int w = 0; w < W; ++w) {
            uint64_t diff = x[w] ^ q[w];
            if (w == W - 1) diff &= last_mask;
            while (diff) {
                const int c = w * 64 + __builtin_ctzll(diff);
                diff &= diff - 1;
                if (part[c] != p) continue;
                const uint32_t uc = uint32_t(col[c]);
                // constrain the basis to v with <v, uc> = 0: the odd vector
                // with the lowest leading bit is dropped and XORed into the
                // other odd ones (their leading bits are higher, so they stay
                // distinct)
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
        }
#pragma unroll
        for (int l = 0; l < kMaxLogD; ++l)
            if (B[l]) return p * Lp + int(B[l]) - 1;
    }
    return -1;
}

// S2: per (query, table) the query's directory bin [start, start+len) in
// table T and the number of entries in it whose key equals the query's key
// (the bucket size, i.e. this table's share of #Collisions).
__global__ void lookup_kernel(const uint32_t *__restrict__ qkeys, int64_t nq, int L,
                              const uint32_t *__restrict__ tkeys, const uint32_t *__restrict__ dir, int64_t n,
                              int dir_bits, uint32_t *__restrict__ rstart, uint32_t *__restrict__ rlen,
                              uint32_t *__restrict__ rmatch) {
    const int64_t total = nq * L;
    const int64_t nb = int64_t(1) << dir_bits;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += int64_t(gridDim.x) * blockDim.x) {
        const int T = int(g / nq);
        const int64_t qi = g - int64_t(T) * nq;
        const uint32_t key = qkeys[g];
        const uint32_t *tk = tkeys + int64_t(T) * n;
        const uint32_t *dr = dir + int64_t(T) * (nb + 1);
        const uint32_t bin = key >> (31 - dir_bits);
        const uint32_t lo = dr[bin], hi = dr[bin + 1];
        uint32_t m = 0;
        for (uint32_t j = lo; j < hi; ++j) m += tk[j] == key;
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

// S3 + emission.  One wave per (query, table) item; lanes stride over the
// query's directory bin and keep the entries of its bucket (equal key).  Each reported (query, id) pair takes a slot from a global cursor
// (one atomic per wave); slots past `cap` are dropped and recounted by the
// host with a larger buffer.
__global__ __launch_bounds__(256) void verify_kernel(
    const uint64_t *__restrict__ pts, int W, int d, const uint64_t *__restrict__ queries, int64_t nq,
    int L, const uint32_t *__restrict__ tkeys, const uint32_t *__restrict__ tids, int64_t n,
    const uint32_t *__restrict__ qkeys, const uint32_t *__restrict__ rstart, const uint32_t *__restrict__ rmatch,
    const uint32_t *__restrict__ rlen, int rq, const int32_t *__restrict__ part,
    const int32_t *__restrict__ col, int t, int mbits, int Lp, uint64_t last_mask,
    unsigned long long *__restrict__ cursor, uint32_t *__restrict__ out_q, uint32_t *__restrict__ out_id,
    int64_t cap, uint32_t *__restrict__ qcount) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x >> 6);
    const int64_t items = nq * L;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t it = __builtin_amdgcn_readfirstlane(wave0); it < items; it += nwaves) {
        if (rmatch[it] == 0) continue;
        const uint32_t cnt = rlen[it];
        const int64_t qi = it / L;
        const int T = int(it - qi * L);
        const uint32_t st = rstart[it];
        const uint32_t qkey = qkeys[int64_t(T) * nq + qi];
        const uint64_t *qp = queries + qi * W;
        const uint32_t *ids = tids + int64_t(T) * n + st;
        const uint32_t *bk = tkeys + int64_t(T) * n + st;
        for (uint32_t j0 = 0; j0 < cnt; j0 += 64) {
            const uint32_t j = j0 + lane;
            bool emit = false;
            uint32_t id = 0;
            if (j < cnt && bk[j] == qkey) {
                id = ids[j];
                const uint64_t *xp = pts + int64_t(id) * W;
                int dist = 0;
                for (int w = 0; w < W; ++w) {
                    uint64_t df = xp[w] ^ qp[w];
                    if (w == W - 1) df &= last_mask;
                    dist += __popcll(df);
                }
                if (dist <= rq)
                    emit = first_shared_table(xp, qp, W, d, part, col, t, mbits, Lp, last_mask) == T;
            }
            const uint64_t bal = __ballot(emit);
            if (bal) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(cursor, (unsigned long long)__popcll(bal));
                base = __shfl(base, 0, 64);
                if (lane == 0) atomicAdd(&qcount[qi], uint32_t(__popcll(bal)));
                if (emit) {
                    const unsigned long long slot = base + __popcll(bal & lt);
                    if (slot < (unsigned long long)cap) {
                        out_q[slot] = uint32_t(qi);
                        out_id[slot] = id;
                    }
                }
            }
        }
    }
}

__global__ void widen_counts_kernel(const uint32_t *__restrict__ c32, int64_t nq, uint64_t *__restrict__ c64) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nq) c64[i] = c32[i];
}

__global__ void set_last_offset_kernel(uint64_t *offsets, int64_t nq, const unsigned long long *cursor) {
    offsets[nq] = *cursor;
}

unsigned grid_for(int64_t work, int per_block, unsigned cap = 1u << 20) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

}  // namespace



namespace {

template <class T>
fclsh_status regrow(T **p, int64_t have, int64_t want, const char *what) {
    if (want <= have && *p) return FCLSH_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(p), size_t(std::max<int64_t>(want, 1)) * sizeof(T)) != hipSuccess)
        return fail(FCLSH_ENOMEM, "device allocation for %s failed", what);
    return FCLSH_OK;
}

}  // namespace

fclsh_status ws_reserve(QueryWorkspace &ws, int64_t nq, int L, int64_t pairs) {
    const int64_t items = nq * L;
    if (items > ws.cap_items) {
        FCLSH_TRY(regrow(&ws.qkeys, 0, items, "query keys"));
        FCLSH_TRY(regrow(&ws.rstart, 0, items, "query ranges"));
        FCLSH_TRY(regrow(&ws.rcount, 0, items, "query ranges"));
        FCLSH_TRY(regrow(&ws.rmatch, 0, items, "query ranges"));
        ws.cap_items = items;
    }
    if (nq + 1 > ws.cap_q) {
        FCLSH_TRY(regrow(&ws.qcount, 0, nq + 1, "query counts"));
        FCLSH_TRY(regrow(&ws.qcount64, 0, nq + 1, "query counts"));
        ws.cap_q = nq + 1;
    }
    if (!ws.cursor) FCLSH_TRY(regrow(&ws.cursor, 0, 1, "cursor"));
    if (!ws.offs1) FCLSH_TRY(regrow(&ws.offs1, 0, 2, "plain offsets"));
    if (pairs > ws.cap_pairs) {
        FCLSH_TRY(regrow(&ws.pq, 0, pairs, "result pairs"));
        FCLSH_TRY(regrow(&ws.pid, 0, pairs, "result pairs"));
        FCLSH_TRY(regrow(&ws.sk, 0, pairs, "result sort"));
        FCLSH_TRY(regrow(&ws.sv, 0, pairs, "result sort"));
        FCLSH_TRY(regrow(&ws.tk, 0, pairs, "result sort"));
        FCLSH_TRY(regrow(&ws.tv, 0, pairs, "result sort"));
        ws.cap_pairs = pairs;
    }
    return FCLSH_OK;
}

void ws_release(QueryWorkspace &ws) {
    void *ps[] = {ws.qkeys, ws.rstart, ws.rcount, ws.rmatch, ws.qcount, ws.qcount64, ws.offs1, ws.cursor,
                  ws.pq, ws.pid, ws.sk, ws.sv, ws.tk, ws.tv};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    ws = QueryWorkspace{};
}

static uint64_t last_word_mask(int d) {
    return (d % 64) ? ((uint64_t(1) << (d % 64)) - 1) : ~uint64_t(0);
}

// S1 + S2 for a batch; leaves keys and ranges in the workspace.
fclsh_status query_lookup(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, hipStream_t st) {
    const int L = ix.prm.L();
    FCLSH_TRY(launch_hash(ix, queries, nq, ws.qkeys, nq, st));
    hipLaunchKernelGGL(lookup_kernel, dim3(grid_for(nq * L, 256)), dim3(256), 0, st, ws.qkeys, nq, L,
                       ix.tkeys, ix.dir, ix.n, ix.dir_bits, ws.rstart, ws.rcount, ws.rmatch);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

fclsh_status query_collisions(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq,
                              uint64_t *coll, hipStream_t st) {
    FCLSH_TRY(ws_reserve(ws, nq, ix.prm.L(), 0));
    FCLSH_TRY(query_lookup(ix, ws, queries, nq, st));
    hipLaunchKernelGGL(collisions_kernel, dim3(grid_for(nq, 256)), dim3(256), 0, st, ws.rmatch, nq,
                       ix.prm.L(), coll);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

// Full batched query into CSR (see fclsh_query_batch).
fclsh_status query_batch(Index &ix, QueryWorkspace &ws, const uint64_t *queries, int64_t nq, int rq,
                         hipStream_t st, uint64_t *offsets, uint32_t *ids, int64_t ids_cap,
                         int64_t *total_out) {
    const int L = ix.prm.L();
    if (nq == 0) {
        FCLSH_HIP(hipMemsetAsync(offsets, 0, 8, st));
        FCLSH_HIP(hipStreamSynchronize(st));
        *total_out = 0;
        return FCLSH_OK;
    }
    int64_t pairs_cap = std::max<int64_t>(ws.cap_pairs, std::max<int64_t>(1 << 16, nq * 8));
    FCLSH_TRY(ws_reserve(ws, nq, L, pairs_cap));
    FCLSH_TRY(query_lookup(ix, ws, queries, nq, st));
    const uint64_t lm = last_word_mask(ix.prm.d);
    unsigned long long total = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        FCLSH_HIP(hipMemsetAsync(ws.cursor, 0, 8, st));
        FCLSH_HIP(hipMemsetAsync(ws.qcount, 0, size_t(nq) * 4, st));
        const int64_t items = nq * L;
        hipLaunchKernelGGL(verify_kernel, dim3(grid_for(items, 4, 65536)), dim3(256), 0, st, ix.pts, ix.W,
                           ix.prm.d, queries, nq, L, ix.tkeys, ix.tids, ix.n, ws.qkeys, ws.rstart, ws.rmatch,
                           ws.rcount, rq, ix.dpart, ix.dcol,
                           ix.prm.t, ix.prm.rp + 1, ix.prm.Lp(), lm, ws.cursor, ws.pq, ws.pid, ws.cap_pairs,
                           ws.qcount);
        FCLSH_HIP(hipGetLastError());
        FCLSH_HIP(hipMemcpyAsync(&total, ws.cursor, 8, hipMemcpyDeviceToHost, st));
        FCLSH_HIP(hipStreamSynchronize(st));
        if (int64_t(total) <= ws.cap_pairs) break;
        FCLSH_TRY(ws_reserve(ws, nq, L, int64_t(total) + (int64_t(total) >> 3)));
    }
    // CSR offsets from the per-query counts
    hipLaunchKernelGGL(widen_counts_kernel, dim3(grid_for(nq, 256)), dim3(256), 0, st, ws.qcount, nq,
                       ws.qcount64);
    FCLSH_HIP(hipGetLastError());
    Scratch scr;
    FCLSH_TRY(exclusive_scan_u64(ws.qcount64, offsets, nq, nullptr, scr, st));
    hipLaunchKernelGGL(set_last_offset_kernel, dim3(1), dim3(1), 0, st, offsets, nq, ws.cursor);
    FCLSH_HIP(hipGetLastError());
    *total_out = int64_t(total);
    if (int64_t(total) > ids_cap) {
        FCLSH_HIP(hipStreamSynchronize(st));
        return fail(FCLSH_ECAPACITY, "%lld ids do not fit the output capacity %lld", (long long)total,
                    (long long)ids_cap);
    }
    if (total > 0) {
        // canonical order: by query, ids ascending (two stable LSD sorts)
        const int idbits = std::max(1, ilog2_ceil(uint64_t(ix.n)));
        const int qbits = std::max(1, ilog2_ceil(uint64_t(nq)));
        FCLSH_TRY(radix_sort_pairs(ws.pid, ws.pq, ws.sk, ws.sv, ws.tk, ws.tv, 1, int64_t(total), 0, idbits, scr,
                                   st));
        FCLSH_TRY(radix_sort_pairs(ws.sv, ws.sk, ws.pq, ids, ws.tk, ws.tv, 1, int64_t(total), 0, qbits, scr, st));
    }
    FCLSH_HIP(hipStreamSynchronize(st));
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
        fclsh_status s = query_batch(ix, ws, queries + i * ix.W, 1, rq, st, ws.offs1,
                                     room > 0 ? ids + run : nullptr, room > 0 ? room : 0, &got);
        if (s == FCLSH_ECAPACITY) {
            over = true;
        } else if (s != FCLSH_OK) {
            return s;
        }
        run += got;
        off[size_t(i) + 1] = uint64_t(run);
    }
    FCLSH_HIP(hipMemcpyAsync(offsets, off.data(), off.size() * 8, hipMemcpyHostToDevice, st));
    FCLSH_HIP(hipStreamSynchronize(st));
    *total_out = run;
    if (over)
        return fail(FCLSH_ECAPACITY, "%lld ids do not fit the output capacity %lld", (long long)run,
                    (long long)ids_cap);
    return FCLSH_OK;
}

}  // namespace fclsh
