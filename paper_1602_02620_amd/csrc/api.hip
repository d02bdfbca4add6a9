// C ABI of the library (declared in include/fclsh.h): argument checking, the
// index object and its device memory, per-stream query workspaces.
#include <map>
#include <mutex>

#include "common.h"

namespace fclsh {


fclsh_status Scratch::get(void **p, size_t bytes, const char *what) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes ? bytes : 1) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FCLSH_ENOMEM, "scratch allocation of %zu bytes for %s failed", bytes, what);
    }
    ptrs.push_back(q);
    *p = q;
    return FCLSH_OK;
}

fclsh_status dev_alloc(Index *ix, void **p, size_t bytes, const char *what) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes ? bytes : 1) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FCLSH_ENOMEM, "device allocation of %zu bytes for %s failed", bytes, what);
    }
    ix->owned.push_back({q, bytes});
    ix->bytes_owned += bytes;
    *p = q;
    return FCLSH_OK;
}

void dev_free_all(Index *ix) {
    for (auto &b : ix->owned) (void)hipFree(b.ptr);
    ix->owned.clear();
    ix->bytes_owned = 0;
}

namespace {

__global__ void copy_points_kernel(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, int64_t total,
                                   int W, uint64_t last_mask) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        uint64_t v = src[i];
        if (int(i % W) == W - 1) v &= last_mask;
        dst[i] = v;
    }
}

uint64_t last_word_mask(int d) { return (d % 64) ? ((uint64_t(1) << (d % 64)) - 1) : ~uint64_t(0); }

}  // namespace

struct IndexHandle {
    Index ix;
    std::mutex mu;
    std::map<hipStream_t, QueryWorkspace *> ws;
    uint32_t *keys = nullptr;  // build scratch, kept for rebuilds
    uint32_t *tk = nullptr;
    uint32_t *tv = nullptr;
    uint32_t *aux = nullptr;
    QueryWorkspace *workspace(hipStream_t st) {
        std::lock_guard<std::mutex> g(mu);
        auto it = ws.find(st);
        if (it != ws.end()) return it->second;
        auto *w = new QueryWorkspace();
        ws[st] = w;
        return w;
    }
};

static size_t estimate_index_bytes(const Params &p, int64_t n, int W, int dir_bits) {
    const size_t L = size_t(p.L());
    size_t b = size_t(n) * W * 8;                        // point copy
    b += 2 * L * size_t(n) * 4;                          // table keys + ids
    b += L * ((size_t(1) << dir_bits) + 1) * 4;          // directories
    b += 3 * L * size_t(n) * 4;                          // build scratch: keys + 2 partition buffers
    b += table_build_scratch_bytes(int64_t(L), n);       // histograms
    return b;
}

static fclsh_status hash_and_bucket(IndexHandle *h, hipStream_t st) {
    Index &ix = h->ix;
    const int64_t L = ix.prm.L();
    if (!h->keys) {
        FCLSH_TRY(dev_alloc(&ix, reinterpret_cast<void **>(&h->keys), size_t(L * ix.n) * 4, "build keys"));
        FCLSH_TRY(dev_alloc(&ix, reinterpret_cast<void **>(&h->tk), size_t(L * ix.n) * 4, "sort buffer"));
        FCLSH_TRY(dev_alloc(&ix, reinterpret_cast<void **>(&h->tv), size_t(L * ix.n) * 4, "sort buffer"));
        FCLSH_TRY(dev_alloc(&ix, reinterpret_cast<void **>(&h->aux), table_build_scratch_bytes(L, ix.n),
                            "table histograms"));
    }
    FCLSH_TRY(launch_hash(ix, ix.pts, ix.n, h->keys, ix.n, st));
    FCLSH_TRY(build_tables_2pass(h->keys, L, ix.n, ix.dir_bits, h->tk, h->tv, h->aux, ix.tkeys, ix.tids, ix.dir,
                                 st));
    FCLSH_HIP(hipStreamSynchronize(st));
    return FCLSH_OK;
}

static fclsh_status build_common(const uint64_t *d_points, int64_t n, Params &&prm, uint64_t budget,
                                 hipStream_t st, fclsh_index *out) {
    if (!out) return fail(FCLSH_EINVAL, "out is null");
    *out = nullptr;
    if (!d_points) return fail(FCLSH_EINVAL, "d_points is null");
    if (n < 1 || n > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
    FCLSH_TRY(check_params(prm));
    if (int64_t(prm.L()) > 65535) return fail(FCLSH_EUNSUPPORTED, "L=%d tables exceed 65535", prm.L());
    auto *h = new IndexHandle();
    Index &ix = h->ix;
    ix.prm = std::move(prm);
    ix.W = words_of(ix.prm.d);
    ix.n = n;
    ix.dir_bits = table_dir_bits(n);
    ix.budget = budget;
    (void)hipGetDevice(&ix.device);
    auto bail = [&](fclsh_status s) {
        dev_free_all(&ix);
        delete h;
        return s;
    };
    if (budget) {
        const size_t need = estimate_index_bytes(ix.prm, n, ix.W, ix.dir_bits);
        if (need > budget)
            return bail(fail(FCLSH_ENOMEM, "index needs about %zu bytes, budget is %llu", need,
                             (unsigned long long)budget));
    }
    const int64_t L = ix.prm.L();
    fclsh_status s;
    if ((s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.pts), size_t(n) * ix.W * 8, "points")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.tkeys), size_t(L * n) * 4, "table keys")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.tids), size_t(L * n) * 4, "table ids")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.dir),
                       size_t(L) * ((size_t(1) << ix.dir_bits) + 1) * 4, "directory")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.dpart), size_t(ix.prm.d) * 4, "params")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.dcol), size_t(ix.prm.d) * 4, "params")))
        return bail(s);
    if ((s = build_hash_plan(&ix))) return bail(s);
    if (hipMemcpy(ix.dpart, ix.prm.part.data(), size_t(ix.prm.d) * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ix.dcol, ix.prm.col.data(), size_t(ix.prm.d) * 4, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(FCLSH_EDEVICE, "parameter upload failed"));
    const int64_t total = n * ix.W;
    unsigned g = unsigned(std::min<int64_t>((total + 255) / 256, 65536));
    hipLaunchKernelGGL(copy_points_kernel, dim3(g), dim3(256), 0, st, d_points, ix.pts, total, ix.W,
                       last_word_mask(ix.prm.d));
    if (hipGetLastError() != hipSuccess) return bail(fail(FCLSH_EDEVICE, "point copy launch failed"));
    if ((s = hash_and_bucket(h, st))) return bail(s);
    *out = reinterpret_cast<fclsh_index>(h);
    return FCLSH_OK;
}

static IndexHandle *handle(fclsh_index idx) { return reinterpret_cast<IndexHandle *>(idx); }

}  // namespace fclsh

using namespace fclsh;

extern "C" {

const char *fclsh_last_error(void) { return last_error_cstr(); }

fclsh_status fclsh_derive_params(int32_t d, int32_t r, uint64_t seed, const fclsh_build_opts *opts,
                                 int32_t *t_out, int32_t *r_part_out, int32_t *part, int32_t *col, uint64_t *b) {
    if (!t_out || !r_part_out || !part || !col || !b) return fail(FCLSH_EINVAL, "null output pointer");
    if (d > kMaxDims) return fail(FCLSH_EUNSUPPORTED, "d=%d exceeds %d", d, kMaxDims);
    Params p;
    FCLSH_TRY(derive_params(d, r, seed, opts, &p));
    *t_out = p.t;
    *r_part_out = p.rp;
    for (int c = 0; c < d; ++c) {
        part[c] = p.part[c];
        col[c] = p.col[c];
        b[c] = p.b[c];
    }
    return FCLSH_OK;
}

fclsh_status fclsh_build_index(const uint64_t *d_points, int64_t n, int32_t d, int32_t r, uint64_t seed,
                               const fclsh_build_opts *opts, void *stream, fclsh_index *out) {
    if (out) *out = nullptr;
    if (d > kMaxDims) return fail(FCLSH_EUNSUPPORTED, "d=%d exceeds %d", d, kMaxDims);
    Params p;
    FCLSH_TRY(derive_params(d, r, seed, opts, &p));
    return build_common(d_points, n, std::move(p), opts ? opts->mem_budget_bytes : 0,
                        reinterpret_cast<hipStream_t>(stream), out);
}

fclsh_status fclsh_build_index_with_params(const uint64_t *d_points, int64_t n, int32_t d, int32_t r, int32_t t,
                                           int32_t r_part, const int32_t *part, const int32_t *col,
                                           const uint64_t *b, uint64_t prime, void *stream, fclsh_index *out) {
    if (out) *out = nullptr;
    if (!part || !col || !b) return fail(FCLSH_EINVAL, "null parameter array");
    if (d <= 0 || d > kMaxDims) return fail(FCLSH_EUNSUPPORTED, "d=%d outside [1, %d]", d, kMaxDims);
    if (prime != 0 && prime != kPrime) return fail(FCLSH_EUNSUPPORTED, "only the prime 2^31-1 is supported");
    Params p;
    p.d = d;
    p.r = r;
    p.t = t;
    p.rp = r_part;
    p.part.assign(part, part + d);
    p.col.assign(col, col + d);
    p.b.assign(b, b + d);
    return build_common(d_points, n, std::move(p), 0, reinterpret_cast<hipStream_t>(stream), out);
}

void fclsh_index_free(fclsh_index idx) {
    if (!idx) return;
    IndexHandle *h = handle(idx);
    for (auto &kv : h->ws) {
        ws_release(*kv.second);
        delete kv.second;
    }
    dev_free_all(&h->ix);
    delete h;
}

fclsh_status fclsh_index_info(fclsh_index idx, int32_t *d, int32_t *r, int32_t *t, int32_t *r_part, int64_t *n,
                              int32_t *L, int32_t *dir_bits) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    const Index &ix = handle(idx)->ix;
    if (d) *d = ix.prm.d;
    if (r) *r = ix.prm.r;
    if (t) *t = ix.prm.t;
    if (r_part) *r_part = ix.prm.rp;
    if (n) *n = ix.n;
    if (L) *L = ix.prm.L();
    if (dir_bits) *dir_bits = ix.dir_bits;
    return FCLSH_OK;
}

fclsh_status fclsh_index_params(fclsh_index idx, int32_t *part, int32_t *col, uint64_t *b) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    const Index &ix = handle(idx)->ix;
    for (int c = 0; c < ix.prm.d; ++c) {
        if (part) part[c] = ix.prm.part[c];
        if (col) col[c] = ix.prm.col[c];
        if (b) b[c] = ix.prm.b[c];
    }
    return FCLSH_OK;
}

fclsh_status fclsh_hash(fclsh_index idx, const uint64_t *d_pts, int64_t m, uint32_t *d_keys, void *stream) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    if (m < 0 || m > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "m=%lld out of range", (long long)m);
    if (m && (!d_pts || !d_keys)) return fail(FCLSH_EINVAL, "null buffer");
    return launch_hash(handle(idx)->ix, d_pts, m, d_keys, m, reinterpret_cast<hipStream_t>(stream));
}

fclsh_status fclsh_index_tables(fclsh_index idx, const uint32_t **d_tkeys, const uint32_t **d_tids,
                                const uint32_t **d_dir, const uint64_t **d_points) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    const Index &ix = handle(idx)->ix;
    if (d_tkeys) *d_tkeys = ix.tkeys;
    if (d_tids) *d_tids = ix.tids;
    if (d_dir) *d_dir = ix.dir;
    if (d_points) *d_points = ix.pts;
    return FCLSH_OK;
}

fclsh_status fclsh_index_rebuild(fclsh_index idx, void *stream) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    return hash_and_bucket(handle(idx), reinterpret_cast<hipStream_t>(stream));
}

fclsh_status fclsh_query_batch(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                               void *stream, uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                               int64_t *total_out) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    if (!total_out || !d_offsets) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || nq > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "nq=%lld out of range", (long long)nq);
    if (nq && !d_queries) return fail(FCLSH_EINVAL, "null queries");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    if (r_query < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (r_query > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", r_query, h->ix.prm.r);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_batch(h->ix, *h->workspace(st), d_queries, nq, r_query, st, d_offsets, d_ids, ids_capacity,
                       total_out);
}

fclsh_status fclsh_query_collisions(fclsh_index idx, const uint64_t *d_queries, int64_t nq, void *stream,
                                    uint64_t *d_collisions) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    if (nq < 0 || (nq && (!d_queries || !d_collisions))) return fail(FCLSH_EINVAL, "bad arguments");
    if (nq == 0) return FCLSH_OK;
    IndexHandle *h = handle(idx);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_collisions(h->ix, *h->workspace(st), d_queries, nq, d_collisions, st);
}

fclsh_status fclsh_query_plain(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                               void *stream, uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                               int64_t *total_out) {
    if (!idx) return fail(FCLSH_EINVAL, "null index");
    if (!total_out || !d_offsets) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || (nq && !d_queries)) return fail(FCLSH_EINVAL, "bad queries");
    IndexHandle *h = handle(idx);
    if (r_query < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (r_query > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", r_query, h->ix.prm.r);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_plain(h->ix, *h->workspace(st), d_queries, nq, r_query, st, d_offsets, d_ids, ids_capacity,
                       total_out);
}

}  // extern "C"
