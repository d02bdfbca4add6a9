// C ABI of the library (declared in include/fclsh.h): argument checking, the
// index object and its device memory, per-stream query workspaces.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

namespace fclsh {


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

// hash, pass-1 histogram, pass-1 scan, pass-1 scatter, pass-1b split, pass-2 fast, pass-2 stable
constexpr int kRebuildPhases = 7;

struct IndexHandle {
    Index ix;
    std::mutex mu;
    std::map<hipStream_t, QueryWorkspace *> ws;
    // build scratch (hash keys, two partition buffers, histograms), held
    // between builds only when the index keeps it (keep_build_scratch, or once
    // it has been rebuilt)
    uint32_t *keys = nullptr;
    uint32_t *tk = nullptr;
    uint32_t *tv = nullptr;
    uint32_t *aux = nullptr;
    uint64_t scratch_bytes = 0;
    bool keep_scratch = false;
    // pass 2's counters of the last build, copied to pinned host memory
    // behind an event (read before the next build chooses its pass-2 form)
    uint32_t *host_cnt = nullptr;
    hipEvent_t cnt_ev = nullptr;
    bool cnt_pending = false;
    BuildMode cnt_mode = BuildMode::kFull;  // form of the build the counters come from
    // graphs captured on the index hold its buffers: fclsh_index_free only
    // marks a handle with live graphs as released, and the last graph's free
    // destroys it
    int live_graphs = 0;
    bool released = false;
    QueryWorkspace *workspace(hipStream_t st) {
        std::lock_guard<std::mutex> g(mu);
        auto it = ws.find(st);
        if (it != ws.end()) return it->second;
        auto *w = new QueryWorkspace();
        ws[st] = w;
        return w;
    }
};

static void free_build_scratch(IndexHandle *h) {
    for (uint32_t **p : {&h->keys, &h->tk, &h->tv, &h->aux}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    h->scratch_bytes = 0;
}

// All four scratch buffers or none.
static fclsh_status alloc_build_scratch(IndexHandle *h) {
    if (h->keys) return FCLSH_OK;
    const Index &ix = h->ix;
    const size_t entries = size_t(ix.prm.L()) * size_t(ix.n);
    const size_t aux = table_build_scratch_bytes(ix.prm.L(), ix.n, ix.dir_bits);
    struct {
        uint32_t **p;
        size_t bytes;
    } want[] = {{&h->keys, entries * 4}, {&h->tk, entries * 4}, {&h->tv, entries * 4}, {&h->aux, aux}};
    for (auto &w : want) {
        if (hipMalloc(reinterpret_cast<void **>(w.p), std::max<size_t>(w.bytes, 1)) != hipSuccess) {
            (void)hipGetLastError();
            *w.p = nullptr;
            free_build_scratch(h);
            return fail(FCLSH_ENOMEM, "device allocation of %zu bytes of build scratch failed", w.bytes);
        }
        h->scratch_bytes += w.bytes;
    }
    return FCLSH_OK;
}

static void destroy_handle(IndexHandle *h) {
    for (auto &kv : h->ws) {
        ws_release(*kv.second);
        delete kv.second;
    }
    h->ws.clear();
    if (h->cnt_ev) (void)hipEventSynchronize(h->cnt_ev);
    if (h->cnt_ev) (void)hipEventDestroy(h->cnt_ev);
    if (h->host_cnt) (void)hipHostFree(h->host_cnt);
    free_build_scratch(h);
    dev_free_all(&h->ix);
    delete h;
}

static void lookup_tuning(Index &ix);

static size_t estimate_index_bytes(const Params &p, int64_t n, int W, int64_t nnz, int dir_bits) {
    const size_t L = size_t(p.L());
    size_t b = p.sparse ? size_t(n + 1) * 8 + size_t(nnz) * 4 : size_t(n) * W * 8;  // point copy
    b += L * size_t(n) * (4 + size_t(table_key_bytes(dir_bits)));  // table ids + keys
    b += L * ((size_t(1) << dir_bits) + 1) * 4;          // directories
    b += 3 * L * size_t(n) * 4;                          // build scratch: keys + 2 partition buffers
    b += table_build_scratch_bytes(int64_t(L), n, dir_bits);  // histograms, group starts, lists
    return b;
}

// The next build's pass-2 form (BuildMode), from pass 2's counters of the
// last build.  A rebuild hashes the index's own points with its fixed hash
// functions, so its groups and bins are those of the last build, whose
// counters therefore predict it exactly:
//   no group sent off the slot branch  -> kSlotAll
//   at most 1 % of the groups          -> kSlotOnly
//   more                               -> kFull.
// (A kSlotAll build does not look at bin sizes: it keeps its form.)  Waits
// for the last build's counters if needed.
static fclsh_status take_build_counts(IndexHandle *h) {
    if (!h->cnt_pending) return FCLSH_OK;
    FCLSH_HIP(hipEventSynchronize(h->cnt_ev));
    h->cnt_pending = false;
    Index &ix = h->ix;
    if (h->cnt_mode == BuildMode::kSlotAll) return FCLSH_OK;
    const int64_t groups =
        int64_t(ix.prm.L()) << (8 + table_split_bits(ix.n, ix.dir_bits) - table_merge_bits(ix.n, ix.dir_bits));
    // groups listed for the second kernel + groups that took the ballot
    // branch (none in a slot-only build)
    const int64_t off_slot = int64_t(h->host_cnt[0]) + int64_t(h->host_cnt[1]);
    ix.build_mode = off_slot == 0              ? BuildMode::kSlotAll
                    : off_slot * 100 <= groups ? BuildMode::kSlotOnly
                                               : BuildMode::kFull;
    return FCLSH_OK;
}

// Enqueues hash + table build on st; sync = wait for it (and take the
// counters) before returning.  marks (optional, kRebuildPhases + 1 events):
// before the hash, after the hash, then after each table kernel.
static fclsh_status hash_and_bucket(IndexHandle *h, hipStream_t st, hipEvent_t *marks = nullptr, bool sync = true) {
    Index &ix = h->ix;
    const int64_t L = ix.prm.L();
    if (!h->host_cnt &&
        hipHostMalloc(reinterpret_cast<void **>(&h->host_cnt), 2 * sizeof(uint32_t), hipHostMallocDefault) !=
            hipSuccess) {
        h->host_cnt = nullptr;
        return fail(FCLSH_ENOMEM, "pinned host allocation failed");
    }
    if (!h->cnt_ev && hipEventCreateWithFlags(&h->cnt_ev, hipEventDisableTiming) != hipSuccess) {
        h->cnt_ev = nullptr;
        return fail(FCLSH_EDEVICE, "hipEventCreate failed");
    }
    FCLSH_TRY(take_build_counts(h));
    FCLSH_TRY(alloc_build_scratch(h));
    if (marks) FCLSH_HIP(hipEventRecord(marks[0], st));
    if (ix.prm.sparse)
        FCLSH_TRY(launch_hash_sparse(ix, CsrRows{ix.sptr, ix.scols, ix.nnz}, ix.n, h->keys, ix.n, st));
    else
        FCLSH_TRY(launch_hash(ix, ix.pts, ix.n, h->keys, ix.n, st));
    if (marks) FCLSH_HIP(hipEventRecord(marks[1], st));
    FCLSH_TRY(build_tables_2pass(h->keys, L, ix.n, ix.dir_bits, h->tk, h->tv, h->aux, ix.tkeys, ix.tids, ix.dir,
                                 ix.build_mode, ix.p2_fallback, st, marks ? marks + 2 : nullptr));
    h->cnt_mode = ix.build_mode;
    FCLSH_HIP(hipMemcpyAsync(h->host_cnt, table_build_counts(h->aux, L, ix.n, ix.dir_bits), 2 * sizeof(uint32_t),
                             hipMemcpyDeviceToHost, st));
    FCLSH_HIP(hipEventRecord(h->cnt_ev, st));
    h->cnt_pending = true;
    if (sync) {
        FCLSH_HIP(hipStreamSynchronize(st));
        FCLSH_TRY(take_build_counts(h));
        if (!h->keep_scratch) free_build_scratch(h);
    }
    return FCLSH_OK;
}

// The device rows of a sparse build, checked before the index copies them.
static fclsh_status check_rows(const CsrRows &rows, int64_t m, int d, hipStream_t st) {
    uint32_t *flag = nullptr;
    if (hipMalloc(&flag, sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FCLSH_ENOMEM, "device allocation of a check flag failed");
    }
    uint32_t bad = 0;
    fclsh_status s = FCLSH_OK;
    if (hipMemsetAsync(flag, 0, sizeof(uint32_t), st) != hipSuccess) s = fail(FCLSH_EDEVICE, "hipMemsetAsync failed");
    if (s == FCLSH_OK) s = csr_check(rows, m, d, flag, 0, st);
    if (s == FCLSH_OK && (hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, st) != hipSuccess ||
                          hipStreamSynchronize(st) != hipSuccess))
        s = fail(FCLSH_EDEVICE, "reading the row check failed");
    (void)hipFree(flag);
    if (s != FCLSH_OK) return s;
    if (bad)
        return fail(FCLSH_EINVAL, "malformed rows:%s%s%s", bad & kCsrBadPtr ? " bad row bounds" : "",
                    bad & kCsrBadCol ? " column outside [0, d)" : "",
                    bad & kCsrBadOrder ? " columns not strictly ascending" : "");
    return FCLSH_OK;
}

// d_points (dense [n][W] words) or rows (sparse; prm.sparse) is the input.
static fclsh_status build_common(const uint64_t *d_points, const CsrRows *rows, int64_t n, Params &&prm,
                                 uint64_t budget, bool keep_scratch, int32_t test_flags, hipStream_t st,
                                 fclsh_index *out) {
    if (!out) return fail(FCLSH_EINVAL, "out is null");
    *out = nullptr;
    if (prm.sparse != (rows != nullptr)) return fail(FCLSH_EINVAL, "point format does not match the parameters");
    if (!rows && !d_points) return fail(FCLSH_EINVAL, "d_points is null");
    if (rows && (!rows->ptr || rows->nnz < 0 || (rows->nnz > 0 && !rows->cols)))
        return fail(FCLSH_EINVAL, "null row arrays or negative nnz");
    if (rows && rows->nnz > 0x7FFFFFFFll) return fail(FCLSH_EUNSUPPORTED, "nnz above 2^31-1");
    if (n < 1 || n > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
    FCLSH_TRY(check_params(prm));
    if (int64_t(prm.L()) > 65535) return fail(FCLSH_EUNSUPPORTED, "L=%d tables exceed 65535", prm.L());
    auto *h = new IndexHandle();
    Index &ix = h->ix;
    ix.prm = std::move(prm);
    ix.W = words_of(ix.prm.d);
    ix.n = n;
    ix.dir_bits = table_dir_bits(n);
    ix.key_bytes = table_key_bytes(ix.dir_bits);
    ix.budget = budget;
    (void)hipGetDevice(&ix.device);
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ix.device) == hipSuccess && prop.multiProcessorCount > 0)
            ix.num_cus = prop.multiProcessorCount;
        (void)hipGetLastError();
    }
    lookup_tuning(ix);
    ix.p2_fallback = (test_flags & FCLSH_TEST_P2_FALLBACK) != 0;
    h->keep_scratch = keep_scratch;
    auto bail = [&](fclsh_status s) {
        destroy_handle(h);
        return s;
    };
    if (rows) ix.nnz = rows->nnz;
    if (budget) {
        const size_t need = estimate_index_bytes(ix.prm, n, ix.W, ix.nnz, ix.dir_bits);
        if (need > budget)
            return bail(fail(FCLSH_ENOMEM, "index needs about %zu bytes, budget is %llu", need,
                             (unsigned long long)budget));
    }
    const int64_t L = ix.prm.L();
    fclsh_status s;
    if (rows && (s = check_rows(*rows, n, ix.prm.d, st))) return bail(s);
    if (rows) {
        if ((s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.sptr), size_t(n + 1) * 8, "point rows")) ||
            (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.scols), size_t(ix.nnz) * 4, "point columns")))
            return bail(s);
    } else if ((s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.pts), size_t(n) * ix.W * 8, "points"))) {
        return bail(s);
    }
    if ((s = dev_alloc(&ix, &ix.tkeys, size_t(L * n) * size_t(ix.key_bytes), "table keys")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.tids), size_t(L * n) * 4, "table ids")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.dir),
                       size_t(L) * ((size_t(1) << ix.dir_bits) + 1) * 4, "directory")) ||
        (s = dev_alloc(&ix, reinterpret_cast<void **>(&ix.dpc), size_t(ix.prm.dd()) * 4, "params")))
        return bail(s);
    if ((s = build_hash_plan(&ix))) return bail(s);
    {
        // (part, column) of each coordinate in one word for the dedupe test:
        // parts and columns (< 2^kMaxLogD) each fit 16 bits
        std::vector<uint32_t> pc(size_t(ix.prm.dd()));
        for (int c = 0; c < ix.prm.dd(); ++c)
            pc[size_t(c)] = uint32_t(ix.prm.part[c]) << 16 | uint32_t(ix.prm.col[c]);
        if (hipMemcpy(ix.dpc, pc.data(), pc.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(FCLSH_EDEVICE, "parameter upload failed"));
    }
    if (rows) {
        if (hipMemcpyAsync(ix.sptr, rows->ptr, size_t(n + 1) * 8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            (ix.nnz > 0 &&
             hipMemcpyAsync(ix.scols, rows->cols, size_t(ix.nnz) * 4, hipMemcpyDeviceToDevice, st) != hipSuccess))
            return bail(fail(FCLSH_EDEVICE, "point row copy failed"));
    } else {
        const int64_t total = n * ix.W;
        unsigned g = unsigned(std::min<int64_t>((total + 255) / 256, 65536));
        hipLaunchKernelGGL(copy_points_kernel, dim3(g), dim3(256), 0, st, d_points, ix.pts, total, ix.W,
                           last_word_mask(ix.prm.d));
        if (hipGetLastError() != hipSuccess) return bail(fail(FCLSH_EDEVICE, "point copy launch failed"));
    }
    if ((s = hash_and_bucket(h, st))) return bail(s);
    *out = reinterpret_cast<fclsh_index>(h);
    return FCLSH_OK;
}

static IndexHandle *handle(fclsh_index idx) { return reinterpret_cast<IndexHandle *>(idx); }

// Process-wide cache of autotuned launch shapes, keyed by index shape and
// device, so that a rebuilt index of the same shape starts tuned.
struct TuneKey {
    int device, d, t, rp, logn;
    bool operator<(const TuneKey &o) const {
        return std::tie(device, d, t, rp, logn) < std::tie(o.device, o.d, o.t, o.rp, o.logn);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, QueryTuning> g_tune_cache;

static TuneKey tune_key(const Index &ix) {
    return TuneKey{ix.device, ix.prm.d, ix.prm.t, ix.prm.rp, ilog2_ceil(uint64_t(ix.n))};
}

static void lookup_tuning(Index &ix) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(ix));
    if (it != g_tune_cache.end()) ix.tuning = it->second;
}

namespace {
__global__ void publish_result_kernel(const QueryCtrl *ctrl, uint64_t *out) {
    out[0] = ctrl->total;
    out[1] = ctrl->status;
}
}  // namespace

static fclsh_status publish_result(QueryWorkspace &ws, uint64_t *d_result, hipStream_t st) {
    hipLaunchKernelGGL(publish_result_kernel, dim3(1), dim3(1), 0, st, ws.ctrl, d_result);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

// Device buffers and events of one autotuning run, released on every exit.
struct DeviceBuffers {
    void *offs = nullptr;
    void *ids = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool alloc(void **p, size_t bytes) {
        if (hipMalloc(p, bytes) == hipSuccess) return true;
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    ~DeviceBuffers() {
        if (offs) (void)hipFree(offs);
        if (ids) (void)hipFree(ids);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Workspace of fclsh_query_batch_noalloc: one array per GPU, in the code
// object's static device memory, so that the call itself allocates nothing.
// In host code `scratch` only names the symbol; its address on a device comes
// from hipGetSymbolAddress with that device current, looked up once per device
// and kept in g_scratch_addr.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_addr;

static fclsh_status scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return FCLSH_OK;
    }
    int cur = -1;
    FCLSH_HIP(hipGetDevice(&cur));
    if (cur != device) FCLSH_HIP(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
        return fail(FCLSH_EDEVICE, "hipGetSymbolAddress of the no-allocation scratch failed: %s",
                    hipGetErrorString(e));
    g_scratch_addr[device] = p;
    *out = p;
    return FCLSH_OK;
}

struct GraphHandle {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    IndexHandle *owner = nullptr;
    QueryWorkspace ws;  // private: no later call on a stream can regrow it
};

// The caller's options, read up to its struct_size; fields past it keep
// their defaults (zero).
static fclsh_status read_opts(const fclsh_build_opts *in, fclsh_build_opts *out) {
    *out = fclsh_build_opts{};
    out->struct_size = sizeof(fclsh_build_opts);
    if (!in) return FCLSH_OK;
    if (in->struct_size < sizeof(uint32_t) || in->struct_size > sizeof(fclsh_build_opts))
        return fail(FCLSH_EINVAL, "opts->struct_size %u outside [4, %zu]", in->struct_size, sizeof(fclsh_build_opts));
    std::memcpy(reinterpret_cast<char *>(out) + sizeof(uint32_t), reinterpret_cast<const char *>(in) + sizeof(uint32_t),
                in->struct_size - sizeof(uint32_t));
    out->struct_size = sizeof(fclsh_build_opts);
    if (out->test_flags & ~FCLSH_TEST_P2_FALLBACK) return fail(FCLSH_EINVAL, "unknown opts->test_flags bits");
    return FCLSH_OK;
}

// A handle a call may use: not null and not released.
static bool usable(fclsh_index idx) {
    return idx && !reinterpret_cast<IndexHandle *>(idx)->released;
}

// A usable handle whose points have the format of the call (dense words or
// sparse rows).
static fclsh_status need_format(fclsh_index idx, bool sparse) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    if (reinterpret_cast<IndexHandle *>(idx)->ix.prm.sparse != sparse)
        return fail(FCLSH_EINVAL, sparse ? "the index holds dense points: use the calls on bit vectors"
                                         : "the index holds sparse points: use the calls on rows");
    return FCLSH_OK;
}

}  // namespace fclsh

using namespace fclsh;

extern "C" {

const char *fclsh_last_error(void) { return last_error_cstr(); }

fclsh_status fclsh_preprocessing(int64_t n, int32_t r, double c, int32_t *replicate, int32_t *partitions) {
    if (!replicate || !partitions) return fail(FCLSH_EINVAL, "null output pointer");
    if (n < 2 || r <= 0 || !(c > 1.0)) return fail(FCLSH_EINVAL, "need n >= 2, r > 0 and c > 1");
    const double logn = std::log2(double(n)), cr = c * double(r);
    *replicate = 1;
    *partitions = 1;
    if (cr < logn) *replicate = int32_t(std::floor(logn / cr));
    else if (cr > logn) *partitions = int32_t(std::min(std::ceil(cr / logn), double(1 << 30)));
    return FCLSH_OK;
}

fclsh_status fclsh_derive_params(int32_t d, int32_t r, uint64_t seed, const fclsh_build_opts *opts,
                                 int32_t *t_out, int32_t *r_part_out, int32_t *part, int32_t *col, uint64_t *b) {
    if (!t_out || !r_part_out || !part || !col || !b) return fail(FCLSH_EINVAL, "null output pointer");
    if (d > kMaxSparseDims) return fail(FCLSH_EUNSUPPORTED, "d=%d exceeds %d", d, kMaxSparseDims);
    fclsh_build_opts o;
    FCLSH_TRY(read_opts(opts, &o));
    Params p;
    // the draws do not depend on the point format; d above kMaxDims is for
    // sparse points only
    FCLSH_TRY(derive_params(d, r, seed, &o, &p, d > kMaxDims));
    *t_out = p.t;
    *r_part_out = p.rp;
    for (int c = 0; c < p.dd(); ++c) {
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
    fclsh_build_opts o;
    FCLSH_TRY(read_opts(opts, &o));
    Params p;
    FCLSH_TRY(derive_params(d, r, seed, &o, &p));
    return build_common(d_points, nullptr, n, std::move(p), o.mem_budget_bytes, o.keep_build_scratch != 0,
                        o.test_flags, reinterpret_cast<hipStream_t>(stream), out);
}

fclsh_status fclsh_build_index_sparse(const int64_t *d_ptr, const int32_t *d_cols, int64_t n, int64_t nnz, int32_t d,
                                      int32_t r, uint64_t seed, const fclsh_build_opts *opts, void *stream,
                                      fclsh_index *out) {
    if (out) *out = nullptr;
    if (d > kMaxSparseDims) return fail(FCLSH_EUNSUPPORTED, "d=%d exceeds %d", d, kMaxSparseDims);
    fclsh_build_opts o;
    FCLSH_TRY(read_opts(opts, &o));
    Params p;
    FCLSH_TRY(derive_params(d, r, seed, &o, &p, true));
    const CsrRows rows{d_ptr, d_cols, nnz};
    return build_common(nullptr, &rows, n, std::move(p), o.mem_budget_bytes, o.keep_build_scratch != 0,
                        o.test_flags, reinterpret_cast<hipStream_t>(stream), out);
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
    return build_common(d_points, nullptr, n, std::move(p), 0, false, 0, reinterpret_cast<hipStream_t>(stream), out);
}

void fclsh_index_free(fclsh_index idx) {
    if (!idx) return;
    IndexHandle *h = handle(idx);
    {
        std::lock_guard<std::mutex> g(h->mu);
        if (h->released) return;
        h->released = true;
        if (h->live_graphs > 0) {
            // the graphs keep the tables, points and parameters; what only
            // later calls would have used goes now
            for (auto &kv : h->ws) {
                ws_release(*kv.second);
                delete kv.second;
            }
            h->ws.clear();
            free_build_scratch(h);
            return;
        }
    }
    destroy_handle(h);
}

fclsh_status fclsh_index_memory(fclsh_index idx, uint64_t *index_bytes, uint64_t *build_scratch_bytes,
                                uint64_t *workspace_bytes) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    IndexHandle *h = handle(idx);
    std::lock_guard<std::mutex> g(h->mu);
    uint64_t w = 0;
    for (auto &kv : h->ws) w += ws_bytes(*kv.second);
    if (index_bytes) *index_bytes = h->ix.bytes_owned;
    if (build_scratch_bytes) *build_scratch_bytes = h->scratch_bytes;
    if (workspace_bytes) *workspace_bytes = w;
    return FCLSH_OK;
}

fclsh_status fclsh_index_info(fclsh_index idx, int32_t *d, int32_t *r, int32_t *t, int32_t *r_part, int64_t *n,
                              int32_t *L, int32_t *dir_bits, int32_t *group_bits) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    const Index &ix = handle(idx)->ix;
    if (d) *d = ix.prm.d;
    if (r) *r = ix.prm.r;
    if (t) *t = ix.prm.t;
    if (r_part) *r_part = ix.prm.rp;
    if (n) *n = ix.n;
    if (L) *L = ix.prm.L();
    if (dir_bits) *dir_bits = ix.dir_bits;
    if (group_bits) *group_bits = 8 + table_split_bits(ix.n, ix.dir_bits) - table_merge_bits(ix.n, ix.dir_bits);
    return FCLSH_OK;
}

fclsh_status fclsh_index_params(fclsh_index idx, int32_t *part, int32_t *col, uint64_t *b) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    const Index &ix = handle(idx)->ix;
    for (int c = 0; c < ix.prm.dd(); ++c) {
        if (part) part[c] = ix.prm.part[c];
        if (col) col[c] = ix.prm.col[c];
        if (b) b[c] = ix.prm.b[c];
    }
    return FCLSH_OK;
}

fclsh_status fclsh_hash(fclsh_index idx, const uint64_t *d_pts, int64_t m, uint32_t *d_keys, void *stream) {
    FCLSH_TRY(need_format(idx, false));
    if (m < 0 || m > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "m=%lld out of range", (long long)m);
    if (m && (!d_pts || !d_keys)) return fail(FCLSH_EINVAL, "null buffer");
    return launch_hash(handle(idx)->ix, d_pts, m, d_keys, m, reinterpret_cast<hipStream_t>(stream));
}

fclsh_status fclsh_hash_sparse(fclsh_index idx, const int64_t *d_ptr, const int32_t *d_cols, int64_t m, int64_t nnz,
                               uint32_t *d_keys, void *stream) {
    FCLSH_TRY(need_format(idx, true));
    if (m < 0 || m > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "m=%lld out of range", (long long)m);
    if (nnz < 0 || (m && (!d_ptr || !d_keys)) || (nnz > 0 && !d_cols)) return fail(FCLSH_EINVAL, "bad buffers");
    return launch_hash_sparse(handle(idx)->ix, CsrRows{d_ptr, d_cols, nnz}, m, d_keys, m,
                              reinterpret_cast<hipStream_t>(stream));
}

fclsh_status fclsh_index_tables(fclsh_index idx, const void **d_tkeys, int32_t *key_bytes, const uint32_t **d_tids,
                                const uint32_t **d_dir, const uint64_t **d_points) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    const Index &ix = handle(idx)->ix;
    if (d_tkeys) *d_tkeys = ix.tkeys;
    if (key_bytes) *key_bytes = ix.key_bytes;
    if (d_tids) *d_tids = ix.tids;
    if (d_dir) *d_dir = ix.dir;
    if (d_points) *d_points = ix.pts;
    return FCLSH_OK;
}

fclsh_status fclsh_index_table_keys(fclsh_index idx, int32_t T0, int32_t T1, uint32_t *d_keys, void *stream) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    const Index &ix = handle(idx)->ix;
    if (T0 < 0 || T1 < T0 || T1 > ix.prm.L() || (T1 > T0 && !d_keys))
        return fail(FCLSH_EINVAL, "tables [%d, %d) outside [0, %d) or null output", T0, T1, ix.prm.L());
    return expand_table_keys(ix.tkeys, ix.key_bytes, ix.dir, ix.n, ix.dir_bits, T0, T1, d_keys,
                             reinterpret_cast<hipStream_t>(stream));
}

fclsh_status fclsh_index_rebuild(fclsh_index idx, void *stream) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    handle(idx)->keep_scratch = true;  // rebuilds keep their scratch
    return hash_and_bucket(handle(idx), reinterpret_cast<hipStream_t>(stream));
}

fclsh_status fclsh_index_build_mode(fclsh_index idx, int32_t *mode) {
    if (!usable(idx) || !mode) return fail(FCLSH_EINVAL, "null argument or released index");
    IndexHandle *h = handle(idx);
    FCLSH_TRY(take_build_counts(h));
    *mode = int32_t(h->ix.build_mode);
    return FCLSH_OK;
}

fclsh_status fclsh_index_rebuild_async(fclsh_index idx, void *stream) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    handle(idx)->keep_scratch = true;
    return hash_and_bucket(handle(idx), reinterpret_cast<hipStream_t>(stream), nullptr, false);
}

fclsh_status fclsh_index_rebuild_timed(fclsh_index idx, void *stream, float *phase_ms, int32_t nphase) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    if (!phase_ms || nphase < kRebuildPhases) return fail(FCLSH_EINVAL, "phase_ms needs %d entries", kRebuildPhases);
    hipEvent_t ev[kRebuildPhases + 1] = {};
    fclsh_status s = FCLSH_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            s = fail(FCLSH_EDEVICE, "hipEventCreate failed");
            break;
        }
    handle(idx)->keep_scratch = true;
    if (s == FCLSH_OK) s = hash_and_bucket(handle(idx), reinterpret_cast<hipStream_t>(stream), ev);
    for (int k = 0; s == FCLSH_OK && k < kRebuildPhases; ++k)
        if (hipEventElapsedTime(&phase_ms[k], ev[k], ev[k + 1]) != hipSuccess)
            s = fail(FCLSH_EDEVICE, "hipEventElapsedTime failed");
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return s;
}

fclsh_status fclsh_query_batch_sparse(fclsh_index idx, const int64_t *d_ptr, const int32_t *d_cols, int64_t nq,
                                      int64_t nnz, int32_t r_query, void *stream, uint64_t *d_offsets,
                                      uint32_t *d_ids, int64_t ids_capacity, int64_t *total_out) {
    FCLSH_TRY(need_format(idx, true));
    if (!total_out || !d_offsets) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || nq > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "nq=%lld out of range", (long long)nq);
    if (nnz < 0 || (nq && !d_ptr) || (nnz > 0 && !d_cols)) return fail(FCLSH_EINVAL, "bad query rows");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    if (r_query < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (r_query > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", r_query, h->ix.prm.r);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const CsrRows rows{d_ptr, d_cols, nnz};
    return query_batch(h->ix, *h->workspace(st), nullptr, nq, r_query, nullptr, st, d_offsets, d_ids, ids_capacity,
                       total_out, &rows);
}

fclsh_status fclsh_query_batch(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                               void *stream, uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                               int64_t *total_out) {
    FCLSH_TRY(need_format(idx, false));
    if (!total_out || !d_offsets) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || nq > 0x7FFFFFFFll) return fail(FCLSH_EINVAL, "nq=%lld out of range", (long long)nq);
    if (nq && !d_queries) return fail(FCLSH_EINVAL, "null queries");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    if (r_query < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (r_query > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", r_query, h->ix.prm.r);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_batch(h->ix, *h->workspace(st), d_queries, nq, r_query, nullptr, st, d_offsets, d_ids,
                       ids_capacity, total_out);
}

fclsh_status fclsh_query_batch_finish(fclsh_index idx, void *stream, const uint64_t *d_offsets, uint32_t *d_ids,
                                      int64_t ids_capacity, int64_t *total_out) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    if (!total_out || !d_offsets) return fail(FCLSH_EINVAL, "null output pointer");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_finish(h->ix, *h->workspace(st), st, d_offsets, d_ids, ids_capacity, total_out);
}

fclsh_status fclsh_query_collisions(fclsh_index idx, const uint64_t *d_queries, int64_t nq, void *stream,
                                    uint64_t *d_collisions) {
    FCLSH_TRY(need_format(idx, false));
    if (nq < 0 || (nq && (!d_queries || !d_collisions))) return fail(FCLSH_EINVAL, "bad arguments");
    if (nq == 0) return FCLSH_OK;
    IndexHandle *h = handle(idx);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_collisions(h->ix, *h->workspace(st), d_queries, nq, d_collisions, st);
}

fclsh_status fclsh_query_cost(fclsh_index idx, const uint64_t *d_queries, int64_t nq, void *stream,
                              uint64_t *d_collisions, uint64_t *d_candidates) {
    FCLSH_TRY(need_format(idx, false));
    if (nq < 0 || nq > 0x7FFFFFFFll || (nq && (!d_queries || !d_collisions || !d_candidates)))
        return fail(FCLSH_EINVAL, "bad arguments");
    if (nq == 0) return FCLSH_OK;
    IndexHandle *h = handle(idx);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_cost(h->ix, *h->workspace(st), d_queries, nq, d_collisions, d_candidates, st);
}

fclsh_status fclsh_query_cost_sparse(fclsh_index idx, const int64_t *d_ptr, const int32_t *d_cols, int64_t nq,
                                     int64_t nnz, void *stream, uint64_t *d_collisions, uint64_t *d_candidates) {
    FCLSH_TRY(need_format(idx, true));
    if (nq < 0 || nq > 0x7FFFFFFFll || nnz < 0 || (nq && (!d_ptr || !d_collisions || !d_candidates)) ||
        (nnz > 0 && !d_cols))
        return fail(FCLSH_EINVAL, "bad arguments");
    if (nq == 0) return FCLSH_OK;
    IndexHandle *h = handle(idx);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const CsrRows rows{d_ptr, d_cols, nnz};
    FCLSH_TRY(check_rows(rows, nq, h->ix.prm.d, st));
    return query_cost(h->ix, *h->workspace(st), nullptr, nq, d_collisions, d_candidates, st, &rows);
}

fclsh_status fclsh_linear_scan(const uint64_t *d_points, int64_t n, int32_t d, const uint64_t *d_queries,
                               int64_t nq, int32_t r, void *stream, uint64_t *d_offsets, uint32_t *d_ids,
                               int64_t ids_capacity, int64_t *total_out) {
    if (!total_out || !d_offsets) return fail(FCLSH_EINVAL, "null output pointer");
    if (n < 1 || n > 0x7FFFFFFFll || !d_points) return fail(FCLSH_EINVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
    if (d < 1) return fail(FCLSH_EINVAL, "d=%d must be positive", d);
    if (r < 0) return fail(FCLSH_EINVAL, "negative radius");
    if (nq < 0 || nq > 65535 || (nq && !d_queries)) return fail(FCLSH_EINVAL, "nq=%lld outside [0, 65535]", (long long)nq);
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (nq == 0) {
        static const uint64_t zero = 0;
        FCLSH_HIP(hipMemcpyAsync(d_offsets, &zero, 8, hipMemcpyHostToDevice, st));
        FCLSH_HIP(hipStreamSynchronize(st));
        *total_out = 0;
        return FCLSH_OK;
    }
    return linear_scan(d_points, n, d, d_queries, nq, r, st, d_offsets, d_ids, ids_capacity, total_out);
}

fclsh_status fclsh_query_plain(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                               void *stream, uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                               int64_t *total_out) {
    FCLSH_TRY(need_format(idx, false));
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

fclsh_status fclsh_query_batch_radii(fclsh_index idx, const uint64_t *d_queries, int64_t nq,
                                     const int32_t *d_radii, int32_t max_radius, void *stream,
                                     uint64_t *d_offsets, uint32_t *d_ids, int64_t ids_capacity,
                                     int64_t *total_out) {
    FCLSH_TRY(need_format(idx, false));
    if (!total_out || !d_offsets) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || nq > 0x7FFFFFFFll || (nq && (!d_queries || !d_radii))) return fail(FCLSH_EINVAL, "bad queries");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    if (max_radius < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (max_radius > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", max_radius, h->ix.prm.r);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return query_batch(h->ix, *h->workspace(st), d_queries, nq, 0, d_radii, st, d_offsets, d_ids, ids_capacity,
                       total_out);
}

fclsh_status fclsh_query_reserve(fclsh_index idx, int64_t max_nq, int64_t pair_capacity,
                                 int64_t spill_capacity, void *stream) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    if (max_nq < 0 || pair_capacity < 1 || spill_capacity < 1) return fail(FCLSH_EINVAL, "bad capacities");
    IndexHandle *h = handle(idx);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    FCLSH_HIP(hipStreamSynchronize(st));  // buffers may be replaced
    return ws_reserve(*h->workspace(st), max_nq, h->ix.prm.L(), pair_capacity, spill_capacity);
}

fclsh_status fclsh_query_batch_async(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                                     const int32_t *d_radii, void *stream, uint64_t *d_offsets, uint32_t *d_ids,
                                     int64_t ids_capacity, uint64_t *d_result) {
    FCLSH_TRY(need_format(idx, false));
    if (!d_offsets || !d_result) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || (nq && !d_queries)) return fail(FCLSH_EINVAL, "bad queries");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    if (r_query < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (r_query > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", r_query, h->ix.prm.r);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    QueryWorkspace &ws = *h->workspace(st);
    FCLSH_TRY(query_batch_async(h->ix, ws, d_queries, nq, r_query, d_radii, st, d_offsets, d_ids, ids_capacity));
    return publish_result(ws, d_result, st);
}

fclsh_status fclsh_query_batch_noalloc(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                                       const int32_t *d_radii, void *stream, uint64_t *d_offsets, uint32_t *d_ids,
                                       int64_t ids_capacity, uint64_t *d_result) {
    FCLSH_TRY(need_format(idx, false));
    if (!d_offsets || !d_result) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || nq > 0x7FFFFFFFll || (nq && !d_queries)) return fail(FCLSH_EINVAL, "bad queries");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    if (r_query < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (r_query > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", r_query, h->ix.prm.r);
    void *base = nullptr;
    FCLSH_TRY(scratch_address(h->ix.device, &base));
    QueryWorkspace ws;
    FCLSH_TRY(ws_carve(ws, base, kNoAllocScratchBytes, nq, h->ix.prm.L()));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    FCLSH_TRY(query_batch_async(h->ix, ws, d_queries, nq, r_query, d_radii, st, d_offsets, d_ids, ids_capacity));
    return publish_result(ws, d_result, st);
}

fclsh_status fclsh_query_graph_create(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                                      const int32_t *d_radii, uint64_t *d_offsets, uint32_t *d_ids,
                                      int64_t ids_capacity, uint64_t *d_result, void *stream,
                                      fclsh_graph *out) {
    if (!out) return fail(FCLSH_EINVAL, "null output pointer");
    *out = nullptr;
    FCLSH_TRY(need_format(idx, false));
    if (!stream) return fail(FCLSH_EINVAL, "graph capture needs a non-null stream");
    if (!d_offsets || !d_result) return fail(FCLSH_EINVAL, "null output pointer");
    if (nq < 0 || (nq && !d_queries)) return fail(FCLSH_EINVAL, "bad queries");
    if (ids_capacity < 0 || (ids_capacity > 0 && !d_ids)) return fail(FCLSH_EINVAL, "bad id buffer");
    IndexHandle *h = handle(idx);
    if (r_query < 0) return fail(FCLSH_EINVAL, "negative query radius");
    if (r_query > h->ix.prm.r)
        return fail(FCLSH_ERADIUS, "query radius %d exceeds the index radius %d", r_query, h->ix.prm.r);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const QueryWorkspace &sws = *h->workspace(st);
    if (nq * h->ix.prm.L() > sws.cap_items || nq + 1 > sws.cap_q || !sws.ctrl || !sws.pq || !sws.spill)
        return fail(FCLSH_EINVAL, "query workspace of the stream not reserved for %lld queries", (long long)nq);
    auto *g = new GraphHandle();
    auto drop = [&](fclsh_status s) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        ws_release(g->ws);
        delete g;
        return s;
    };
    FCLSH_HIP(hipStreamSynchronize(st));
    fclsh_status s = ws_reserve(g->ws, std::max<int64_t>(nq, sws.cap_q - 1), h->ix.prm.L(), sws.cap_pairs,
                                sws.cap_spill);
    if (s != FCLSH_OK) return drop(s);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return drop(fail(FCLSH_EDEVICE, "hipStreamBeginCapture failed"));
    s = query_batch_async(h->ix, g->ws, d_queries, nq, r_query, d_radii, st, d_offsets, d_ids, ids_capacity);
    if (s == FCLSH_OK) s = publish_result(g->ws, d_result, st);
    const hipError_t e = hipStreamEndCapture(st, &g->graph);
    if (s != FCLSH_OK) return drop(s);
    if (e != hipSuccess) return drop(fail(FCLSH_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e)));
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        g->exec = nullptr;
        return drop(fail(FCLSH_EDEVICE, "hipGraphInstantiate failed"));
    }
    {
        std::lock_guard<std::mutex> lk(h->mu);
        ++h->live_graphs;
    }
    g->owner = h;
    *out = reinterpret_cast<fclsh_graph>(g);
    return FCLSH_OK;
}

fclsh_status fclsh_graph_launch(fclsh_graph graph, void *stream) {
    if (!graph) return fail(FCLSH_EINVAL, "null graph");
    FCLSH_HIP(hipGraphLaunch(reinterpret_cast<GraphHandle *>(graph)->exec, reinterpret_cast<hipStream_t>(stream)));
    return FCLSH_OK;
}

void fclsh_graph_free(fclsh_graph graph) {
    if (!graph) return;
    auto *g = reinterpret_cast<GraphHandle *>(graph);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    ws_release(g->ws);  // hipFree waits for the device, so no replay is still running
    IndexHandle *h = g->owner;
    delete g;
    if (!h) return;
    bool last = false;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        last = --h->live_graphs == 0 && h->released;
    }
    if (last) destroy_handle(h);
}

fclsh_status fclsh_index_set_tuning(fclsh_index idx, int32_t tile, int32_t blocks_per_cu) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    if (tile < 64 || tile > (1 << 20) || blocks_per_cu < 1 || blocks_per_cu > 64)
        return fail(FCLSH_EINVAL, "tile in [64, 2^20], blocks per CU in [1, 64]");
    QueryTuning &tu = handle(idx)->ix.tuning;
    tu.tile = tile;
    tu.blocks_per_cu = blocks_per_cu;
    return FCLSH_OK;
}

fclsh_status fclsh_index_set_schedule(fclsh_index idx, int32_t schedule) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    if (schedule != kScheduleStatic && schedule != kScheduleClaim) return fail(FCLSH_EINVAL, "schedule must be 0 or 1");
    handle(idx)->ix.tuning.schedule = schedule;
    return FCLSH_OK;
}

fclsh_status fclsh_index_get_schedule(fclsh_index idx, int32_t *schedule) {
    if (!usable(idx) || !schedule) return fail(FCLSH_EINVAL, "null argument or released index");
    *schedule = handle(idx)->ix.tuning.schedule;
    return FCLSH_OK;
}

fclsh_status fclsh_index_get_tuning(fclsh_index idx, int32_t *tile, int32_t *blocks_per_cu) {
    if (!usable(idx)) return fail(FCLSH_EINVAL, "null or released index");
    if (tile) *tile = handle(idx)->ix.tuning.tile;
    if (blocks_per_cu) *blocks_per_cu = handle(idx)->ix.tuning.blocks_per_cu;
    return FCLSH_OK;
}

fclsh_status fclsh_autotune(fclsh_index idx, const uint64_t *d_queries, int64_t nq, int32_t r_query,
                            void *stream, int32_t *tile_out, int32_t *blocks_out, float *best_ms_out) {
    FCLSH_TRY(need_format(idx, false));
    if (nq < 1 || !d_queries) return fail(FCLSH_EINVAL, "autotuning needs a sample batch");
    IndexHandle *h = handle(idx);
    if (r_query < 0 || r_query > h->ix.prm.r) return fail(FCLSH_ERADIUS, "bad query radius");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    QueryWorkspace &ws = *h->workspace(st);
    Index &ix = h->ix;
    const QueryTuning saved = ix.tuning;
    DeviceBuffers buf;
    // the answer size of the sample (the id buffer is sized to it once)
    int64_t total = 0;
    if (!buf.alloc(&buf.offs, size_t(nq + 1) * 8)) return fail(FCLSH_ENOMEM, "autotune buffers");
    fclsh_status s = query_batch(ix, ws, d_queries, nq, r_query, nullptr, st, static_cast<uint64_t *>(buf.offs),
                                 nullptr, 0, &total);
    if (s != FCLSH_OK && s != FCLSH_ECAPACITY) return s;
    if (!buf.alloc(&buf.ids, size_t(std::max<int64_t>(total, 1)) * 4)) return fail(FCLSH_ENOMEM, "autotune buffers");
    uint64_t *offs = static_cast<uint64_t *>(buf.offs);
    uint32_t *ids = static_cast<uint32_t *>(buf.ids);
    if (hipEventCreate(&buf.e0) != hipSuccess || hipEventCreate(&buf.e1) != hipSuccess)
        return fail(FCLSH_EDEVICE, "hipEventCreate failed");
    const int tiles[] = {64, 128, 256, 512, 1024, 4096};
    const int bpcs[] = {2, 4, 8, 16};
    const int schedules[] = {kScheduleStatic, kScheduleClaim};
    float best = -1.0f;
    QueryTuning best_t = saved;
    for (int tl : tiles)
        for (int bp : bpcs)
            for (int sc : schedules) {
                ix.tuning = QueryTuning{tl, bp, sc};
                // the synchronous path first: it grows the spill queue and the
                // pair buffer until this shape's run is complete
                int64_t got = 0;
                s = query_batch(ix, ws, d_queries, nq, r_query, nullptr, st, offs, ids, total, &got);
                if (s != FCLSH_OK) {
                    ix.tuning = saved;
                    return s;
                }
                FCLSH_HIP(hipEventRecord(buf.e0, st));
                for (int rep = 0; rep < 3; ++rep) {
                    s = query_batch_async(ix, ws, d_queries, nq, r_query, nullptr, st, offs, ids, total);
                    if (s != FCLSH_OK) {
                        (void)hipStreamSynchronize(st);
                        ix.tuning = saved;
                        return s;
                    }
                }
                FCLSH_HIP(hipEventRecord(buf.e1, st));
                FCLSH_HIP(hipEventSynchronize(buf.e1));
                QueryCtrl c{};
                FCLSH_HIP(hipMemcpy(&c, ws.ctrl, sizeof c, hipMemcpyDeviceToHost));
                if (c.status != 0) continue;  // an overflowing run skipped work: not a valid timing
                float ms = 0;
                FCLSH_HIP(hipEventElapsedTime(&ms, buf.e0, buf.e1));
                ms /= 3;
                if (best < 0 || ms < best) {
                    best = ms;
                    best_t = ix.tuning;
                }
            }
    if (best < 0) {
        ix.tuning = saved;
        return fail(FCLSH_EDEVICE, "no launch shape completed the sample batch");
    }
    ix.tuning = best_t;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[tune_key(ix)] = best_t;
    }
    if (tile_out) *tile_out = best_t.tile;
    if (blocks_out) *blocks_out = best_t.blocks_per_cu;
    if (best_ms_out) *best_ms_out = best;
    return FCLSH_OK;
}

}  // extern "C"
