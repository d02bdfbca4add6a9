// Generic device-wide primitives: a stable least-significant-digit radix sort
// of (uint32 key, uint32 value) pairs over 8-bit digits, batched over
// equal-length segments, and an exclusive scan of uint64 values.  They put the
// query results in canonical order (by query, ids ascending) and build CSR
// offsets.  Each radix pass is
//   histogram  per (segment, tile) digit counts, in LDS
//   scan       per segment, exclusive scan in digit-major, tile-minor order
//   scatter    per tile: stable ranks from wave ballots (each lane learns the
//              lanes holding its digit from 8 ballots), per-wave running
//              counts in LDS, a block-local reorder in LDS so that each
//              digit's run is written out contiguously.
// Without input values, the first pass takes each element's index as value.
#include "common.h"

namespace fclsh {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 16;                  // rounds of 64 per wave
constexpr int kTile = kThreads * kItems;    // 4096 elements per tile
constexpr int kRadix = 256;

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t *__restrict__ keys,
                                                              int64_t len, int shift, int bits,
                                                              uint32_t *__restrict__ hist,
                                                              int nblk) {
    __shared__ uint32_t h[kRadix];
    const int seg = blockIdx.y;
    const int blk = blockIdx.x;
    const int R = 1 << bits;
    for (int i = threadIdx.x; i < R; i += kThreads) h[i] = 0;
    __syncthreads();
    const uint32_t *kp = keys + int64_t(seg) * len;
    const int64_t beg = int64_t(blk) * kTile;
    const int64_t end = min(len, beg + kTile);
    const uint32_t mask = uint32_t(R - 1);
    for (int64_t e = beg + threadIdx.x; e < end; e += kThreads)
        atomicAdd(&h[(kp[e] >> shift) & mask], 1u);
    __syncthreads();
    for (int dgt = threadIdx.x; dgt < R; dgt += kThreads)
        hist[(int64_t(seg) * R + dgt) * nblk + blk] = h[dgt];
}

// Block-wide exclusive scan of one value per thread (1024 threads max).
template <int NT>
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t *sh, uint64_t *total) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    uint64_t x = v;
    // inclusive scan within the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (tid == 0) {
        uint64_t run = 0;
        for (int w = 0; w < NT / 64; ++w) {
            const uint64_t c = sh[w];
            sh[w] = run;
            run += c;
        }
        sh[NT / 64] = run;
    }
    __syncthreads();
    const uint64_t res = x - v + sh[wave];
    if (total) *total = sh[NT / 64];
    __syncthreads();
    return res;
}

// Per segment: exclusive scan of cnt[seg][0..count) in place, plus `add`
// (the segment's base offset) on every element.
__global__ __launch_bounds__(1024) void seg_scan_kernel(uint32_t *__restrict__ cnt, int64_t count,
                                                        int64_t seg_base_stride) {
    __shared__ uint64_t sh[1024 / 64 + 1];
    const int seg = blockIdx.x;
    uint32_t *c = cnt + int64_t(seg) * count;
    const int64_t per = (count + 1023) / 1024;
    const int64_t beg = min(count, int64_t(threadIdx.x) * per);
    const int64_t end = min(count, beg + per);
    uint64_t sum = 0;
    for (int64_t i = beg; i < end; ++i) sum += c[i];
    uint64_t run = block_excl_scan<1024>(sum, sh, nullptr) + uint64_t(seg) * uint64_t(seg_base_stride);
    for (int64_t i = beg; i < end; ++i) {
        const uint32_t x = c[i];
        c[i] = uint32_t(run);  // offsets are relative within the segment's base
        run += x;
    }
    (void)seg_base_stride;
}

__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t len, int shift, int bits, const uint32_t *__restrict__ offs,
    int nblk) {
    __shared__ uint32_t wc[kWaves][kRadix];  // per-wave running counts, then wave offsets
    __shared__ uint32_t dstart[kRadix];      // block-local start of each digit
    __shared__ uint32_t gpos[kRadix];        // global start of this tile's run of each digit
    __shared__ uint32_t sk[kTile];
    __shared__ uint32_t sv[kTile];
    __shared__ uint64_t scan_sh[kThreads / 64 + 1];

    const int seg = blockIdx.y;
    const int blk = blockIdx.x;
    const int R = 1 << bits;
    const uint32_t mask = uint32_t(R - 1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t segoff = int64_t(seg) * len;
    const int64_t beg = int64_t(blk) * kTile;
    const int cnt = int(min<int64_t>(kTile, len - beg));

    for (int i = threadIdx.x; i < kWaves * kRadix; i += kThreads) (&wc[0][0])[i] = 0;
    for (int dgt = threadIdx.x; dgt < R; dgt += kThreads)
        gpos[dgt] = offs[(int64_t(seg) * R + dgt) * nblk + blk];
    __syncthreads();

    uint32_t rk[kItems], rv[kItems], rr[kItems];
    volatile uint32_t *mywc = wc[wave];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int e = wave * (64 * kItems) + it * 64 + lane;
        const bool ok = e < cnt;
        uint32_t key = 0, val = 0;
        if (ok) {
            key = kin[segoff + beg + e];
            val = vin ? vin[segoff + beg + e] : uint32_t(beg + e);
        }
        const uint32_t dg = (key >> shift) & mask;
        uint64_t same = __ballot(ok);
        for (int b = 0; b < bits; ++b) {
            const uint64_t bb = __ballot((dg >> b) & 1u);
            same &= ((dg >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t before = uint32_t(__popcll(same & lt));
        const uint32_t base = ok ? mywc[dg] : 0u;
        // the lowest lane of each digit group advances the running count
        if (ok && before == 0) mywc[dg] = base + uint32_t(__popcll(same));
        rk[it] = key;
        rv[it] = val;
        rr[it] = ok ? base + before : 0xFFFFFFFFu;
    }
    __syncthreads();
    // per digit: wave offsets and block total
    uint32_t tot = 0;
    if (threadIdx.x < R) {
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = wc[w][threadIdx.x];
            wc[w][threadIdx.x] = tot;
            tot += c;
        }
    }
    const uint64_t ds = block_excl_scan<kThreads>(threadIdx.x < R ? tot : 0u, scan_sh, nullptr);
    if (threadIdx.x < R) dstart[threadIdx.x] = uint32_t(ds);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        if (rr[it] != 0xFFFFFFFFu) {
            const uint32_t dg = (rk[it] >> shift) & mask;
            const uint32_t lp = dstart[dg] + wc[wave][dg] + rr[it];
            sk[lp] = rk[it];
            sv[lp] = rv[it];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kThreads) {
        const uint32_t key = sk[j];
        const uint32_t dg = (key >> shift) & mask;
        const int64_t dst = segoff + int64_t(gpos[dg]) + (j - int64_t(dstart[dg]));
        kout[dst] = key;
        vout[dst] = sv[j];
    }
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of uint64 (three phases, recursive on the partials).
// ---------------------------------------------------------------------------
constexpr int kScanNT = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanNT * kScanPer;

__global__ __launch_bounds__(kScanNT) void scan_reduce_kernel(const uint64_t *__restrict__ in,
                                                              int64_t n, uint64_t *__restrict__ part) {
    __shared__ uint64_t sh[kScanNT / 64 + 1];
    const int64_t beg = int64_t(blockIdx.x) * kScanTile;
    uint64_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = beg + int64_t(k) * kScanNT + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint64_t tot;
    (void)block_excl_scan<kScanNT>(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanNT) void scan_apply_kernel(const uint64_t *__restrict__ in,
                                                             uint64_t *__restrict__ out, int64_t n,
                                                             const uint64_t *__restrict__ part) {
    __shared__ uint64_t sh[kScanNT / 64 + 1];
    const int64_t beg = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanPer;
    uint64_t v[kScanPer];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = beg + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    uint64_t run = block_excl_scan<kScanNT>(s, sh, nullptr) + (part ? part[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = beg + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

__global__ void scan_total_kernel(const uint64_t *in, const uint64_t *excl, int64_t n, uint64_t *total) {
    *total = n ? excl[n - 1] + in[n - 1] : 0;
}

}  // namespace

fclsh_status radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                              uint32_t *vals_out, uint32_t *tmp_keys, uint32_t *tmp_vals,
                              int64_t nseg, int64_t len, int begin_bit, int end_bit, Scratch &scr,
                              hipStream_t st) {
    if (nseg == 0 || len == 0) return FCLSH_OK;
    if (len > 0xFFFFFFFFll) return fail(FCLSH_EINVAL, "segment too long for the radix sort");
    if (nseg > 65535) return fail(FCLSH_EINVAL, "too many segments for one radix sort");
    const int nblk = int((len + kTile - 1) / kTile);
    int npass = (end_bit - begin_bit + 7) / 8;
    if (npass <= 0) {
        FCLSH_HIP(hipMemcpyAsync(keys_out, keys_in, size_t(nseg * len) * 4, hipMemcpyDeviceToDevice, st));
        return FCLSH_OK;
    }
    uint32_t *hist;
    FCLSH_TRY(scr.get(&hist, size_t(nseg) * kRadix * nblk, "radix histogram"));
    // ping-pong so that the last pass writes keys_out / vals_out
    const uint32_t *ck = keys_in;
    const uint32_t *cv = vals_in;
    for (int ps = 0; ps < npass; ++ps) {
        const int shift = begin_bit + 8 * ps;
        const int bits = std::min(8, end_bit - shift);
        const bool last = ps == npass - 1;
        const bool to_out = ((npass - 1 - ps) % 2) == 0;
        uint32_t *nk = to_out ? keys_out : tmp_keys;
        uint32_t *nv = to_out ? vals_out : tmp_vals;
        (void)last;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nblk, unsigned(nseg)), dim3(kThreads), 0, st, ck, len,
                           shift, bits, hist, nblk);
        FCLSH_HIP(hipGetLastError());
        hipLaunchKernelGGL(seg_scan_kernel, dim3(unsigned(nseg)), dim3(1024), 0, st, hist,
                           int64_t(1 << bits) * nblk, int64_t(0));
        FCLSH_HIP(hipGetLastError());
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblk, unsigned(nseg)), dim3(kThreads), 0, st, ck, cv,
                           nk, nv, len, shift, bits, hist, nblk);
        FCLSH_HIP(hipGetLastError());
        ck = nk;
        cv = nv;
    }
    return FCLSH_OK;
}

int64_t scan_partials_needed(int64_t n) {
    int64_t need = 0;
    for (int64_t m = (n + kScanTile - 1) / kScanTile; m > 1; m = (m + kScanTile - 1) / kScanTile) need += m;
    return need + 1;
}

fclsh_status exclusive_scan_u64_ws(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *partials,
                                   hipStream_t st) {
    if (n <= 0) return FCLSH_OK;
    const int64_t nblk = (n + kScanTile - 1) / kScanTile;
    if (nblk == 1) {
        hipLaunchKernelGGL(scan_apply_kernel, dim3(1), dim3(kScanNT), 0, st, in, out, n, (const uint64_t *)nullptr);
        FCLSH_HIP(hipGetLastError());
        return FCLSH_OK;
    }
    uint64_t *part = partials;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(unsigned(nblk)), dim3(kScanNT), 0, st, in, n, part);
    FCLSH_HIP(hipGetLastError());
    FCLSH_TRY(exclusive_scan_u64_ws(part, part, nblk, partials + nblk, st));
    hipLaunchKernelGGL(scan_apply_kernel, dim3(unsigned(nblk)), dim3(kScanNT), 0, st, in, out, n,
                       (const uint64_t *)part);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

fclsh_status exclusive_scan_u64(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *total,
                                Scratch &scr, hipStream_t st) {
    if (n <= 0) {
        if (total) FCLSH_HIP(hipMemsetAsync(total, 0, 8, st));
        return FCLSH_OK;
    }
    const int64_t nblk = (n + kScanTile - 1) / kScanTile;
    uint64_t *last_in = nullptr;
    if (total) {
        // keep the last input: the scan may run in place
        FCLSH_TRY(scr.get(&last_in, 1, "scan"));
        FCLSH_HIP(hipMemcpyAsync(last_in, in + n - 1, 8, hipMemcpyDeviceToDevice, st));
    }
    if (nblk == 1) {
        hipLaunchKernelGGL(scan_apply_kernel, dim3(1), dim3(kScanNT), 0, st, in, out, n,
                           (const uint64_t *)nullptr);
        FCLSH_HIP(hipGetLastError());
    } else {
        uint64_t *part;
        FCLSH_TRY(scr.get(&part, size_t(nblk), "scan partials"));
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(unsigned(nblk)), dim3(kScanNT), 0, st, in, n, part);
        FCLSH_HIP(hipGetLastError());
        FCLSH_TRY(exclusive_scan_u64(part, part, nblk, nullptr, scr, st));
        hipLaunchKernelGGL(scan_apply_kernel, dim3(unsigned(nblk)), dim3(kScanNT), 0, st, in, out, n,
                           (const uint64_t *)part);
        FCLSH_HIP(hipGetLastError());
    }
    if (total) {
        hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, st, last_in, out + n - 1, int64_t(1),
                           total);
        FCLSH_HIP(hipGetLastError());
    }
    return FCLSH_OK;
}

}  // namespace fclsh
