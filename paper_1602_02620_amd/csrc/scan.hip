// Device-wide exclusive scan of uint64 values, used for the CSR offsets of a
// query batch.  Three phases: per-tile sums, a scan of the tile sums
// (recursive on the partials), and per-tile exclusive scans plus the tile's
// base.  The caller provides the partials (scan_partials_needed(n) entries),
// so the scan allocates nothing and can be captured in a HIP graph.
#include "common.h"

namespace fclsh {

namespace {

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

}  // namespace

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

}  // namespace fclsh
