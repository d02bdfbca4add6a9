// Linear scan (the baseline of Sec. 4, and the ground truth recall is
// measured against): for each query, every point at Hamming distance <= r,
// ids ascending.  Two passes over (query, chunk of kChunk points) tiles:
//   count   per tile, the number of points within r;
//   scan    one exclusive scan of the tile counts in (query, chunk) order,
//           which is also the output order, gives every tile its first
//           output position and every query its CSR offset;
//   write   per tile, a block-wide prefix of the match flags places each
//           matching id at its position.
// The points and queries are W-word rows; pad bits of the last word are
// masked.
#include <algorithm>

#include "common.h"

namespace fclsh {

namespace {

constexpr int kLinNT = 256;
constexpr int kLinPer = 16;                   // points per thread per tile
constexpr int kChunk = kLinNT * kLinPer;      // points per tile

__device__ inline int distance(const uint64_t *__restrict__ x, const uint64_t *__restrict__ q, int W,
                               uint64_t last_mask) {
    int dist = 0;
    for (int w = 0; w < W; ++w) {
        uint64_t df = x[w] ^ q[w];
        if (w == W - 1) df &= last_mask;
        dist += __popcll(df);
    }
    return dist;
}

// Thread t takes points t, t + kLinNT, ... of the tile (coalesced rows).
__global__ __launch_bounds__(kLinNT) void lin_count_kernel(const uint64_t *__restrict__ pts, int64_t n,
                                                           const uint64_t *__restrict__ qs, int W,
                                                           uint64_t last_mask, int r, int64_t nchunk,
                                                           uint64_t *__restrict__ counts) {
    __shared__ uint32_t wsum[kLinNT / 64];
    const int64_t q = blockIdx.y;
    const int64_t c = blockIdx.x;
    const uint64_t *qp = qs + q * W;
    uint32_t cnt = 0;
    for (int k = 0; k < kLinPer; ++k) {
        const int64_t i = c * kChunk + int64_t(k) * kLinNT + threadIdx.x;
        if (i < n) cnt += distance(pts + i * W, qp, W, last_mask) <= r;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += uint32_t(__shfl_xor(int(cnt), o, 64));
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kLinNT / 64; ++w) s += wsum[w];
        counts[q * nchunk + c] = s;
    }
}

// Points of a tile in ascending order: point k*kLinNT + t is the (k, t)-th
// in a round-major order, so the block prefix runs over rounds, then lanes.
__global__ __launch_bounds__(kLinNT) void lin_write_kernel(const uint64_t *__restrict__ pts, int64_t n,
                                                           const uint64_t *__restrict__ qs, int W,
                                                           uint64_t last_mask, int r, int64_t nchunk,
                                                           const uint64_t *__restrict__ base,
                                                           uint32_t *__restrict__ ids, int64_t ids_cap) {
    __shared__ uint32_t wsum[kLinNT / 64 + 1];
    const int64_t q = blockIdx.y;
    const int64_t c = blockIdx.x;
    const uint64_t *qp = qs + q * W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t pos = base[q * nchunk + c];
    for (int k = 0; k < kLinPer; ++k) {
        const int64_t i = c * kChunk + int64_t(k) * kLinNT + threadIdx.x;
        const bool hit = i < n && distance(pts + i * W, qp, W, last_mask) <= r;
        const uint64_t bal = __ballot(hit);
        if (lane == 0) wsum[wave] = uint32_t(__popcll(bal));
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int w = 0; w < kLinNT / 64; ++w) {
            before += w < wave ? wsum[w] : 0u;
            total += wsum[w];
        }
        if (hit) {
            const uint64_t at = pos + before + uint32_t(__popcll(bal & lt));
            if (at < uint64_t(ids_cap)) ids[at] = uint32_t(i);
        }
        pos += total;
        __syncthreads();
    }
}

__global__ void lin_offsets_kernel(const uint64_t *__restrict__ base, const uint64_t *__restrict__ counts,
                                   int64_t nq, int64_t nchunk, uint64_t *__restrict__ offsets) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < nq) offsets[q] = base[q * nchunk];
    if (q == nq) {
        const int64_t last = nq * nchunk - 1;
        offsets[nq] = base[last] + counts[last];
    }
}

uint64_t mask_of(int d) { return (d % 64) ? ((uint64_t(1) << (d % 64)) - 1) : ~uint64_t(0); }

}  // namespace

fclsh_status linear_scan(const uint64_t *pts, int64_t n, int d, const uint64_t *qs, int64_t nq, int r,
                         hipStream_t st, uint64_t *offsets, uint32_t *ids, int64_t ids_cap, int64_t *total_out) {
    const int W = words_of(d);
    const int64_t nchunk = (n + kChunk - 1) / kChunk;
    const int64_t tiles = nq * nchunk;
    if (nchunk > 0x7FFFFFFF || nq > 65535)
        return fail(FCLSH_EINVAL, "linear scan: at most 65535 queries per call");
    const int64_t npart = scan_partials_needed(tiles);
    uint64_t *buf = nullptr;
    const size_t bytes = size_t(2 * tiles + npart) * 8;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FCLSH_ENOMEM, "device allocation of %zu bytes for the linear scan failed", bytes);
    }
    uint64_t *counts = buf, *base = buf + tiles, *part = buf + 2 * tiles;
    fclsh_status s = FCLSH_OK;
    const dim3 grid{unsigned(nchunk), unsigned(nq), 1u};
    hipLaunchKernelGGL(lin_count_kernel, grid, dim3(kLinNT), 0, st, pts, n, qs, W, mask_of(d), r, nchunk, counts);
    if (hipGetLastError() != hipSuccess) s = fail(FCLSH_EDEVICE, "linear scan count launch failed");
    if (s == FCLSH_OK) s = exclusive_scan_u64_ws(counts, base, tiles, part, st);
    if (s == FCLSH_OK) {
        hipLaunchKernelGGL(lin_offsets_kernel, dim3(unsigned((nq + 256) / 256)), dim3(256), 0, st, base, counts, nq,
                           nchunk, offsets);
        if (hipGetLastError() != hipSuccess) s = fail(FCLSH_EDEVICE, "linear scan offsets launch failed");
    }
    uint64_t total = 0;
    if (s == FCLSH_OK) {
        if (hipMemcpyAsync(&total, offsets + nq, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            s = fail(FCLSH_EDEVICE, "linear scan: reading the result size failed");
    }
    if (s == FCLSH_OK && int64_t(total) <= ids_cap && total > 0) {
        hipLaunchKernelGGL(lin_write_kernel, grid, dim3(kLinNT), 0, st, pts, n, qs, W, mask_of(d), r, nchunk, base,
                           ids, ids_cap);
        if (hipGetLastError() != hipSuccess) s = fail(FCLSH_EDEVICE, "linear scan write launch failed");
    }
    const hipError_t e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (s == FCLSH_OK && e != hipSuccess) s = fail(FCLSH_EDEVICE, "linear scan failed: %s", hipGetErrorString(e));
    if (s != FCLSH_OK) return s;
    *total_out = int64_t(total);
    if (int64_t(total) > ids_cap)
        return fail(FCLSH_ECAPACITY, "%lld ids do not fit the output capacity %lld", (long long)total,
                    (long long)ids_cap);
    return FCLSH_OK;
}

}  // namespace fclsh
