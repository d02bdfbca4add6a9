// Validation of points given by their nonzero coordinates (CSR rows): the
// kernels that read such rows clamp and skip what is malformed, and this
// check reports it.
#include <algorithm>

#include "common.h"

namespace fclsh {

namespace {

// Densifies m rows into bit vectors of W words each (out must be zero):
// a wave per row, lanes striding over its nonzeros; columns outside [0, d)
// are skipped.
__global__ void csr_densify_kernel(const int64_t *__restrict__ ptr, const int32_t *__restrict__ cols, int64_t m,
                                   int64_t nnz, int d, int W, unsigned long long *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; i < m;
         i += (int64_t(gridDim.x) * blockDim.x) >> 6) {
        const int64_t a = min(max(ptr[i], int64_t(0)), nnz);
        const int64_t b = min(max(ptr[i + 1], a), nnz);
        for (int64_t e = a + lane; e < b; e += 64) {
            const uint32_t c = uint32_t(cols[e]);
            if (c < uint32_t(d)) atomicOr(&out[i * W + (c >> 6)], 1ull << (c & 63));
        }
    }
}

__global__ void zero_words_kernel(unsigned long long *__restrict__ p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0ull;
}

// A wave per row (grid-stride over rows): the row's bounds, then its
// columns, each lane comparing its column with the one before it.
__global__ void csr_check_kernel(const int64_t *__restrict__ ptr, const int32_t *__restrict__ cols, int64_t m,
                                 int64_t nnz, int d, uint32_t *flag, int shift) {
    uint32_t bad = 0;
    const int lane = threadIdx.x & 63;
    const int64_t w0 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (w0 == 0 && lane == 0 && (ptr[0] != 0 || ptr[m] != nnz)) bad |= kCsrBadPtr;
    for (int64_t i = w0; i < m; i += (int64_t(gridDim.x) * blockDim.x) >> 6) {
        const int64_t a = ptr[i], b = ptr[i + 1];
        if (a < 0 || b < a || b > nnz) {
            bad |= kCsrBadPtr;
            continue;
        }
        for (int64_t e = a + lane; e < b; e += 64) {
            const int32_t c = cols[e];
            if (c < 0 || c >= d) bad |= kCsrBadCol;
            if (e > a && c <= cols[e - 1]) bad |= kCsrBadOrder;
        }
    }
    if (bad) atomicOr(flag, bad << shift);
}

}  // namespace

fclsh_status csr_check(const CsrRows &rows, int64_t m, int d, uint32_t *flag, int shift, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((m + 3) / 4, 4096);  // four rows per block of four waves
    hipLaunchKernelGGL(csr_check_kernel, dim3(unsigned(std::max<int64_t>(blocks, 1))), dim3(256), 0, st, rows.ptr,
                       rows.cols, m, rows.nnz, d, flag, shift);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

fclsh_status csr_densify(const CsrRows &rows, int64_t m, int d, uint64_t *out, hipStream_t st) {
    const int W = words_of(d);
    const int64_t words = m * W;
    auto *o = reinterpret_cast<unsigned long long *>(out);
    hipLaunchKernelGGL(zero_words_kernel, dim3(unsigned(std::clamp<int64_t>((words + 255) / 256, 1, 4096))), dim3(256),
                       0, st, o, words);
    FCLSH_HIP(hipGetLastError());
    hipLaunchKernelGGL(csr_densify_kernel, dim3(unsigned(std::clamp<int64_t>((m + 3) / 4, 1, 4096))), dim3(256), 0,
                       st, rows.ptr, rows.cols, m, rows.nnz, d, W, o);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

}  // namespace fclsh
