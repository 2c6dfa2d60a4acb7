// Input check of the validation mode: the operands must be canonical CSR
// (Section 2.1.1) before any kernel gathers through them.
//
// Two launches per matrix, in stream order:
//   k_check_rpt  rpt monotone, rpt[0] >= 0 and rpt[rows] - rpt[0] == nnz
//                (the caller's entry count), so every entry index that the
//                row pointer names lies in [rpt[0], rpt[0] + nnz);
//   k_check_col  only when the first found nothing: every column index in
//                [0, cols) and strictly ascending inside its row.
// Each failure sets a bit of *flags (1 = row pointer, 2 = column index out
// of range, 4 = columns not strictly ascending); the second kernel reads
// col only after the first has cleared the row pointer, so a bad row
// pointer never leads to an out-of-range read.
#include "opsp_internal.h"

namespace opsp {

__global__ __launch_bounds__(256) void k_check_rpt(int64_t rows, int64_t nnz,
                                                   const int64_t *__restrict__ rpt,
                                                   unsigned int *__restrict__ flags) {
    const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i0 == 0) bad = rpt[0] < 0 || rpt[rows] - rpt[0] != nnz;
    for (int64_t i = i0; i < rows; i += (int64_t)gridDim.x * 256) bad |= rpt[i + 1] < rpt[i];
    if (__ballot(bad) && lane_id() == 0) atomicOr(flags, 1u);
}

// One wave per row (grid-stride over rows): lane l checks entries
// rpt[i] + l, rpt[i] + l + 64, ... against the entry before each.
__global__ __launch_bounds__(256) void k_check_col(int64_t rows, int64_t cols,
                                                   const int64_t *__restrict__ rpt,
                                                   const int32_t *__restrict__ col,
                                                   unsigned int *__restrict__ flags) {
    if (*flags & 1u) return;   // row pointer rejected: col is not read
    const int l = lane_id();
    const int64_t waves = (int64_t)gridDim.x * 4;
    unsigned int f = 0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < rows; i += waves) {
        const int64_t p0 = rpt[i], p1 = rpt[i + 1];
        for (int64_t p = p0 + l; p < p1; p += 64) {
            const int32_t c = col[p];
            if (c < 0 || (int64_t)c >= cols) f |= 2u;
            if (p > p0 && col[p - 1] >= c) f |= 4u;
        }
    }
    const unsigned int u = (__ballot(f & 2u) ? 2u : 0u) | (__ballot(f & 4u) ? 4u : 0u);
    if (u && l == 0) atomicOr(flags, u);
}

hipError_t launch_check_csr(int64_t rows, int64_t cols, int64_t nnz, const int64_t *rpt,
                            const int32_t *col, unsigned int *flags, hipStream_t s) {
    int64_t g = (rows + 1 + 255) / 256;
    g = g < 2048 ? (g > 0 ? g : 1) : 2048;
    hipLaunchKernelGGL(k_check_rpt, dim3((unsigned)g), dim3(256), 0, s, rows, nnz, rpt, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || rows == 0 || nnz == 0) return e;
    int64_t gc = (rows + 3) / 4;
    gc = gc < 4096 ? gc : 4096;
    hipLaunchKernelGGL(k_check_col, dim3((unsigned)gc), dim3(256), 0, s, rows, cols, rpt, col, flags);
    return hipGetLastError();
}

}  // namespace opsp
