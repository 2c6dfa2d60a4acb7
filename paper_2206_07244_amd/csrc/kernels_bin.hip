// Setup step, the two binning passes and the row-pointer scan
// (OpSparse Section 5, setup step; Section 5.1 Alg. 1-3; Section 5.3).
//
// gfx950 design: counting is done per wave with ballots (one LDS atomic per
// wave per bin instead of one per lane), ranks inside a bin come from
// mbcnt over the ballot mask, and each workgroup issues one global atomic
// per bin.  The numeric second pass also performs the in-place exclusive
// scan that turns per-row nnz (kept in C.rpt) into C's row pointer.
#include "opsp_internal.h"

namespace opsp {

// ---------------------------------------------------------------------------
// Setup: n_prod_i = sum over A_i* of len(B_k*), written into C.rpt[i]
// (Section 5.3 reuses C.rpt for n_prod), fused with the first symbolic
// binning pass (Alg. 1).  Each wave owns 64 consecutive rows and walks the
// flat range of their A entries with coalesced loads, so one long row does
// not serialise a single lane.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_setup(int64_t M, const int64_t *__restrict__ arpt,
                                               const int32_t *__restrict__ acol,
                                               const int64_t *__restrict__ brpt,
                                               int64_t *__restrict__ nprod, Bounds bd,
                                               Counters *__restrict__ ctr,
                                               int32_t *__restrict__ f_alen,
                                               int32_t *__restrict__ f_bmax) {
    __shared__ int64_t rs[4][65];
    __shared__ unsigned long long acc[4][64];
    __shared__ unsigned int bmx[4][64];
    __shared__ unsigned long long hist[16];
    __shared__ unsigned long long s_tot, s_max;

    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (threadIdx.x < 16) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) { s_tot = 0; s_max = 0; }
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 64;
    const int nrows = (int)(M - r0 < 0 ? 0 : (M - r0 > 64 ? 64 : M - r0));
    if (nrows > 0) {
        rs[w][l] = arpt[r0 + (l < nrows ? l : nrows)];
        if (l == 0) rs[w][64] = arpt[r0 + nrows];
    }
    acc[w][l] = 0;
    bmx[w][l] = 0;
    __syncthreads();

    if (nrows > 0) {
        const int64_t e0 = rs[w][0], e1 = rs[w][64];
        for (int64_t e = e0 + l; e < e1; e += 64) {
            const int k = acol[e];
            const int64_t len = brpt[k + 1] - brpt[k];
            // largest r in [0, nrows) with rs[r] <= e (rows may be empty)
            int lo = 0, hi = nrows - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rs[w][mid] <= e) lo = mid; else hi = mid - 1;
            }
            atomicAdd(&acc[w][lo], (unsigned long long)len);
            atomicMax(&bmx[w][lo], (unsigned)(len > 0xffffffffll ? 0xffffffffll : len));
        }
    }
    __syncthreads();

    const bool valid = l < nrows;
    const int64_t i = r0 + l;
    const unsigned long long v = valid ? acc[w][l] : 0ull;
    if (valid) {
        nprod[i] = (int64_t)v;
        if (f_alen) f_alen[i] = (int32_t)(rs[w][l + 1] - rs[w][l]);
        if (f_bmax) f_bmax[i] = (int32_t)bmx[w][l];
    }
    const int b = valid ? bin_of((int64_t)v, bd) : -1;
    for (int j = 0; j < bd.nslots; ++j) {
        const unsigned long long m = __ballot(b == j);
        if (l == 0 && m) atomicAdd(&hist[j], (unsigned long long)__popcll(m));
    }
    const unsigned long long ws = wave_sum(v), wm = wave_max(v);
    if (l == 0) {
        atomicAdd(&s_tot, ws);
        atomicMax(&s_max, wm);
    }
    __syncthreads();
    if ((int)threadIdx.x < bd.nslots && hist[threadIdx.x])
        atomicAdd(&ctr->size[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 0) {
        atomicAdd(&ctr->total, s_tot);
        atomicMax(&ctr->maxv, s_max);
    }
}

// ---------------------------------------------------------------------------
// First binning pass over existing values (Alg. 1), plus the total
// (Section 5.4: nnz(C) is summed inside the numeric binning's first pass)
// and 256-row block sums for the row-pointer scan.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hist(int64_t M, const int64_t *__restrict__ v, Bounds bd,
                                              Counters *__restrict__ ctr,
                                              unsigned long long *__restrict__ blocksum) {
    __shared__ unsigned long long hist[16];
    __shared__ unsigned long long s_tot, s_max;
    const int l = threadIdx.x & 63;
    if (threadIdx.x < 16) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) { s_tot = 0; s_max = 0; }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = i < M;
    const unsigned long long x = valid ? (unsigned long long)v[i] : 0ull;
    const int b = valid ? bin_of((int64_t)x, bd) : -1;
    for (int j = 0; j < bd.nslots; ++j) {
        const unsigned long long m = __ballot(b == j);
        if (l == 0 && m) atomicAdd(&hist[j], (unsigned long long)__popcll(m));
    }
    const unsigned long long ws = wave_sum(x), wm = wave_max(x);
    if (l == 0) {
        atomicAdd(&s_tot, ws);
        atomicMax(&s_max, wm);
    }
    __syncthreads();
    if ((int)threadIdx.x < bd.nslots && hist[threadIdx.x])
        atomicAdd(&ctr->size[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 0) {
        atomicAdd(&ctr->total, s_tot);
        atomicMax(&ctr->maxv, s_max);
        if (blocksum) blocksum[blockIdx.x] = s_tot;
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of the block sums (one workgroup, chunks of 1024 with a
// running carry).  The grand total is nnz(C) = C.rpt[M].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t nblk,
                                                      unsigned long long *__restrict__ bs,
                                                      int64_t *__restrict__ total_out) {
    __shared__ unsigned long long wtot[16];
    __shared__ unsigned long long carry;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c = 0; c < nblk; c += 1024) {
        const int64_t i = c + threadIdx.x;
        const unsigned long long x = i < nblk ? bs[i] : 0ull;
        const unsigned long long incl = wave_incl_scan(x);
        if (l == 63) wtot[w] = incl;
        __syncthreads();
        unsigned long long pre = carry;
        for (int ww = 0; ww < w; ++ww) pre += wtot[ww];
        if (i < nblk) bs[i] = pre + incl - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry = pre + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total_out = (int64_t)carry;
}

// ---------------------------------------------------------------------------
// Second binning pass (Alg. 2): each row id is written to its bin's segment
// of `bins`.  A wave ballots per bin, lanes take their rank from mbcnt, the
// workgroup reserves one slice per bin with a single global atomic, and the
// bin's start offset is the exclusive sum of the (complete) bin sizes.
// With SCAN, v[] (per-row nnz in C.rpt) becomes C's row pointer in place:
// every row is read and written by the same thread, so no other thread can
// observe a half-updated value.
// ---------------------------------------------------------------------------
template <bool SCAN>
__global__ __launch_bounds__(256) void k_scatter(int64_t M, int64_t *__restrict__ v, Bounds bd,
                                                 Counters *__restrict__ ctr,
                                                 int32_t *__restrict__ bins,
                                                 const unsigned long long *__restrict__ blockbase) {
    __shared__ unsigned int wcnt[4][16];
    __shared__ unsigned long long base[16];
    __shared__ unsigned long long wsum[4];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = i < M;
    const int64_t x = valid ? v[i] : 0;
    const int b = valid ? bin_of(x, bd) : -1;
    int rank = 0;
    for (int j = 0; j < bd.nslots; ++j) {
        const unsigned long long m = __ballot(b == j);
        if (b == j) rank = mbcnt(m);
        if (l == 0) wcnt[w][j] = (unsigned)__popcll(m);
    }
    unsigned long long incl = 0;
    if (SCAN) {
        incl = wave_incl_scan((unsigned long long)x);
        if (l == 63) wsum[w] = incl;
    }
    __syncthreads();
    if (bins && (int)threadIdx.x < bd.nslots) {
        const int j = threadIdx.x;
        const unsigned long long tot = (unsigned long long)wcnt[0][j] + wcnt[1][j] + wcnt[2][j] + wcnt[3][j];
        unsigned long long off = 0;
        for (int jj = 0; jj < j; ++jj) off += ctr->size[jj];
        base[j] = off + (tot ? atomicAdd(&ctr->fill[j], tot) : 0ull);
    }
    __syncthreads();
    if (valid && bins) {
        unsigned long long pos = base[b];
        for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][b];
        bins[pos + rank] = (int32_t)i;
    }
    if (SCAN && valid) {
        unsigned long long pre = blockbase[blockIdx.x];
        for (int ww = 0; ww < w; ++ww) pre += wsum[ww];
        v[i] = (int64_t)(pre + incl - (unsigned long long)x);
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_setup(const DevCSR &A, const DevCSR &B, int64_t *nprod, const Bounds &bd,
                        Counters *ctr, int32_t *f_alen, int32_t *f_bmax, hipStream_t s) {
    if (A.rows == 0) return hipSuccess;
    const int64_t grid = (A.rows + 255) / 256;
    hipLaunchKernelGGL(k_setup, dim3((unsigned)grid), dim3(256), 0, s, A.rows, A.rpt, A.col, B.rpt,
                       nprod, bd, ctr, f_alen, f_bmax);
    return hipGetLastError();
}

hipError_t launch_hist(int64_t M, const int64_t *v, const Bounds &bd, Counters *ctr,
                       unsigned long long *blocksum, hipStream_t s) {
    if (M == 0) return hipSuccess;
    const int64_t grid = (M + 255) / 256;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)grid), dim3(256), 0, s, M, v, bd, ctr, blocksum);
    return hipGetLastError();
}

hipError_t launch_scan_blocks(int64_t nblk, unsigned long long *blocksum, int64_t *total_out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, nblk, blocksum, total_out);
    return hipGetLastError();
}

hipError_t launch_scatter(int64_t M, int64_t *v, const Bounds &bd, Counters *ctr, int32_t *bins,
                          const unsigned long long *blockbase, bool scan, hipStream_t s) {
    if (M == 0) return hipSuccess;
    const int64_t grid = (M + 255) / 256;
    if (scan)
        hipLaunchKernelGGL(k_scatter<true>, dim3((unsigned)grid), dim3(256), 0, s, M, v, bd, ctr,
                           bins, blockbase);
    else
        hipLaunchKernelGGL(k_scatter<false>, dim3((unsigned)grid), dim3(256), 0, s, M, v, bd, ctr,
                           bins, blockbase);
    return hipGetLastError();
}

}  // namespace opsp
