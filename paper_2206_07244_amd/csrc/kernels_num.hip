// Numeric step (OpSparse Section 5.2 Alg. 5, Section 5.6.2 kernel
// configuration): hashing, condensing and sorting of every row of C, stored
// at C.rpt[i] in C.col / C.val.
//
// Hashing: compare-and-swap on the key; when the slot is empty or already
// holds the key the product a_ik * b_kj is added with an LDS FP64 atomic
// (ds_add_f64); otherwise the next slot is probed.
//
// Condensing (Section 5.6.2): occupied slots are packed to the front of the
// table.  Positions come from a wave ballot prefix (mbcnt) plus per-wave
// totals, instead of one shared-counter atomic per entry.
//
// Sorting (the paper leaves the algorithm open): the packed (key, value)
// pairs are sorted in LDS with a bitonic network whose first comparator of
// every merge is mirrored, so all comparators are ascending and the
// power-of-two padding can stay virtual (+inf keys never move).  Bin 0 rows
// (at most a few dozen entries) use rank counting.  Bin 7 rows live in
// global-memory tables and are ordered by an LDS bitmap of their column
// range: the rank of a column is the popcount of the bitmap below it.
#include <limits.h>

#include "opsp_internal.h"

namespace opsp {

// Returns false when no slot was found after T probes (cannot happen when the
// bin bounds hold; reported instead of spinning).
__device__ __forceinline__ bool num_insert_lds(int *keys, double *vals, uint32_t T, int key,
                                               double v) {
    uint32_t s = hslot(key, T);
    for (uint32_t n = 0; n < T; ++n) {
        const int old = atomicCAS(&keys[s], -1, key);
        if (old == -1 || old == key) {
            atomicAdd(&vals[s], v);
            return true;
        }
        s = next_slot(s, T);
    }
    return false;
}

// ---------------------------------------------------------------------------
// bin 0: GL lanes per row; rank counting over the packed keys
// ---------------------------------------------------------------------------
template <int GL, int T>
__global__ __launch_bounds__(256) void k_num_group(
    int64_t nrows, const int32_t *__restrict__ bins, int64_t bin_off,
    const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const double *__restrict__ aval, const int64_t *__restrict__ brpt,
    const int32_t *__restrict__ bcol, const double *__restrict__ bval,
    const int64_t *__restrict__ crpt, int32_t *__restrict__ ccol, double *__restrict__ cval,
    Counters *__restrict__ ctr) {
    constexpr int RPW = 256 / GL;
    constexpr int ITEMS = (T + GL - 1) / GL;
    __shared__ double vals[RPW * T];
    __shared__ int keys[RPW * T];
    __shared__ int ck[RPW * T];
    const int slot = threadIdx.x / GL, g = threadIdx.x % GL;
    const int64_t idx = (int64_t)blockIdx.x * RPW + slot;
    const bool active = idx < nrows;
    int *tk = keys + slot * T;
    double *tv = vals + slot * T;
    int *pk = ck + slot * T;
    for (int s = g; s < T; s += GL) { tk[s] = -1; tv[s] = 0.0; }
    __syncthreads();
    int64_t row = 0;
    if (active) {
        row = bins ? (int64_t)bins[bin_off + idx] : bin_off + idx;
        const int64_t a1 = arpt[row + 1];
        for (int64_t p = arpt[row] + g; p < a1; p += GL) {
            const int k = acol[p];
            const double a = aval[p];
            const int64_t b1 = brpt[k + 1];
            for (int64_t q = brpt[k]; q < b1; ++q)
                if (!num_insert_lds(tk, tv, T, bcol[q], a * bval[q])) atomicAdd(&ctr->error, 1u);
        }
    }
    __syncthreads();
    // pack keys: lane g owns slots g, g+GL, ...
    int c = 0;
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
        const int s = g + m * GL;
        if (s < T && tk[s] >= 0) ++c;
    }
    int incl = c;
#pragma unroll
    for (int o = 1; o < GL; o <<= 1) {
        const int y = __shfl_up(incl, o, GL);
        if (g >= o) incl += y;
    }
    const int n = __shfl(incl, GL - 1, GL);
    int pos = incl - c;
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
        const int s = g + m * GL;
        if (s < T && tk[s] >= 0) pk[pos++] = tk[s];
    }
    __syncthreads();
    if (active) {
        const int64_t base = crpt[row];
        const int64_t cap = crpt[row + 1] - base;
        if (g == 0 && cap != n) atomicAdd(&ctr->error, 1u);
#pragma unroll
        for (int m = 0; m < ITEMS; ++m) {
            const int s = g + m * GL;
            if (s < T) {
                const int key = tk[s];
                if (key >= 0) {
                    int rank = 0;
                    for (int j = 0; j < n; ++j) rank += pk[j] < key;
                    if (rank < cap) {
                        ccol[base + rank] = key;
                        cval[base + rank] = tv[s];
                    }
                }
            }
        }
    }
}

// Ascending bitonic sort of keys[0..n) with their values (mirrored first
// comparator per merge; positions >= n are virtual +inf and never touched).
template <int NT, bool WT>
__device__ __forceinline__ void team_bitonic(int *keys, double *vals, int n, int t) {
    if (n < 2) return;
    const int P = (int)pow2_at_least((uint64_t)n);
    for (int k = 2; k <= P; k <<= 1) {
        const int h = k >> 1;
        for (int c = t; c < (P >> 1); c += NT) {
            const int blk = c / h, off = c - blk * h;
            const int i = blk * k + off, j = blk * k + k - 1 - off;
            if (j < n) {
                const int ki = keys[i], kj = keys[j];
                if (ki > kj) {
                    keys[i] = kj; keys[j] = ki;
                    const double vi = vals[i];
                    vals[i] = vals[j]; vals[j] = vi;
                }
            }
        }
        team_sync<WT>();
        for (int d = h >> 1; d > 0; d >>= 1) {
            for (int c = t; c < (P >> 1); c += NT) {
                const int i = 2 * d * (c / d) + (c % d), j = i + d;
                if (j < n) {
                    const int ki = keys[i], kj = keys[j];
                    if (ki > kj) {
                        keys[i] = kj; keys[j] = ki;
                        const double vi = vals[i];
                        vals[i] = vals[j]; vals[j] = vi;
                    }
                }
            }
            team_sync<WT>();
        }
    }
}

// ---------------------------------------------------------------------------
// bins 1-6: one team (wave for W == 64, else the workgroup) per row
// ---------------------------------------------------------------------------
template <int W, int T>
__global__ __launch_bounds__(W == 64 ? 256 : W) void k_num_row(
    int64_t nrows, const int32_t *__restrict__ bins, int64_t bin_off,
    const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const double *__restrict__ aval, const int64_t *__restrict__ brpt,
    const int32_t *__restrict__ bcol, const double *__restrict__ bval,
    const int64_t *__restrict__ crpt, int32_t *__restrict__ ccol, double *__restrict__ cval,
    int log_g, Counters *__restrict__ ctr) {
    constexpr bool WT = (W == 64);
    constexpr int R = WT ? 4 : 1;
    constexpr int NW = W / 64;
    constexpr int ITEMS = (T + W - 1) / W;
    __shared__ double vals[R * T];
    __shared__ int keys[R * T];
    __shared__ int wtot[R * NW];

    const int team = threadIdx.x / W, t = threadIdx.x % W;
    const int wv = t >> 6, l = t & 63;
    const int64_t idx = (int64_t)blockIdx.x * R + team;
    const bool active = idx < nrows;
    int *tk = keys + team * T;
    double *tv = vals + team * T;
    for (int s = t; s < T; s += W) { tk[s] = -1; tv[s] = 0.0; }
    team_sync<WT>();

    int64_t row = 0;
    if (active) {
        row = bins ? (int64_t)bins[bin_off + idx] : bin_off + idx;
        const int G = 1 << log_g;
        const int ngroups = W >> log_g;
        const int gid = t >> log_g, gl = t & (G - 1);
        const int64_t a1 = arpt[row + 1];
        for (int64_t p = arpt[row] + gid; p < a1; p += ngroups) {
            const int k = acol[p];
            const double a = aval[p];
            const int64_t b1 = brpt[k + 1];
            for (int64_t q = brpt[k] + gl; q < b1; q += G)
                if (!num_insert_lds(tk, tv, T, bcol[q], a * bval[q])) atomicAdd(&ctr->error, 1u);
        }
    }
    team_sync<WT>();

    // condense into registers, then pack to the front of the table
    int rk[ITEMS];
    double rv[ITEMS];
    int c = 0;
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
        const int s = t + m * W;
        rk[m] = -1;
        rv[m] = 0.0;
        if (s < T) {
            rk[m] = tk[s];
            if (rk[m] >= 0) { rv[m] = tv[s]; ++c; }
        }
    }
    const int incl = wave_incl_scan(c);
    int n, pos;
    if constexpr (WT) {
        n = __shfl(incl, 63);
        pos = incl - c;
    } else {
        if (l == 63) wtot[wv] = incl;
        __syncthreads();
        int pre = 0;
        n = 0;
        for (int i = 0; i < NW; ++i) {
            const int x = wtot[i];
            if (i < wv) pre += x;
            n += x;
        }
        pos = pre + incl - c;
    }
    team_sync<WT>();
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
        if (rk[m] >= 0) {
            tk[pos] = rk[m];
            tv[pos] = rv[m];
            ++pos;
        }
    }
    team_sync<WT>();
    team_bitonic<W, WT>(tk, tv, n, t);
    if (active) {
        const int64_t base = crpt[row];
        const int64_t cap = crpt[row + 1] - base;
        if (t == 0 && cap != n) atomicAdd(&ctr->error, 1u);
        const int nw = cap < n ? (int)cap : n;
        for (int e = t; e < nw; e += W) {
            ccol[base + e] = tk[e];
            cval[base + e] = tv[e];
        }
    }
}

// ---------------------------------------------------------------------------
// bin 7: global-memory tables (one slab per persistent workgroup), ordered
// through LDS bitmaps of 2^19 columns at a time.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_num_global(
    int64_t nrows, const int32_t *__restrict__ bins, int64_t bin_off,
    const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const double *__restrict__ aval, const int64_t *__restrict__ brpt,
    const int32_t *__restrict__ bcol, const double *__restrict__ bval,
    const int64_t *__restrict__ crpt, int32_t *__restrict__ ccol, double *__restrict__ cval,
    int *slab_keys, double *slab_vals, int64_t slab_entries, int log_g,
    Counters *__restrict__ ctr) {
    constexpr int CW = NUM_GLOBAL_CHUNK_WORDS;
    constexpr int CBITS = CW * 32;
    constexpr int WPT = CW / 1024;  // bitmap words per thread
    __shared__ unsigned int bitmap[CW];
    __shared__ unsigned int prefix[CW];
    __shared__ unsigned int red[16];
    __shared__ int s_min, s_max;

    int *tk = slab_keys + (int64_t)blockIdx.x * slab_entries;
    double *tv = slab_vals + (int64_t)blockIdx.x * slab_entries;
    const int t = threadIdx.x, wv = t >> 6, l = t & 63;
    const int G = 1 << log_g;
    const int ngroups = 1024 >> log_g;
    const int gid = t >> log_g, gl = t & (G - 1);

    for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int64_t row = bins ? (int64_t)bins[bin_off + r] : bin_off + r;
        const int64_t base = crpt[row];
        const int64_t n = crpt[row + 1] - base;
        uint32_t T = pow2_at_least((uint64_t)(2 * n > 64 ? 2 * n : 64));
        if ((int64_t)T > slab_entries) T = (uint32_t)slab_entries;
        for (uint32_t s = t; s < T; s += 1024) { tk[s] = -1; tv[s] = 0.0; }
        if (t == 0) { s_min = INT_MAX; s_max = -1; }
        __syncthreads();

        int kmin = INT_MAX, kmax = -1;
        const int64_t a1 = arpt[row + 1];
        for (int64_t p = arpt[row] + gid; p < a1; p += ngroups) {
            const int k = acol[p];
            const double a = aval[p];
            const int64_t b1 = brpt[k + 1];
            for (int64_t q = brpt[k] + gl; q < b1; q += G) {
                const int key = bcol[q];
                kmin = key < kmin ? key : kmin;
                kmax = key > kmax ? key : kmax;
                uint32_t s = hslot(key, T);
                uint32_t pr = 0;
                for (; pr < T; ++pr) {
                    const int old = atomicCAS(&tk[s], -1, key);
                    if (old == -1 || old == key) {
                        unsafeAtomicAdd(&tv[s], a * bval[q]);
                        break;
                    }
                    s = next_slot(s, T);
                }
                if (pr == T) atomicAdd(&ctr->error, 1u);
            }
        }
        kmin = wave_min(kmin);
        kmax = wave_max(kmax);
        if (l == 0) {
            atomicMin(&s_min, kmin);
            atomicMax(&s_max, kmax);
        }
        __syncthreads();
        const int lo = s_min, hi = s_max;
        int64_t run = 0;
        for (int64_t c0 = lo; c0 <= hi; c0 += CBITS) {
            for (int w = t; w < CW; w += 1024) bitmap[w] = 0u;
            __syncthreads();
            for (uint32_t s = t; s < T; s += 1024) {
                const int key = ld_coherent(&tk[s]);
                if (key >= 0 && key >= c0 && key < c0 + CBITS) {
                    const int b = key - (int)c0;
                    atomicOr(&bitmap[b >> 5], 1u << (b & 31));
                }
            }
            __syncthreads();
            // exclusive popcount prefix over the chunk's words
            unsigned int loc[WPT];
            unsigned int sum = 0;
#pragma unroll
            for (int i = 0; i < WPT; ++i) {
                loc[i] = sum;
                sum += __popc(bitmap[t * WPT + i]);
            }
            const unsigned int incl = wave_incl_scan(sum);
            if (l == 63) red[wv] = incl;
            __syncthreads();
            unsigned int pre = 0, tot = 0;
            for (int i = 0; i < 16; ++i) {
                if (i < wv) pre += red[i];
                tot += red[i];
            }
            pre += incl - sum;
#pragma unroll
            for (int i = 0; i < WPT; ++i) prefix[t * WPT + i] = pre + loc[i];
            __syncthreads();
            for (uint32_t s = t; s < T; s += 1024) {
                const int key = ld_coherent(&tk[s]);
                if (key >= 0 && key >= c0 && key < c0 + CBITS) {
                    const int b = key - (int)c0;
                    const int64_t rank =
                        run + prefix[b >> 5] + __popc(bitmap[b >> 5] & ((1u << (b & 31)) - 1u));
                    if (rank < n) {
                        ccol[base + rank] = key;
                        cval[base + rank] = ld_coherent(&tv[s]);
                    }
                }
            }
            run += tot;
            __syncthreads();
        }
        if (t == 0 && run != n) atomicAdd(&ctr->error, 1u);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
template <int W, int T>
static hipError_t go_row(const NumArgs &a, hipStream_t s) {
    constexpr int R = (W == 64) ? 4 : 1;
    const int64_t grid = (a.nrows + R - 1) / R;
    hipLaunchKernelGGL((k_num_row<W, T>), dim3((unsigned)grid), dim3(W * R), 0, s, a.nrows, a.bins,
                       a.bin_off, a.A.rpt, a.A.col, a.A.val, a.B.rpt, a.B.col, a.B.val, a.crpt,
                       a.ccol, a.cval, a.log_g, a.ctr);
    return hipGetLastError();
}

hipError_t launch_numeric_bin(int bin, const NumArgs &a, hipStream_t s) {
    if (a.nrows == 0) return hipSuccess;
    switch (bin) {
        case 0: {
            constexpr int RPW = 256 / NUM_GL;
            const int64_t grid = (a.nrows + RPW - 1) / RPW;
            hipLaunchKernelGGL((k_num_group<NUM_GL, NUM_T[0]>), dim3((unsigned)grid), dim3(256), 0, s,
                               a.nrows, a.bins, a.bin_off, a.A.rpt, a.A.col, a.A.val, a.B.rpt,
                               a.B.col, a.B.val, a.crpt, a.ccol, a.cval, a.ctr);
            return hipGetLastError();
        }
        case 1: return go_row<NUM_W[1], NUM_T[1]>(a, s);
        case 2: return go_row<NUM_W[2], NUM_T[2]>(a, s);
        case 3: return go_row<NUM_W[3], NUM_T[3]>(a, s);
        case 4: return go_row<NUM_W[4], NUM_T[4]>(a, s);
        case 5: return go_row<NUM_W[5], NUM_T[5]>(a, s);
        case 6: return go_row<NUM_W[6], NUM_T[6]>(a, s);
        case NUM_GLOBAL_BIN: {
            if (a.grid <= 0) return hipSuccess;
            hipLaunchKernelGGL(k_num_global, dim3((unsigned)a.grid), dim3(1024), 0, s, a.nrows,
                               a.bins, a.bin_off, a.A.rpt, a.A.col, a.A.val, a.B.rpt, a.B.col,
                               a.B.val, a.crpt, a.ccol, a.cval, a.slab_keys, a.slab_vals,
                               a.slab_entries, a.log_g, a.ctr);
            return hipGetLastError();
        }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace opsp
