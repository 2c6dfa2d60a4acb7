// Setup step, the two binning passes and the row-pointer scan
// (OpSparse Section 5, setup step; Section 5.1 Alg. 1-3; Section 5.3).
//
// gfx950 design: every 256-row block counts its rows per bin with wave
// ballots and LDS, and writes its counts, value total and value maximum to a
// per-block record instead of issuing global atomics (thousands of blocks
// hitting one counter serialise in L2).  One finalize workgroup turns the
// records into bin sizes, per-block bin offsets (exclusive scans over blocks)
// and, for the numeric step, per-block row-pointer offsets.  The second pass
// then places every row with no global atomic at all: rows of a bin appear in
// ascending order, so the bin lists are deterministic.
#include <limits.h>

#include "opsp_internal.h"

namespace opsp {

// ---------------------------------------------------------------------------
// Setup: n_prod_i = sum over A_i* of len(B_k*), written into C.rpt[i]
// (Section 5.3 reuses C.rpt for n_prod), fused with the first symbolic
// binning pass (Alg. 1).  Each wave owns 64 consecutive rows and walks the
// flat range of their A entries with coalesced loads, so one long row does
// not serialise a single lane.  Rows of more than SETUP_TILE entries are
// listed instead, with their tiles, and left out of the block's record:
// k_setup_long walks the tiles on many workgroups and k_setup_fin bins each
// listed row into its block's record.
// ---------------------------------------------------------------------------
__global__ void k_setup_init(LongHead *lh) {
    if (threadIdx.x == 0) lh->packed = 0;
}

__global__ __launch_bounds__(256) void k_setup(int64_t M, const int64_t *__restrict__ arpt,
                                               const int32_t *__restrict__ acol,
                                               const int64_t *__restrict__ brpt,
                                               int64_t *__restrict__ nprod, Bounds bd,
                                               BlockParts parts,
                                               int32_t *__restrict__ f_alen,
                                               int32_t *__restrict__ f_bmax,
                                               const int4 *__restrict__ brec,
                                               int2 *__restrict__ rng) {
    __shared__ int64_t rs[4][65];
    __shared__ unsigned long long acc[4][64];
    __shared__ unsigned int bmx[4][64];
    __shared__ int clo[4][64], chi[4][64];
    __shared__ int lng[4][64];   // row handed to k_setup_long
    __shared__ unsigned int hist[BIN_SLOTS];
    __shared__ unsigned long long s_tot, s_max;

    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (threadIdx.x < BIN_SLOTS) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) { s_tot = 0; s_max = 0; }
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 64;
    const int nrows = (int)(M - r0 < 0 ? 0 : (M - r0 > 64 ? 64 : M - r0));
    if (nrows > 0) {
        rs[w][l] = arpt[r0 + (l < nrows ? l : nrows)];
        if (l == 0) rs[w][64] = arpt[r0 + nrows];
    }
    acc[w][l] = 0;
    bmx[w][l] = 0;
    clo[w][l] = INT_MAX;
    chi[w][l] = -1;
    __syncthreads();
    const bool range = rng != nullptr;   // column range of each row's output

    // Short rows (the wave's longest at most 64 entries), or rows of up to
    // 256 entries whose longest is at most twice the wave's mean (finite
    // element rows: 81 entries for 3 unknowns on a 27-point stencil): every
    // lane walks its own row, accumulating in registers; no per-entry row
    // search and no LDS atomics.  Otherwise the wave walks the flat range of
    // its rows' entries, so that one long row does not serialise a single
    // lane.
    const int64_t my_len = (nrows > 0 && l < nrows) ? rs[w][l + 1] - rs[w][l] : 0;
    const int64_t wmax = wave_max(my_len), wtot = nrows > 0 ? rs[w][64] - rs[w][0] : 0;
    const bool lane_rows = nrows > 0 && (wmax <= 64 || (wmax <= 256 && wmax * nrows <= 2 * wtot));
    {
        // long rows go to the tile list: one reservation per wave (a 64-bit
        // add of its rows and tiles).  If the list is full, which only an A
        // whose rows span more entries than its nnz can cause, the wave walks
        // those rows itself and blanks the slots it reserved.
        const bool lr = my_len > SETUP_TILE;
        const int n = lr ? (int)((my_len + SETUP_TILE - 1) / SETUP_TILE) : 0;
        const unsigned long long m = __ballot(lr);
        bool handed = false;
        if (m) {   // uniform over the wave
            const int incl = wave_incl_scan(n);
            const int tot = __shfl(incl, 63);
            const int nr = (int)__popcll(m), rk = mbcnt(m);
            unsigned long long base = 0;
            if (l == 0)
                base = atomicAdd(&parts.lh->packed,
                                 ((unsigned long long)nr << 32) | (unsigned long long)(unsigned)tot);
            base = __shfl(base, 0);
            const uint32_t s0 = (uint32_t)(base >> 32), i0 = (uint32_t)base;
            const bool fits = (uint64_t)s0 + nr <= parts.cap_rows && (uint64_t)i0 + tot <= parts.cap_items;
            const uint32_t slot = s0 + (uint32_t)rk, it0 = i0 + (uint32_t)(incl - n);
            if (lr && fits) {
                parts.lrows[slot] = LongRow{(int32_t)(r0 + l), n, (int32_t)it0, 0};
                for (int j = 0; j < n; ++j) parts.litems[it0 + j] = make_int2((int)slot, j);
                handed = true;
            } else if (lr) {
                if (slot < parts.cap_rows) parts.lrows[slot] = LongRow{-1, 0, 0, 0};
                for (int j = 0; j < n; ++j)
                    if (it0 + (uint32_t)j < parts.cap_items) parts.litems[it0 + j] = make_int2(-1, 0);
            }
        }
        lng[w][l] = handed ? 1 : 0;
    }
    __syncthreads();
    if (lane_rows) {
        unsigned long long a = 0;
        unsigned int bm = 0;
        int mn = INT_MAX, mx = -1;
        const int64_t p0 = l < nrows ? rs[w][l] : 0;
        for (int64_t p = p0; p < p0 + my_len; p += 4) {
            int k[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) k[u] = p + u < p0 + my_len ? acol[p + u] : -1;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k[u] < 0) continue;
                int64_t len;
                if (range) {
                    const int4 r = brec[k[u]];
                    len = r.x;
                    if (len > 0) {
                        mn = r.y < mn ? r.y : mn;
                        mx = r.z > mx ? r.z : mx;
                    }
                } else {
                    len = brpt[k[u] + 1] - brpt[k[u]];
                }
                a += (unsigned long long)len;
                const unsigned int lc = (unsigned)(len > 0xffffffffll ? 0xffffffffll : len);
                bm = lc > bm ? lc : bm;
            }
        }
        acc[w][l] = a;
        bmx[w][l] = bm;
        clo[w][l] = mn;
        chi[w][l] = mx;
    } else if (nrows > 0) {
        const int64_t e0 = rs[w][0], e1 = rs[w][64];
        // four entries per lane per step so that their gathers overlap; the
        // loop is uniform over the wave (lanes past the end hold no entry),
        // as the wave reductions below need every lane
        for (int64_t eb0 = e0; eb0 < e1;) {
            {   // jump over a row handed to the tiles (uniform)
                int lo = 0, hi = nrows - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (rs[w][mid] <= eb0) lo = mid; else hi = mid - 1;
                }
                if (lng[w][lo]) {
                    eb0 = rs[w][lo + 1];
                    continue;
                }
            }
            const int64_t eb = eb0 + l;
            eb0 += 256;
            int64_t len[4];
            int2 fl[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = eb + 64 * u;
                const int k = e < e1 ? acol[e] : -1;
                if (range) {   // one 16-byte record per B row: length, first, last column
                    const int4 r = k >= 0 ? brec[k] : make_int4(-1, INT_MAX, -1, 0);
                    len[u] = r.x;
                    fl[u] = make_int2(r.y, r.z);
                } else {
                    len[u] = k >= 0 ? brpt[k + 1] - brpt[k] : -1;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = eb + 64 * u;
                const bool ok0 = len[u] >= 0;
                // largest r in [0, nrows) with rs[r] <= e (rows may be empty)
                int lo = 0, hi = nrows - 1;
                while (ok0 && lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (rs[w][mid] <= e) lo = mid; else hi = mid - 1;
                }
                const bool ok = ok0 && !lng[w][lo];
                const unsigned lc = ok ? (unsigned)(len[u] > 0xffffffffll ? 0xffffffffll : len[u]) : 0u;
                const bool fr = range && ok && len[u] > 0;
                // lanes hold consecutive entries, so lane 0 has the lowest
                // row; when every lane with an entry is in that row (a long
                // row), reduce over the wave and update the row once instead
                // of 64 lanes contending for one LDS word
                const int lo0 = __builtin_amdgcn_readfirstlane(lo);
                if (__ballot(ok && lo != lo0) == 0ull) {
                    const unsigned long long sa = wave_sum(ok ? (unsigned long long)len[u] : 0ull);
                    const unsigned sm = wave_max(lc);
                    const int smin = wave_min(fr ? fl[u].x : INT_MAX);
                    const int smax = wave_max(fr ? fl[u].y : -1);
                    if (l == 0 && __ballot(ok) != 0ull) {
                        acc[w][lo0] += sa;
                        bmx[w][lo0] = sm > bmx[w][lo0] ? sm : bmx[w][lo0];
                        clo[w][lo0] = smin < clo[w][lo0] ? smin : clo[w][lo0];
                        chi[w][lo0] = smax > chi[w][lo0] ? smax : chi[w][lo0];
                    }
                    continue;
                }
                if (!ok) continue;
                atomicAdd(&acc[w][lo], (unsigned long long)len[u]);
                atomicMax(&bmx[w][lo], lc);
                if (fr) {
                    atomicMin(&clo[w][lo], fl[u].x);
                    atomicMax(&chi[w][lo], fl[u].y);
                }
            }
        }
    }
    __syncthreads();

    const bool valid = l < nrows;
    const int64_t i = r0 + l;
    const unsigned long long v = valid ? acc[w][l] : 0ull;
    // a handed row starts from n_prod 0, no range and b_max 0 here; the
    // tiles add to them and bin it
    if (valid) {
        nprod[i] = (int64_t)v;
        if (f_alen) f_alen[i] = (int32_t)(rs[w][l + 1] - rs[w][l]);
        if (f_bmax) f_bmax[i] = (int32_t)bmx[w][l];
        if (range) rng[i] = make_int2(clo[w][l], chi[w][l]);
    }
    const int b = valid && !lng[w][l]
                      ? (range ? bin_of_row((int64_t)v, bd, make_int2(clo[w][l], chi[w][l]))
                               : bin_of((int64_t)v, bd))
                      : -1;
    for (int j = 0; j < bd.nslots; ++j) {
        const unsigned long long m = __ballot(b == j);
        if (l == 0 && m) atomicAdd(&hist[j], (unsigned)__popcll(m));
    }
    const unsigned long long ws = wave_sum(v), wm = wave_max(v);
    if (l == 0) {
        atomicAdd(&s_tot, ws);
        atomicMax(&s_max, wm);
    }
    __syncthreads();
    if ((int)threadIdx.x < BIN_SLOTS) parts.hist[(int64_t)blockIdx.x * BIN_SLOTS + threadIdx.x] = hist[threadIdx.x];
    if (threadIdx.x == 0) {
        parts.tot[blockIdx.x] = s_tot;
        parts.mx[blockIdx.x] = s_max;
    }
}

// ---------------------------------------------------------------------------
// Long rows listed by k_setup.  k_setup_long: persistent waves over the
// tiles, each tile's sum of B row lengths, largest B row and column range
// into its slot.  k_setup_fin: one wave per long row combines its tiles,
// writes the row's n_prod / b_max / range and counts the row in its 256-row
// block's record (bin, total, maximum), as k_setup does for the other rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_setup_long(const int64_t *__restrict__ arpt,
                                                    const int32_t *__restrict__ acol,
                                                    const int64_t *__restrict__ brpt,
                                                    BlockParts parts,
                                                    const int4 *__restrict__ brec) {
    constexpr int EPL = SETUP_TILE / 64;   // entries per lane, EPL / 4 rounds of four gathers
    static_assert(EPL % 4 == 0, "whole rounds");
    const int l = threadIdx.x & 63;
    const bool range = brec != nullptr;
    const uint32_t req = (uint32_t)parts.lh->packed;
    const uint32_t nit = req < parts.cap_items ? req : parts.cap_items;
    const uint32_t nw = gridDim.x * 4;
    for (uint32_t it = blockIdx.x * 4 + (threadIdx.x >> 6); it < nit; it += nw) {
        const int2 item = parts.litems[it];
        if (item.x < 0) continue;   // uniform over the wave
        const int64_t row = parts.lrows[item.x].row;
        const int64_t a0 = arpt[row] + (int64_t)item.y * SETUP_TILE;
        const int64_t a1r = arpt[row + 1];
        const int64_t a1 = a0 + SETUP_TILE < a1r ? a0 + SETUP_TILE : a1r;
        unsigned long long sum = 0;
        unsigned bm = 0;
        int mn = INT_MAX, mx = -1;
#pragma unroll
        for (int q = 0; q < EPL; q += 4) {
            int k[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = a0 + l + 64 * (q + u);
                k[u] = e < a1 ? acol[e] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k[u] < 0) continue;
                int64_t len;
                if (range) {
                    const int4 r = brec[k[u]];
                    len = r.x;
                    if (len > 0) {
                        mn = r.y < mn ? r.y : mn;
                        mx = r.z > mx ? r.z : mx;
                    }
                } else {
                    len = brpt[k[u] + 1] - brpt[k[u]];
                }
                sum += (unsigned long long)len;
                const unsigned lc = (unsigned)(len > 0xffffffffll ? 0xffffffffll : len);
                bm = lc > bm ? lc : bm;
            }
        }
        sum = wave_sum(sum);
        bm = wave_max(bm);
        mn = wave_min(mn);
        mx = wave_max(mx);
        if (l == 0) parts.lpart[it] = LongPart{sum, bm, mn, mx, 0};
    }
}

__global__ __launch_bounds__(256) void k_setup_fin(int64_t *__restrict__ nprod, Bounds bd,
                                                   BlockParts parts, int32_t *__restrict__ f_bmax,
                                                   int2 *__restrict__ rng) {
    const int l = threadIdx.x & 63;
    const uint32_t req = (uint32_t)(parts.lh->packed >> 32);
    const uint32_t nr = req < parts.cap_rows ? req : parts.cap_rows;
    const uint32_t nw = gridDim.x * 4;
    for (uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < nr; r += nw) {
        const LongRow lr = parts.lrows[r];
        if (lr.row < 0) continue;   // uniform over the wave
        unsigned long long sum = 0;
        unsigned bm = 0;
        int mn = INT_MAX, mx = -1;
        for (int j = l; j < lr.ntiles; j += 64) {
            const LongPart p = parts.lpart[lr.it0 + j];
            sum += p.sum;
            bm = p.bmax > bm ? p.bmax : bm;
            mn = p.lo < mn ? p.lo : mn;
            mx = p.hi > mx ? p.hi : mx;
        }
        sum = wave_sum(sum);
        bm = wave_max(bm);
        mn = wave_min(mn);
        mx = wave_max(mx);
        if (l == 0) {
            const int64_t i = lr.row;
            nprod[i] = (int64_t)sum;
            if (f_bmax) f_bmax[i] = (int32_t)(bm > 0x7fffffffu ? 0x7fffffffu : bm);
            if (rng) rng[i] = make_int2(mn, mx);
            const int b = rng ? bin_of_row((int64_t)sum, bd, make_int2(mn, mx)) : bin_of((int64_t)sum, bd);
            const int64_t blk = i >> 8;
            atomicAdd(&parts.hist[blk * BIN_SLOTS + b], 1u);
            atomicAdd(&parts.tot[blk], sum);
            atomicMax(&parts.mx[blk], sum);
        }
    }
}

// ---------------------------------------------------------------------------
// First binning pass over existing values (Alg. 1), with the per-block total
// (Section 5.4 sums nnz(C) inside the numeric binning's first pass).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hist(int64_t M, const int64_t *__restrict__ v, Bounds bd,
                                              BlockParts parts) {
    __shared__ unsigned int hist[BIN_SLOTS];
    __shared__ unsigned long long s_tot, s_max;
    const int l = threadIdx.x & 63;
    if (threadIdx.x < BIN_SLOTS) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) { s_tot = 0; s_max = 0; }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = i < M;
    const unsigned long long x = valid ? (unsigned long long)v[i] : 0ull;
    const int b = valid ? bin_of((int64_t)x, bd) : -1;
    for (int j = 0; j < bd.nslots; ++j) {
        const unsigned long long m = __ballot(b == j);
        if (l == 0 && m) atomicAdd(&hist[j], (unsigned)__popcll(m));
    }
    const unsigned long long ws = wave_sum(x), wm = wave_max(x);
    if (l == 0) {
        atomicAdd(&s_tot, ws);
        atomicMax(&s_max, wm);
    }
    __syncthreads();
    if ((int)threadIdx.x < BIN_SLOTS) parts.hist[(int64_t)blockIdx.x * BIN_SLOTS + threadIdx.x] = hist[threadIdx.x];
    if (threadIdx.x == 0) {
        parts.tot[blockIdx.x] = s_tot;
        parts.mx[blockIdx.x] = s_max;
    }
}

// ---------------------------------------------------------------------------
// Finalize (one workgroup of 1024 threads): blocks are taken 1024 at a time,
// one per thread, and the next 1024 blocks' records are loaded while the
// current ones are scanned.  Each thread loads its block's record (16 bin
// counts with four 16-byte loads, the total and the maximum); the workgroup
// scans every bin slot and the totals (wave scans; then, per value, a
// 16-lane scan of the 16 wave sums, which also advances a running carry
// across chunks) and writes the exclusive offsets back in place: per bin
// slot the block's offset inside the bin, and with SCAN the block's
// row-pointer offset.  Bin sizes, grand total and maximum go to `ctr`.
// ---------------------------------------------------------------------------
template <bool SCAN>
__global__ __launch_bounds__(1024) void k_finalize(int64_t nblk, int nslots, BlockParts parts,
                                                   Counters *__restrict__ ctr,
                                                   int64_t *__restrict__ total_out) {
    constexpr int NV = BIN_SLOTS + 1;               // bin slots + totals
    __shared__ unsigned long long wred[NV][16];     // per-wave inclusive sums
    __shared__ unsigned long long wpre[NV][16];     // carry + exclusive prefix of wred
    __shared__ unsigned long long carry[NV];
    __shared__ unsigned long long wmx[16];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    // this step's failure / error counters start from zero
    if (t == 0) {
        ctr->fail = 0u;
        ctr->error = 0u;
        ctr->sched[0] = 0ull;
        ctr->sched[1] = 0ull;
    }
    if (t < NV) carry[t] = 0;
    unsigned long long mx = 0;
    // block b's record (zeros past the last block; the index is clamped so
    // that the loads need no branch)
    unsigned int h[BIN_SLOTS];
    unsigned long long tt, m;
    auto load = [&](int64_t b, unsigned int *hh, unsigned long long &t_, unsigned long long &m_) {
        const bool ok = b < nblk;
        const int64_t bb = ok ? b : nblk - 1;
        const uint4 *src = reinterpret_cast<const uint4 *>(parts.hist + bb * BIN_SLOTS);
#pragma unroll
        for (int q = 0; q < BIN_SLOTS / 4; ++q) {
            const uint4 v4 = src[q];
            hh[4 * q] = ok ? v4.x : 0u;
            hh[4 * q + 1] = ok ? v4.y : 0u;
            hh[4 * q + 2] = ok ? v4.z : 0u;
            hh[4 * q + 3] = ok ? v4.w : 0u;
        }
        const unsigned long long tv = parts.tot[bb], mv = parts.mx[bb];
        t_ = ok ? tv : 0ull;
        m_ = ok ? mv : 0ull;
    };
    load(t, h, tt, m);
    __syncthreads();
    for (int64_t c = 0; c < nblk; c += 1024) {
        const int64_t b = c + t;
        const bool ok = b < nblk;
        unsigned int hn[BIN_SLOTS];
        unsigned long long ttn, mn;
        load(b + 1024, hn, ttn, mn);   // next chunk, in flight during this one
        mx = m > mx ? m : mx;
        unsigned int incl[BIN_SLOTS];
#pragma unroll
        for (int j = 0; j < BIN_SLOTS; ++j) {
            incl[j] = j < nslots ? wave_incl_scan(h[j]) : 0u;
            if (l == 63) wred[j][w] = incl[j];
        }
        const unsigned long long inclt = wave_incl_scan(tt);
        if (l == 63) wred[BIN_SLOTS][w] = inclt;
        __syncthreads();
        if (t < NV * 16) {   // value j = t / 16, wave ww = t % 16: lanes of one wave
            const int j = t >> 4, ww = t & 15;
            const unsigned long long v = wred[j][ww];
            const unsigned long long cj = carry[j];
            unsigned long long inc = v;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const unsigned long long y = __shfl_up(inc, o, 16);
                if (ww >= o) inc += y;
            }
            wpre[j][ww] = cj + inc - v;
            if (ww == 15) carry[j] = cj + inc;   // after every lane of the group read cj
        }
        __syncthreads();
        if (ok) {
            unsigned int outv[BIN_SLOTS];
#pragma unroll
            for (int j = 0; j < BIN_SLOTS; ++j)
                outv[j] = (unsigned)(wpre[j][w] + incl[j] - h[j]);
            uint4 *dst = reinterpret_cast<uint4 *>(parts.hist + b * BIN_SLOTS);
#pragma unroll
            for (int q = 0; q < BIN_SLOTS / 4; ++q)
                dst[q] = make_uint4(outv[4 * q], outv[4 * q + 1], outv[4 * q + 2], outv[4 * q + 3]);
            if (SCAN) parts.tot[b] = wpre[BIN_SLOTS][w] + inclt - tt;
        }
#pragma unroll
        for (int j = 0; j < BIN_SLOTS; ++j) h[j] = hn[j];
        tt = ttn;
        m = mn;
    }
    mx = wave_max(mx);
    if (l == 0) wmx[w] = mx;
    __syncthreads();
    if (t < nslots) ctr->size[t] = carry[t];
    if (t == 0) {
        unsigned long long mm = 0;
        for (int i = 0; i < 16; ++i) mm = wmx[i] > mm ? wmx[i] : mm;
        ctr->maxv = mm;
        ctr->total = carry[BIN_SLOTS];
        if (total_out) *total_out = (int64_t)carry[BIN_SLOTS];
    }
}

// ---------------------------------------------------------------------------
// Second binning pass (Alg. 2): row i goes to position
//   start(bin) + offset of its block inside the bin + rank inside the block,
// where the rank comes from per-wave ballots (mbcnt) and per-wave counts.
// With SCAN, v[] (per-row nnz in C.rpt) becomes C's row pointer in place:
// every row is read and written by the same thread.
// ---------------------------------------------------------------------------
template <bool SCAN>
__global__ __launch_bounds__(256) void k_scatter(int64_t M, int64_t *v, Bounds bd,
                                                 const Counters *__restrict__ ctr,
                                                 int32_t *__restrict__ bins, BlockParts parts,
                                                 int64_t *vout, int skip_full,
                                                 const int2 *__restrict__ rng) {
    __shared__ unsigned int wcnt[4][BIN_SLOTS];
    __shared__ unsigned long long base[BIN_SLOTS];
    __shared__ unsigned long long wsum[4];
    if (!SCAN && skip_full) {
        // one bin holds every row: its rows are read in order, no list
        for (int j = 0; j < bd.nslots; ++j)
            if ((int64_t)ctr->size[j] == M) return;   // uniform over the grid
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = i < M;
    const int64_t x = valid ? v[i] : 0;
    const int b = valid ? (rng ? bin_of_row(x, bd, rng[i]) : bin_of(x, bd)) : -1;
    int rank = 0;
    if (bins) {
        for (int j = 0; j < bd.nslots; ++j) {
            const unsigned long long m = __ballot(b == j);
            if (b == j) rank = mbcnt(m);
            if (l == 0) wcnt[w][j] = (unsigned)__popcll(m);
        }
    }
    unsigned long long incl = 0;
    if (SCAN) {
        incl = wave_incl_scan((unsigned long long)x);
        if (l == 63) wsum[w] = incl;
    }
    if (bins && (int)threadIdx.x < bd.nslots) {
        const int j = threadIdx.x;
        unsigned long long off = 0;
        for (int jj = 0; jj < j; ++jj) off += ctr->size[jj];
        base[j] = off + parts.hist[(int64_t)blockIdx.x * BIN_SLOTS + j];
    }
    __syncthreads();
    if (valid && bins) {
        unsigned long long pos = base[b];
        for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][b];
        bins[pos + rank] = (int32_t)i;
    }
    if (SCAN && valid) {
        unsigned long long pre = parts.tot[blockIdx.x];
        for (int ww = 0; ww < w; ++ww) pre += wsum[ww];
        vout[i] = (int64_t)(pre + incl - (unsigned long long)x);
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_setup(const DevCSR &A, const DevCSR &B, int64_t *nprod, const Bounds &bd,
                        const BlockParts &parts, int32_t *f_alen, int32_t *f_bmax, hipStream_t s,
                        const int4 *brec, int2 *rng) {
    if (A.rows == 0) return hipSuccess;
    const int64_t grid = (A.rows + 255) / 256;
    hipLaunchKernelGGL(k_setup_init, dim3(1), dim3(64), 0, s, parts.lh);
    hipLaunchKernelGGL(k_setup, dim3((unsigned)grid), dim3(256), 0, s, A.rows, A.rpt, A.col, B.rpt,
                       nprod, bd, parts, f_alen, f_bmax, brec, brec ? rng : nullptr);
    // long rows: fixed grids of two workgroups per CU of gfx950 (R-MAT
    // scale 20 lists ~6,200 rows in ~17,600 tiles)
    hipLaunchKernelGGL(k_setup_long, dim3(512), dim3(256), 0, s, A.rpt, A.col, B.rpt, parts, brec);
    hipLaunchKernelGGL(k_setup_fin, dim3(512), dim3(256), 0, s, nprod, bd, parts, f_bmax,
                       brec ? rng : nullptr);
    return hipGetLastError();
}

// Length, first and last column of every row of B in one 16-byte record,
// so that the setup step reads one record per A entry (instead of two row
// bounds) and also gets each row's output column range; with `dup` the
// fourth field flags a row with the same columns as the row before it (the
// symbolic step skips such a row when the A row also holds the one before
// it), else it is zero.
constexpr int64_t DUP_MAX = 256;
__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0) *p = 0ull;
}

__global__ __launch_bounds__(256) void k_brange(int64_t K, const int64_t *__restrict__ brpt,
                                                const int32_t *__restrict__ bcol,
                                                int4 *__restrict__ brec, int dup,
                                                unsigned long long *__restrict__ ndup) {
    __shared__ unsigned int s_dup;   // flagged rows of the workgroup (with ndup)
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (ndup && threadIdx.x == 0) s_dup = 0u;
    int d = 0;
    if (k < K) {
        const int64_t b0 = brpt[k], b1 = brpt[k + 1];
        // rows of up to DUP_MAX entries whose length and end columns match
        // are compared in full; the compare has no early exit so that its
        // loads can be in flight together
        if (dup && k > 0 && b1 > b0) {
            const int64_t p0 = brpt[k - 1], L = b1 - b0;
            if (b0 - p0 == L && L <= DUP_MAX && bcol[p0] == bcol[b0] && bcol[b0 - 1] == bcol[b1 - 1]) {
                int diff = 0;
#pragma unroll 8
                for (int64_t e = 1; e + 1 < L; ++e) diff |= bcol[p0 + e] ^ bcol[b0 + e];
                d = diff == 0;
            }
        }
        brec[k] = b1 > b0 ? make_int4((int)(b1 - b0), bcol[b0], bcol[b1 - 1], d)
                          : make_int4(0, INT_MAX, -1, 0);
    }
    if (ndup) {   // uniform: per-wave counts into LDS, one global atomic per workgroup
        __syncthreads();
        const unsigned long long m = __ballot(d != 0);
        if ((threadIdx.x & 63) == 0 && m) atomicAdd(&s_dup, (unsigned int)__popcll(m));
        __syncthreads();
        if (threadIdx.x == 0 && s_dup) atomicAdd(ndup, (unsigned long long)s_dup);
    }
}

hipError_t launch_brange(const DevCSR &B, int4 *brec, bool dup, unsigned long long *ndup,
                         hipStream_t s) {
    if (!dup) ndup = nullptr;
    if (ndup) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ndup);
    if (B.rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_brange, dim3((unsigned)((B.rows + 255) / 256)), dim3(256), 0, s, B.rows,
                       B.rpt, B.col, brec, dup ? 1 : 0, ndup);
    return hipGetLastError();
}

// Rows of A with the same columns as the row before them (rows of 1 to
// DUP_MAX entries; the compare as in k_brange).
__global__ __launch_bounds__(256) void k_arow_same(int64_t M, const int64_t *__restrict__ arpt,
                                                   const int32_t *__restrict__ acol,
                                                   uint8_t *__restrict__ same) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    int d = 0;
    if (r > 0) {
        const int64_t a0 = arpt[r], a1 = arpt[r + 1], p0 = arpt[r - 1], L = a1 - a0;
        if (L > 0 && a0 - p0 == L && L <= DUP_MAX && acol[p0] == acol[a0] && acol[a0 - 1] == acol[a1 - 1]) {
            int diff = 0;
#pragma unroll 8
            for (int64_t e = 1; e + 1 < L; ++e) diff |= acol[p0 + e] ^ acol[a0 + e];
            d = diff == 0;
        }
    }
    same[r] = (uint8_t)d;
}

// Distance of each row to the first row of its run of identical rows; a
// row at a multiple of ARUN_CAP starts a run, so the walk back is short.
__global__ __launch_bounds__(256) void k_arow_run(int64_t M, const int4 *__restrict__ brec,
                                                  const uint8_t *__restrict__ same,
                                                  uint8_t *__restrict__ arun) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    int d = 0;
    while (((r - d) & (ARUN_CAP - 1)) != 0 && (brec ? brec[r - d].w : (int)same[r - d]) != 0) ++d;
    arun[r] = (uint8_t)d;
}

__global__ __launch_bounds__(256) void k_arow_copy(int64_t M, const uint8_t *__restrict__ arun,
                                                   int64_t *__restrict__ nnz) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    const int d = arun[r];
    if (d) nnz[r] = nnz[r - d];   // the run's first row has d = 0: not written here
}

hipError_t launch_arun(const DevCSR &A, const int4 *brec, uint8_t *same, uint8_t *arun,
                       hipStream_t s) {
    if (A.rows == 0) return hipSuccess;
    const dim3 grid((unsigned)((A.rows + 255) / 256));
    if (!brec) hipLaunchKernelGGL(k_arow_same, grid, dim3(256), 0, s, A.rows, A.rpt, A.col, same);
    hipLaunchKernelGGL(k_arow_run, grid, dim3(256), 0, s, A.rows, brec, (const uint8_t *)same, arun);
    return hipGetLastError();
}

hipError_t launch_arun_copy(int64_t M, const uint8_t *arun, int64_t *nnz, hipStream_t s) {
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_arow_copy, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, M, arun, nnz);
    return hipGetLastError();
}

hipError_t launch_hist(int64_t M, const int64_t *v, const Bounds &bd, const BlockParts &parts,
                       hipStream_t s) {
    if (M == 0) return hipSuccess;
    const int64_t grid = (M + 255) / 256;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)grid), dim3(256), 0, s, M, v, bd, parts);
    return hipGetLastError();
}

hipError_t launch_finalize(int64_t M, int nslots, const BlockParts &parts, Counters *ctr,
                           int64_t *total_out, bool scan, hipStream_t s) {
    const int64_t nblk = (M + 255) / 256;
    if (scan)
        hipLaunchKernelGGL(k_finalize<true>, dim3(1), dim3(1024), 0, s, nblk, nslots, parts, ctr,
                           total_out);
    else
        hipLaunchKernelGGL(k_finalize<false>, dim3(1), dim3(1024), 0, s, nblk, nslots, parts, ctr,
                           total_out);
    return hipGetLastError();
}

hipError_t launch_scatter(int64_t M, int64_t *v, const Bounds &bd, const Counters *ctr,
                          int32_t *bins, const BlockParts &parts, bool scan, hipStream_t s,
                          int64_t *vout, bool device_identity, const int2 *rng) {
    if (M == 0) return hipSuccess;
    const int64_t grid = (M + 255) / 256;
    if (!vout) vout = v;
    if (scan)
        hipLaunchKernelGGL(k_scatter<true>, dim3((unsigned)grid), dim3(256), 0, s, M, v, bd, ctr,
                           bins, parts, vout, 0, nullptr);
    else
        hipLaunchKernelGGL(k_scatter<false>, dim3((unsigned)grid), dim3(256), 0, s, M, v, bd, ctr,
                           bins, parts, vout, device_identity ? 1 : 0, rng);
    return hipGetLastError();
}

}  // namespace opsp
