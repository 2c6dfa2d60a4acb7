// Symbolic step (OpSparse Section 5.2 Alg. 4, Section 5.6.1 kernel
// configuration): the number of distinct columns of every row of C, written
// over n_prod in C.rpt.
//
// Hashing: one compare-and-swap per probe (the paper's "single access"):
// the returned old value says whether the slot was empty (new key), held the
// key (duplicate) or another key (probe the next slot).
//
// gfx950 mapping of the work of one row:
//  * bin 0: 8 lanes per row, 32 rows per 256-lane workgroup; each lane takes
//    every 8th entry of A's row and walks that B row alone (tiny rows);
//  * bin 1: one wave per row (4 rows per workgroup, wave-level sync only);
//  * bins 2-7: one workgroup per row;
//  in bins 1-8 the products of the row are enumerated flat (row_products):
//  every lane handles one product per 64-product window, whatever the
//  lengths of the B rows.
//  * bin 7 uses all 160 KB of LDS and abandons a row as soon as its distinct
//    count passes the abort threshold (0.8 of the table, Section 5.6.1);
//  * bin 8 recomputes abandoned rows with per-workgroup global-memory tables
//    sized from the row's own bound min(n_prod, N), persistent workgroups.
#include "opsp_internal.h"

namespace opsp {

// 1 = new key, 0 = key already present, -1 = no free slot after T probes
// (cannot happen when the bin bounds hold; reported instead of spinning).
__device__ __forceinline__ int sym_insert_lds(int *tab, uint32_t T, int key) {
    uint32_t s = hslot(key, T);
    for (uint32_t n = 0; n < T; ++n) {
        const int old = hash_claim(&tab[s], key);
        if (old == -1) return 1;
        if (old == key) return 0;
        s = next_slot(s, T);
    }
    return -1;
}

// ---------------------------------------------------------------------------
// bin 0: GL lanes per row (eight waves per SIMD requested: the
// occupancy is otherwise capped at seven by scalar registers)
// ---------------------------------------------------------------------------
template <int GL, int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_sym_group(RowSrc src, const int64_t *__restrict__ arpt,
                                                   const int32_t *__restrict__ acol,
                                                   const int64_t *__restrict__ brpt,
                                                   const int32_t *__restrict__ bcol,
                                                   int64_t *__restrict__ nnz,
                                                   Counters *__restrict__ ctr) {
    constexpr int RPW = 256 / GL;
    __shared__ int tab[RPW * T];
    src.resolve();
    const int slot = threadIdx.x / GL, g = threadIdx.x % GL;
    int *t = tab + slot * T;
    for (int64_t b0 = (int64_t)blockIdx.x * RPW; b0 < src.nrows; b0 += (int64_t)gridDim.x * RPW) {
        const int64_t idx = b0 + slot;
        const bool active = idx < src.nrows;
        for (int s = g; s < T; s += GL) t[s] = -1;
        __syncthreads();
        int cnt = 0;
        int64_t row = 0;
        if (active) {
            row = src.row(idx);
            const int64_t a1 = arpt[row + 1];
            for (int64_t p = arpt[row] + g; p < a1; p += GL) {
                const int k = acol[p];
                const int64_t b1 = brpt[k + 1];
                // GRP_U keys of the B row are loaded before any is inserted
                // (indices past the row end re-read its first key, unused)
                for (int64_t q = brpt[k]; q < b1; q += GRP_U) {
                    int kk[GRP_U];
#pragma unroll
                    for (int u = 0; u < GRP_U; ++u) kk[u] = bcol[q + u < b1 ? q + u : q];
#pragma unroll
                    for (int u = 0; u < GRP_U; ++u) {
                        if (q + u < b1) {
                            const int r = sym_insert_lds(t, T, kk[u]);
                            if (r < 0) atomicAdd(&ctr->error, 1u);
                            else cnt += r;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int o = GL / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, GL);
        if (active && g == 0) nnz[row] = cnt;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// bins 1-7: one team (a wave for W == 64, else the workgroup) per row
// ---------------------------------------------------------------------------
template <int W, int T, bool ABORT, bool PERSIST>
// Eight waves per SIMD requested where the LDS allows them: wave teams
// (scalar registers would otherwise cap the occupancy at seven), and the
// 512- and 1024-thread teams whose tables let two or four workgroups share a
// CU (at more than 64 vector registers only one would fit: rmat 2^20
// symbolic 46.8 -> 42.9 ms).
__global__ __launch_bounds__(W == 64 ? 256 : W) __attribute__((amdgpu_waves_per_eu((W == 64 || (W >= 512 && T <= 20448)) ? 8 : 1))) void k_sym_row(
    RowSrc src, const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const int64_t *__restrict__ brpt, const int32_t *__restrict__ bcol, int64_t *__restrict__ nnz,
    int abort_thr, Counters *__restrict__ ctr, int32_t *__restrict__ fail_list,
    const int2 *__restrict__ rng, const int4 *__restrict__ brec, const uint8_t *__restrict__ arun) {
    constexpr bool WT = (W == 64);
    constexpr int R = WT ? 4 : 1;
    constexpr int NW = W / 64;  // waves per team
    __shared__ __align__(16) int tab[R * T];
    __shared__ int s_cnt[R];
    __shared__ int s_abort[R];
    __shared__ int red[NW];
    src.resolve();

    // the team index is uniform over each wave: keep it (and all per-row
    // values derived from it) in scalar registers
    const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / W), t = threadIdx.x % W;
    int *tb = tab + team * T;
    const int64_t stride = PERSIST ? (int64_t)gridDim.x * R : src.nrows + R;
    for (int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * R; b0 < src.nrows; b0 += stride) {
        const int64_t idx = b0 + team;
        bool active = idx < src.nrows;
        // A row whose output columns span a range that fits a bitmap of at
        // most TP words (TP = the largest power of two <= T) is counted in
        // that bitmap (an atomic OR per product, a popcount at the end)
        // instead of the hash table: same count, no probing.  Column offset o sets bit o >> lg of word
        // o & (nw - 1), so neighbouring columns land in different words
        // (different banks, no serialised ORs on one word).
        constexpr int TP = 1 << (31 - __builtin_clz(T));
        int64_t row = 0, a0 = 0, a1 = 0;
        bool bm = false;
        int lo = 0, nwords = 0, lgw = 0;
        uint32_t span = 0;
        if (active) {
            row = src.row(idx);
            a0 = arpt[row];   // issued together with the range and n_prod loads
            a1 = arpt[row + 1];
            if (rng) {
                const int2 r = rng[row];
                const int64_t np = nnz[row];
                lo = r.x;
                const int64_t sp = (int64_t)r.y - lo + 1;
                if (sp <= 32ll * TP) {
                    int nw = 1;
                    while (32ll * nw < sp) nw <<= 1;
                    // the largest bin counts by bitmap whenever it fits (no
                    // abandoned rows); the others when the bitmap is small
                    // against the row's products, and always for rows with
                    // more products than the table has slots (routed here by
                    // their range, bin_of_row)
                    if ((ABORT ? nw <= 2 * np : (2 * nw <= np || np > T)) || sp <= 0) {
                        bm = true;
                        nwords = sp > 0 ? nw : 0;
                        span = sp > 0 ? (uint32_t)sp : 0u;
                        lgw = 31 - __builtin_clz((unsigned)nw);
                    }
                }
            }
            // a row with the columns of the row before it is counted by its
            // run's first row (the count is copied after the symbolic step)
            if (arun && arun[row]) {
                active = false;
                bm = false;
            }
        }
        team_sync<WT>();   // the previous row of this team is done with the table
        // 16-byte LDS stores where the sizes allow (T and the bitmap's
        // power-of-two word count are multiples of 4 words)
        static_assert(T % 4 == 0, "vector clears");
        if (bm) {
            if (nwords >= 4) {
                uint4 *p4 = reinterpret_cast<uint4 *>(tb);
                for (int s = t; s < (nwords >> 2); s += W) p4[s] = make_uint4(0u, 0u, 0u, 0u);
            } else {
                for (int s = t; s < nwords; s += W) tb[s] = 0;
            }
        } else {
            int4 *p4 = reinterpret_cast<int4 *>(tb);
            for (int s = t; s < T / 4; s += W) p4[s] = make_int4(-1, -1, -1, -1);
        }
        if (t == 0) { s_cnt[team] = 0; s_abort[team] = 0; }
        team_sync<WT>();

        int cnt = 0;
        if (active && bm) {
            const uint32_t wmask = (uint32_t)nwords - 1u;
            auto set = [&](bool ok, int key) {
                const uint32_t o = (uint32_t)(key - lo);
                if (ok && o < span) atomicOr((unsigned int *)&tb[o & wmask], 1u << (o >> lgw));
            };
            row_products<false, (W >= 512 ? (ABORT ? SYM_ABORT_D : WIDE_D) : 1)>(a0, a1, acol, (const double *)nullptr, brpt, bcol, (const double *)nullptr, t >> 6, NW, set,
                                [] { return false; }, brec);
        } else if (active) {
            auto ins = [&](bool ok, int key) {
                const int nw = sym_insert_wave(tb, (uint32_t)T, ok, key, &ctr->error);
                if constexpr (ABORT) {
                    const unsigned long long m = __ballot(nw);
                    const int nm = (int)__popcll(m);
                    if (nm && lane_id() == 0) {
                        if (atomicAdd(&s_cnt[team], nm) + nm > abort_thr) s_abort[team] = 1;
                    }
                } else {
                    cnt += nw;
                }
            };
            auto stop = [&]() -> bool {
                if constexpr (ABORT) return *(volatile int *)&s_abort[team] != 0;
                else return false;
            };
            row_products<false, (W >= 512 ? (ABORT ? SYM_ABORT_D : WIDE_D) : 1)>(a0, a1, acol, (const double *)nullptr, brpt, bcol, (const double *)nullptr, t >> 6, NW, ins, stop,
                brec);
        }
        if (bm) {   // uniform over the team
            team_sync<WT>();
            if (nwords >= 4) {
                const uint4 *p4 = reinterpret_cast<const uint4 *>(tb);
                for (int s = t; s < (nwords >> 2); s += W) {
                    const uint4 v = p4[s];
                    cnt += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
                }
            } else {
                for (int s = t; s < nwords; s += W) cnt += __popc((unsigned int)tb[s]);
            }
        }
        if (ABORT && !bm) {
            team_sync<WT>();
            if (active && t == 0) {
                if (s_abort[team]) {
                    const unsigned f = atomicAdd(&ctr->fail, 1u);
                    fail_list[f] = (int32_t)row;
                } else {
                    nnz[row] = s_cnt[team];
                }
            }
        } else {
            cnt = wave_sum(cnt);
            if constexpr (WT) {
                if (active && t == 0) nnz[row] = cnt;
            } else {
                if ((t & 63) == 0) red[t >> 6] = cnt;
                __syncthreads();
                if (active && t == 0) {
                    int sum = 0;
                    for (int i = 0; i < NW; ++i) sum += red[i];
                    nnz[row] = sum;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// bin 8: rows too long for the LDS tables.  With the row's column range
// known, the distinct columns are counted in an LDS bitmap of 2^20 columns,
// one pass over the row's products per 2^20-column window of the range
// (a product is a bit set; no probing, no global table).  Rows whose range
// needs more than SW_MAXPASS windows, and every row when no ranges were
// computed, use a global-memory hash table, one slab per workgroup.  Rows
// are taken from a counter (the longest rows would otherwise pile up on a
// few workgroups of a round-robin assignment).
// ---------------------------------------------------------------------------
constexpr int SW_WORDS = 1 << (SW_LG - 5);

__global__ __launch_bounds__(1024) void k_sym_global(
    RowSrc src, const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const int64_t *__restrict__ brpt, const int32_t *__restrict__ bcol, int64_t *__restrict__ nnz,
    int64_t ncols, int *slabs, int64_t slab_entries, const int2 *__restrict__ rng,
    unsigned long long *sched, Counters *__restrict__ ctr, const int4 *__restrict__ brec) {
    __shared__ unsigned int bm[SW_WORDS];
    __shared__ int red[16];
    __shared__ long long s_r;
    src.resolve();
    int *tb = slabs ? slabs + (int64_t)blockIdx.x * slab_entries : nullptr;
    const int t = threadIdx.x, wv = t >> 6, l = t & 63;
    int64_t r = blockIdx.x;
    while (true) {
        if (sched) {
            if (t == 0) s_r = (long long)take_row(sched, src.nrows);
            __syncthreads();
            r = (int64_t)s_r;
        }
        if (r >= src.nrows) break;   // uniform
        const int64_t row = src.row(r);
        const int64_t a0 = arpt[row], a1 = arpt[row + 1];
        int64_t lo = 0, span = -1;
        if (rng) {
            const int2 rg = rng[row];
            lo = rg.x;
            span = (int64_t)rg.y - rg.x + 1;
        }
        if (rng && span <= ((int64_t)SW_MAXPASS << SW_LG)) {
            int64_t total = 0;
            for (int64_t w0 = 0; w0 < span; w0 += (1 << SW_LG)) {
                const int64_t rest = span - w0;
                const uint32_t wlen = rest < (1 << SW_LG) ? (uint32_t)rest : (1u << SW_LG);
                const uint32_t words = (wlen + 31) >> 5;
                for (uint32_t i = t; i < words; i += 1024) bm[i] = 0u;
                __syncthreads();
                const uint32_t base = (uint32_t)(lo + w0);
                row_products<false, WIDE_D>(a0, a1, acol, (const double *)nullptr, brpt, bcol, (const double *)nullptr, wv, 16,
                                    [&](bool ok, int key) {
                                        const uint32_t o = (uint32_t)key - base;
                                        if (ok && o < wlen) atomicOr(&bm[o >> 5], 1u << (o & 31));
                                    },
                                    [] { return false; }, brec);
                __syncthreads();
                unsigned int c = 0;
                for (uint32_t i = t; i < words; i += 1024) c += __popc(bm[i]);
                c = wave_sum(c);
                if (l == 0) red[wv] = (int)c;
                __syncthreads();
                for (int i = 0; i < 16; ++i) total += red[i];
                __syncthreads();
            }
            if (t == 0) nnz[row] = total < 0 ? 0 : total;
        } else {
            // C.rpt[row] still holds n_prod for rows that reach this kernel
            const int64_t np = nnz[row];
            const int64_t bound = np < ncols ? np : ncols;
            uint32_t T = pow2_at_least((uint64_t)(2 * bound > 64 ? 2 * bound : 64));
            if ((int64_t)T > slab_entries) T = (uint32_t)slab_entries;
            for (uint32_t s = t; s < T; s += 1024) tb[s] = -1;
            __syncthreads();
            int cnt = 0;
            auto ins = [&](bool ok, int key) { cnt += sym_insert_wave(tb, T, ok, key, &ctr->error); };
            row_products<false, WIDE_D>(a0, a1, acol, (const double *)nullptr, brpt, bcol, (const double *)nullptr, wv, 16, ins,
                                [] { return false; }, brec);
            cnt = wave_sum(cnt);
            if (l == 0) red[wv] = cnt;
            __syncthreads();
            if (t == 0) {
                int64_t sum = 0;
                for (int i = 0; i < 16; ++i) sum += red[i];
                nnz[row] = sum;
            }
        }
        __syncthreads();
        if (!sched) r += gridDim.x;
    }
}

// ---------------------------------------------------------------------------
static int64_t grid_for(const SymArgs &a, int64_t per_wg) {
    if (a.grid > 0) return a.grid;
    return (a.src.nrows + per_wg - 1) / per_wg;
}

template <int W, int T, bool ABORT>
static hipError_t go_row(const SymArgs &a, hipStream_t s) {
    constexpr int R = (W == 64) ? 4 : 1;
    const int64_t grid = grid_for(a, R);
    if (grid <= 0) return hipSuccess;
    if (a.grid > 0)
        hipLaunchKernelGGL((k_sym_row<W, T, ABORT, true>), dim3((unsigned)grid), dim3(W * R), 0, s,
                           a.src, a.A.rpt, a.A.col, a.B.rpt, a.B.col, a.nnz, a.abort_thr, a.ctr,
                           a.fail_list, a.rng, a.brec, a.arun);
    else
        hipLaunchKernelGGL((k_sym_row<W, T, ABORT, false>), dim3((unsigned)grid), dim3(W * R), 0, s,
                           a.src, a.A.rpt, a.A.col, a.B.rpt, a.B.col, a.nnz, a.abort_thr, a.ctr,
                           a.fail_list, a.rng, a.brec, a.arun);
    return hipGetLastError();
}

hipError_t launch_symbolic_bin(int bin, const SymArgs &a, hipStream_t s) {
    if (!a.src.dctr && !a.src.count && a.src.nrows == 0) return hipSuccess;
    switch (bin) {
        case 0: {
            const int64_t grid = grid_for(a, 256 / GROUP_GL[a.gv]);
            if (grid <= 0) return hipSuccess;
            switch (a.gv) {
                case 1:
                    hipLaunchKernelGGL((k_sym_group<GROUP_GL[1], SYM_T0[1]>), dim3((unsigned)grid), dim3(256), 0,
                                       s, a.src, a.A.rpt, a.A.col, a.B.rpt, a.B.col, a.nnz, a.ctr);
                    break;
                case 2:
                    hipLaunchKernelGGL((k_sym_group<GROUP_GL[2], SYM_T0[2]>), dim3((unsigned)grid), dim3(256), 0,
                                       s, a.src, a.A.rpt, a.A.col, a.B.rpt, a.B.col, a.nnz, a.ctr);
                    break;
                default:
                    hipLaunchKernelGGL((k_sym_group<GROUP_GL[0], SYM_T0[0]>), dim3((unsigned)grid), dim3(256), 0,
                                       s, a.src, a.A.rpt, a.A.col, a.B.rpt, a.B.col, a.nnz, a.ctr);
            }
            return hipGetLastError();
        }
        case 1: return go_row<SYM_W[1], SYM_T[1], false>(a, s);
        case 2: return go_row<SYM_W[2], SYM_T[2], false>(a, s);
        case 3: return go_row<SYM_W[3], SYM_T[3], false>(a, s);
        case 4: return go_row<SYM_W[4], SYM_T[4], false>(a, s);
        case 5: return go_row<SYM_W[5], SYM_T[5], false>(a, s);
        case 6: return go_row<SYM_W[6], SYM_T[6], false>(a, s);
        case 7: return go_row<SYM_W[7], SYM_T[7], true>(a, s);
        case SYM_GLOBAL_BIN: {
            if (a.grid <= 0) return hipSuccess;
            hipLaunchKernelGGL(k_sym_global, dim3((unsigned)a.grid), dim3(1024), 0, s, a.src, a.A.rpt,
                               a.A.col, a.B.rpt, a.B.col, a.nnz, a.B.cols, a.slab, a.slab_entries,
                               a.rng, a.sched, a.ctr, a.brec);
            return hipGetLastError();
        }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace opsp
