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

// Value types.  The kernels read A and B and write C in the product's value
// type V (double, or float for the FP32 product) and form each product
// a_ik * b_kj in V, but their LDS tables and global tables always sum in
// FP64: on gfx950 the LDS FP32 atomic add (ds_add_f32) runs at about 1/20 of
// the rate of ds_add_f64 (0.33 against 7.5 lane operations per CU per clock,
// measured), and an FP64 sum rounded once is the more accurate anyway.

// Value pointers of the launch arguments in the product's value type.
template <class V>
struct VPtrs {
    const V *aval, *bval;
    V *cval, *slab_vals;
    explicit VPtrs(const NumArgs &a)
        : aval((const V *)a.A.val), bval((const V *)a.B.val), cval((V *)a.cval),
          slab_vals((V *)a.slab_vals) {}
};


// Returns false when no slot was found after T probes (cannot happen when the
// bin bounds hold; reported instead of spinning).
template <class V>
__device__ __forceinline__ bool num_insert_lds(int *keys, V *vals, uint32_t T, int key, V v) {
    uint32_t s = hslot(key, T);
    for (uint32_t n = 0; n < T; ++n) {
        const int old = hash_claim(&keys[s], key);
        if (old == -1 || old == key) {
            atomicAdd(&vals[s], v);
            return true;
        }
        s = next_slot(s, T);
    }
    return false;
}

// Accumulate one product per lane (lanes with ok == false take part without
// one): compare-and-swap the key, then add the product to the slot holding it
// (Alg. 5).  The probe loop is uniform over the wave and bounded by T
// iterations with a scalar counter.  Returns 1 when this lane's key was new.
template <class KeyT, class ValT, class AddF>
__device__ __forceinline__ int num_insert_wave(KeyT *keys, ValT *vals, uint32_t T, bool ok, int key,
                                               ValT v, unsigned int *err, AddF &&add) {
    bool pend = ok;
    int isnew = 0;
    uint32_t s = ok ? hslot(key, T) : 0u;
    for (uint32_t it = 0; __ballot(pend); ++it) {
        if (it >= T) {
            if (pend) atomicAdd(err, 1u);
            break;
        }
        if (pend) {
            const int old = hash_claim(&keys[s], key);
            const bool hit = (old == -1) | (old == key);
            if (hit) add(&vals[s], v);
            isnew = old == -1;
            pend = !hit;
            s = hit ? s : next_slot(s, T);
        }
    }
    return isnew;
}

// ---------------------------------------------------------------------------
// One-phase step (the upper-bound alternative of Section 2.2, with predicted
// per-row capacities in place of a bound): where a finished row goes.
// ---------------------------------------------------------------------------

// Start index for the n entries of `row`: its slot when they fit, else a
// range of the overflow arena; -1 when the arena is exhausted.
__device__ __forceinline__ int64_t lrn_place(const Learn &L, int64_t row, int64_t n) {
    const int64_t o = L.off ? L.off[row] : 0;
    const int64_t cap = L.off ? L.off[row + 1] - o : 0;
    if (n <= cap) return o;
    const unsigned long long a = atomicAdd(&L.lc->arena_used, (unsigned long long)n);
    if ((int64_t)a + n <= L.arena_cap) {
        atomicAdd(&L.lc->slot_overflow, 1u);
        return L.arena_base + (int64_t)a;
    }
    return -1;
}

// Queue `row` for the exact recompute (mode 2), with its output bound.
__device__ __forceinline__ void lrn_retry(const Learn &L, int64_t row, bool table_full) {
    const unsigned f = atomicAdd(&L.lc->retry, 1u);
    L.retry[f] = (int32_t)row;
    const int64_t np = L.nprod[row];
    atomicAdd(&L.lc->retry_ub, (unsigned long long)(np < L.ncols ? np : L.ncols));
    if (table_full) atomicAdd(&L.lc->table_overflow, 1u);
}

__device__ __forceinline__ void lrn_done(const Learn &L, int64_t row, int64_t n, int64_t base) {
    L.nnz[row] = n;
    L.loc[row] = base + L.loc_bias;
}

// ---------------------------------------------------------------------------
// bin 0: GL lanes per row (eight waves per SIMD requested: the
// occupancy is otherwise capped at seven by scalar registers); rank counting over the packed keys
// ---------------------------------------------------------------------------
template <int GL, int T, bool LRN, class V>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_num_group(
    RowSrc src, const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const V *__restrict__ aval, const int64_t *__restrict__ brpt,
    const int32_t *__restrict__ bcol, const V *__restrict__ bval,
    const int64_t *__restrict__ crpt, int32_t *__restrict__ ccol, V *__restrict__ cval,
    Counters *__restrict__ ctr, Learn L) {
    constexpr int RPW = 256 / GL;
    constexpr int ITEMS = (T + GL - 1) / GL;
    __shared__ double vals[RPW * T];   // sums in FP64 for either value type
    __shared__ int keys[RPW * T];
    __shared__ int ck[RPW * T];
    __shared__ int s_full[RPW];   // one-phase: the row's table filled up
    src.resolve();
    const int slot = threadIdx.x / GL, g = threadIdx.x % GL;
    int *tk = keys + slot * T;
    double *tv = vals + slot * T;
    int *pk = ck + slot * T;
    for (int64_t b0 = (int64_t)blockIdx.x * RPW; b0 < src.nrows; b0 += (int64_t)gridDim.x * RPW) {
        const int64_t idx = b0 + slot;
        const bool active = idx < src.nrows;
        for (int s = g; s < T; s += GL) { tk[s] = -1; tv[s] = 0.0; }
        if (LRN && g == 0) s_full[slot] = 0;
        __syncthreads();
        int64_t row = 0, c0 = 0, c1 = 0;
        if (active) {
            row = src.row(idx);
            const int64_t a1 = arpt[row + 1];
            if constexpr (!LRN) {   // the row's place in C, used at the end
                c0 = crpt[row];
                c1 = crpt[row + 1];
            }
            for (int64_t p = arpt[row] + g; p < a1; p += GL) {
                const int k = acol[p];
                const V a = aval[p];
                const int64_t b1 = brpt[k + 1];
                bool full = false;
                // GRP_U entries of the B row are loaded before any is
                // inserted (indices past the row end re-read its first entry,
                // unused)
                for (int64_t q = brpt[k]; q < b1 && !full; q += GRP_U) {
                    int kk[GRP_U];
                    V vv[GRP_U];
#pragma unroll
                    for (int u = 0; u < GRP_U; ++u) {
                        const int64_t qq = q + u < b1 ? q + u : q;
                        kk[u] = bcol[qq];
                        vv[u] = bval[qq];
                    }
#pragma unroll
                    for (int u = 0; u < GRP_U; ++u) {
                        if (q + u < b1 && !full && !num_insert_lds(tk, tv, T, kk[u], (double)(a * vv[u]))) {
                            if constexpr (LRN) {
                                s_full[slot] = 1;
                                full = true;
                            } else {
                                atomicAdd(&ctr->error, 1u);
                            }
                        }
                    }
                }
                if (LRN && (full || *(volatile int *)&s_full[slot])) break;
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
        int64_t base = 0, cap = 0;
        if (active) {
            if constexpr (LRN) {
                int64_t b = -1;
                if (s_full[slot]) {
                    if (g == 0) lrn_retry(L, row, true);
                } else if (g == 0) {
                    b = lrn_place(L, row, n);
                    if (b < 0) lrn_retry(L, row, false);
                    else lrn_done(L, row, n, b);
                }
                base = __shfl(b, 0, GL);
                cap = base < 0 ? 0 : n;
            } else {
                base = c0;
                cap = c1 - c0;
                if (g == 0 && cap != n) atomicAdd(&ctr->error, 1u);
            }
        }
        if (active && cap > 0) {
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
        __syncthreads();
    }
}

// Ascending bitonic sort of keys[0..n) carrying an int payload (mirrored
// first comparator per merge; positions >= n are virtual +inf and never
// touched).  All index arithmetic is shifts and masks.
template <int NT, bool WT, class P>
__device__ __forceinline__ void team_bitonic(int *keys, P *pay, int n, int t) {
    if (n < 2) return;
    int lgP = 0;
    while ((1 << lgP) < n) ++lgP;
    const int half = 1 << (lgP - 1);
    auto ce = [&](int i, int j) {
        if (j < n) {
            const int ki = keys[i], kj = keys[j];
            if (ki > kj) {
                keys[i] = kj;
                keys[j] = ki;
                const P pi = pay[i];
                pay[i] = pay[j];
                pay[j] = pi;
            }
        }
    };
    for (int lk = 1; lk <= lgP; ++lk) {
        const int lh = lk - 1;
        const int hmask = (1 << lh) - 1;
        for (int c = t; c < half; c += NT) {
            const int blk = c >> lh, off = c & hmask;
            const int i = (blk << lk) + off;
            const int j = (blk << lk) + (1 << lk) - 1 - off;
            ce(i, j);
        }
        team_sync<WT>();
        for (int ld = lh - 1; ld >= 0; --ld) {
            const int dmask = (1 << ld) - 1;
            for (int c = t; c < half; c += NT) {
                const int i = ((c >> ld) << (ld + 1)) + (c & dmask);
                ce(i, i + (1 << ld));
            }
            team_sync<WT>();
        }
    }
}

// Reductions over a team (a wave, or the NW waves of a workgroup through the
// LDS scratch `red`, which holds at least 3*NW ints).
template <bool WT, int NW>
__device__ __forceinline__ void team_min_max_sum(int &mn, int &mx, int &sum, int *red) {
    mn = wave_min(mn);
    mx = wave_max(mx);
    sum = wave_sum(sum);
    if constexpr (!WT) {
        const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
        if (l == 0) {
            red[wv] = mn;
            red[NW + wv] = mx;
            red[2 * NW + wv] = sum;
        }
        __syncthreads();
        mn = red[0];
        mx = red[NW];
        sum = red[2 * NW];
        for (int i = 1; i < NW; ++i) {
            mn = red[i] < mn ? red[i] : mn;
            mx = red[NW + i] > mx ? red[NW + i] : mx;
            sum += red[2 * NW + i];
        }
        __syncthreads();
    }
}

// Exclusive prefix of one int per lane over the team, plus the team total.
template <bool WT, int NW>
__device__ __forceinline__ int team_excl_scan(int x, int &total, int *red) {
    const int incl = wave_incl_scan(x);
    if constexpr (WT) {
        total = __builtin_amdgcn_readlane(incl, 63);
        return incl - x;
    } else {
        const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
        if (l == 63) red[wv] = incl;
        __syncthreads();
        int pre = 0;
        total = 0;
        for (int i = 0; i < NW; ++i) {
            const int y = red[i];
            if (i < wv) pre += y;
            total += y;
        }
        __syncthreads();
        return pre + incl - x;
    }
}

// ---------------------------------------------------------------------------
// bins 1-6: one team (wave for W == 64, else the workgroup) per row
//
// Ordering after hashing.  The occupied slots are packed into (key, slot)
// pairs at the front of the key array, and each lane then holds the pairs
// e = t, t + W, ...  An entry's rank is computed with a two-level bitmap of
// the row's column range [kmin, kmax], built in the freed key array:
//   level 1: one bit per block of 32 columns, with u16 popcount prefixes per
//            word, numbers the non-empty blocks;
//   level 0: one 32-bit word per non-empty block (at most n), with u16
//            prefixes, holds the columns themselves;
// rank = prefix0[block number] + popcount of the block word below the column.
// Values stay in the hash table and are read through the slot.  Rows whose
// range does not fit the level-1 bitmap sort the pairs with the bitonic
// network instead; with binning ratios below 1.5 pairs may not fit at all and
// entries are ranked by counting over the table.
// ---------------------------------------------------------------------------
template <int W, int T, bool LRN, class V, bool MRG = false>
// wave teams: eight waves per SIMD requested (scalar registers would
// otherwise cap the occupancy at seven).  Merged runs hold up to NUM_RUN
// values per window and would spill within the 64 registers of that
// occupancy; teams of up to 256 lanes then ask for seven (72 registers, no
// spills; 2.38 -> 2.28 ms against the unconstrained 74 registers and six
// waves on the 3x3-block stencil 40^3)
__global__ __launch_bounds__(W == 64 ? 256 : W) __attribute__((amdgpu_waves_per_eu(MRG ? (W <= 256 ? 7 : 1) : (W == 64 ? 8 : 1)))) void k_num_row(
    RowSrc src, const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const V *__restrict__ aval, const int64_t *__restrict__ brpt,
    const int32_t *__restrict__ bcol, const V *__restrict__ bval,
    const int64_t *__restrict__ crpt, int32_t *__restrict__ ccol, V *__restrict__ cval,
    Counters *__restrict__ ctr, Learn L, const int2 *__restrict__ rng,
    const int4 *__restrict__ dup) {
    // MRG: entries whose B rows repeat the previous entry's column set are
    // merged into one table update per column (row_products, `dup` = B's row
    // records)
    static_assert(!(MRG && LRN), "runs are merged in the two-phase step only");
    constexpr int RN = MRG ? NUM_RUN : 1;
    constexpr bool WT = (W == 64);
    constexpr int R = WT ? 4 : 1;
    constexpr int NW = W / 64;
    constexpr int ITEMS = (T + W - 1) / W;
    constexpr int NPACK = (4 * T) / 6;               // pairs that fit the key array
    constexpr int EMAX = (NPACK + W - 1) / W;         // packed pairs per lane
    // one-phase: abandon the row once its distinct count passes THR.  Until a
    // wave sees the count above THR it inserts at most one more window of 64
    // keys, so the table never holds more than THR + W <= T keys.
    constexpr int THR = (4 * T) / 5 < T - W ? (4 * T) / 5 : T - W;
    static_assert(THR > 0, "table too small for the one-phase bound");
    __shared__ double vals[R * T];   // sums in FP64 for either value type
    __shared__ int keys[R * T];
    __shared__ int red[3 * NW];
    __shared__ int s_cnt[R];
    __shared__ long long s_base[R];

    src.resolve();
    // the team index is uniform over each wave: keep it (and all per-row
    // values derived from it) in scalar registers
    const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / W), t = threadIdx.x % W;
    const int wv = t >> 6;
    int *tk = keys + team * T;
    double *tv = vals + team * T;
    // one team per row (grids are sized from the numeric bin counts, which
    // are always read back before this step); every lane of the team makes
    // the same early returns
    auto do_row = [&](const int64_t idx) {
    const bool active = idx < src.nrows;
    // A row whose output columns span at most T positions accumulates into a
    // dense array of that range (values) plus a bitmap (occupancy): no
    // probing, and the rank of a column is a popcount.
    int64_t row = 0, a0 = 0, a1 = 0, c0 = 0, c1 = 0;
    bool dn = false;
    int lo = 0, dspan = 0;
    if (active) {
        row = src.row(idx);
        a0 = arpt[row];   // issued together with the range load
        a1 = arpt[row + 1];
        if constexpr (!LRN) {   // and the row's place in C, used at the end
            c0 = crpt[row];
            c1 = crpt[row + 1];
        }
        if (rng) {
            const int2 r = rng[row];
            lo = r.x;
            const int64_t sp = (int64_t)r.y - lo + 1;
            if (sp <= T) {
                dn = true;
                dspan = sp > 0 ? (int)sp : 0;
            }
        }
    }
    const int nwd = (dspan + 31) >> 5;
    team_sync<WT>();   // the previous row of this team is done with the table
    if (dn) {
        for (int s = t; s < dspan; s += W) tv[s] = 0.0;
        for (int s = t; s < nwd; s += W) tk[s] = 0;
    } else {
        for (int s = t; s < T; s += W) { tk[s] = -1; tv[s] = 0.0; }
    }
    if (LRN && t == 0) s_cnt[team] = 0;
    team_sync<WT>();

    // where the n entries of the row go: (base, cap), base < 0 = skip
    auto place = [&](int n, int64_t &base, int64_t &cap) {
        if constexpr (LRN) {
            if (active && t == 0) {
                const int64_t b = lrn_place(L, row, n);
                if (b < 0) lrn_retry(L, row, false);
                else lrn_done(L, row, n, b);
                s_base[team] = b;
            }
            team_sync<WT>();
            base = active ? (int64_t)s_base[team] : -1;
            cap = n;
        } else {
            base = active ? c0 : -1;
            cap = active ? c1 - c0 : 0;
            if (active && t == 0 && cap != n) atomicAdd(&ctr->error, 1u);
        }
    };

    if (dn) {   // uniform over the team
        if (active) {
            unsigned int *bits = reinterpret_cast<unsigned int *>(tk);
            auto acc = [&](bool ok, int key, auto v) {
                const uint32_t o = (uint32_t)(key - lo);
                if (ok && o < (uint32_t)dspan) {
                    atomicOr(&bits[o >> 5], 1u << (o & 31));
                    atomicAdd(&tv[o], (double)v);
                }
            };
            row_products<true, (W >= 512 ? WIDE_D : 1), V, RN>(a0, a1, acol, aval, brpt, bcol, bval, wv,
                                                                NW, acc, [] { return false; }, dup);
        }
        team_sync<WT>();
        // exclusive popcount prefix per bitmap word, after the words
        unsigned int *bits = reinterpret_cast<unsigned int *>(tk);
        int *pre = tk + nwd;
        const int q = (nwd + W - 1) / W;
        const int w0 = t * q, w1 = w0 + q < nwd ? w0 + q : nwd;
        int sum = 0;
        for (int w = w0; w < w1; ++w) sum += __popc(bits[w]);
        int n;
        int p0 = team_excl_scan<WT, NW>(sum, n, red);
        for (int w = w0; w < w1; ++w) {
            pre[w] = p0;
            p0 += __popc(bits[w]);
        }
        team_sync<WT>();
        int64_t base, cap;
        place(n, base, cap);
        if (base < 0 || n == 0) return;   // uniform over the team
        for (int o = t; o < dspan; o += W) {
            const unsigned int word = bits[o >> 5];
            const unsigned int bit = 1u << (o & 31);
            if (word & bit) {
                const int rank = pre[o >> 5] + __popc(word & (bit - 1u));
                if (rank < cap) {
                    ccol[base + rank] = lo + o;
                    cval[base + rank] = tv[o];
                }
            }
        }
        return;
    }

    // one-phase: distinct keys inserted so far.  A one-wave team keeps the
    // count in a scalar register; larger teams add into LDS.
    int wcnt = 0;
    if (active) {
        auto ins = [&](bool ok, int key, auto v) {
            const int nw = num_insert_wave(tk, tv, (uint32_t)T, ok, key, (double)v, &ctr->error,
                                           [](double *p, double x) { atomicAdd(p, x); });
            if constexpr (LRN) {
                const int nm = (int)__popcll(__ballot(nw));
                if constexpr (WT) wcnt += nm;
                else if (nm && lane_id() == 0) atomicAdd(&s_cnt[team], nm);
            }
        };
        auto stop = [&]() -> bool {
            if constexpr (LRN && WT) return wcnt > THR;
            else if constexpr (LRN) return *(volatile int *)&s_cnt[team] > THR;
            else return false;
        };
        row_products<true, (W >= 512 ? WIDE_D : 1), V, RN>(a0, a1, acol, aval, brpt, bcol, bval, wv, NW,
                                                            ins, stop, dup);
    }
    team_sync<WT>();
    if constexpr (LRN) {
        if ((WT ? wcnt : s_cnt[team]) > THR) {   // uniform over the team
            if (active && t == 0) lrn_retry(L, row, true);
            return;
        }
    }

    // count, range and keys of this lane's slots (s = t + m*W)
    int rk[ITEMS];
    int c = 0, kmin = INT_MAX, kmax = -1;
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
        const int s = t + m * W;
        rk[m] = s < T ? tk[s] : -1;
        if (rk[m] >= 0) {
            ++c;
            kmin = rk[m] < kmin ? rk[m] : kmin;
            kmax = rk[m] > kmax ? rk[m] : kmax;
        }
    }
    int n = c;
    team_min_max_sum<WT, NW>(kmin, kmax, n, red);
    int64_t base, cap;
    place(n, base, cap);
    if (LRN && base < 0) return;   // uniform over the team
    if (n == 0) return;            // uniform over the team

    if (n > NPACK) {
        // rank by counting against the intact table
        if (active) {
#pragma unroll
            for (int m = 0; m < ITEMS; ++m) {
                if (rk[m] >= 0) {
                    int rank = 0;
                    for (int s2 = 0; s2 < T; ++s2) {
                        const int k2 = tk[s2];
                        rank += (k2 >= 0) & (k2 < rk[m]);
                    }
                    if (rank < cap) {
                        ccol[base + rank] = rk[m];
                        cval[base + rank] = tv[t + m * W];
                    }
                }
            }
        }
        return;
    }

    // pack (key, slot) pairs: keys in tk[0..n), u16 slots after them
    int tot;
    int pos = team_excl_scan<WT, NW>(c, tot, red);
    team_sync<WT>();   // every lane has read its slots
    unsigned short *ps = reinterpret_cast<unsigned short *>(tk + n);
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
        if (rk[m] >= 0) {
            tk[pos] = rk[m];
            ps[pos] = (unsigned short)(t + m * W);
            ++pos;
        }
    }
    team_sync<WT>();

    // A one-wave row of at most 64 entries: lane e holds packed entry e, and
    // its rank is the number of the other lanes' keys below its own (keys are
    // distinct), read lane by lane from registers.
    if constexpr (WT) {
        if (n <= 64) {   // uniform over the wave
            const int key = t < n ? tk[t] : INT_MAX;
            const int sl = t < n ? (int)ps[t] : 0;
            const int nn = __builtin_amdgcn_readfirstlane(n);
            int rank = 0;
            for (int j = 0; j < nn; ++j) rank += __builtin_amdgcn_readlane(key, j) < key ? 1 : 0;
            if (active && t < n && rank < cap) {
                ccol[base + rank] = key;
                cval[base + rank] = tv[sl];
            }
            return;
        }
    }

    // level-1 words (even count keeps level 0 4-byte aligned)
    const int span = kmax - kmin + 1;
    const int nblk1 = (int)(((int64_t)span + 31) >> 5);
    int l1w = (nblk1 + 31) >> 5;
    l1w += l1w & 1;
    const bool two_level = 6 * l1w + 6 * n <= 4 * T;
    if (!two_level) {
        team_bitonic<W, WT>(tk, ps, n, t);
        if (active) {
            const int nw = cap < n ? (int)cap : n;
            for (int e = t; e < nw; e += W) {
                ccol[base + e] = tk[e];
                cval[base + e] = tv[ps[e]];
            }
        }
        return;
    }

    // pairs per lane in use (uniform): the loops below stop there instead of
    // running all EMAX steps with the lanes masked off
    const int jn = __builtin_amdgcn_readfirstlane((n + W - 1) / W);
    int ek[EMAX], es[EMAX];
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {
        const int e = t + j * W;
        ek[j] = e < n ? tk[e] : -1;
        es[j] = e < n ? (int)ps[e] : 0;
    }
    team_sync<WT>();   // the pairs are in registers; the key array is free

    unsigned int *L1 = reinterpret_cast<unsigned int *>(tk);
    unsigned short *P1 = reinterpret_cast<unsigned short *>(L1 + l1w);
    unsigned int *L0 = reinterpret_cast<unsigned int *>(P1 + l1w);
    unsigned short *P0 = reinterpret_cast<unsigned short *>(L0 + n);
    for (int w = t; w < l1w; w += W) L1[w] = 0u;
    for (int w = t; w < n; w += W) L0[w] = 0u;
    team_sync<WT>();
    int eb[EMAX];
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {
        if (j >= jn) break;
        eb[j] = (ek[j] - kmin) >> 5;
        if (ek[j] >= 0) atomicOr(&L1[eb[j] >> 5], 1u << (eb[j] & 31));
    }
    team_sync<WT>();
    // level-1 prefixes: lane t owns words [t*q1, t*q1 + q1)
    {
        const int q1 = (l1w + W - 1) / W;
        const int w0 = t * q1, w1 = w0 + q1 < l1w ? w0 + q1 : l1w;
        int sum = 0;
        for (int w = w0; w < w1; ++w) sum += __popc(L1[w]);
        int nb;
        int pre = team_excl_scan<WT, NW>(sum, nb, red);
        for (int w = w0; w < w1; ++w) {
            P1[w] = (unsigned short)pre;
            pre += __popc(L1[w]);
        }
    }
    team_sync<WT>();
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {
        if (j >= jn) break;
        if (ek[j] >= 0) {
            const int b = eb[j];
            eb[j] = P1[b >> 5] + __popc(L1[b >> 5] & ((1u << (b & 31)) - 1u));
            atomicOr(&L0[eb[j]], 1u << ((ek[j] - kmin) & 31));
        }
    }
    team_sync<WT>();
    // level-0 prefixes over the non-empty blocks (at most n words)
    {
        const int q0 = (n + W - 1) / W;
        const int w0 = t * q0, w1 = w0 + q0 < n ? w0 + q0 : n;
        int sum = 0;
        for (int w = w0; w < w1; ++w) sum += __popc(L0[w]);
        int nn;
        int pre = team_excl_scan<WT, NW>(sum, nn, red);
        for (int w = w0; w < w1; ++w) {
            P0[w] = (unsigned short)pre;
            pre += __popc(L0[w]);
        }
    }
    team_sync<WT>();
    if (active) {
#pragma unroll
        for (int j = 0; j < EMAX; ++j) {
            if (j >= jn) break;
            if (ek[j] >= 0) {
                const int bit = (ek[j] - kmin) & 31;
                const int rank = P0[eb[j]] + __popc(L0[eb[j]] & ((1u << bit) - 1u));
                if (rank < cap) {
                    ccol[base + rank] = ek[j];
                    cval[base + rank] = tv[es[j]];
                }
            }
        }
    }
    };
    do_row(xcd_block(blockIdx.x, gridDim.x) * R + team);
}

// ---------------------------------------------------------------------------
// bin 7: global-memory tables (one slab per persistent workgroup), ordered
// through LDS bitmaps of 2^19 columns at a time.
// ---------------------------------------------------------------------------
template <bool LRN, class V>
__global__ __launch_bounds__(1024) void k_num_global(
    RowSrc src, const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const V *__restrict__ aval, const int64_t *__restrict__ brpt,
    const int32_t *__restrict__ bcol, const V *__restrict__ bval,
    const int64_t *__restrict__ crpt, int32_t *__restrict__ ccol, V *__restrict__ cval,
    int *slab_keys, double *slab_vals, int64_t slab_entries, Counters *__restrict__ ctr, Learn L) {
    constexpr int CW = NUM_GLOBAL_CHUNK_WORDS;
    constexpr int CBITS = CW * 32;
    constexpr int WPT = CW / 1024;  // bitmap words per thread
    __shared__ unsigned int bitmap[CW];
    __shared__ unsigned int prefix[CW];
    __shared__ unsigned int red[16];
    __shared__ int s_min, s_max;
    __shared__ unsigned int s_cnt;
    __shared__ long long s_base;

    src.resolve();
    int *tk = slab_keys + (int64_t)blockIdx.x * slab_entries;
    double *tv = slab_vals + (int64_t)blockIdx.x * slab_entries;
    const int t = threadIdx.x, wv = t >> 6, l = t & 63;

    for (int64_t r = blockIdx.x; r < src.nrows; r += gridDim.x) {
        const int64_t row = src.row(r);
        int64_t base = 0, n = 0;
        uint32_t T, thr = 0xffffffffu;
        if constexpr (LRN) {
            // mode 1: table from the predicted capacity, abandoned past thr
            // (at most one more window of 64 keys per wave after a wave sees
            // the count above thr: thr + 1024 <= T for T >= 8192);
            // mode 2: table from the row's bound min(n_prod, N), never full
            int64_t sz;
            if (L.mode == 1) {
                sz = L.off[row + 1] - L.off[row];
                T = pow2_at_least((uint64_t)(2 * sz > 8192 ? 2 * sz : 8192));
            } else {
                const int64_t np = L.nprod[row];
                sz = np < L.ncols ? np : L.ncols;
                T = pow2_at_least((uint64_t)(2 * sz > 64 ? 2 * sz : 64));
            }
            if ((int64_t)T > slab_entries) T = (uint32_t)slab_entries;
            if (L.mode == 1) thr = (T / 5) * 4 < T - 1024 ? (T / 5) * 4 : T - 1024;
        } else {
            base = crpt[row];
            n = crpt[row + 1] - base;
            T = pow2_at_least((uint64_t)(2 * n > 64 ? 2 * n : 64));
            if ((int64_t)T > slab_entries) T = (uint32_t)slab_entries;
        }
        for (uint32_t s = t; s < T; s += 1024) { tk[s] = -1; tv[s] = 0.0; }
        if (t == 0) { s_min = INT_MAX; s_max = -1; s_cnt = 0u; }
        __syncthreads();

        int kmin = INT_MAX, kmax = -1;
        auto ins = [&](bool ok, int key, V v) {
            if (ok) {
                kmin = key < kmin ? key : kmin;
                kmax = key > kmax ? key : kmax;
            }
            const int nw = num_insert_wave(tk, tv, T, ok, key, (double)v, &ctr->error,
                                           [](double *p, double x) { unsafeAtomicAdd(p, x); });
            if constexpr (LRN) {
                const unsigned nm = (unsigned)__popcll(__ballot(nw));
                if (nm && l == 0) atomicAdd(&s_cnt, nm);
            }
        };
        auto stop = [&]() -> bool {
            if constexpr (LRN) return *(volatile unsigned int *)&s_cnt > thr;
            else return false;
        };
        row_products<true, WIDE_D>(arpt[row], arpt[row + 1], acol, aval, brpt, bcol, bval, wv, 16, ins, stop);
        kmin = wave_min(kmin);
        kmax = wave_max(kmax);
        if (l == 0) {
            atomicMin(&s_min, kmin);
            atomicMax(&s_max, kmax);
        }
        __syncthreads();
        if constexpr (LRN) {
            n = (int64_t)s_cnt;
            if (t == 0) {
                int64_t b = -1;
                if (n > (int64_t)thr) {
                    lrn_retry(L, row, true);
                } else {
                    b = lrn_place(L, row, n);
                    if (b < 0) lrn_retry(L, row, false);
                    else lrn_done(L, row, n, b);
                }
                s_base = b;
            }
            __syncthreads();
            base = (int64_t)s_base;
            if (base < 0) continue;   // uniform; no barrier is pending
        }
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
// bin 7, rows with a known column range: bucketed dense accumulation.
// A long row's products are partitioned by BK_CW-column chunk of its output
// range into a per-workgroup staging buffer (a counting pass, a scan over
// the chunks, a scatter pass), then each chunk is accumulated densely in
// LDS (an FP64 add and an occupancy bit per product) and emitted in column
// order through a popcount prefix.  Global traffic is sequential (the
// staging writes and reads) instead of one random global atomic per product.
// The dense array and the bitmap are re-zeroed only where written.  Two
// workgroups share a CU, so that one's barriers and LDS round trips overlap
// the other's work.
// ---------------------------------------------------------------------------
constexpr int BK_T = 512;           // threads per workgroup (two workgroups per CU: one's
                                    // barriers and serial steps overlap the other's work)
constexpr int BK_NW = BK_T / 64;    // waves per workgroup
constexpr int BK_LG = 13;
constexpr int BK_CW = 1 << BK_LG;   // columns per chunk (a dense array of 64 KB)
constexpr int BK_NB = 2048;         // chunks per row at most
static_assert(BK_NB >= (int)(BUCKET_MAX_COLS >> BK_LG), "chunk counters");
static_assert(BK_NB % BK_T == 0, "chunk scan");
static_assert(BK_CW / 16 == BK_T, "one thread per 16 columns in the emission");
constexpr int BK_U = 4;             // staged products in flight per thread
constexpr int BK_ORD = 2048;        // ranks ordered per emission round

// Position of chunk column o in the dense array: the low four bits are XORed
// with the index of o's 16-column group, so that the threads of an emission
// step, each reading the lowest remaining column of its own group, spread
// over the LDS banks (randomly addressed accumulation does not care).
__device__ __forceinline__ uint32_t bk_swz(uint32_t o) { return o ^ ((o >> 4) & 15u); }

template <bool LRN, class V>
__global__ __launch_bounds__(BK_T) void k_num_bucket(
    RowSrc src, const int64_t *__restrict__ arpt, const int32_t *__restrict__ acol,
    const V *__restrict__ aval, const int64_t *__restrict__ brpt,
    const int32_t *__restrict__ bcol, const V *__restrict__ bval,
    const int64_t *__restrict__ crpt, int32_t *__restrict__ ccol, V *__restrict__ cval,
    const int2 *__restrict__ rng, unsigned short *stage_keys, V *stage_vals, int64_t stage_cap,
    Counters *__restrict__ ctr, Learn L) {
    // dense accumulator of one chunk; while the products are counted and
    // scattered (before any chunk is accumulated) its first BK_NB / 2 words
    // hold the chunk counters
    __shared__ double dense[BK_CW];   // sums in FP64 for either value type
    __shared__ unsigned int bits[BK_CW / 32];
    __shared__ unsigned int off[BK_NB + 1];
    __shared__ unsigned short ord[BK_ORD];   // chunk column of each rank in the current round
    __shared__ unsigned int red[BK_NW];
    __shared__ long long s_base;
    __shared__ long long s_r;

    src.resolve();
    const int t = threadIdx.x, wv = t >> 6, l = t & 63;
    unsigned int *cc = reinterpret_cast<unsigned int *>(dense);
    // a staged product is its column's offset in its chunk (2 bytes) and its value
    unsigned short *sk = stage_keys + (int64_t)blockIdx.x * stage_cap;
    V *sv = stage_vals + (int64_t)blockIdx.x * stage_cap;
    for (int i = t; i < BK_CW; i += BK_T) dense[i] = 0.0;
    for (int i = t; i < BK_CW / 32; i += BK_T) bits[i] = 0u;

    // rows from the launch's counter: row lengths here vary by orders of
    // magnitude, and a round-robin assignment leaves a few workgroups with
    // most of the work
    auto fetch = [&]() -> int64_t {
        __syncthreads();   // every thread is done with the previous s_r
        if (t == 0) s_r = (long long)take_row(ctr->sched, src.nrows);
        __syncthreads();
        return (int64_t)s_r;
    };
    for (int64_t r = fetch(); r < src.nrows; r = fetch()) {
        const int64_t row = src.row(r);
        const int64_t a0 = arpt[row], a1 = arpt[row + 1];
        const int2 rg = rng[row];
        int64_t base = 0, n = 0;
        if constexpr (!LRN) {
            base = crpt[row];
            n = crpt[row + 1] - base;
        }
        const int lo = rg.x;
        const int64_t span = (int64_t)rg.y - lo + 1;
        if (span <= 0) {   // no products (uniform; no barrier pending)
            if (LRN && t == 0) lrn_done(L, row, 0, L.off ? L.off[row] : 0);
            continue;
        }
        const int nb = (int)((span + BK_CW - 1) >> BK_LG);
        for (int i = t; i < nb; i += BK_T) cc[i] = 0u;
        __syncthreads();
        // Lanes of a window that hold consecutive products of one sorted B
        // row mostly fall in one chunk: runs of equal chunks in consecutive
        // lanes are found with one lane shuffle and a ballot, and the run's
        // first lane updates the chunk's counter for the whole run (the
        // same-address LDS atomics of many lanes are what serialise).
        auto runs = [&](bool in, int c, int &head_lane, int &run_len) {
            const int l = lane_id();
            const int cp = __builtin_amdgcn_ds_bpermute((l > 0 ? l - 1 : 0) << 2, c);
            const unsigned long long bnd = __ballot(l == 0 || cp != c);
            const unsigned long long le = l == 63 ? ~0ull : ((2ull << l) - 1ull);
            head_lane = 63 - __clzll((long long)(bnd & le));
            const unsigned long long after = bnd & ~le;
            const int next = after ? __ffsll((long long)after) - 1 : 64;
            run_len = in ? next - head_lane : 0;
        };
        // 1. products per chunk
        row_products<false, WIDE_D>(a0, a1, acol, (const V *)nullptr, brpt, bcol, (const V *)nullptr, wv, BK_NW,
                                  [&](bool ok, int key) {
                                      const uint32_t o = (uint32_t)(key - lo);
                                      const bool in = ok && o < (uint64_t)span;
                                      const int c = in ? (int)(o >> BK_LG) : -1;
                                      int h, n;
                                      runs(in, c, h, n);
                                      if (in && h == lane_id()) atomicAdd(&cc[c], (unsigned int)n);
                                  },
                                  [] { return false; });
        __syncthreads();
        // 2. chunk offsets (exclusive scan, BK_NB / BK_T consecutive chunks
        //    per thread)
        {
            constexpr int PT = BK_NB / BK_T;
            unsigned int x[PT], sum = 0;
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                const int q = t * PT + u;
                x[u] = q < nb ? cc[q] : 0u;
                sum += x[u];
            }
            const unsigned int incl = wave_incl_scan(sum);
            if (l == 63) red[wv] = incl;
            __syncthreads();
            unsigned int pre = 0, tot = 0;
            for (int i = 0; i < BK_NW; ++i) {
                if (i < wv) pre += red[i];
                tot += red[i];
            }
            pre += incl - sum;
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                const int q = t * PT + u;
                if (q < nb) {
                    off[q] = pre;
                    cc[q] = pre;   // running fill position of the chunk
                }
                pre += x[u];
            }
            if (t == 0) off[nb] = tot;
            __syncthreads();
        }
        // 3. scatter the products into their chunks; lanes of a wave that
        //    hit one chunk take consecutive positions (coalesced stores)
        //    (every lane stores: one without a product writes the
        //    workgroup's spare last entry, so that no branch sits around the
        //    stores, which count with the loads in flight)
        row_products<true, WIDE_D>(a0, a1, acol, aval, brpt, bcol, bval, wv, BK_NW,
                                   [&](bool ok, int key, V v) {
                                       const uint32_t o = (uint32_t)(key - lo);
                                       const bool in = ok && o < (uint64_t)span;
                                       const int c = in ? (int)(o >> BK_LG) : -1;
                                       int h, n;
                                       runs(in, c, h, n);
                                       const int l = lane_id();
                                       unsigned int b = 0u;
                                       if (in && h == l) b = atomicAdd(&cc[c], (unsigned int)n);
                                       b = (unsigned int)__builtin_amdgcn_ds_bpermute(h << 2, (int)b);
                                       const unsigned int p = in ? b + (unsigned int)(l - h)
                                                                 : (unsigned int)(stage_cap - 1);
                                       sk[p] = (unsigned short)(o & (BK_CW - 1));
                                       sv[p] = v;
                                   },
                                   [] { return false; });
        // once every wave has scattered, the counters lent by the dense array
        // are zeroed, and the staging writes of every wave are visible to the
        // reads below (plain loads, so that several are in flight per thread)
        __threadfence();
        __syncthreads();
        for (int i = t; i < BK_NB / 2; i += BK_T) dense[i] = 0.0;
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // One-phase step: the row goes to its slot while it fits.  Its size
        // is only counted (distinct columns of the chunks not yet emitted)
        // once the next chunk's products could overflow the slot; if the
        // exact size does not fit, the row moves to the arena (the entries
        // already emitted are copied there) or, when the arena is full, to
        // the recompute list.
        int64_t cap = n;
        bool known = !LRN;
        if constexpr (LRN) {   // no slots in the recompute pass: straight to the arena
            base = L.off ? L.off[row] : 0;
            cap = L.off ? L.off[row + 1] - base : 0;
        }
        // distinct columns of chunks [b0, nb) (bits is clear before and after)
        auto count_from = [&](int b0) -> int64_t {
            int64_t tot_n = 0;
            for (int b = b0; b < nb; ++b) {
                const unsigned int p0 = off[b], p1 = off[b + 1];
                if (p0 == p1) continue;   // uniform
                for (unsigned int p = p0 + t; p < p1; p += BK_T * BK_U) {
                    int ck[BK_U];
#pragma unroll
                    for (int u = 0; u < BK_U; ++u) {
                        const unsigned int q = p + (unsigned int)BK_T * u;
                        ck[u] = q < p1 ? (int)sk[q] : -1;
                    }
#pragma unroll
                    for (int u = 0; u < BK_U; ++u) {
                        if (ck[u] < 0) continue;
                        const uint32_t o = (uint32_t)ck[u];
                        atomicOr(&bits[o >> 5], 1u << (o & 31));
                    }
                }
                __syncthreads();
                unsigned int c = t < BK_CW / 32 ? __popc(bits[t]) : 0u;
                if (t < BK_CW / 32) bits[t] = 0u;
                c = wave_sum(c);
                if (l == 0) red[wv] = c;
                __syncthreads();
                for (int i = 0; i < BK_NW; ++i) tot_n += red[i];
                __syncthreads();
            }
            return tot_n;
        };
        // 4. per chunk: dense accumulation, then emission.  Thread t owns
        //    the 16 columns [16 t, 16 t + 16) of the chunk: a wave scan (DPP)
        //    and one exchange over the waves give its first rank, and it
        //    stores its columns in order.  The first staged products of the
        //    next nonempty chunk are loaded while the current chunk is
        //    emitted (chunks of long sparse rows hold a few hundred products:
        //    their load latency would dominate).
        int64_t run = 0;
        int kk[BK_U];
        V vv[BK_U];
        auto preload = [&](int bb) {
            const unsigned int q0 = off[bb], q1 = off[bb + 1];
#pragma unroll
            for (int u = 0; u < BK_U; ++u) {
                const unsigned int q = q0 + t + (unsigned int)BK_T * u;
                kk[u] = q < q1 ? (int)sk[q] : -1;
                vv[u] = q < q1 ? sv[q] : 0.0;
            }
        };
        const unsigned short *bits16 = reinterpret_cast<const unsigned short *>(bits);
        int b = 0;
        while (b < nb && off[b] == off[b + 1]) ++b;   // uniform
        if (b < nb) preload(b);
        bool dropped = false;
        while (b < nb) {
            const unsigned int p0 = off[b], p1 = off[b + 1];
            const int c0 = lo + (b << BK_LG);
            if constexpr (LRN) {
                if (!known && run + (int64_t)(p1 - p0) > cap) {   // uniform
                    const int64_t ex = run + count_from(b);
                    known = true;
                    if (ex > cap) {
                        if (t == 0) {
                            int64_t nb2 = -1;
                            const unsigned long long a =
                                atomicAdd(&L.lc->arena_used, (unsigned long long)ex);
                            if ((int64_t)a + ex <= L.arena_cap) {
                                atomicAdd(&L.lc->slot_overflow, 1u);
                                nb2 = L.arena_base + (int64_t)a;
                            } else {
                                lrn_retry(L, row, false);
                            }
                            s_base = nb2;
                        }
                        // the entries emitted so far are visible to every
                        // thread of the workgroup before they are moved
                        __threadfence();
                        __syncthreads();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        const int64_t nbase = (int64_t)s_base;
                        if (nbase < 0) {   // uniform
                            dropped = true;
                            break;
                        }
                        for (int64_t i = t; i < run; i += BK_T) {
                            ccol[nbase + i] = ld_coherent(&ccol[base + i]);
                            cval[nbase + i] = ld_coherent(&cval[base + i]);
                        }
                        base = nbase;
                    }
                    cap = ex;
                }
            }
            auto accumulate = [&]() {
#pragma unroll
                for (int u = 0; u < BK_U; ++u) {
                    if (kk[u] < 0) continue;
                    const uint32_t o = (uint32_t)kk[u];
                    atomicAdd(&dense[bk_swz(o)], (double)vv[u]);
                    atomicOr(&bits[o >> 5], 1u << (o & 31));
                }
            };
            accumulate();
            for (unsigned int p = p0 + (unsigned int)(BK_T * BK_U); p < p1; p += (unsigned int)(BK_T * BK_U)) {
#pragma unroll
                for (int u = 0; u < BK_U; ++u) {
                    const unsigned int q = p + t + (unsigned int)BK_T * u;
                    kk[u] = q < p1 ? (int)sk[q] : -1;
                    vv[u] = q < p1 ? sv[q] : 0.0;
                }
                accumulate();
            }
            __syncthreads();
            int bn = b + 1;
            while (bn < nb && off[bn] == off[bn + 1]) ++bn;   // uniform
            if (bn < nb) preload(bn);
            const unsigned int m0 = bits16[t];
            const int c = __popc(m0);
            const int incl = wave_incl_scan_dpp(c);
            if (l == 63) red[wv] = (unsigned int)incl;
            __syncthreads();
            unsigned int pre = 0, tot = 0;
#pragma unroll
            for (int i = 0; i < BK_NW; ++i) {
                const unsigned int r = red[i];
                pre += i < wv ? r : 0u;
                tot += r;
            }
            pre += (unsigned int)(incl - c);   // rank of thread t's first column
            // rounds of BK_ORD ranks: every thread writes the columns of its
            // ranks in the round into ord[], then the ranks are stored in order
            // (thread k takes ranks k, k + BK_T, ...: coalesced stores to C)
            for (unsigned int r0 = 0; r0 < tot; r0 += BK_ORD) {
                if (pre < r0 + BK_ORD && pre + (unsigned int)c > r0) {
                    unsigned int m = m0;
                    unsigned int k = pre;
                    while (m) {
                        const int bit = __ffs(m) - 1;
                        m &= m - 1u;
                        if (k >= r0 && k < r0 + BK_ORD) ord[k - r0] = (unsigned short)((t << 4) + bit);
                        ++k;
                    }
                }
                __syncthreads();
                const unsigned int cnt = tot - r0 < (unsigned int)BK_ORD ? tot - r0 : (unsigned int)BK_ORD;
                for (unsigned int k = t; k < cnt; k += BK_T) {
                    const uint32_t o = ord[k];
                    const uint32_t q = bk_swz(o);
                    const V v = (V)dense[q];
                    dense[q] = 0.0;
                    const int64_t kr = run + r0 + k;
                    if (kr < cap) {   // C is not read again here: keep it out of the caches
                        __builtin_nontemporal_store(c0 + (int)o, &ccol[base + kr]);
                        __builtin_nontemporal_store(v, &cval[base + kr]);
                    }
                }
                __syncthreads();
            }
            if (t < BK_CW / 32) bits[t] = 0u;
            run += tot;
            __syncthreads();
            b = bn;
        }
        if constexpr (LRN) {
            if (!dropped && t == 0) {
                if (run > cap) atomicAdd(&ctr->error, 1u);
                lrn_done(L, row, run, base);
            }
        } else {
            if (t == 0 && run != n) atomicAdd(&ctr->error, 1u);
        }
        __syncthreads();
    }
}

template <class V>
static hipError_t go_bucket(const NumArgs &a, hipStream_t s) {
    const VPtrs<V> v(a);
    if (a.lrn.mode > 0)
        hipLaunchKernelGGL((k_num_bucket<true, V>), dim3((unsigned)a.grid), dim3(BK_T), 0, s, a.src, a.A.rpt,
                           a.A.col, v.aval, a.B.rpt, a.B.col, v.bval, a.crpt, a.ccol, v.cval, a.rng,
                           (unsigned short *)a.slab_keys, v.slab_vals, a.slab_entries, a.ctr, a.lrn);
    else
        hipLaunchKernelGGL((k_num_bucket<false, V>), dim3((unsigned)a.grid), dim3(BK_T), 0, s, a.src, a.A.rpt,
                           a.A.col, v.aval, a.B.rpt, a.B.col, v.bval, a.crpt, a.ccol, v.cval, a.rng,
                           (unsigned short *)a.slab_keys, v.slab_vals, a.slab_entries, a.ctr, a.lrn);
    return hipGetLastError();
}

hipError_t launch_numeric_bucket(const NumArgs &a, hipStream_t s) {
    if (a.grid <= 0 || !a.rng) return hipSuccess;
    if (a.fp32 && a.lrn.mode > 0) return hipErrorInvalidValue;   // one-phase step: FP64 only
    return a.fp32 ? go_bucket<float>(a, s) : go_bucket<double>(a, s);
}

// ---------------------------------------------------------------------------
// One-phase step, last stage: copy every row from where the numeric step
// left it (its slot, the arena, or the second arena of recomputed rows) to
// its place in C.  Work is split by output entries, CH per wave: a wave finds
// the row holding its first entry with a 64-way search of C.rpt, then walks
// 64 rows at a time with their bounds and sources staged in LDS; every lane
// copies one entry per step, so reads and writes are coalesced within rows
// and writes are contiguous across them.
// ---------------------------------------------------------------------------
constexpr int COMPACT_CH = 4096;

__global__ __launch_bounds__(256) void k_compact(int64_t M, int64_t nnzC,
                                                 const int64_t *__restrict__ crpt,
                                                 const int64_t *__restrict__ loc,
                                                 const int32_t *__restrict__ tcol,
                                                 const double *__restrict__ tval, int64_t tsize,
                                                 const int32_t *__restrict__ acol2,
                                                 const double *__restrict__ aval2,
                                                 int32_t *__restrict__ ccol,
                                                 double *__restrict__ cval) {
    __shared__ int64_t s_rs[4][65];
    __shared__ int64_t s_src[4][64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t chunk = (int64_t)blockIdx.x * 4 + w;
    const int64_t e0 = chunk * COMPACT_CH;
    if (e0 >= nnzC) return;   // uniform per wave; no workgroup barrier follows
    const int64_t e1 = e0 + COMPACT_CH < nnzC ? e0 + COMPACT_CH : nnzC;
    // last row r with crpt[r] <= e0 (the row holding entry e0): 64-way search
    int64_t lo = 0, hi = M;   // crpt[lo] <= e0, and hi == M or crpt[hi] > e0
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t p = lo + (int64_t)l * step;
        const bool le = p < hi && crpt[p] <= e0;
        const int c = (int)__popcll(__ballot(le));   // >= 1: p = lo holds
        const int64_t nlo = lo + (int64_t)(c - 1) * step;
        const int64_t nhi = nlo + step < hi ? nlo + step : hi;
        lo = nlo;
        hi = nhi;
    }
    int64_t r = lo;
    int64_t pos = e0;
    while (pos < e1) {
        // stage rows r .. r+63: starts (65 bounds) and source indices
        const int64_t rr = r + l;
        s_rs[w][l] = crpt[rr < M ? rr : M];
        if (l == 0) s_rs[w][64] = crpt[r + 64 < M ? r + 64 : M];
        s_src[w][l] = rr < M ? loc[rr] : 0;
        wave_lds_sync();
        const int64_t wend_rows = s_rs[w][64];
        const int64_t stop = wend_rows < e1 ? wend_rows : e1;
        for (int64_t b = pos; b < stop; b += 64) {
            const int64_t e = b + l;
            if (e < stop) {
                // last staged row j with start <= e
                int j = 0;
#pragma unroll
                for (int h = 32; h > 0; h >>= 1)
                    if (s_rs[w][j + h] <= e) j += h;
                const int64_t src = s_src[w][j] + (e - s_rs[w][j]);
                int32_t cv;
                double vv;
                if (src < tsize) {
                    cv = tcol[src];
                    vv = tval[src];
                } else {
                    cv = acol2[src - tsize];
                    vv = aval2[src - tsize];
                }
                ccol[e] = cv;
                cval[e] = vv;
            }
        }
        pos = stop;
        r += 64;
        wave_lds_sync();   // every lane is done with the staged rows
    }
}

hipError_t launch_compact(int64_t M, int64_t nnzC, const int64_t *crpt, const int64_t *loc,
                          const int32_t *tcol, const double *tval, int64_t tsize,
                          const int32_t *acol2, const double *aval2, int32_t *ccol, double *cval,
                          hipStream_t s) {
    if (nnzC <= 0 || M <= 0) return hipSuccess;
    const int64_t chunks = (nnzC + COMPACT_CH - 1) / COMPACT_CH;
    const int64_t grid = (chunks + 3) / 4;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)grid), dim3(256), 0, s, M, nnzC, crpt, loc, tcol,
                       tval, tsize, acol2, aval2, ccol, cval);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
static int64_t grid_for(const NumArgs &a, int64_t per_wg) {
    if (a.grid > 0) return a.grid;
    return (a.src.nrows + per_wg - 1) / per_wg;
}

template <int W, int T, class V>
static hipError_t go_row_v(const NumArgs &a, hipStream_t s) {
    constexpr int R = (W == 64) ? 4 : 1;
    const int64_t grid = (a.src.nrows + R - 1) / R;   // one team per row
    if (grid <= 0) return hipSuccess;
    const VPtrs<V> v(a);
    if (a.lrn.mode == 1)
        hipLaunchKernelGGL((k_num_row<W, T, true, V>), dim3((unsigned)grid), dim3(W * R), 0, s, a.src,
                           a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval, a.crpt, a.ccol,
                           v.cval, a.ctr, a.lrn, a.rng, nullptr);
    else if (a.brec && a.lrn.mode == 0)
        hipLaunchKernelGGL((k_num_row<W, T, false, V, true>), dim3((unsigned)grid), dim3(W * R), 0, s,
                           a.src, a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval, a.crpt, a.ccol,
                           v.cval, a.ctr, a.lrn, a.rng, a.brec);
    else
        hipLaunchKernelGGL((k_num_row<W, T, false, V>), dim3((unsigned)grid), dim3(W * R), 0, s, a.src,
                           a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval, a.crpt, a.ccol,
                           v.cval, a.ctr, a.lrn, a.rng, nullptr);
    return hipGetLastError();
}

template <int W, int T>
static hipError_t go_row(const NumArgs &a, hipStream_t s) {
    return a.fp32 ? go_row_v<W, T, float>(a, s) : go_row_v<W, T, double>(a, s);
}

template <class V>
static hipError_t go_group(const NumArgs &a, hipStream_t s) {
    const int gv = a.lrn.mode == 1 ? 0 : a.gv;
    const int64_t grid = grid_for(a, 256 / GROUP_GL[gv]);
    if (grid <= 0) return hipSuccess;
    const VPtrs<V> v(a);
    if (a.lrn.mode == 1)
        hipLaunchKernelGGL((k_num_group<GROUP_GL[0], NUM_T0[0], true, V>), dim3((unsigned)grid),
                           dim3(256), 0, s, a.src, a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval,
                           a.crpt, a.ccol, v.cval, a.ctr, a.lrn);
    else if (gv == 1)
        hipLaunchKernelGGL((k_num_group<GROUP_GL[1], NUM_T0[1], false, V>), dim3((unsigned)grid),
                           dim3(256), 0, s, a.src, a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval,
                           a.crpt, a.ccol, v.cval, a.ctr, a.lrn);
    else if (gv == 2)
        hipLaunchKernelGGL((k_num_group<GROUP_GL[2], NUM_T0[2], false, V>), dim3((unsigned)grid),
                           dim3(256), 0, s, a.src, a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval,
                           a.crpt, a.ccol, v.cval, a.ctr, a.lrn);
    else
        hipLaunchKernelGGL((k_num_group<GROUP_GL[0], NUM_T0[0], false, V>), dim3((unsigned)grid),
                           dim3(256), 0, s, a.src, a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval,
                           a.crpt, a.ccol, v.cval, a.ctr, a.lrn);
    return hipGetLastError();
}

template <class V>
static hipError_t go_global(const NumArgs &a, hipStream_t s) {
    if (a.grid <= 0) return hipSuccess;
    const VPtrs<V> v(a);
    if (a.lrn.mode > 0)
        hipLaunchKernelGGL((k_num_global<true, V>), dim3((unsigned)a.grid), dim3(1024), 0, s, a.src,
                           a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval, a.crpt, a.ccol, v.cval,
                           a.slab_keys, (double *)a.slab_vals, a.slab_entries, a.ctr, a.lrn);
    else
        hipLaunchKernelGGL((k_num_global<false, V>), dim3((unsigned)a.grid), dim3(1024), 0, s, a.src,
                           a.A.rpt, a.A.col, v.aval, a.B.rpt, a.B.col, v.bval, a.crpt, a.ccol, v.cval,
                           a.slab_keys, (double *)a.slab_vals, a.slab_entries, a.ctr, a.lrn);
    return hipGetLastError();
}

hipError_t launch_numeric_bin(int bin, const NumArgs &a, hipStream_t s) {
    if (!a.src.dctr && !a.src.count && a.src.nrows == 0) return hipSuccess;
    if (a.fp32 && a.lrn.mode > 0) return hipErrorInvalidValue;   // one-phase step: FP64 only
    switch (bin) {
        case 0: return a.fp32 ? go_group<float>(a, s) : go_group<double>(a, s);
        case 1: return go_row<NUM_W[1], NUM_T[1]>(a, s);
        case 2: return go_row<NUM_W[2], NUM_T[2]>(a, s);
        case 3: return go_row<NUM_W[3], NUM_T[3]>(a, s);
        case 4: return go_row<NUM_W[4], NUM_T[4]>(a, s);
        case 5: return go_row<NUM_W[5], NUM_T[5]>(a, s);
        case 6: return go_row<NUM_W[6], NUM_T[6]>(a, s);
        case NUM_GLOBAL_BIN: return a.fp32 ? go_global<float>(a, s) : go_global<double>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace opsp
