// Device-side helpers shared by the opsp kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace opsp {

constexpr int WAVE = 64;

// Multiplicative (Fibonacci) hashing, Knuth TAOCP vol. 3 §6.4: the key is
// multiplied by floor(2^32 / golden ratio) and the high bits of the 32-bit
// product are range-reduced to [0, T) with a multiply-high (Lemire's
// fast range reduction), so any table size T works without a division.
// It plays the role of the paper's "key * HASH_SCALE mod t" (Section 5.2).
constexpr uint32_t HASH_MUL = 2654435769u;

__device__ __forceinline__ uint32_t hslot(int32_t key, uint32_t T) {
    return __umulhi((uint32_t)key * HASH_MUL, T);
}

__device__ __forceinline__ uint32_t next_slot(uint32_t s, uint32_t T) {
    ++s;
    return s == T ? 0u : s;
}

// Bin bounds of one binning step (Section 5.1): row value v goes to the
// first bin j < nb-1 with v <= ub[j], else to bin nb-1.  `force` >= 0 routes
// every row that fits bin `force` (v <= ub[force], or force >= nb-1) there.
struct Bounds {
    int32_t nb;       // natural bins
    int32_t force;    // -1 = off
    int32_t nslots;   // histogram slots (>= nb, > force)
    int32_t span_bin; // symbolic step: bin of rows routed by their column range (-1 = off)
    int64_t ub[16];
    int64_t span_max;        // ... whose output column range is at most this wide
    int64_t span_nprod_max;  // ... and whose n_prod is at most this
};

__device__ __forceinline__ int bin_of(int64_t v, const Bounds &b) {
    int j = 0;
    while (j < b.nb - 1 && v > b.ub[j]) ++j;
    if (b.force >= 0 && (b.force >= b.nb - 1 || v <= b.ub[b.force])) j = b.force;
    return j;
}

// Symbolic bin of a row from its n_prod and output column range: a row whose
// range is narrow enough for the one-wave kernel's bitmap is counted there
// whatever its n_prod (up to a cap), instead of in a table sized for n_prod
// distinct columns (rows of high compression ratio: thousands of products,
// a few hundred outputs).  No effect without ranges or with a forced bin.
__device__ __forceinline__ int bin_of_row(int64_t v, const Bounds &b, int2 rg) {
    int j = bin_of(v, b);
    if (b.span_bin >= 0 && b.force < 0 && j > b.span_bin && rg.y >= rg.x &&
        (int64_t)rg.y - rg.x + 1 <= b.span_max && v <= b.span_nprod_max)
        j = b.span_bin;
    return j;
}

// Device counters of one binning step (one per step, zeroed before use).
struct Counters {
    unsigned long long size[16];    // rows per bin
    unsigned long long fill[16];    // rows already placed per bin (pass 2)
    unsigned long long total;       // sum of row values (n_prod or nnz)
    unsigned long long maxv;        // largest row value
    unsigned int fail;              // rows abandoned by the LDS table (symbolic)
    unsigned int error;             // internal consistency failures
    unsigned long long sched[2];    // row counter, finished workgroups (take_row)
    unsigned long long dups;        // B rows that repeat the row before them (k_brange)
    unsigned long long pad[3];
};

// Counters of the one-phase (predicted-capacity) numeric step, zeroed
// before use.
struct LearnCtr {
    unsigned long long arena_used;   // entries taken from the overflow arena
    unsigned long long retry_ub;     // sum of min(n_prod, N) over rows to recompute
    unsigned long long nprod_total;  // sum of n_prod (capacity kernel)
    unsigned long long nprod_max;
    unsigned int retry;              // rows pushed to the recompute list
    unsigned int table_overflow;     // rows abandoned because their table filled up
    unsigned int slot_overflow;      // rows stored in the arena (slot too small)
    unsigned int error;
};

// Arguments of the one-phase numeric step (mode 0 = the exact two-phase
// step, which ignores them).  Mode 1: every row has a slot of its predicted
// capacity at off[row] in temporary arrays; a row that outgrows its slot is
// stored in the overflow arena, a row whose table fills up is abandoned to
// the recompute list.  Mode 2 (global-table kernel only): rows of the
// recompute list, tables sized from min(n_prod, N), stored in a second arena
// that holds their upper bounds.
struct Learn {
    int mode;
    int pad;
    const int64_t *off;       // slot offsets, off[M] = total (mode 1)
    const int64_t *nprod;     // n_prod per row
    int64_t *nnz;             // out: exact nnz per row
    int64_t *loc;             // out: index of the row's first entry
    int64_t loc_bias;         // added to the recorded index (second arena)
    int64_t ncols;            // N
    int64_t arena_base;       // first arena index in the written arrays
    int64_t arena_cap;        // arena capacity in entries
    LearnCtr *lc;
    int32_t *retry;           // recompute list (capacity M)
};

// Where a kernel finds the rows of its bin.  Host mode: `nrows` rows listed
// from position `off` of `bins` (rows off, off+1, ... when bins == NULL).
// Device mode (used by captured graphs, whose grids cannot depend on the
// data): with `dctr` the bin's size and start are read from the binning
// counters; with `count` the row count is read from device memory.  Kernels
// walk their rows with grid-stride loops, so any grid size is valid.
struct RowSrc {
    const int32_t *bins;
    int64_t off, nrows;
    const Counters *dctr;
    const unsigned int *count;
    int bin;
    // with dctr: the number of rows of the whole matrix (0 = unknown); a bin
    // that holds all of them is read in row order without the list (the
    // all-rows-in-one-bin case of Section 5.1, decided on the device)
    int64_t all;
    __device__ __forceinline__ void resolve() {
        if (dctr) {
            nrows = (int64_t)dctr->size[bin];
            int64_t o = 0;
            for (int j = 0; j < bin; ++j) o += (int64_t)dctr->size[j];
            off = o;
            if (all > 0 && nrows == all) {
                bins = nullptr;
                off = 0;
            }
        }
        if (count) nrows = (int64_t)*count;
    }
    __device__ __forceinline__ int64_t row(int64_t idx) const {
        return bins ? (int64_t)bins[off + idx] : off + idx;
    }
};

// Workgroups of a launch are dispatched round-robin over the 8 XCDs of the
// chip, each with its own L2.  This bijection on [0, n) gives XCD x the
// contiguous logical blocks [x q + min(x, r), ...) (q = n / 8, r = n % 8),
// so neighbouring rows, which read overlapping rows of B, share an L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t n) {
    const int64_t q = n / NUM_XCD, r = n % NUM_XCD;
    const int64_t x = bid % NUM_XCD, local = bid / NUM_XCD;
    return x * q + (x < r ? x : r) + local;
}

// Dynamic row assignment of a persistent launch (called by thread 0 of a
// workgroup): sched[0] hands out row indices, sched[1] counts workgroups
// that found no row left.  The last workgroup of the grid to finish resets
// both to zero, so that the next launch on the stream starts from zero; by
// then every other workgroup has left its loop.  Every workgroup of the
// grid must call this until it returns a value >= nrows.
__device__ __forceinline__ int64_t take_row(unsigned long long *sched, int64_t nrows) {
    const unsigned long long r = atomicAdd(&sched[0], 1ull);
    if ((int64_t)r >= nrows) {
        const unsigned long long d = atomicAdd(&sched[1], 1ull);
        if (d == (unsigned long long)gridDim.x - 1ull) {
            atomicExch(&sched[0], 0ull);
            atomicExch(&sched[1], 0ull);
        }
    }
    return (int64_t)r;
}

// Wave helpers ---------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ int mbcnt(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

// Inclusive prefix sum across the wave.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(v, o);
        if (l >= o) v += y;
    }
    return v;
}

// Inclusive prefix sum across the wave with DPP moves (no LDS round trips):
// shifts by 1, 2, 4, 8 lanes within each row of 16 lanes, then lane 15 of a
// row added into the next row and lane 31 into the upper half (row_bcast).
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// Synchronise the lanes of one wave through LDS: every LDS write issued
// before is visible to every lane of the wave after.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A "team" processes one row: one wave (WAVE_TEAM) or the whole workgroup.
template <bool WAVE_TEAM>
__device__ __forceinline__ void team_sync() {
    if constexpr (WAVE_TEAM) wave_lds_sync();
    else __syncthreads();
}

__device__ __forceinline__ uint32_t pow2_at_least(uint64_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Loads that bypass the per-CU vector cache: used to read global hash tables
// that were last written by device-scope atomics.
__device__ __forceinline__ int ld_coherent(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coherent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_coherent(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace opsp

namespace opsp {

__device__ __forceinline__ int64_t readlane64(int64_t v, int s) {
    const int lo = __builtin_amdgcn_readlane((int)(uint64_t)v, s);
    const int hi = __builtin_amdgcn_readlane((int)((uint64_t)v >> 32), s);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int s) {
    return __longlong_as_double(readlane64(__double_as_longlong(v), s));
}

__device__ __forceinline__ int bpermute(int v, int src_lane) {
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}

__device__ __forceinline__ int64_t bpermute64(int64_t v, int src_lane) {
    const int lo = bpermute((int)(uint64_t)v, src_lane);
    const int hi = bpermute((int)((uint64_t)v >> 32), src_lane);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Claim of hash slot *p for `key`; returns the slot's previous content: -1
// = the key was inserted here, `key` = it was already here, anything else =
// the slot holds another key (probe on).  The single-access form of Alg. 4
// and 5 is one compare-and-swap per probe, its returned value reused
// (Section 5.2).  Built with OPSP_HASH_MULTI_ACCESS=1 the slot is read first
// and swapped only when it reads empty: the multiple-access form that the
// paper's ablation compares with (Section 6.3.2); same result.  A slot
// changes once, from -1 to its key, so a stale read is harmless.
#ifndef OPSP_HASH_MULTI_ACCESS
#define OPSP_HASH_MULTI_ACCESS 0
#endif
template <class P>
__device__ __forceinline__ int hash_claim(P *p, int key) {
#if OPSP_HASH_MULTI_ACCESS
    const int cur = (int)*(volatile P *)p;
    if (cur == key) return key;
    if (cur != -1) return cur;
#endif
    return (int)atomicCAS(p, (P)-1, (P)key);
}

// Symbolic hashing: insert one key per lane (lanes with ok == false take part without a key).
// The probe loop is uniform over the wave and bounded by T iterations with a
// scalar counter; every probe is a single compare-and-swap (Alg. 4).
// Returns 1 when this lane's key was new.
template <class Tab>
__device__ __forceinline__ int sym_insert_wave(Tab *tab, uint32_t T, bool ok, int key,
                                               unsigned int *err) {
    bool pend = ok;
    int isnew = 0;
    uint32_t s = ok ? hslot(key, T) : 0u;
    for (uint32_t it = 0; __ballot(pend); ++it) {
        if (it >= T) {
            if (pend) atomicAdd(err, 1u);
            break;
        }
        if (pend) {
            const int old = hash_claim(&tab[s], key);
            const bool hit = (old == -1) | (old == key);
            isnew = old == -1;
            pend = !hit;
            s = hit ? s : next_slot(s, T);
        }
    }
    return isnew;
}

// Value of lane s (readlane) / of lane src_lane (bpermute) for the value
// types of the numeric step (FP64 as two 32-bit halves, FP32 as one).
__device__ __forceinline__ double readlane_v(double v, int s) { return readlane_f64(v, s); }
__device__ __forceinline__ float readlane_v(float v, int s) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), s));
}
__device__ __forceinline__ double bpermute_v(double v, int src_lane) {
    return __longlong_as_double(bpermute64(__double_as_longlong(v), src_lane));
}
__device__ __forceinline__ float bpermute_v(float v, int src_lane) {
    return __int_as_float(bpermute(__float_as_int(v), src_lane));
}

// Products of one window handed to the numeric step: a[0] * b[0], or, for an
// entry that leads a run of up to RUN entries whose B rows share one column
// set (see row_products), the sum of the run's products a[r] * b[r] at one
// column.  Each product is rounded to the value type and the sum is taken in
// FP64, as the tables add them.
template <class V, int RUN>
struct WinProd {
    V a[RUN], b[RUN];
    __device__ __forceinline__ auto value() const {
        if constexpr (RUN == 1) {
            return a[0] * b[0];
        } else {
            double s = (double)(V)(a[0] * b[0]);
#pragma unroll
            for (int r = 1; r < RUN; ++r) s += (double)(V)(a[r] * b[r]);
            return s;
        }
    }
};

// Longest run of entries with one B-row pattern that the numeric step merges
// (3 unknowns per node in 3-D elasticity).
constexpr int NUM_RUN = 3;

// Enumeration of the intermediate products of one row of C = A*B
// (Eq. 2: C_i* = sum over k in A_i* of A_ik * B_k*), spread over `nwaves`
// waves of which the caller is wave `wv`.
//
// A's row is taken in chunks of 64 entries; every wave loads the chunk (lane j
// holds entry j's B-row start, length and value a_j).  Each chunk is then
// walked in 64-lane windows in one of two ways, whichever issues fewer
// instructions for that chunk:
//  * grouped: when every referenced B row has at most G <= 64 entries, a
//    window gives 64/G consecutive entries a group of G lanes each; lane
//    (g, r) handles entry e0+g, position r.  The entry's start, length and
//    value arrive with one ds_bpermute per 32-bit field.
//  * flat: lanes take 64 consecutive products of the chunk; a lane finds its
//    entry by walking (with scalar readlanes) the entries that start inside
//    the window, after taking the entry that covers the window's first
//    product.  Used for long or irregular B rows.
// Windows go round-robin to the waves.  B loads of the next D windows are
// issued before the current window's products are handed to `f(ok, key, a * b)`
// (`f(ok, key)` for the symbolic step); every lane calls f once per window,
// `ok` says whether it holds a product.  `stop()` is polled once per window
// and ends the enumeration for the whole wave.
// Repeated B-row patterns (`dup`: B's row records, .w = 1 when a row has the
// same columns as the row before it; blocks of unknowns per node in finite
// elements): when A holds k - 1 and k and B row k repeats row k - 1, entry k
// adds no column of its own.  The symbolic step skips such an entry.  The
// numeric step with RUN > 1 gives a run of up to RUN such entries (within a
// chunk) to the run's first entry, which walks its B row once and hands f
// the run's summed products (WinProd) per column: one table update where
// there were up to RUN.  The rows of a run are consecutive in B with one
// length L, so product r of position p sits at p + r*L.
template <bool NUMERIC, int D = 1, class V = double, int RUN = 1, class F, class Stop>
__device__ __forceinline__ void row_products(int64_t a0, int64_t a1, const int32_t *__restrict__ acol,
                                             const V *__restrict__ aval,
                                             const int64_t *__restrict__ brpt,
                                             const int32_t *__restrict__ bcol,
                                             const V *__restrict__ bval, int wv_in, int nwaves,
                                             F &&f, Stop &&stop, const int4 *__restrict__ dup = nullptr) {
    static_assert(RUN == 1 || NUMERIC, "runs are merged by the numeric step only");
    using P = WinProd<V, RUN>;
    const int l = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(wv_in);   // wave-uniform: window indices in SGPRs
    int k_last = -2;   // symbolic with dup: the previous chunk's last B row
    for (int64_t c0 = a0; c0 < a1; c0 += 64) {
        const int64_t j = c0 + l;
        const bool v = j < a1;
        int k = 0;
        V av = 0;
        if (v) {
            k = acol[j];
            if constexpr (NUMERIC) av = aval[j];
        }
        const int64_t b0 = v ? brpt[k] : 0;
        int len = v ? (int)(brpt[k + 1] - b0) : 0;
        // run of the entry (RUN > 1): ar[r] the value of its r-th entry and
        // rn the entries in the run (lanes that are not a run's first: 0)
        V ar[RUN];
        ar[0] = av;
        int rn = 1;
        if constexpr (!NUMERIC) {
            if (dup) {   // uniform: the previous entry from the next lane down
                int kp = __shfl_up(k, 1);
                if (l == 0) kp = k_last;
                k_last = __builtin_amdgcn_readlane(k, 63);   // lanes past the end are not read again
                if (v && k > 0 && kp == k - 1 && dup[k].w) len = 0;
            }
        } else if constexpr (RUN > 1) {
#pragma unroll
            for (int r = 1; r < RUN; ++r) ar[r] = 0;
            if (dup) {   // uniform
                const int kp = __shfl_up(k, 1);
                const bool fol = v && l > 0 && k > 0 && kp == k - 1 && dup[k].w;
                const unsigned long long fm = __ballot(fol);
                const unsigned long long upto = (2ull << l) - 1;   // lanes 0..l
                // lane 0 never follows: the run's first lane is the highest
                // lane at or below l that does not follow
                const int top = 63 - __clzll((long long)(~fm & upto));
                const bool lead = !fol || (l - top) % RUN == 0;
                const unsigned long long nxt = __ballot(lead) & ~upto;
                rn = lead ? (nxt ? __ffsll((long long)nxt) - 1 - l : 64 - l) : 0;
#pragma unroll
                for (int r = 1; r < RUN; ++r) {
                    const V x = bpermute_v(av, l + r < 64 ? l + r : 63);
                    ar[r] = r < rn ? x : V(0);
                }
                if (!lead) len = 0;
            }
        }
        const int nent = (int)(a1 - c0 < 64 ? a1 - c0 : 64);
        const int lmax = wave_max(len);
        const int64_t total = (int64_t)wave_sum((long long)len);
        if (total == 0) continue;
        int lg = 0;
        while ((1 << lg) < lmax) ++lg;
        const int per = 64 >> lg;                         // entries per window
        const int64_t win_grouped = (nent + per - 1) / per;
        const int64_t win_flat = (total + 63) / 64;
        // a flat window costs about twice a grouped one (entry walk)
        const bool grouped = lg <= 6 && win_grouped <= 2 * win_flat;
        // loads of the run's further products (RUN > 1): position ix of the
        // first row, rows of length el, crn entries in the run
        auto load_run = [&](P &pv, bool ok, int64_t ix, int el, int crn) {
#pragma unroll
            for (int r = 1; r < RUN; ++r) {
                const bool okr = ok && r < crn;
                const V bw = bval[okr ? ix + (int64_t)r * el : 0];
                pv.b[r] = okr ? bw : V(0);
            }
        };
        // windows wv, wv + nwaves, ... of nwin with D + 1 windows of loads in
        // flight: slot d is consumed, then refilled with the window D + 1
        // places ahead.  Windows past the last hold no products (every lane
        // has ok false) and are fetched and consumed like the others, so the
        // loop body has no branch around its loads.  Returns true when
        // stop() ended the row.
        auto pipelined = [&](int64_t nwin, auto &&fetchw) -> bool {
            constexpr int S = D + 1;
            int key[S];
            P pv[S];
            bool ok[S];
#pragma unroll
            for (int d = 0; d < S; ++d) fetchw(wv + (int64_t)nwaves * d, key[d], pv[d], ok[d]);
            for (int64_t w = wv; w < nwin; w += (int64_t)nwaves * S) {
#pragma unroll
                for (int d = 0; d < S; ++d) {
                    if constexpr (NUMERIC) f(ok[d], key[d], pv[d].value());
                    else f(ok[d], key[d]);
                    if (stop()) return true;
                    fetchw(w + (int64_t)nwaves * (d + S), key[d], pv[d], ok[d]);
                }
            }
            return false;
        };
        // one window at a time, the next one's loads issued before the
        // current one is consumed
        auto paired = [&](int64_t w, int64_t step, int64_t end, auto &&fetchw) {
            int key, key1;
            P pv, pv1;
            bool ok, ok1;
            fetchw(w, key, pv, ok);
            while (true) {
                const int64_t wn = w + step;
                const bool more = wn < end;
                fetchw(wn, key1, pv1, ok1);   // past the last window: no products
                if constexpr (NUMERIC) f(ok, key, pv.value());
                else f(ok, key);
                if (!more || stop()) break;
                w = wn;
                key = key1;
                pv = pv1;
                ok = ok1;
            }
        };

        if (grouped) {
            const int g = l >> lg, r = l & ((1 << lg) - 1);
            auto fetch = [&](int64_t w, int &key, P &pv, bool &ok) {
                const int e = (int)w * per + g;
                const int src = e < 64 ? e : 63;
                const int64_t eb0 = bpermute64(b0, src);
                const int elen = bpermute(len, src);
                if constexpr (NUMERIC) {
#pragma unroll
                    for (int q = 0; q < RUN; ++q) pv.a[q] = bpermute_v(ar[q], src);
                }
                ok = e < nent && r < elen;
                // every lane loads (index 0 when it holds no product): no
                // divergent branch around the loads, so that the wait before
                // a window's use leaves the next windows' loads in flight
                const int64_t ix = ok ? eb0 + r : 0;
                const int kv = bcol[ix];
                key = ok ? kv : -1;
                if constexpr (NUMERIC) {
                    const V bw = bval[ix];
                    pv.b[0] = ok ? bw : V(0);
                    if constexpr (RUN > 1) load_run(pv, ok, ix, elen, bpermute(rn, src));
                }
            };
            if (wv >= win_grouped) continue;
            if constexpr (D > 1) {
                if (pipelined(win_grouped, fetch)) break;
                continue;
            }
            paired(wv, nwaves, win_grouped, fetch);
        } else {
            const int64_t incl = wave_incl_scan((int64_t)len);
            const int64_t off = incl - len;
            const int64_t base = b0 - off;
            const bool starts = len > 0;
            auto fetch = [&](int64_t w0, int &key, P &pv, bool &ok) {
                const unsigned long long cov = __ballot(starts && off <= w0);
                int s = 63 - __clzll((long long)cov);
                int64_t cb = readlane64(base, s);
                int cl = 0, crn = 1;   // RUN > 1: the entry's row length and run
                auto take = [&](int src) {
                    if constexpr (NUMERIC) {
#pragma unroll
                        for (int q = 0; q < RUN; ++q) pv.a[q] = readlane_v(ar[q], src);
                    }
                    if constexpr (RUN > 1) {
                        cl = __builtin_amdgcn_readlane(len, src);
                        crn = __builtin_amdgcn_readlane(rn, src);
                    }
                };
                take(s);
                unsigned long long in = __ballot(starts && off > w0 && off < w0 + 64);
                const int64_t p = w0 + l;
                while (in) {
                    s = __ffsll((long long)in) - 1;
                    in &= in - 1;
                    const int64_t os = readlane64(off, s);
                    if (p >= os) {
                        cb = readlane64(base, s);
                        take(s);
                    }
                }
                ok = p < total;
                const int64_t ix = ok ? cb + p : 0;
                const int kv = bcol[ix];
                key = ok ? kv : -1;
                if constexpr (NUMERIC) {
                    const V bw = bval[ix];
                    pv.b[0] = ok ? bw : V(0);
                    if constexpr (RUN > 1) load_run(pv, ok, ix, cl, crn);
                }
            };
            const int64_t stride = (int64_t)nwaves * 64;
            const int64_t w0 = (int64_t)wv * 64;
            if (w0 >= total) continue;
            if constexpr (D > 1) {
                auto fetch_w = [&](int64_t w, int &key, P &pv, bool &ok) {
                    fetch(w * 64, key, pv, ok);
                };
                if (pipelined(win_flat, fetch_w)) break;
                continue;
            }
            paired(w0, stride, total, fetch);
        }
        if (stop()) break;
    }
}

}  // namespace opsp
