// Host-side declarations of the kernel launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "opsp_dev.h"
#include "opsp_tables.h"

namespace opsp {

inline int64_t pow2_host(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Device-memory cache (opsp_alloc.hip): stream-ordered reuse of blocks
// without HIP calls on the hot path.
hipError_t cache_alloc(void **out, size_t bytes, hipStream_t s);
hipError_t cache_free(void *p, hipStream_t s);

struct DevCSR {
    int64_t rows, cols;
    const int64_t *rpt;
    const int32_t *col;
    const void *val;         // double, or float for the FP32 product
};

// ---- binning / setup / scan (kernels_bin.hip) -----------------------------
// Histogram slots per 256-row block (>= the bins of either step).
constexpr int BIN_SLOTS = 16;

// Rows of more than SETUP_TILE entries of A are walked by the setup step in
// tiles of SETUP_TILE entries, one wave per tile, instead of by the wave
// that owns them (R-MAT's heaviest rows are adjacent: one wave's 64 rows can
// hold a quarter of a million entries).
constexpr int SETUP_TILE = 512;
struct LongHead { unsigned long long packed; unsigned long long pad; };   // rows << 32 | tiles
struct LongRow { int32_t row, ntiles, it0, pad; };                       // row < 0: unused slot
struct LongPart { unsigned long long sum; uint32_t bmax; int32_t lo, hi, pad; };

// Per-block records of the first binning pass (256 rows per block), and the
// setup step's list of long rows and their tiles.
struct BlockParts {
    unsigned int *hist;          // [nblk][BIN_SLOTS] rows per bin; exclusive over blocks after finalize
    unsigned long long *tot;     // [nblk] sum of row values; exclusive scan after a scanning finalize
    unsigned long long *mx;      // [nblk] max row value
    LongHead *lh;                // counts of lrows / litems (setup step only)
    LongRow *lrows;              // [cap_rows]
    int2 *litems;                // [cap_items] (slot in lrows or -1, tile of the row)
    LongPart *lpart;             // [cap_items] per-tile sums
    uint32_t cap_rows, cap_items;
};

// Bytes of the records of M rows whose A holds nnzA entries (the long-row
// list is sized so that any A whose rows span at most nnzA entries fits:
// at most nnzA / SETUP_TILE rows and 2 nnzA / SETUP_TILE + 1 tiles).
inline void block_parts_caps(int64_t nnzA, uint32_t *cr, uint32_t *ci) {
    const int64_t r = nnzA / SETUP_TILE + 1, t = 2 * r;
    const int64_t lim = (int64_t)1 << 30;
    *cr = (uint32_t)(r < lim ? r : lim);
    *ci = (uint32_t)(t < lim ? t : lim);
}
inline size_t block_parts_bytes(int64_t M, int64_t nnzA) {
    const int64_t nblk = M > 0 ? (M + 255) / 256 : 1;
    uint32_t cr, ci;
    block_parts_caps(nnzA, &cr, &ci);
    size_t b = (sizeof(unsigned int) * BIN_SLOTS + 2 * sizeof(unsigned long long)) * (size_t)nblk;
    b = (b + 15) & ~(size_t)15;
    return b + sizeof(LongHead) + sizeof(LongRow) * cr + (sizeof(int2) + sizeof(LongPart)) * ci;
}
inline BlockParts block_parts_at(void *p, int64_t M, int64_t nnzA) {
    const int64_t nblk = M > 0 ? (M + 255) / 256 : 1;
    BlockParts q;
    q.tot = (unsigned long long *)p;
    q.mx = q.tot + nblk;
    q.hist = (unsigned int *)(q.mx + nblk);
    size_t b = (sizeof(unsigned int) * BIN_SLOTS + 2 * sizeof(unsigned long long)) * (size_t)nblk;
    b = (b + 15) & ~(size_t)15;
    block_parts_caps(nnzA, &q.cap_rows, &q.cap_items);
    q.lh = (LongHead *)((char *)p + b);
    q.lrows = (LongRow *)((char *)p + b + sizeof(LongHead));
    q.lpart = (LongPart *)(q.lrows + q.cap_rows);
    q.litems = (int2 *)(q.lpart + q.cap_items);
    return q;
}

// Length, first and last column of every row of B (0, INT_MAX, -1 for
// empty rows) as int4 records; .w = 1 when the row has the same columns as
// the row before it (compared for rows of at most 256 entries).
// With `dup`, the fourth field flags a row that repeats the row before it,
// and `ndup` (optional; zeroed first) receives the number of flagged rows.
hipError_t launch_brange(const DevCSR &B, int4 *brec, bool dup, unsigned long long *ndup,
                         hipStream_t s);
// Rows of A with the columns of the row before them: arun[i] = distance of
// row i to the first row of its run (0: counted itself); runs are cut at
// multiples of ARUN_CAP rows.  `brec` (B's records with repeated-pattern
// flags) stands in for the row compare when A and B are one matrix; else
// `same` (M bytes) holds the compare.  launch_arun_copy gives each row the
// symbolic count of its run's first row.
constexpr int ARUN_CAP = 32;
hipError_t launch_arun(const DevCSR &A, const int4 *brec, uint8_t *same, uint8_t *arun,
                       hipStream_t s);
hipError_t launch_arun_copy(int64_t M, const uint8_t *arun, int64_t *nnz, hipStream_t s);
// Setup step fused with the first binning pass: n_prod per row into `nprod`,
// per-block bin counts / totals / maxima into `parts` (which must come from
// block_parts_at with A's nnz); optional features
// (a_len, b_max) and, given B's row records `brec`, the column range
// (lo, hi) of each row's output (the smallest first and largest last column
// of the B rows it references; INT_MAX / -1 for rows without products).
hipError_t launch_setup(const DevCSR &A, const DevCSR &B, int64_t *nprod, const Bounds &bd,
                        const BlockParts &parts, int32_t *f_alen, int32_t *f_bmax, hipStream_t s,
                        const int4 *brec = nullptr, int2 *rng = nullptr);
// First binning pass over existing row values (numeric step).
hipError_t launch_hist(int64_t M, const int64_t *v, const Bounds &bd, const BlockParts &parts,
                       hipStream_t s);
// Reduce the block records into bin sizes, total and max (ctr); scan the
// per-block bin counts; with `scan`, also scan the block totals and write the
// grand total to *total_out.
hipError_t launch_finalize(int64_t M, int nslots, const BlockParts &parts, Counters *ctr,
                           int64_t *total_out, bool scan, hipStream_t s);
// Second binning pass: scatter row ids into `bins` (may be NULL when no
// bins are needed); with `scan`, also write the exclusive offsets of v[] to
// vout[] (NULL = in place).  With `device_identity` (no scan), nothing is
// written when one bin holds every row: readers given RowSrc::all take the
// rows in order then.  `rng` (symbolic step, no scan): the rows' output
// column ranges, for the range rule of bin_of_row (the setup kernel must
// have binned with the same ranges).
hipError_t launch_scatter(int64_t M, int64_t *v, const Bounds &bd, const Counters *ctr,
                          int32_t *bins, const BlockParts &parts, bool scan, hipStream_t s,
                          int64_t *vout = nullptr, bool device_identity = false,
                          const int2 *rng = nullptr);

// ---- input check of the validation mode (kernels_check.hip) ----------------
// Sets bits of *flags (zeroed before): 1 = rpt not monotone, rpt[0] < 0 or
// rpt[rows] - rpt[0] != nnz; 2 = a column index outside [0, cols); 4 =
// columns not strictly ascending in a row.  col is read only when bit 1
// stays clear.
hipError_t launch_check_csr(int64_t rows, int64_t cols, int64_t nnz, const int64_t *rpt,
                            const int32_t *col, unsigned int *flags, hipStream_t s);

// ---- symbolic step (kernels_sym.hip) ---------------------------------------
struct SymArgs {
    DevCSR A, B;
    int64_t *nnz;            // in: n_prod per row (C.rpt); out: distinct columns per row
    RowSrc src;              // rows of the bin
    int abort_thr;           // bin 7: abandon a row above this many keys
    Counters *ctr;           // fail / error counters
    int32_t *fail_list;      // abandoned rows (bin 7)
    int *slab;               // global tables (bin 8)
    int64_t slab_entries;
    int64_t grid;            // fixed grid (persistent launch); 0 = one team per row
    const int2 *rng;         // optional column range of each row (setup step): rows
                             // with a narrow range are counted with a bitmap
    unsigned long long *sched;  // bin 8: Counters::sched of the launch, zero on entry
                                // (null: rows assigned round-robin)
    int gv;                  // bin 0 variant (GROUP_GL / SYM_T0)
    const int4 *brec;        // optional B row records (launch_brange): rows that
                             // repeat the previous entry's column set are skipped
    const uint8_t *arun;     // optional (launch_arun): rows of A counted by the
                             // first row of their run are skipped (bins 1-7)
};
// Average B row length from which the symbolic step looks for repeated
// row patterns.
constexpr int64_t DUP_MIN_AVG = 48;
hipError_t launch_symbolic_bin(int bin, const SymArgs &a, hipStream_t s);
// Workgroups per CU of a symbolic bin kernel launched persistently (its rows
// counted on the device): several times what one CU holds, so that the
// hardware hands a freed slot to a waiting workgroup (dynamic balance over
// rows of uneven cost) while each workgroup still strides over many rows;
// workgroups that find no row left exit at once.  Measured on one MI355X
// against full residency only: the 27-point stencil's one-wave bin 1.33 ->
// 1.16 ms, the block stencil's symbolic step 3.27 -> 2.77 ms, R-MAT 2^20
// 49.3 -> 46.7 ms.
inline int sym_wg_per_cu(int bin) {
    switch (bin) {
        case 0: return 64;           // 256-lane workgroups, 8 resident
        case 1: return 128;          // 256 lanes (4 one-wave rows), 8 resident
        case 2: return 64;           // 128 lanes, 16 resident
        case 3: return 32;
        case 4: return 16;
        case 5: case 6: return 8;
        default: return 4;           // bin 7: 160 KB of LDS, 1 resident
    }
}
// Rows one workgroup of a symbolic bin kernel takes at a time.
inline int sym_rows_per_wg(int bin, int gv = 0) {
    return bin == 0 ? 256 / GROUP_GL[gv] : (bin == 1 ? 4 : 1);
}

// ---- numeric step (kernels_num.hip) ----------------------------------------
struct NumArgs {
    DevCSR A, B;
    const int64_t *crpt;     // C row pointer (exclusive offsets, crpt[M] = nnz)
    int32_t *ccol;
    void *cval;              // double, or float when fp32
    RowSrc src;              // rows of the bin
    Counters *ctr;           // error counter
    int *slab_keys;          // global tables (bin 7)
    void *slab_vals;         // value type of the product
    int64_t slab_entries;
    int64_t grid;
    Learn lrn;               // one-phase step (lrn.mode > 0); crpt unused then
    const int2 *rng;         // optional column range of each row (setup step): rows
                             // with a narrow range accumulate densely (bins 1-6)
    int gv;                  // bin 0 variant (GROUP_GL / NUM_T0); the one-phase
                             // step uses variant 0
    int fp32;                // values are float (A, B, C and the tables); two-phase only
    const int4 *brec;        // optional B row records with repeated-pattern flags
                             // (launch_brange with dup): bins 1-6 merge runs of
                             // entries whose B rows share one column set
};
hipError_t launch_numeric_bin(int bin, const NumArgs &a, hipStream_t s);
// Bin 7 by bucketed dense accumulation (rows with a column range in `rng`;
// the matrix must have at most BUCKET_MAX_COLS columns).  slab_keys /
// slab_vals / slab_entries are the staging buffers, one per workgroup of
// the grid: slab_entries >= the largest n_prod of the bin's rows + 1 (the
// last entry takes the stores of lanes without a product).
constexpr int64_t BUCKET_MAX_COLS = (int64_t)1 << 24;
constexpr int BUCKET_WG_PER_CU = 2;   // workgroups of the bucketed kernel per CU
hipError_t launch_numeric_bucket(const NumArgs &a, hipStream_t s);

// Copy the rows of the one-phase step from the temporary arrays (entries
// [0, tsize)) and the second arena (indices tsize.. in `loc`) into C.
hipError_t launch_compact(int64_t M, int64_t nnzC, const int64_t *crpt, const int64_t *loc,
                          const int32_t *tcol, const double *tval, int64_t tsize,
                          const int32_t *acol2, const double *aval2, int32_t *ccol, double *cval,
                          hipStream_t s);

// ---- predictor (kernels_mlp.hip) -------------------------------------------
constexpr int MLP_NPARAM = 4481;
// log2(1 + v) features of every row from the integer features.
hipError_t launch_mlp_features(int64_t M, const int32_t *alen, const int64_t *nprod,
                               const int32_t *bmax, float *X, hipStream_t s);
hipError_t launch_mlp_forward(const uint16_t *P, const float *X, int64_t n, float *y, hipStream_t s);
// Gradient of the mean squared error (tau == 0) or of the mean pinball
// loss of level tau over n rows; `part` holds ceil(n / 64) * (MLP_NPARAM + 1)
// floats.
hipError_t launch_mlp_grad(const uint16_t *P, const float *X, const float *T, int64_t n, float tau,
                           float *part, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *master, float *m, float *v, const float *g, float lr, float b1,
                           float b2, float eps, float c1, float c2, uint16_t *P, hipStream_t s);
// Capacities of every row (predictor kind 0 = network, 1 = min(n_prod, N),
// 2 = n_prod / ratio) into cap[0..M), with per-block numeric-bin records and
// the n_prod total and maximum in lc.
struct CapArgs {
    int kind;
    int pad;
    const uint16_t *P;
    double margin, ratio, scale;
    int64_t ncols;
    float *pred;             // optional: the network's outputs (written)
    const float *pred_in;    // network outputs computed before (NULL = run it here)
    const double *calib;     // calibration sums [3][CAL_OCT] (launch_cal_sum), or NULL
    const unsigned long long *calmax;   // largest ratio per octave, double bits
};
hipError_t launch_mlp_caps(int64_t M, const CapArgs &ca, const int32_t *alen, const int64_t *nprod,
                           const int32_t *bmax, int64_t *cap, const Bounds &bd,
                           const BlockParts &parts, LearnCtr *lc, hipStream_t s);
// Network outputs for every row from the integer features.
hipError_t launch_mlp_pred(int64_t M, const uint16_t *P, const int32_t *alen, const int64_t *nprod,
                           const int32_t *bmax, float *pred, hipStream_t s);
// Calibration sample of the predicted sizes.  Eligible rows have a_len >= 2,
// 1 <= n_prod < 2^(CAL_MAX_OCT + 1) and a column range of at most
// CAL_SPAN_MAX columns (so that the bin-8 bitmap kernel counts them); they
// are grouped by the octave o = floor(log2 n_prod).  launch_cal_hist adds
// the number of eligible rows of each octave into hist[CAL_OCT];
// launch_cal_pick turns an octave's count c into its quota
// quota[o] = K = min(c, clamp(CAL_OCT_PRODUCTS >> o, CAL_MIN_ROWS, per_octave))
// and appends the eligible rows with u(i) * c < K * 2^32 to `list` (u: the
// high half of MurmurHash3's fmix64 of the row index, so each row is picked
// with probability K / c); after the picked rows are counted exactly into exact[row],
// launch_cal_sum adds, per octave, their sizes into calib[o], their estimates
// 2^pred - 1 clamped to [min(b_max, U), U] into calib[CAL_OCT + o] and 1 into
// calib[2 CAL_OCT + o], and keeps the largest size / estimate in calmax[o]
// (bit pattern of the double; both zeroed before).  The capacity kernel
// scales the rows of an octave with at least CAL_MIN_ROWS counted rows by
// calmax[o]; other rows are not scaled.
constexpr int CAL_OCT = 64;
constexpr int64_t CAL_SPAN_MAX = (int64_t)SW_MAXPASS << SW_LG;
constexpr int64_t CAL_OCT_PRODUCTS = (int64_t)1 << 24;
constexpr int CAL_MIN_ROWS = 4;
constexpr int CAL_MAX_OCT = 20;
hipError_t launch_cal_hist(int64_t M, const int32_t *alen, const int64_t *nprod, const int2 *rng,
                           unsigned long long *hist, hipStream_t s);
hipError_t launch_cal_pick(int64_t M, const int32_t *alen, const int64_t *nprod, const int2 *rng,
                           const unsigned long long *hist, int64_t per_octave,
                           unsigned long long *quota, int32_t *list, unsigned int *count,
                           hipStream_t s);
hipError_t launch_cal_sum(const int32_t *list, const unsigned int *count, const int64_t *nprod,
                          const int32_t *bmax, const float *pred, const int64_t *exact, int64_t ncols,
                          double *calib, unsigned long long *calmax, hipStream_t s);

}  // namespace opsp
