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

struct DevCSR {
    int64_t rows, cols;
    const int64_t *rpt;
    const int32_t *col;
    const double *val;
};

// ---- binning / setup / scan (kernels_bin.hip) -----------------------------
// Setup step fused with the first binning pass: n_prod per row into `nprod`,
// per-bin row counts, total and max into `ctr`; optional per-row features.
hipError_t launch_setup(const DevCSR &A, const DevCSR &B, int64_t *nprod, const Bounds &bd,
                        Counters *ctr, int32_t *f_alen, int32_t *f_bmax, hipStream_t s);
// First binning pass over existing row values (numeric step): counts, total,
// max and per-256-row block sums (for the scan).
hipError_t launch_hist(int64_t M, const int64_t *v, const Bounds &bd, Counters *ctr,
                       unsigned long long *blocksum, hipStream_t s);
// Exclusive scan of the block sums; writes the grand total to *total_out.
hipError_t launch_scan_blocks(int64_t nblk, unsigned long long *blocksum, int64_t *total_out,
                              hipStream_t s);
// Second binning pass: scatter row ids into `bins` (may be NULL when no
// bins are needed); with `scan`, also turn v[] into exclusive offsets.
hipError_t launch_scatter(int64_t M, int64_t *v, const Bounds &bd, Counters *ctr, int32_t *bins,
                          const unsigned long long *blockbase, bool scan, hipStream_t s);

// ---- symbolic step (kernels_sym.hip) ---------------------------------------
struct SymArgs {
    DevCSR A, B;
    int64_t *nnz;            // in: n_prod per row (C.rpt); out: distinct columns per row
    const int32_t *bins;     // row list of the bin (NULL = identity rows bin_off..)
    int64_t bin_off;         // offset of the bin in `bins`
    int64_t nrows;           // rows in the bin
    int log_g;               // lanes streaming one B row = 1 << log_g
    int abort_thr;           // bin 7: abandon a row above this many keys
    Counters *ctr;           // fail counter
    int32_t *fail_list;      // abandoned rows (bin 7)
    int *slab;               // global tables (bin 8)
    int64_t slab_entries;
    int64_t grid;            // persistent grid for bin 8
    const unsigned int *count_dev;  // bin 8: device row count (NULL = nrows)
};
hipError_t launch_symbolic_bin(int bin, const SymArgs &a, hipStream_t s);

// ---- numeric step (kernels_num.hip) ----------------------------------------
struct NumArgs {
    DevCSR A, B;
    const int64_t *crpt;     // C row pointer (exclusive offsets, crpt[M] = nnz)
    int32_t *ccol;
    double *cval;
    const int32_t *bins;
    int64_t bin_off;
    int64_t nrows;
    int log_g;
    Counters *ctr;           // error counter
    int *slab_keys;          // global tables (bin 7)
    double *slab_vals;
    int64_t slab_entries;
    int64_t grid;
};
hipError_t launch_numeric_bin(int bin, const NumArgs &a, hipStream_t s);

}  // namespace opsp
