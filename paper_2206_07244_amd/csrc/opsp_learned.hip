// Entry points of the row-size predictor and of the one-phase product with
// predicted capacities (see include/opsp.h).
//
// One-phase flow (the alternative of Section 2.2, capacities from the
// predictor instead of a bound):
//   1 setup       n_prod, a_len, b_max per row (the setup kernel of the
//                 two-phase path with its feature outputs);
//   2 capacities  network inference (matrix cores) -> cap per row, fused with
//                 the first numeric binning pass over the capacities;
//                 finalize + second pass: numeric bins by capacity and the
//                 capacities scanned into slot offsets; one read-back;
//   3 numeric     the hash-accumulate kernels of the numeric step in their
//                 one-phase form: a row's sorted entries go to its slot, or
//                 to the overflow arena when it outgrew the slot; a row whose
//                 table passes the fill threshold is abandoned to a list;
//   4 scan        exact nnz per row scanned into C.rpt (out of place, so a
//                 recompute can still add rows); one read-back of nnz(C) and
//                 the overflow counters;
//   5 recompute   only when rows were abandoned: the global-table kernel with
//                 tables sized from min(n_prod, N) into a second arena, then
//                 the scan again (a third read-back);
//   6 copy        C allocated, rows copied from slots / arenas into C.
#include <cmath>
#include <cstddef>
#include <new>
#include <string.h>

#include "opsp.h"
#include "opsp_host_util.h"

using namespace opsp;
using namespace opsp::host;

namespace {

constexpr int64_t ARENA_MIN = 1 << 16;

// Workgroups of the bucketed kernel: BUCKET_WG_PER_CU per CU at most,
// staging (12 bytes per product of the longest row, per workgroup) within
// the staging budget.
int64_t bucket_grid(int64_t rows, int cus, int64_t max_nprod) {
    int64_t g = rows < (int64_t)cus * BUCKET_WG_PER_CU ? rows : (int64_t)cus * BUCKET_WG_PER_CU;
    const int64_t per = (max_nprod > 1 ? max_nprod : 1) * 12;
    const int64_t fit = STAGING_BUDGET / per;
    if (g > fit) g = fit > 1 ? fit : 1;
    return g;
}

struct LearnedCounters {
    Counters num;      // numeric bins by capacity; total = sum of capacities
    Counters scan;     // scan of the exact row sizes; total = nnz(C)
    LearnCtr lc;
    double calib[3 * CAL_OCT];            // calibration sums per n_prod octave
    unsigned long long cal_hist[CAL_OCT];  // eligible rows per octave
    unsigned long long cal_quota[CAL_OCT];
    unsigned long long cal_max[CAL_OCT];   // largest exact / estimate per octave (bits)
    unsigned long long cal_sched[2];       // row counter of the exact count
    unsigned int cal_n;                    // picked rows
};
constexpr int64_t CAL_PER_OCTAVE_DEFAULT = 64;
static_assert(sizeof(LearnedCounters) <= PINNED_BYTES, "read-back buffer");

opsp_status check_predictor(const opsp_predictor *p) {
    if (!p || p->version != OPSP_PREDICTOR_VERSION) return OPSP_ERR_INVALID;
    if (p->kind < OPSP_PRED_MLP || p->kind > OPSP_PRED_RATIO) return OPSP_ERR_INVALID;
    if (p->kind == OPSP_PRED_MLP && !p->params) return OPSP_ERR_INVALID;
    if (!(p->margin >= 0.0) || !std::isfinite(p->margin)) return OPSP_ERR_INVALID;
    if (p->kind == OPSP_PRED_RATIO && !(p->ratio > 0.0 && std::isfinite(p->ratio))) return OPSP_ERR_INVALID;
    if (p->cap_scale < 0.0 || !std::isfinite(p->cap_scale)) return OPSP_ERR_INVALID;
    return OPSP_OK;
}

// Scan of the exact row sizes nz[0..M) into crpt[0..M] and its read-back.
opsp_status scan_sizes(int64_t M, int64_t *nz, int64_t *crpt, const BlockParts &parts,
                       LearnedCounters *d, LearnedCounters *h, hipStream_t s) {
    Bounds none;
    memset(&none, 0, sizeof(none));
    none.nb = 1;
    none.nslots = 1;
    CHK(launch_hist(M, nz, none, parts, s));
    CHK(launch_finalize(M, 1, parts, &d->scan, crpt + M, true, s));
    CHK(launch_scatter(M, nz, none, &d->scan, nullptr, parts, true, s, crpt));
    CHK(read_back(h, d, sizeof(LearnedCounters), s));
    return OPSP_OK;
}

opsp_status run_learned(const opsp_csr *A, const opsp_csr *B, opsp_csr *C, const opsp_predictor *pr,
                        const opsp_config *cfg, opsp_stats *stats, hipStream_t s) {
    int dev = 0, cus = 256;
    opsp_status st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    const int64_t M = A->rows, N = B->cols;
    if (cfg && cfg->validate) {
        const opsp_csr *X[2] = {A, B};
        st = validate_csr(X, 2, s);
        if (st != OPSP_OK) return st;
    }
    Timer tm(cfg && cfg->stage_timing, s);
    opsp_stats S;
    memset(&S, 0, sizeof(S));
    Arena ar(s);
    void *p = nullptr;
    CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)(M + 1)));
    int64_t *crpt = (int64_t *)p;
    if (M == 0) {
        CHK(hipMemsetAsync(crpt, 0, sizeof(int64_t), s));
        ar.keep(crpt);
        C->rows = 0;
        C->cols = N;
        C->rpt = crpt;
        if (stats) *stats = S;
        return OPSP_OK;
    }
    const int64_t nblk = (M + 255) / 256;
    CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)(M + 1)));
    int64_t *np = (int64_t *)p;
    CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)(M + 1)));
    int64_t *off = (int64_t *)p;
    CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)(M + 1)));
    int64_t *nz = (int64_t *)p;
    CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)M));
    int64_t *loc = (int64_t *)p;
    CHK(ar.alloc(&p, sizeof(int32_t) * (size_t)M * 4));
    int32_t *alen = (int32_t *)p, *bmax = alen + M, *bins = alen + 2 * M, *retry = alen + 3 * M;
    const bool ranges = !(cfg && cfg->version >= 2 && cfg->hash_all_rows);
    const int64_t cal_k = pr->calib_rows == 0 ? CAL_PER_OCTAVE_DEFAULT : pr->calib_rows;
    const bool calib = pr->kind == OPSP_PRED_MLP && cal_k > 0;
    int2 *rng = nullptr;
    int4 *bfl = nullptr;   // output column range per row, B's row bounds
    if (ranges || calib) {   // the calibration needs the ranges too
        CHK(ar.alloc(&p, sizeof(int2) * (size_t)M));
        rng = (int2 *)p;
        CHK(ar.alloc(&p, sizeof(int4) * (size_t)(B->rows > 0 ? B->rows : 1)));
        bfl = (int4 *)p;
    }
    CHK(ar.alloc(&p, block_parts_bytes(M, A->nnz)));
    const BlockParts parts = block_parts_at(p, M, A->nnz);
    CHK(ar.alloc(&p, sizeof(LearnedCounters)));
    LearnedCounters *dc = (LearnedCounters *)p;
    LearnedCounters hc;

    const Bounds bs = make_bounds(0, sym_ratio(cfg), -1);
    const Bounds bn = config_bounds(1, cfg, 0);   // the one-phase bin 0 kernel is variant 0
    const DevCSR dA = dev_of(A), dB = dev_of(B);

    // 1-2 setup, capacities, numeric bins by capacity, slot offsets
    tm.mark();
    CHK(hipMemsetAsync(&dc->lc, 0, sizeof(LearnedCounters) - offsetof(LearnedCounters, lc), s));
    if (bfl) CHK(launch_brange(dB, bfl, false, nullptr, s));
    CHK(launch_setup(dA, dB, np, bs, parts, alen, bmax, s, bfl, rng));
    CapArgs ca;
    memset(&ca, 0, sizeof(ca));
    ca.kind = pr->kind;
    ca.P = pr->params;
    ca.margin = pr->margin;
    ca.ratio = pr->ratio > 0 ? pr->ratio : 1.0;
    ca.scale = pr->cap_scale > 0 ? pr->cap_scale : 1.0;
    ca.ncols = N;
    ca.pred = pr->pred_out;
    if (calib) {
        // network outputs first, then the exactly counted sample (picked
        // per octave of n_prod), then the calibrated capacities
        float *pred = pr->pred_out;
        if (!pred) {
            CHK(ar.alloc(&p, sizeof(float) * (size_t)M));
            pred = (float *)p;
        }
        CHK(launch_mlp_pred(M, pr->params, alen, np, bmax, pred, s));
        CHK(launch_cal_hist(M, alen, np, rng, dc->cal_hist, s));
        CHK(ar.alloc(&p, sizeof(int32_t) * (size_t)M));
        int32_t *list = (int32_t *)p;
        CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)M));
        int64_t *exact = (int64_t *)p;
        CHK(launch_cal_pick(M, alen, np, rng, dc->cal_hist, cal_k, dc->cal_quota, list, &dc->cal_n, s));
        // exact sizes of the picked rows: the bin-8 bitmap windows (every
        // picked range fits them), one row per workgroup from a counter
        SymArgs g;
        memset(&g, 0, sizeof(g));
        g.A = dA;
        g.B = dB;
        g.nnz = exact;
        g.src.bins = list;
        g.src.count = &dc->cal_n;
        g.ctr = &dc->num;
        g.rng = rng;
        g.sched = dc->cal_sched;
        g.grid = cus;
        CHK(launch_symbolic_bin(SYM_GLOBAL_BIN, g, s));
        CHK(launch_cal_sum(list, &dc->cal_n, np, bmax, pred, exact, N, dc->calib, dc->cal_max, s));
        ca.pred_in = pred;
        ca.calib = dc->calib;
        ca.calmax = dc->cal_max;
    }
    CHK(launch_mlp_caps(M, ca, alen, np, bmax, off, bn, parts, &dc->lc, s));
    if (pr->cap_out)
        CHK(hipMemcpyAsync(pr->cap_out, off, sizeof(int64_t) * (size_t)M, hipMemcpyDeviceToDevice, s));
    CHK(launch_finalize(M, bn.nslots, parts, &dc->num, off + M, true, s));
    CHK(launch_scatter(M, off, bn, &dc->num, bins, parts, true, s));
    tm.mark();
    CHK(read_back(&hc, dc, sizeof(LearnedCounters), s));
    const int64_t cap_total = (int64_t)hc.num.total;
    const int64_t cap_max = (int64_t)hc.num.maxv;
    S.nprod = (int64_t)hc.lc.nprod_total;
    S.max_row_nprod = (int64_t)hc.lc.nprod_max;
    S.cap_total = cap_total;
    {
        double ex = 0.0, es = 0.0;
        for (int o = 0; o < CAL_OCT; ++o) {
            ex += hc.calib[o];
            es += hc.calib[CAL_OCT + o];
        }
        S.calib_scale = es > 0.0 ? ex / es : 1.0;   // the sample's overall ratio
    }
    if (cap_max > INT32_MAX) return OPSP_ERR_OVERFLOW;
    int64_t nsz[OPSP_NUM_BINS], noff[OPSP_NUM_BINS];
    for (int j = 0; j < OPSP_NUM_BINS; ++j) {
        nsz[j] = (int64_t)hc.num.size[j];
        S.num_bin_rows[j] = nsz[j];
        noff[j] = j ? noff[j - 1] + nsz[j - 1] : 0;
    }

    // 3 one-phase numeric into slots + arena
    const int64_t arena_cap = cap_total / 8 > ARENA_MIN ? cap_total / 8 : ARENA_MIN;
    const int64_t tsize = cap_total + arena_cap;
    CHK(ar.alloc(&p, sizeof(int32_t) * (size_t)tsize));
    int32_t *tcol = (int32_t *)p;
    CHK(ar.alloc(&p, sizeof(double) * (size_t)tsize));
    double *tval = (double *)p;
    NumArgs na;
    memset(&na, 0, sizeof(na));
    na.A = dA;
    na.B = dB;
    na.ccol = tcol;
    na.cval = tval;
    na.ctr = &dc->num;
    na.rng = ranges ? rng : nullptr;
    na.lrn.mode = 1;
    na.lrn.off = off;
    na.lrn.nprod = np;
    na.lrn.nnz = nz;
    na.lrn.loc = loc;
    na.lrn.loc_bias = 0;
    na.lrn.ncols = N;
    na.lrn.arena_base = cap_total;
    na.lrn.arena_cap = arena_cap;
    na.lrn.lc = &dc->lc;
    na.lrn.retry = retry;
    for (int b = NUM_GLOBAL_BIN; b >= 0; --b) {
        if (nsz[b] == 0) continue;
        na.src = host_rows(bins, noff[b], nsz[b]);
        na.grid = 0;
        if (b == NUM_GLOBAL_BIN && ranges && N <= BUCKET_MAX_COLS) {
            // long rows: bucketed dense accumulation (never overflows)
            void *pk = nullptr, *pv = nullptr;
            const int64_t grid = bucket_grid(nsz[b], cus, S.max_row_nprod);
            const int64_t sc = (S.max_row_nprod > 1 ? S.max_row_nprod : 1) + 1;   // + spare entry
            CHK(ar.alloc(&pk, sizeof(int) * (size_t)(sc * grid)));
            CHK(ar.alloc(&pv, sizeof(double) * (size_t)(sc * grid)));
            NumArgs ba = na;
            ba.slab_keys = (int *)pk;
            ba.slab_vals = (double *)pv;
            ba.slab_entries = sc;
            ba.grid = grid;
            CHK(launch_numeric_bucket(ba, s));
            continue;
        }
        if (b == NUM_GLOBAL_BIN) {
            const int64_t entries = pow2_host(2 * cap_max > 8192 ? 2 * cap_max : 8192);
            const int64_t grid = nsz[b] < (int64_t)cus * NUM_GLOBAL_WG_PER_CU ? nsz[b]
                                                                               : (int64_t)cus * NUM_GLOBAL_WG_PER_CU;
            void *pk = nullptr, *pv = nullptr;
            CHK(ar.alloc(&pk, sizeof(int) * (size_t)(entries * grid)));
            CHK(ar.alloc(&pv, sizeof(double) * (size_t)(entries * grid)));
            na.slab_keys = (int *)pk;
            na.slab_vals = (double *)pv;
            na.slab_entries = entries;
            na.grid = grid;
        }
        CHK(launch_numeric_bin(b, na, s));
    }
    tm.mark();

    // 4 exact sizes -> C.rpt
    st = scan_sizes(M, nz, crpt, parts, dc, &hc, s);
    if (st != OPSP_OK) return st;
    if (hc.num.error || hc.lc.error) return OPSP_ERR_INTERNAL;

    // 5 recompute abandoned rows (tables sized from min(n_prod, N))
    int32_t *a2col = nullptr;
    double *a2val = nullptr;
    const int64_t nretry = (int64_t)hc.lc.retry;
    S.retry_rows = nretry;
    S.table_overflow_rows = (int64_t)hc.lc.table_overflow;
    S.slot_overflow_rows = (int64_t)hc.lc.slot_overflow;
    S.arena_entries = (int64_t)hc.lc.arena_used < arena_cap ? (int64_t)hc.lc.arena_used : arena_cap;
    if (nretry > 0) {
        const int64_t ub = (int64_t)hc.lc.retry_ub;
        CHK(ar.alloc(&p, sizeof(int32_t) * (size_t)(ub > 0 ? ub : 1)));
        a2col = (int32_t *)p;
        CHK(ar.alloc(&p, sizeof(double) * (size_t)(ub > 0 ? ub : 1)));
        a2val = (double *)p;
        NumArgs ra = na;
        ra.ccol = a2col;
        ra.cval = a2val;
        ra.src = host_rows(retry, 0, nretry);
        ra.lrn.mode = 2;
        ra.lrn.off = nullptr;
        ra.lrn.loc_bias = tsize;
        ra.lrn.arena_base = 0;
        ra.lrn.arena_cap = ub;
        // the second arena starts empty: count its use from zero
        CHK(hipMemsetAsync(&dc->lc.arena_used, 0, sizeof(unsigned long long), s));
        if (ranges && N <= BUCKET_MAX_COLS) {
            // bucketed dense accumulation: staging for the longest row
            const int64_t sc = (S.max_row_nprod > 1 ? S.max_row_nprod : 1) + 1;   // + spare entry
            const int64_t g2 = bucket_grid(nretry, cus, sc);
            void *sk = nullptr, *sv = nullptr;
            CHK(ar.alloc(&sk, sizeof(int) * (size_t)(sc * g2)));
            CHK(ar.alloc(&sv, sizeof(double) * (size_t)(sc * g2)));
            ra.slab_keys = (int *)sk;
            ra.slab_vals = (double *)sv;
            ra.slab_entries = sc;
            ra.grid = g2;
            CHK(launch_numeric_bucket(ra, s));
        } else {
            // global hash tables sized from min(n_prod, N)
            const int64_t bmx = S.max_row_nprod < N ? S.max_row_nprod : N;
            const int64_t entries = pow2_host(2 * bmx > 64 ? 2 * bmx : 64);
            const int64_t grid = nretry < (int64_t)cus ? nretry : (int64_t)cus;
            void *pk = nullptr, *pv = nullptr;
            CHK(ar.alloc(&pk, sizeof(int) * (size_t)(entries * grid)));
            CHK(ar.alloc(&pv, sizeof(double) * (size_t)(entries * grid)));
            ra.slab_keys = (int *)pk;
            ra.slab_vals = (double *)pv;
            ra.slab_entries = entries;
            ra.grid = grid;
            CHK(launch_numeric_bin(NUM_GLOBAL_BIN, ra, s));
        }
        st = scan_sizes(M, nz, crpt, parts, dc, &hc, s);
        if (st != OPSP_OK) return st;
        if (hc.num.error || hc.lc.error || (int64_t)hc.lc.retry != nretry) return OPSP_ERR_INTERNAL;
    }
    const int64_t nnzC = (int64_t)hc.scan.total;
    S.nnz = nnzC;
    S.max_row_nnz = (int64_t)hc.scan.maxv;

    // 6 C and the copy
    void *pc = nullptr, *pv = nullptr;
    if (nnzC > 0) {
        CHK(ar.alloc(&pc, sizeof(int32_t) * (size_t)nnzC));
        CHK(ar.alloc(&pv, sizeof(double) * (size_t)nnzC));
    }
    tm.mark();
    CHK(launch_compact(M, nnzC, crpt, loc, tcol, tval, tsize, a2col, a2val, (int32_t *)pc,
                       (double *)pv, s));
    tm.mark();
    ar.keep(crpt);
    ar.keep(pc);
    ar.keep(pv);
    C->rows = M;
    C->cols = N;
    C->nnz = nnzC;
    C->rpt = crpt;
    C->col = (int32_t *)pc;
    C->val = (double *)pv;
    if (stats) {
        if (tm.on) {
            (void)hipStreamSynchronize(s);
            for (int k = 0; k < 4; ++k) S.ms_stage[k] = tm.between(k, k + 1);
            S.ms_stage[4] = tm.between(0, 4);
        }
        *stats = S;
    }
    return OPSP_OK;
}

}  // namespace

extern "C" {

opsp_status opsp_row_features(const opsp_csr *A, const opsp_csr *B, int32_t *a_len, int64_t *n_prod,
                              int32_t *b_max, void *stream) {
    opsp_status st = check_inputs(A, B);
    if (st != OPSP_OK) return st;
    int dev = 0, cus = 0;
    st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    const int64_t M = A->rows;
    if (M == 0) return OPSP_OK;
    hipStream_t s = (hipStream_t)stream;
    Arena ar(s);
    void *p = nullptr;
    const int64_t nblk = (M + 255) / 256;
    CHK(ar.alloc(&p, block_parts_bytes(M, A->nnz)));
    const BlockParts parts = block_parts_at(p, M, A->nnz);
    int64_t *np = n_prod;
    if (!np) {
        CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)M));
        np = (int64_t *)p;
    }
    CHK(launch_setup(dev_of(A), dev_of(B), np, make_bounds(0, 1.2, -1), parts, a_len, b_max, s));
    return OPSP_OK;
}

opsp_status opsp_mlp_features(const opsp_csr *A, const opsp_csr *B, float *X, void *stream) {
    opsp_status st = check_inputs(A, B);
    if (st != OPSP_OK) return st;
    const int64_t M = A->rows;
    if (M > 0 && !X) return OPSP_ERR_INVALID;
    if (M == 0) return OPSP_OK;
    hipStream_t s = (hipStream_t)stream;
    Arena ar(s);
    void *p = nullptr;
    {
        hipError_t e = ar.alloc(&p, (sizeof(int64_t) + 2 * sizeof(int32_t)) * (size_t)M);
        if (e != hipSuccess) return status_of(e);
    }
    int64_t *np = (int64_t *)p;
    int32_t *al = (int32_t *)(np + M), *bm = al + M;
    st = opsp_row_features(A, B, al, np, bm, stream);
    if (st != OPSP_OK) return st;
    CHK(launch_mlp_features(M, al, np, bm, X, s));
    return OPSP_OK;
}

opsp_status opsp_mlp_forward(const uint16_t *params, const float *X, int64_t n, float *y,
                             void *stream) {
    if (n < 0 || (n > 0 && (!params || !X || !y))) return OPSP_ERR_INVALID;
    if (n == 0) return OPSP_OK;
    int dev = 0, cus = 0;
    opsp_status st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    CHK(launch_mlp_forward(params, X, n, y, (hipStream_t)stream));
    return OPSP_OK;
}

opsp_status opsp_mlp_grad(const uint16_t *params, const float *X, const float *target, int64_t n,
                          float tau, float *grad, float *loss, void *stream) {
    if (n < 1 || !params || !X || !target || !grad) return OPSP_ERR_INVALID;
    if (!(tau >= 0.f && tau < 1.f)) return OPSP_ERR_INVALID;
    int dev = 0, cus = 0;
    opsp_status st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Arena ar(s);
    void *p = nullptr;
    const int64_t nblk = (n + 63) / 64;
    CHK(ar.alloc(&p, sizeof(float) * (size_t)(nblk * (MLP_NPARAM + 1))));
    CHK(launch_mlp_grad(params, X, target, n, tau, (float *)p, grad, loss, s));
    return OPSP_OK;
}

opsp_status opsp_mlp_adam(float *master, float *m, float *v, const float *grad, int64_t step,
                          float lr, float beta1, float beta2, float eps, uint16_t *params,
                          void *stream) {
    if (!master || !m || !v || !grad || !params || step < 1) return OPSP_ERR_INVALID;
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || !(lr >= 0.f))
        return OPSP_ERR_INVALID;
    int dev = 0, cus = 0;
    opsp_status st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    const double c1 = 1.0 / (1.0 - pow((double)beta1, (double)step));
    const double c2 = 1.0 / (1.0 - pow((double)beta2, (double)step));
    CHK(launch_mlp_adam(master, m, v, grad, lr, beta1, beta2, eps, (float)c1, (float)c2, params,
                        (hipStream_t)stream));
    return OPSP_OK;
}

opsp_status opsp_spgemm_learned(const opsp_csr *A, const opsp_csr *B, opsp_csr *C,
                                const opsp_predictor *predictor, const opsp_config *config,
                                opsp_stats *stats, void *stream) {
    if (!C) return OPSP_ERR_INVALID;
    memset(C, 0, sizeof(*C));
    opsp_status st = check_inputs(A, B);
    if (st != OPSP_OK) return st;
    st = check_config(config);
    if (st != OPSP_OK) return st;
    st = check_predictor(predictor);
    if (st != OPSP_OK) return st;
    st = run_learned(A, B, C, predictor, config, stats, (hipStream_t)stream);
    if (st != OPSP_OK) memset(C, 0, sizeof(*C));
    return st;
}

}  // extern "C"
