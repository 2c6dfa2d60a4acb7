// Batched SpGEMM: many independent products C_p = A_p * B_p as ONE
// block-diagonal product over the concatenation of their rows.
//
// Rows of C are independent (Section 2.1), so stacking the A_p row-wise,
// shifting A_p's column indices to the position of B_p inside the stacked B,
// and stacking the B_p gives a single matrix product whose row i (belonging
// to problem p) touches only B_p's rows and yields exactly row i of C_p.  One
// pass of every stage (setup, both binnings, symbolic, scan, numeric) then
// covers all problems, so small problems share the GPU instead of each paying
// its own launches and host synchronisations.
//
// Execution is two captured graphs per batch:
//   G1 (structure): gather of the stacked row pointers / column indices,
//      setup + first binning, finalize, second binning, the symbolic bin
//      kernels launched persistently (their bin sizes are only known on the
//      device), the global-table kernel for aborted rows, numeric binning +
//      row-pointer scan, per-problem row-pointer bounds, and the copy of the
//      counters and bounds into pinned host memory;
//   -- one host read-back: nnz(C), numeric bin sizes, per-problem nnz --
//   G2 (values): gather of the stacked values and the numeric bin kernels
//      with exact grids.
// G1 is captured at creation; G2 after the first read-back (and again only
// if the numeric bin sizes change).  Both are replayed by later executions.
// Every result C_p is a view: its row pointer points into the stacked row
// pointer (absolute offsets) and its col/val pointers are the stacked
// arrays, all owned by the batch object.
#include <stddef.h>
#include <string.h>

#include <vector>

#include "opsp.h"
#include "opsp_internal.h"
#include "opsp_host_util.h"

using namespace opsp;

namespace {

struct ProbDesc {
    int64_t row0;        // first row of A_p (and C_p) in the stack
    int64_t annz0;       // first entry of A_p in the stack
    int64_t brow0;       // first row of B_p in the stacked B
    int64_t bnnz0;       // first entry of B_p in the stacked B
    int64_t M, K;        // rows of A_p, rows of B_p
    const int64_t *arpt;
    const int32_t *acol;
    const double *aval;
    const int64_t *brpt;
    const int32_t *bcol;
    const double *bval;
};

// Stacked row pointers and column indices (blockIdx.y = problem).
__global__ __launch_bounds__(256) void k_gather_struct(const ProbDesc *__restrict__ pd,
                                                       int64_t *__restrict__ arpt,
                                                       int32_t *__restrict__ acol,
                                                       int64_t *__restrict__ brpt,
                                                       int32_t *__restrict__ bcol) {
    const ProbDesc d = pd[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t a0 = d.arpt[0], b0 = d.brpt[0];
    for (int64_t i = t0; i <= d.M; i += stride) arpt[d.row0 + i] = d.annz0 + (d.arpt[i] - a0);
    const int64_t an = d.arpt[d.M] - a0;
    const int32_t shift = (int32_t)d.brow0;
    for (int64_t e = t0; e < an; e += stride) acol[d.annz0 + e] = d.acol[a0 + e] + shift;
    for (int64_t i = t0; i <= d.K; i += stride) brpt[d.brow0 + i] = d.bnnz0 + (d.brpt[i] - b0);
    const int64_t bn = d.brpt[d.K] - b0;
    for (int64_t e = t0; e < bn; e += stride) bcol[d.bnnz0 + e] = d.bcol[b0 + e];
}

// Stacked values.
__global__ __launch_bounds__(256) void k_gather_vals(const ProbDesc *__restrict__ pd,
                                                     double *__restrict__ aval,
                                                     double *__restrict__ bval) {
    const ProbDesc d = pd[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t a0 = d.arpt[0], b0 = d.brpt[0];
    const int64_t an = d.arpt[d.M] - a0, bn = d.brpt[d.K] - b0;
    for (int64_t e = t0; e < an; e += stride) aval[d.annz0 + e] = d.aval[a0 + e];
    for (int64_t e = t0; e < bn; e += stride) bval[d.bnnz0 + e] = d.bval[b0 + e];
}

// C row-pointer value at the first row of every problem (and the end).
__global__ void k_prob_bounds(const ProbDesc *__restrict__ pd, int32_t count,
                              const int64_t *__restrict__ crpt, int64_t total_rows,
                              int64_t *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < count) out[p] = crpt[pd[p].row0];
    if (p == count) out[p] = crpt[total_rows];
}

opsp_status status_of_hip(hipError_t e) {
    if (e == hipSuccess) return OPSP_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return OPSP_ERR_ALLOC;
    return OPSP_ERR_HIP;
}

#define BCHK(x)                                          \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) return status_of_hip(e_);  \
    } while (0)

}  // namespace

struct opsp_batch {
    int32_t count = 0;
    int device = 0;
    int cus = 256;
    std::vector<ProbDesc> desc;
    std::vector<int64_t> N;          // columns of each problem
    int64_t M = 0, K = 0, nnzA = 0, nnzB = 0, Nmax = 0;
    int64_t sym_ub[8] = {};
    Bounds bs, bn;
    int gv = 0;                      // bin 0 variant (lanes per row, table size)
    // device memory (cache blocks)
    std::vector<std::pair<void *, size_t>> owned;
    ProbDesc *d_desc = nullptr;
    int64_t *arpt = nullptr, *brpt = nullptr, *crpt = nullptr;
    int32_t *acol = nullptr, *bcol = nullptr, *bins = nullptr, *fail = nullptr;
    double *aval = nullptr, *bval = nullptr;
    BlockParts parts{};
    Counters *ctr = nullptr;         // [0] symbolic, [1] numeric
    int64_t *d_bounds = nullptr;     // count + 1
    int *slab8 = nullptr;
    int64_t slab8_entries = 0, slab8_grid = 0;
    // C storage
    int32_t *ccol = nullptr;
    double *cval = nullptr;
    int64_t ccap = 0;
    int *slab7k = nullptr;
    double *slab7v = nullptr;
    int64_t slab7_entries = 0, slab7_grid = 0;
    // host read-back (pinned): counters + bounds
    void *h_buf = nullptr;
    // graphs
    hipGraphExec_t g1 = nullptr, g2 = nullptr;
    // the batch's own stream: graphs are captured and replayed on it (the
    // caller's stream may be the legacy NULL stream, which cannot be
    // captured); events order it after / before the caller's stream
    hipStream_t cs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int64_t g2_sizes[OPSP_NUM_BINS] = {};
    int64_t g2_nnz = -1;
    int64_t last_nnz = 0, last_nprod = 0, last_max_nnz = 0;
    hipStream_t stream = nullptr;

    Counters *h_ctr() { return (Counters *)h_buf; }
    int64_t *h_bounds() { return (int64_t *)((char *)h_buf + 2 * sizeof(Counters)); }
};

namespace {

hipError_t balloc(opsp_batch *b, void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = cache_alloc(p, bytes, s);
    if (e == hipSuccess) b->owned.push_back({*p, bytes});
    return e;
}

void bfree_all(opsp_batch *b, hipStream_t s) {
    for (auto &pp : b->owned) (void)cache_free(pp.first, s);
    b->owned.clear();
}

opsp_status capture_g1(opsp_batch *b, hipStream_t s) {
    const DevCSR A{b->M, b->K, b->arpt, b->acol, b->aval};
    const DevCSR B{b->K, b->Nmax, b->brpt, b->bcol, b->bval};
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    auto body = [&]() -> hipError_t {
        hipError_t e;
        hipLaunchKernelGGL(k_gather_struct, dim3(64, (unsigned)b->count), dim3(256), 0, s, b->d_desc,
                           b->arpt, b->acol, b->brpt, b->bcol);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_setup(A, B, b->crpt, b->bs, b->parts, nullptr, nullptr, s)) != hipSuccess) return e;
        if ((e = launch_finalize(b->M, b->bs.nslots, b->parts, &b->ctr[0], nullptr, false, s)) != hipSuccess) return e;
        if ((e = launch_scatter(b->M, b->crpt, b->bs, &b->ctr[0], b->bins, b->parts, false, s)) != hipSuccess) return e;
        SymArgs sa;
        memset(&sa, 0, sizeof(sa));
        sa.gv = b->gv;
        sa.A = A;
        sa.B = B;
        sa.nnz = b->crpt;
        sa.ctr = &b->ctr[0];
        sa.fail_list = b->fail;
        sa.abort_thr = (int)(0.8 * SYM_T[7]);
        for (int bin = 7; bin >= 0; --bin) {
            memset(&sa.src, 0, sizeof(sa.src));
            sa.src.bins = b->bins;
            sa.src.dctr = &b->ctr[0];
            sa.src.bin = bin;
            int64_t g = (int64_t)b->cus * sym_wg_per_cu(bin);
            const int64_t R = sym_rows_per_wg(bin, b->gv);
            const int64_t need = (b->M + R - 1) / R;
            sa.grid = g < need ? g : need;
            if (sa.grid < 1) sa.grid = 1;
            if ((e = launch_symbolic_bin(bin, sa, s)) != hipSuccess) return e;
            if (bin == 7 && b->slab8) {
                SymArgs gl = sa;
                memset(&gl.src, 0, sizeof(gl.src));
                gl.src.bins = b->fail;
                gl.src.count = &b->ctr[0].fail;
                gl.slab = b->slab8;
                gl.slab_entries = b->slab8_entries;
                gl.grid = b->slab8_grid;
                gl.sched = b->ctr[0].sched;
                if ((e = launch_symbolic_bin(SYM_GLOBAL_BIN, gl, s)) != hipSuccess) return e;
            }
        }
        if ((e = launch_hist(b->M, b->crpt, b->bn, b->parts, s)) != hipSuccess) return e;
        if ((e = launch_finalize(b->M, b->bn.nslots, b->parts, &b->ctr[1], b->crpt + b->M, true, s)) != hipSuccess) return e;
        if ((e = launch_scatter(b->M, b->crpt, b->bn, &b->ctr[1], b->bins, b->parts, true, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_prob_bounds, dim3((unsigned)((b->count + 256) / 256)), dim3(256), 0, s, b->d_desc,
                           b->count, b->crpt, b->M, b->d_bounds);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(b->h_buf, b->ctr, 2 * sizeof(Counters), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        return hipMemcpyAsync(b->h_bounds(), b->d_bounds, sizeof(int64_t) * (size_t)(b->count + 1),
                              hipMemcpyDeviceToHost, s);
    };
    hipError_t eb = body();
    hipError_t ee = hipStreamEndCapture(s, &graph);
    if (eb != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return status_of_hip(eb);
    }
    BCHK(ee);
    hipError_t ei = hipGraphInstantiate(&b->g1, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    BCHK(ei);
    return OPSP_OK;
}

opsp_status capture_g2(opsp_batch *b, const int64_t *sizes, hipStream_t s) {
    const DevCSR A{b->M, b->K, b->arpt, b->acol, b->aval};
    const DevCSR B{b->K, b->Nmax, b->brpt, b->bcol, b->bval};
    if (b->g2) {
        (void)hipGraphExecDestroy(b->g2);
        b->g2 = nullptr;
    }
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    auto body = [&]() -> hipError_t {
        hipError_t e;
        hipLaunchKernelGGL(k_gather_vals, dim3(64, (unsigned)b->count), dim3(256), 0, s, b->d_desc,
                           b->aval, b->bval);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        NumArgs na;
        memset(&na, 0, sizeof(na));
        na.gv = b->gv;
        na.A = A;
        na.B = B;
        na.crpt = b->crpt;
        na.ccol = b->ccol;
        na.cval = b->cval;
        na.ctr = &b->ctr[1];
        int64_t off = 0, offs[OPSP_NUM_BINS];
        for (int j = 0; j < OPSP_NUM_BINS; ++j) {
            offs[j] = off;
            off += sizes[j];
        }
        for (int bin = NUM_GLOBAL_BIN; bin >= 0; --bin) {
            if (sizes[bin] == 0) continue;
            memset(&na.src, 0, sizeof(na.src));
            na.src.bins = b->bins;
            na.src.off = offs[bin];
            na.src.nrows = sizes[bin];
            na.grid = 0;
            if (bin == NUM_GLOBAL_BIN) {
                na.slab_keys = b->slab7k;
                na.slab_vals = b->slab7v;
                na.slab_entries = b->slab7_entries;
                na.grid = b->slab7_grid;
            }
            if ((e = launch_numeric_bin(bin, na, s)) != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t eb = body();
    hipError_t ee = hipStreamEndCapture(s, &graph);
    if (eb != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return status_of_hip(eb);
    }
    BCHK(ee);
    hipError_t ei = hipGraphInstantiate(&b->g2, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    BCHK(ei);
    for (int j = 0; j < OPSP_NUM_BINS; ++j) b->g2_sizes[j] = sizes[j];
    return OPSP_OK;
}

void batch_release(opsp_batch *b) {
    if (!b) return;
    if (b->cs) (void)hipStreamSynchronize(b->cs);
    if (b->g1) (void)hipGraphExecDestroy(b->g1);
    if (b->g2) (void)hipGraphExecDestroy(b->g2);
    b->g1 = b->g2 = nullptr;
    // the batch's stream is idle: its blocks go back to the cache for the
    // default stream
    bfree_all(b, nullptr);
    if (b->h_buf) (void)hipHostFree(b->h_buf);
    b->h_buf = nullptr;
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    b->ev_in = b->ev_out = nullptr;
    b->cs = nullptr;
}

}  // namespace

extern "C" {

opsp_status opsp_batch_create(int32_t count, const opsp_csr *A, const opsp_csr *B,
                              const opsp_config *cfg, opsp_batch **out, void *stream) {
    if (!out) return OPSP_ERR_INVALID;
    *out = nullptr;
    if (count < 1 || count > 65535 || !A || !B) return OPSP_ERR_INVALID;
    {
        const opsp_status cs = opsp::host::check_config(cfg);
        if (cs != OPSP_OK) return cs;
    }
    hipStream_t user = (hipStream_t)stream;
    opsp_batch *b = new (std::nothrow) opsp_batch();
    if (!b) return OPSP_ERR_ALLOC;
    b->count = count;
    b->stream = user;
    opsp_status st = OPSP_OK;
    auto fail = [&](opsp_status x) {
        batch_release(b);
        delete b;
        return x;
    };
    if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
        return fail(OPSP_ERR_HIP);
    // inputs were produced on the caller's stream
    if (hipEventRecord(b->ev_in, user) != hipSuccess || hipStreamWaitEvent(b->cs, b->ev_in, 0) != hipSuccess)
        return fail(OPSP_ERR_HIP);
    hipStream_t s = b->cs;
    if (hipGetDevice(&b->device) != hipSuccess) return fail(OPSP_ERR_NO_DEVICE);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
        return fail(OPSP_ERR_NO_DEVICE);
    b->cus = cus > 0 ? cus : 256;

    if (cfg && cfg->validate) {
        // every operand canonical before the structure graph gathers through them
        std::vector<const opsp_csr *> X;
        X.reserve(2 * (size_t)count);
        for (int p = 0; p < count; ++p) {
            if (!opsp::host::csr_ok(&A[p]) || !opsp::host::csr_ok(&B[p])) return fail(OPSP_ERR_INVALID);
            X.push_back(&A[p]);
            X.push_back(&B[p]);
        }
        st = opsp::host::validate_csr(X.data(), (int)X.size(), s);
        if (st != OPSP_OK) return fail(st);
    }
    // problem layout
    b->desc.resize(count);
    b->N.resize(count);
    int64_t row = 0, annz = 0, brow = 0, bnnz = 0;
    for (int p = 0; p < count; ++p) {
        const opsp_csr &a = A[p], &bb = B[p];
        if (a.rows < 0 || a.cols < 0 || bb.rows < 0 || bb.cols < 0 || a.nnz < 0 || bb.nnz < 0)
            return fail(OPSP_ERR_INVALID);
        if (!a.rpt || !bb.rpt || (a.nnz && (!a.col || !a.val)) || (bb.nnz && (!bb.col || !bb.val)))
            return fail(OPSP_ERR_INVALID);
        if (a.cols != bb.rows) return fail(OPSP_ERR_SHAPE);
        ProbDesc &d = b->desc[p];
        d.row0 = row;
        d.annz0 = annz;
        d.brow0 = brow;
        d.bnnz0 = bnnz;
        d.M = a.rows;
        d.K = bb.rows;
        d.arpt = a.rpt;
        d.acol = a.col;
        d.aval = a.val;
        d.brpt = bb.rpt;
        d.bcol = bb.col;
        d.bval = bb.val;
        b->N[p] = bb.cols;
        if (bb.cols > b->Nmax) b->Nmax = bb.cols;
        row += a.rows;
        annz += a.nnz;
        brow += bb.rows;
        bnnz += bb.nnz;
    }
    if (brow > INT32_MAX || b->Nmax > INT32_MAX) return fail(OPSP_ERR_SHAPE);
    b->M = row;
    b->K = brow;
    b->nnzA = annz;
    b->nnzB = bnnz;
    // the batch's kernels route every row by its natural bin
    opsp_config c2;
    memset(&c2, 0, sizeof(c2));
    if (cfg) memcpy(&c2, cfg, cfg->version >= 3   ? sizeof(opsp_config)
                              : cfg->version == 2 ? offsetof(opsp_config, streams)
                                                  : offsetof(opsp_config, sym_bounds));
    c2.force_sym_bin = c2.force_num_bin = -1;
    b->gv = opsp::host::gv_of(&c2);
    b->bs = opsp::host::config_bounds(0, &c2, b->gv);
    b->bn = opsp::host::config_bounds(1, &c2, b->gv);

    // device memory
    void *p = nullptr;
    const int64_t nblk = (b->M + 255) / 256;
#define BA(ptr, type, n)                                                   \
    do {                                                                   \
        hipError_t e_ = balloc(b, &p, sizeof(type) * (size_t)(n), s);      \
        if (e_ != hipSuccess) return fail(status_of_hip(e_));              \
        ptr = (type *)p;                                                   \
    } while (0)
    BA(b->d_desc, ProbDesc, count);
    BA(b->arpt, int64_t, b->M + 1);
    BA(b->acol, int32_t, annz > 0 ? annz : 1);
    BA(b->aval, double, annz > 0 ? annz : 1);
    BA(b->brpt, int64_t, b->K + 1);
    BA(b->bcol, int32_t, bnnz > 0 ? bnnz : 1);
    BA(b->bval, double, bnnz > 0 ? bnnz : 1);
    BA(b->crpt, int64_t, b->M + 1);
    BA(b->bins, int32_t, b->M > 0 ? b->M : 1);
    BA(b->fail, int32_t, b->M > 0 ? b->M : 1);
    BA(b->ctr, Counters, 2);
    BA(b->d_bounds, int64_t, count + 1);
    {
        hipError_t e_ = balloc(b, &p, block_parts_bytes(b->M, annz), s);
        if (e_ != hipSuccess) return fail(status_of_hip(e_));
        b->parts = block_parts_at(p, b->M, annz);
    }
    // symbolic global tables: a row reaches them only if it has more than
    // the abort threshold of distinct columns, i.e. if N_p > 0.8 * t7
    if (b->Nmax > (int64_t)(0.8 * SYM_T[7])) {
        b->slab8_entries = pow2_host(2 * b->Nmax);
        const int64_t budget = (int64_t)2 << 30;   // bytes for all slabs
        int64_t g = budget / (b->slab8_entries * 4);
        if (g > (int64_t)b->cus * SYM_GLOBAL_WG_PER_CU) g = (int64_t)b->cus * SYM_GLOBAL_WG_PER_CU;
        if (g < 1) return fail(OPSP_ERR_SHAPE);
        b->slab8_grid = g;
        BA(b->slab8, int, b->slab8_entries * g);
    }
#undef BA
    if (hipHostMalloc(&b->h_buf, 2 * sizeof(Counters) + sizeof(int64_t) * (size_t)(count + 1),
                      hipHostMallocDefault) != hipSuccess)
        return fail(OPSP_ERR_ALLOC);
    if (hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(ProbDesc) * (size_t)count, hipMemcpyHostToDevice,
                       s) != hipSuccess)
        return fail(OPSP_ERR_HIP);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(OPSP_ERR_HIP);
    if (b->M > 0) {
        st = capture_g1(b, s);
        if (st != OPSP_OK) return fail(st);
    }
    *out = b;
    return OPSP_OK;
}

opsp_status opsp_batch_execute(opsp_batch *b, opsp_csr *C, opsp_stats *stats, void *stream) {
    if (!b || !C) return OPSP_ERR_INVALID;
    hipStream_t user = (hipStream_t)stream;
    hipStream_t s = b->cs;
    b->stream = user;
    for (int p = 0; p < b->count; ++p) memset(&C[p], 0, sizeof(opsp_csr));
    // order the batch's stream after the caller's work (inputs, earlier reads
    // of the views), and the caller's stream after the batch's work below
    BCHK(hipEventRecord(b->ev_in, user));
    BCHK(hipStreamWaitEvent(s, b->ev_in, 0));
    auto join = [&]() -> hipError_t {
        hipError_t e = hipEventRecord(b->ev_out, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(user, b->ev_out, 0);
        return e;
    };
    if (b->M == 0) {
        for (int p = 0; p < b->count; ++p) {
            C[p].rows = 0;
            C[p].cols = b->N[p];
            C[p].rpt = b->crpt;
        }
        int64_t zero = 0;
        BCHK(hipMemcpyAsync(b->crpt, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
        BCHK(hipStreamSynchronize(s));
        BCHK(join());
        return OPSP_OK;
    }
    BCHK(hipGraphLaunch(b->g1, s));
    BCHK(hipStreamSynchronize(s));
    Counters *hc = b->h_ctr();
    if (hc[0].error || hc[1].error) return OPSP_ERR_INTERNAL;
    const int64_t nnz = (int64_t)hc[1].total;
    const int64_t max_nnz = (int64_t)hc[1].maxv;
    if (max_nnz > INT32_MAX) return OPSP_ERR_OVERFLOW;
    int64_t sizes[OPSP_NUM_BINS];
    for (int j = 0; j < OPSP_NUM_BINS; ++j) sizes[j] = (int64_t)hc[1].size[j];
    bool recapture = !b->g2 || b->g2_nnz != nnz;
    for (int j = 0; j < OPSP_NUM_BINS; ++j) recapture |= sizes[j] != b->g2_sizes[j];
    void *p = nullptr;
    if (nnz > b->ccap) {
        // grow the C storage (released blocks stay in the library cache)
        if (b->ccol) (void)cache_free(b->ccol, s);
        if (b->cval) (void)cache_free(b->cval, s);
        b->ccol = nullptr;
        b->cval = nullptr;
        b->ccap = 0;
        BCHK(cache_alloc(&p, sizeof(int32_t) * (size_t)nnz, s));
        b->ccol = (int32_t *)p;
        BCHK(cache_alloc(&p, sizeof(double) * (size_t)nnz, s));
        b->cval = (double *)p;
        b->ccap = nnz;
        recapture = true;
    }
    if (sizes[NUM_GLOBAL_BIN] > 0) {
        const int64_t entries = pow2_host(2 * max_nnz > 64 ? 2 * max_nnz : 64);
        const int64_t grid = sizes[NUM_GLOBAL_BIN] < (int64_t)b->cus * NUM_GLOBAL_WG_PER_CU
                                 ? sizes[NUM_GLOBAL_BIN]
                                 : (int64_t)b->cus * NUM_GLOBAL_WG_PER_CU;
        if (entries > b->slab7_entries || grid > b->slab7_grid) {
            if (b->slab7k) (void)cache_free(b->slab7k, s);
            if (b->slab7v) (void)cache_free(b->slab7v, s);
            b->slab7k = nullptr;
            b->slab7v = nullptr;
            BCHK(cache_alloc(&p, sizeof(int) * (size_t)(entries * grid), s));
            b->slab7k = (int *)p;
            BCHK(cache_alloc(&p, sizeof(double) * (size_t)(entries * grid), s));
            b->slab7v = (double *)p;
            b->slab7_entries = entries;
            b->slab7_grid = grid;
            recapture = true;
        }
    }
    if (recapture) {
        opsp_status st = capture_g2(b, sizes, s);
        if (st != OPSP_OK) return st;
        b->g2_nnz = nnz;
    }
    BCHK(hipGraphLaunch(b->g2, s));
    BCHK(join());
    const int64_t *bnd = b->h_bounds();
    for (int q = 0; q < b->count; ++q) {
        C[q].rows = b->desc[q].M;
        C[q].cols = b->N[q];
        C[q].rpt = b->crpt + b->desc[q].row0;
        C[q].col = nnz > 0 ? b->ccol : nullptr;
        C[q].val = nnz > 0 ? b->cval : nullptr;
        const int64_t next = q + 1 < b->count ? bnd[q + 1] : bnd[b->count];
        C[q].nnz = next - bnd[q];
    }
    b->last_nnz = nnz;
    b->last_nprod = (int64_t)hc[0].total;
    b->last_max_nnz = max_nnz;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->nprod = (int64_t)hc[0].total;
        stats->nnz = nnz;
        stats->max_row_nprod = (int64_t)hc[0].maxv;
        stats->max_row_nnz = max_nnz;
        for (int j = 0; j < OPSP_SYM_BINS; ++j) stats->sym_bin_rows[j] = (int64_t)hc[0].size[j];
        stats->sym_bin_rows[SYM_GLOBAL_BIN] += (int64_t)hc[0].fail;
        for (int j = 0; j < OPSP_NUM_BINS; ++j) stats->num_bin_rows[j] = sizes[j];
    }
    return OPSP_OK;
}

void opsp_batch_destroy(opsp_batch *b) {
    if (!b) return;
    if (b->cs) (void)hipStreamSynchronize(b->cs);
    if (b->ccol) (void)cache_free(b->ccol, nullptr);
    if (b->cval) (void)cache_free(b->cval, nullptr);
    if (b->slab7k) (void)cache_free(b->slab7k, nullptr);
    if (b->slab7v) (void)cache_free(b->slab7v, nullptr);
    batch_release(b);
    delete b;
}

opsp_status opsp_spgemm_batched(int32_t count, const opsp_csr *A, const opsp_csr *B, opsp_csr *C,
                                const opsp_config *cfg, opsp_batch **owner, void *stream) {
    if (!owner) return OPSP_ERR_INVALID;
    *owner = nullptr;
    opsp_batch *b = nullptr;
    opsp_status st = opsp_batch_create(count, A, B, cfg, &b, stream);
    if (st != OPSP_OK) return st;
    st = opsp_batch_execute(b, C, nullptr, stream);
    if (st != OPSP_OK) {
        opsp_batch_destroy(b);
        return st;
    }
    *owner = b;
    return OPSP_OK;
}

}  // extern "C"
