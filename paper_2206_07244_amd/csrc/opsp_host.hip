// Host orchestration and the C ABI of opsp (see include/opsp.h).
//
// Flow of one product (OpSparse Section 5, six steps):
//   1 setup      C.rpt allocated; n_prod per row written into it, fused with
//                the first symbolic binning pass (Alg. 1); workspace
//                allocation is stream-ordered and overlaps the kernel.
//   2 sym. bins  second pass (Alg. 2), or the all-in-one-bin shortcut
//                (Alg. 3: rows are their own ids, no list written), decided
//                on the device from the bin sizes.
//   3 symbolic   per-bin kernels, biggest bins first (Section 5.5), launched
//                persistently with their row counts read on the device; bin
//                7 aborts rows into the global-table kernel.
//   4 num. bins  first pass over nnz with the nnz(C) total (Section 5.4);
//                the one read-back of the product (nnz(C), bin sizes).
//   5 alloc+scan C.col/C.val come from the stream-ordered pool while the
//                scan + second pass run (Section 5.4); C.rpt is scanned in
//                place (Section 5.3).
//   6 numeric    per-bin kernels, global-table bin first.
// Every allocation comes from the device's default memory pool with an
// unbounded release threshold, so after warm-up allocation is a pool hit
// and never synchronises the device.
#include <atomic>
#include <mutex>
#include <new>
#include <string.h>

#include "opsp.h"
#include "opsp_internal.h"
#include "opsp_host_util.h"

using namespace opsp;

struct opsp_plan {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t M = 0, K = 0, N = 0;
    int64_t nnzC = 0;
    int64_t max_nnz = 0;
    int64_t *crpt = nullptr;            // C row pointer (owned)
    int32_t *bins = nullptr;            // numeric bins (owned; NULL = identity)
    int64_t num_size[OPSP_NUM_BINS] = {};
    int64_t num_off[OPSP_NUM_BINS] = {};
    int identity_bin = -1;              // bin holding all rows when bins == NULL
    bool check = false;
    int64_t fixed_grid = 0;             // > 0: every bin kernel runs persistently with this grid
    int streams = 1;                    // streams the numeric bin kernels are spread over
    int gv = 0;                         // bin 0 variant (lanes per row, table size)
    bool fp32 = false;                  // FP32 values (opsp_spgemm_f32)
    Counters *ctr = nullptr;            // device counters (numeric step), owned
    int2 *range = nullptr;              // output column range (lo, hi) per row (owned)
    int4 *brec = nullptr;               // B row records with repeated-pattern flags, when
                                        // the numeric step merges such entries (owned)
    opsp_stats stats = {};
};

namespace {
const char *kVersion = "opsp 0.1.0 (gfx950)";
}  // namespace

// Fixed device scratch of opsp_spgemm_numeric_noalloc (the long-row bin's
// staging or global tables).  Every device that loads the library holds its
// own copy until the process ends.  On the host the array's name is not a
// device address: host code uses only the per-device address that
// hipGetSymbolAddress returns (scratch_address below).
static __device__ __align__(256) unsigned char scratch[OPSP_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_addr[64];

// Address of `scratch` on device `dev`, which must be current; looked up once
// per device.
opsp_status scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? OPSP_ERR_ALLOC : OPSP_ERR_HIP;
        if (!p) return OPSP_ERR_HIP;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return OPSP_OK;
}

// A caller-provided device region that replaces the allocations of the
// long-row numeric bin.
struct ScratchBuf {
    char *p;
    int64_t bytes;
};

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }
}  // namespace

namespace opsp {
namespace host {

namespace {
struct DeviceInfo {
    bool ready = false;
    int cus = 256;
    hipStream_t side[MAX_STREAMS - 1] = {};   // library-owned, default priority
    int nside = 0;
};
std::mutex g_mu;
DeviceInfo g_dev[64];

// Per-thread events that fork the bin kernels of a step onto the side
// streams and join them back (created once per device and thread).
struct ForkEvents {
    int dev = -1;
    hipEvent_t ev[MAX_STREAMS] = {};
    bool ok = false;
    bool get(int d) {
        if (dev == d) return ok;
        release();
        dev = d;
        ok = true;
        for (int i = 0; i < MAX_STREAMS; ++i)
            if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
                ev[i] = nullptr;
                ok = false;
            }
        return ok;
    }
    void release() {
        for (int i = 0; i < MAX_STREAMS; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        for (auto &e : ev) e = nullptr;
        dev = -1;
    }
    ~ForkEvents() { release(); }
};
thread_local ForkEvents t_fork;

// Per-thread pinned host buffer for the small counter read-backs.
struct PinnedBuf {
    void *h = nullptr;
    void *get() {
        if (!h && hipHostMalloc(&h, PINNED_BYTES, hipHostMallocDefault) != hipSuccess) h = nullptr;
        return h;
    }
    ~PinnedBuf() {
        if (h) (void)hipHostFree(h);
    }
};
thread_local PinnedBuf t_pinned;
}  // namespace

opsp_status status_of(hipError_t e) {
    if (e == hipSuccess) return OPSP_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return OPSP_ERR_ALLOC;
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return OPSP_ERR_NO_DEVICE;
    return OPSP_ERR_HIP;
}

opsp_status init_device(int *dev_out, int *cus_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return status_of(e);
    if (dev < 0 || dev >= 64) return OPSP_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_dev[dev].ready) {
        hipMemPool_t pool;
        e = hipDeviceGetDefaultMemPool(&pool, dev);
        if (e != hipSuccess) return status_of(e);
        uint64_t thr = UINT64_MAX;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        if (e != hipSuccess) return status_of(e);
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return status_of(e);
        g_dev[dev].cus = cus > 0 ? cus : 256;
        // side streams for concurrent bin kernels; without them every bin
        // runs on the calling stream
        g_dev[dev].nside = 0;
        for (int i = 0; i < MAX_STREAMS - 1; ++i) {
            if (hipStreamCreateWithFlags(&g_dev[dev].side[i], hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                break;
            }
            ++g_dev[dev].nside;
        }
        g_dev[dev].ready = true;
    }
    *dev_out = dev;
    *cus_out = g_dev[dev].cus;
    return OPSP_OK;
}

int streams_of(const opsp_config *c) {
    const int want = (c && c->version >= 3 && c->streams > 0) ? c->streams : DEFAULT_STREAMS;
    return want < MAX_STREAMS ? want : MAX_STREAMS;
}

Fork::Fork(hipStream_t main, int want) : s{main}, n(1) {
    int dev = 0;
    if (want <= 1 || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const int avail = g_dev[dev].nside + 1;
        n = want < avail ? want : avail;
        for (int i = 1; i < n; ++i) s[i] = g_dev[dev].side[i - 1];
    }
    if (n > 1 && !t_fork.get(dev)) n = 1;
    ev = t_fork.ev;
}

hipError_t Fork::begin() {
    if (n <= 1) return hipSuccess;
    hipError_t e = hipEventRecord(ev[0], s[0]);
    for (int i = 1; i < n && e == hipSuccess; ++i) e = hipStreamWaitEvent(s[i], ev[0], 0);
    return e;
}

hipError_t Fork::end() {
    if (n <= 1) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int i = 1; i < n && e == hipSuccess; ++i) {
        e = hipEventRecord(ev[i], s[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s[0], ev[i], 0);
    }
    return e;
}

bool csr_ok(const opsp_csr *X) {
    if (!X) return false;
    if (X->rows < 0 || X->cols < 0 || X->nnz < 0) return false;
    if (!X->rpt) return false;
    if (X->nnz > 0 && (!X->col || !X->val)) return false;
    return true;
}

opsp_status check_inputs(const opsp_csr *A, const opsp_csr *B) {
    if (!csr_ok(A) || !csr_ok(B)) return OPSP_ERR_INVALID;
    if (A->cols != B->rows) return OPSP_ERR_SHAPE;
    if (B->cols > INT32_MAX || A->cols > INT32_MAX) return OPSP_ERR_SHAPE;
    return OPSP_OK;
}

DevCSR dev_of(const opsp_csr *X) {
    return DevCSR{X->rows, X->cols, X->rpt, X->col, X->val};
}

double sym_ratio(const opsp_config *c) { return (c && c->sym_ratio > 0) ? c->sym_ratio : 1.2; }
double num_ratio(const opsp_config *c) { return (c && c->num_ratio > 0) ? c->num_ratio : 2.0; }

// Upper bounds by the ratio rule of Section 5.7.
int64_t bound_for(int step, int64_t t, double ratio) {
    const double x = step == 0 ? (double)t : (double)(t + 1);
    int64_t b = (int64_t)(x / ratio + 1e-9);
    // guard against the division landing just above an integer
    while (b > 0 && (double)b * ratio > x + 1e-9) --b;
    if (step == 1 && b > t) b = t;
    return b;
}

int gv_of(const opsp_config *c) {
    return (c && c->version >= 3) ? group_variant(c->group_lanes) : 0;
}

Bounds make_bounds(int step, double ratio, int force, int gv) {
    Bounds b;
    memset(&b, 0, sizeof(b));
    b.span_bin = -1;
    if (step == 0) {
        b.nb = SYM_NLDS;                    // bins 0..7 natural; 8 only by force
        // rows whose output range fits the one-wave kernel's bitmap (32 bits
        // per table word) go to bin 1 up to 2^13 products (one wave walks
        // them in at most 128 windows of 64)
        b.span_bin = 1;
        b.span_max = 32ll * SYM_T[1];
        b.span_nprod_max = 1ll << 13;
        for (int j = 0; j < SYM_NLDS - 1; ++j) b.ub[j] = bound_for(0, j ? SYM_T[j] : SYM_T0[gv], ratio);
        b.nslots = SYM_NLDS + 1;
    } else {
        b.nb = NUM_NLDS + 1;                // bins 0..6 LDS, 7 global
        for (int j = 0; j < NUM_NLDS; ++j) b.ub[j] = bound_for(1, j ? NUM_T[j] : NUM_T0[gv], ratio);
        b.nslots = NUM_NLDS + 1;
    }
    b.force = force;
    return b;
}

Bounds config_bounds(int step, const opsp_config *c, int gv) {
    const int force = c ? (step == 0 ? c->force_sym_bin : c->force_num_bin) : -1;
    Bounds b = make_bounds(step, step == 0 ? sym_ratio(c) : num_ratio(c), force, gv);
    if (c && c->version >= 2) {
        const int64_t *eb = step == 0 ? c->sym_bounds : c->num_bounds;
        for (int j = 0; j < 7; ++j)
            if (eb[j] != 0) b.ub[j] = eb[j];
    }
    return b;
}

opsp_status check_config(const opsp_config *c) {
    if (!c) return OPSP_OK;
    if (c->version < 1 || c->version > 3) return OPSP_ERR_INVALID;
    if (c->version >= 3 && (c->streams < 0 || c->streams > MAX_STREAMS)) return OPSP_ERR_INVALID;
    if (c->version >= 3 && group_variant(c->group_lanes) < 0) return OPSP_ERR_INVALID;
    const int gv = gv_of(c);
    if (c->sym_ratio != 0 && !(c->sym_ratio >= 1.0)) return OPSP_ERR_INVALID;
    if (c->num_ratio != 0 && !(c->num_ratio >= 1.0)) return OPSP_ERR_INVALID;
    if (c->force_sym_bin < -1 || c->force_sym_bin > SYM_GLOBAL_BIN) return OPSP_ERR_INVALID;
    if (c->force_num_bin < -1 || c->force_num_bin > NUM_GLOBAL_BIN) return OPSP_ERR_INVALID;
    if (c->b_lanes != 0) return OPSP_ERR_INVALID;
    if (c->version >= 2) {
        for (int j = 0; j < 7; ++j) {
            if (c->sym_bounds[j] < -1 || c->sym_bounds[j] > (j ? SYM_T[j] : SYM_T0[gv])) return OPSP_ERR_INVALID;
            if (c->num_bounds[j] < -1 || c->num_bounds[j] > (j ? NUM_T[j] : NUM_T0[gv])) return OPSP_ERR_INVALID;
        }
    }
    return OPSP_OK;
}

hipError_t read_back(void *dst, const void *src, size_t bytes, hipStream_t s) {
    void *pin = bytes <= PINNED_BYTES ? t_pinned.get() : nullptr;
    if (!pin) {
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    }
    hipError_t e = hipMemcpyAsync(pin, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) memcpy(dst, pin, bytes);
    return e;
}

hipError_t read_counters(Counters *dst, const Counters *src, size_t count, hipStream_t s) {
    return read_back(dst, src, sizeof(Counters) * count, s);
}


opsp_status validate_csr(const opsp_csr *const *X, int n, hipStream_t s) {
    Arena ar(s);
    void *p = nullptr;
    CHK(ar.alloc(&p, sizeof(unsigned int) * (size_t)(n > 0 ? n : 1)));
    unsigned int *flags = (unsigned int *)p;
    CHK(hipMemsetAsync(flags, 0, sizeof(unsigned int) * (size_t)n, s));
    for (int k = 0; k < n; ++k)
        CHK(launch_check_csr(X[k]->rows, X[k]->cols, X[k]->nnz, X[k]->rpt, X[k]->col, flags + k, s));
    unsigned int h[64];
    for (int k0 = 0; k0 < n; k0 += 64) {
        const int m = n - k0 < 64 ? n - k0 : 64;
        CHK(read_back(h, flags + k0, sizeof(unsigned int) * (size_t)m, s));
        for (int k = 0; k < m; ++k)
            if (h[k]) return OPSP_ERR_INVALID;
    }
    return OPSP_OK;
}

RowSrc host_rows(const int32_t *bins, int64_t off, int64_t nrows) {
    RowSrc r;
    memset(&r, 0, sizeof(r));
    r.bins = bins;
    r.off = off;
    r.nrows = nrows;
    return r;
}

}  // namespace host
}  // namespace opsp

using namespace opsp::host;

namespace {

// Steps 1-5: everything up to C's row pointer and the numeric bins.
opsp_status run_symbolic(const opsp_csr *A, const opsp_csr *B, const opsp_config *cfg,
                         hipStream_t s, opsp_plan *plan, Timer &tm) {
    int dev = 0, cus = 256;
    opsp_status st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    const int64_t M = A->rows, N = B->cols;
    plan->device = dev;
    plan->stream = s;
    plan->M = M;
    plan->K = A->cols;
    plan->N = N;
    plan->check = cfg && cfg->validate;
    plan->fixed_grid = cfg ? cfg->fixed_grid : 0;
    plan->streams = streams_of(cfg);
    if (plan->check) {
        const opsp_csr *X[2] = {A, B};
        opsp_status vs = validate_csr(X, 2, s);
        if (vs != OPSP_OK) return vs;
    }

    Arena ar(s);
    void *p = nullptr;
    CHK(ar.alloc(&p, sizeof(int64_t) * (size_t)(M + 1)));
    int64_t *crpt = (int64_t *)p;
    CHK(ar.alloc(&p, sizeof(Counters) * 2));
    Counters *ctrS = (Counters *)p, *ctrN = ctrS + 1;
    if (M == 0) {
        CHK(hipMemsetAsync(ctrS, 0, sizeof(Counters) * 2, s));
        CHK(hipMemsetAsync(crpt, 0, sizeof(int64_t), s));
        ar.keep(crpt);
        ar.keep(ctrS);
        plan->crpt = crpt;
        plan->ctr = ctrN;
        return OPSP_OK;
    }
    const int64_t nblk = (M + 255) / 256;
    CHK(ar.alloc(&p, sizeof(int32_t) * (size_t)M));
    int32_t *bins = (int32_t *)p;
    // output column range per row (narrow rows avoid the hash tables), from
    // the first and last column of every row of B
    int2 *rng = nullptr;
    int4 *bfl = nullptr;
    if (!(cfg && cfg->version >= 2 && cfg->hash_all_rows)) {
        CHK(ar.alloc(&p, sizeof(int2) * (size_t)M));
        rng = (int2 *)p;
        CHK(ar.alloc(&p, sizeof(int4) * (size_t)(B->rows > 0 ? B->rows : 1)));
        bfl = (int4 *)p;
    }
    CHK(ar.alloc(&p, block_parts_bytes(M, A->nnz)));
    const BlockParts parts = block_parts_at(p, M, A->nnz);

    const int gv = gv_of(cfg);
    plan->gv = gv;
    const Bounds bs = config_bounds(0, cfg, gv);
    const Bounds bn = config_bounds(1, cfg, gv);
    const DevCSR dA = dev_of(A), dB = dev_of(B);

    // 1 setup + first symbolic binning pass
    tm.mark();
    // rows that repeat the previous entry's B-row pattern are skipped when B
    // looks like a matrix of node blocks (long rows: 3 unknowns of a 27-point
    // node give 81); elsewhere the check would cost more than it finds
    const bool dup = bfl && B->nnz >= DUP_MIN_AVG * B->rows;
    if (bfl) CHK(launch_brange(dB, bfl, dup, &ctrS->dups, s));
    CHK(launch_setup(dA, dB, crpt, bs, parts, nullptr, nullptr, s, bfl, rng));
    tm.mark();   // setup (with the first binning pass fused in) done
    CHK(launch_finalize(M, bs.nslots, parts, ctrS, nullptr, false, s));

    // 2 second pass; the all-rows-in-one-bin case (Alg. 3) is decided on the
    //   device: no list is written and the bin kernel reads rows in order
    CHK(launch_scatter(M, crpt, bs, ctrS, bins, parts, false, s, nullptr, true, rng));
    tm.mark();

    // 3 symbolic, biggest bins first.  The bin sizes stay on the device:
    //   every bin kernel is launched persistently and reads its row count
    //   from the counters, so the host does not wait here (Section 5.5: no
    //   synchronisation until every kernel is launched).  Only global hash
    //   tables (matrices without a usable column range) are sized from the
    //   largest n_prod, which takes one read-back.
    SymArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.A = dA;
    sa.B = dB;
    sa.nnz = crpt;
    sa.ctr = ctrS;
    sa.rng = rng;
    sa.gv = gv;
    sa.brec = dup ? bfl : nullptr;
    // rows of A with the columns of the row before them (the rows of one
    // node) have the same count: only the first row of each run is counted,
    // and the others copy it after the symbolic bins
    uint8_t *arun = nullptr;
    if (bfl && M > 1 && A->nnz >= DUP_MIN_AVG * M) {
        const bool one = dup && A->rpt == B->rpt && A->col == B->col && A->rows == B->rows;
        uint8_t *same = nullptr;
        if (!one) {
            CHK(ar.alloc(&p, (size_t)M));
            same = (uint8_t *)p;
        }
        CHK(ar.alloc(&p, (size_t)M));
        arun = (uint8_t *)p;
        CHK(launch_arun(dA, one ? bfl : nullptr, same, arun, s));
    }
    sa.arun = arun;
    const bool need_slab = !rng || N > ((int64_t)SW_MAXPASS << SW_LG);
    int *slab = nullptr;
    int64_t slab_entries = 0;
    const int64_t sgrid = M < (int64_t)cus * SYM_GLOBAL_WG_PER_CU ? M : (int64_t)cus * SYM_GLOBAL_WG_PER_CU;
    if (need_slab) {
        Counters hS;
        CHK(read_counters(&hS, ctrS, 1, s));
        const int64_t bound = (int64_t)hS.maxv < N ? (int64_t)hS.maxv : N;
        slab_entries = pow2_host(2 * bound > 64 ? 2 * bound : 64);
    }
    int32_t *fail_list = nullptr;
    CHK(ar.alloc(&p, sizeof(int32_t) * (size_t)M));   // rows abandoned by bin 7 (at most all)
    fail_list = (int32_t *)p;
    auto grid_of = [&](int b) -> int64_t {
        if (plan->fixed_grid > 0) return plan->fixed_grid;
        const int64_t R = sym_rows_per_wg(b, gv);
        const int64_t need = (M + R - 1) / R;
        const int64_t g = (int64_t)cus * sym_wg_per_cu(b);
        return g < need ? g : need;
    };
    auto global_args = [&](const RowSrc &src) {
        SymArgs g = sa;
        g.src = src;
        g.slab = slab;
        g.slab_entries = slab_entries;
        g.sched = ctrS->sched;
        g.grid = sgrid;
        return g;
    };
    Fork fk(s, plan->streams);
    CHK(fk.begin());
    for (int b = 7; b >= 0; --b) {
        memset(&sa.src, 0, sizeof(sa.src));
        sa.src.bins = bins;
        sa.src.dctr = ctrS;
        sa.src.bin = b;
        sa.src.all = M;
        sa.grid = grid_of(b);
        if (b == 7) {
            const double frac = cfg && cfg->sym_abort_fraction != 0 ? cfg->sym_abort_fraction : 0.8;
            int64_t thr = frac < 0 ? -1 : (int64_t)(frac * SYM_T[7]);
            const int64_t cap = SYM_T[7] - SYM_W[7] - 1;
            if (thr > cap) thr = cap;
            sa.abort_thr = (int)thr;
            sa.fail_list = fail_list;
        }
        CHK(launch_symbolic_bin(b, sa, fk.on(b, 7)));
        if (b == 7) {
            // the global-table allocation overlaps the bin-7 kernel (Section 5.4)
            if (slab_entries > 0) {
                CHK(ar.alloc(&p, sizeof(int) * (size_t)(slab_entries * sgrid)));
                slab = (int *)p;
            }
            RowSrc fr;
            memset(&fr, 0, sizeof(fr));
            fr.bins = fail_list;
            fr.count = &ctrS->fail;
            CHK(launch_symbolic_bin(SYM_GLOBAL_BIN, global_args(fr), s));
        }
    }
    if (bs.force == SYM_GLOBAL_BIN) {
        // rows routed straight to the global tables
        RowSrc gr;
        memset(&gr, 0, sizeof(gr));
        gr.bins = bins;
        gr.dctr = ctrS;
        gr.bin = SYM_GLOBAL_BIN;
        gr.all = M;
        CHK(launch_symbolic_bin(SYM_GLOBAL_BIN, global_args(gr), s));
    }
    CHK(fk.end());
    if (arun) CHK(launch_arun_copy(M, arun, crpt, s));
    tm.mark();

    // 4 numeric binning, first pass with nnz(C)
    CHK(launch_hist(M, crpt, bn, parts, s));
    CHK(launch_finalize(M, bn.nslots, parts, ctrN, crpt + M, true, s));
    Counters hc[2];
    CHK(read_counters(hc, ctrS, 2, s));   // the one wait of the product
    const Counters &hN = hc[1];
    plan->stats.nprod = (int64_t)hc[0].total;
    plan->stats.max_row_nprod = (int64_t)hc[0].maxv;
    for (int j = 0; j < bs.nslots; ++j)
        plan->stats.sym_bin_rows[j < OPSP_SYM_BINS ? j : OPSP_SYM_BINS - 1] = (int64_t)hc[0].size[j];
    plan->nnzC = (int64_t)hN.total;
    plan->max_nnz = (int64_t)hN.maxv;
    plan->stats.nnz = plan->nnzC;
    plan->stats.max_row_nnz = plan->max_nnz;
    if (plan->max_nnz > INT32_MAX) return OPSP_ERR_OVERFLOW;
    plan->stats.sym_bin_rows[SYM_GLOBAL_BIN] += (int64_t)hc[0].fail;

    // 5 scan C.rpt in place + numeric bins
    int identity = -1;
    for (int j = 0; j < bn.nslots; ++j) {
        plan->num_size[j] = (int64_t)hN.size[j];
        plan->stats.num_bin_rows[j] = plan->num_size[j];
        if (plan->num_size[j] == M) identity = j;
    }
    for (int j = 1; j < bn.nslots; ++j) plan->num_off[j] = plan->num_off[j - 1] + plan->num_size[j - 1];
    CHK(launch_scatter(M, crpt, bn, ctrN, identity >= 0 ? nullptr : bins, parts, true, s));
    tm.mark();
    ar.keep(crpt);
    ar.keep(ctrS);
    if (rng) ar.keep(rng);
    plan->range = rng;
    // the numeric bins merge runs of repeated B rows only when at least a
    // third of B's rows repeat the row before them: the merged kernels cost
    // more registers and lane permutes per window (wide rows without
    // repeats: numeric 3.3 -> 5.1 ms), and pay off on node blocks (two
    // thirds repeated: 4.5 -> 2.3 ms)
    const bool merge = dup && hc[0].dups * 3 >= (unsigned long long)B->rows;
    if (merge) ar.keep(bfl);
    plan->brec = merge ? bfl : nullptr;
    if (identity < 0) ar.keep(bins);
    plan->identity_bin = identity;
    plan->crpt = crpt;
    plan->bins = identity >= 0 ? nullptr : bins;
    plan->ctr = ctrN;
    return OPSP_OK;
}

// Step 6 into caller-visible C arrays.
// With `scr`, the long-row bin works in that region (its grid cut to fit)
// instead of allocating; OPSP_ERR_SCRATCH when one workgroup's share does
// not fit.
opsp_status run_numeric(opsp_plan *plan, const opsp_csr *A, const opsp_csr *B, int32_t *ccol,
                        double *cval, hipStream_t s, Timer *kt = nullptr,
                        const ScratchBuf *scr = nullptr) {
    int dev = 0, cus = 256;
    opsp_status st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    if (plan->M == 0 || plan->nnzC == 0) return OPSP_OK;
    Arena ar(s);
    NumArgs na;
    memset(&na, 0, sizeof(na));
    na.gv = plan->gv;
    na.fp32 = plan->fp32 ? 1 : 0;
    const size_t vsize = plan->fp32 ? sizeof(float) : sizeof(double);
    na.A = dev_of(A);
    na.B = dev_of(B);
    na.crpt = plan->crpt;
    na.ccol = ccol;
    na.cval = cval;
    na.ctr = plan->ctr;
    na.rng = plan->range;
    na.brec = plan->brec;
    const int gb = NUM_GLOBAL_BIN;
    bool first = true;
    void *pk = nullptr, *pv = nullptr;
    Fork fk(s, scr ? 1 : plan->streams);
    CHK(fk.begin());
    for (int b = gb; b >= 0; --b) {
        const int64_t rows = plan->num_size[b];
        if (rows == 0) continue;
        na.src = host_rows((plan->identity_bin == b) ? nullptr : plan->bins,
                           (plan->identity_bin == b) ? 0 : plan->num_off[b], rows);
        na.grid = 0;
        if (plan->fixed_grid > 0 && b == 0) na.grid = plan->fixed_grid < rows ? plan->fixed_grid : rows;
        if (b == gb && plan->range && plan->N <= BUCKET_MAX_COLS) {
            // bucketed dense accumulation: staging for the largest n_prod per
            // workgroup, within the staging budget
            // (+1: the spare entry of lanes without a product)
            const int64_t cap = (plan->stats.max_row_nprod > 1 ? plan->stats.max_row_nprod : 1) + 1;
            int64_t grid = rows < (int64_t)cus * BUCKET_WG_PER_CU ? rows : (int64_t)cus * BUCKET_WG_PER_CU;
            const int64_t fit = STAGING_BUDGET / (cap * 12);
            if (grid > fit) grid = fit > 1 ? fit : 1;
            if (scr) {
                const int64_t g = (scr->bytes - 256) / (cap * 12);
                if (g < 1) return OPSP_ERR_SCRATCH;
                if (grid > g) grid = g;
                pk = scr->p;
                pv = scr->p + align256(cap * grid * (int64_t)sizeof(int));
            } else {
                CHK(ar.alloc(&pk, sizeof(int) * (size_t)(cap * grid)));
                CHK(ar.alloc(&pv, vsize * (size_t)(cap * grid)));
            }
            na.slab_keys = (int *)pk;
            na.slab_vals = (double *)pv;
            na.slab_entries = cap;
            na.grid = grid;
            if (kt) kt->mark();
            CHK(launch_numeric_bucket(na, s));
            if (kt) kt->mark();
            first = false;
            continue;
        }
        if (b == gb) {
            const int64_t entries = pow2_host(2 * plan->max_nnz > 64 ? 2 * plan->max_nnz : 64);
            int64_t grid = rows < (int64_t)cus * NUM_GLOBAL_WG_PER_CU ? rows : (int64_t)cus * NUM_GLOBAL_WG_PER_CU;
            if (scr) {
                const int64_t g = (scr->bytes - 256) / (entries * 12);
                if (g < 1) return OPSP_ERR_SCRATCH;
                if (grid > g) grid = g;
                pk = scr->p;
                pv = scr->p + align256(entries * grid * (int64_t)sizeof(int));
            } else {
                CHK(ar.alloc(&pk, sizeof(int) * (size_t)(entries * grid)));
                CHK(ar.alloc(&pv, sizeof(double) * (size_t)(entries * grid)));   // FP64 sums
            }
            na.slab_keys = (int *)pk;
            na.slab_vals = (double *)pv;
            na.slab_entries = entries;
            na.grid = grid;
        }
        if (kt && b == gb) kt->mark();
        CHK(launch_numeric_bin(b, na, fk.on(b, gb)));
        if (kt && b == gb) kt->mark();
        first = false;
    }
    (void)first;
    CHK(fk.end());
    return OPSP_OK;
}

opsp_status check_errors(opsp_plan *plan, hipStream_t s) {
    if (!plan->ctr) return OPSP_OK;
    Counters h[2];   // symbolic and numeric counters share one allocation
    CHK(read_counters(h, plan->ctr - 1, 2, s));
    return (h[0].error || h[1].error) ? OPSP_ERR_INTERNAL : OPSP_OK;
}

void plan_release(opsp_plan *plan, hipStream_t s) {
    if (!plan) return;
    if (plan->crpt) (void)cache_free(plan->crpt, s);
    if (plan->bins) (void)cache_free(plan->bins, s);
    if (plan->range) (void)cache_free(plan->range, s);
    plan->range = nullptr;
    if (plan->brec) (void)cache_free(plan->brec, s);
    plan->brec = nullptr;
    if (plan->ctr) (void)cache_free(plan->ctr - 1, s);  // both counters share one allocation
    plan->crpt = nullptr;
    plan->bins = nullptr;
    plan->ctr = nullptr;
}

}  // namespace

// ===========================================================================
extern "C" {

const char *opsp_version(void) { return kVersion; }

const char *opsp_status_string(opsp_status s) {
    switch (s) {
        case OPSP_OK: return "OPSP_OK";
        case OPSP_ERR_INVALID: return "OPSP_ERR_INVALID: invalid argument";
        case OPSP_ERR_SHAPE: return "OPSP_ERR_SHAPE: incompatible or oversized shapes";
        case OPSP_ERR_ALLOC: return "OPSP_ERR_ALLOC: device allocation failed";
        case OPSP_ERR_OVERFLOW: return "OPSP_ERR_OVERFLOW: count exceeds its index type";
        case OPSP_ERR_HIP: return "OPSP_ERR_HIP: HIP runtime error";
        case OPSP_ERR_INTERNAL: return "OPSP_ERR_INTERNAL: internal consistency check failed";
        case OPSP_ERR_NO_DEVICE: return "OPSP_ERR_NO_DEVICE: no usable device";
        case OPSP_ERR_SCRATCH:
            return "OPSP_ERR_SCRATCH: the product needs more than the fixed scratch of the "
                   "no-allocation entry point";
    }
    return "unknown opsp status";
}

}  // extern "C"

namespace {
// The whole two-phase product; values are FP64, or FP32 when `fp32` (the
// val pointers of A, B and C then point to float).
opsp_status two_phase(const opsp_csr *A, const opsp_csr *B, opsp_csr *C, const opsp_config *config,
                      opsp_stats *stats, void *stream, bool fp32) {
    if (!C) return OPSP_ERR_INVALID;
    memset(C, 0, sizeof(*C));
    opsp_status st = check_inputs(A, B);
    if (st != OPSP_OK) return st;
    st = check_config(config);
    if (st != OPSP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    opsp_plan plan;
    plan.fp32 = fp32;
    Timer tm(config && config->stage_timing, s);
    st = run_symbolic(A, B, config, s, &plan, tm);
    if (st != OPSP_OK) {
        plan_release(&plan, s);
        return st;
    }
    void *pc = nullptr, *pv = nullptr;
    if (plan.nnzC > 0) {
        hipError_t e = cache_alloc(&pc, sizeof(int32_t) * (size_t)plan.nnzC, s);
        if (e == hipSuccess) e = cache_alloc(&pv, (fp32 ? sizeof(float) : sizeof(double)) * (size_t)plan.nnzC, s);
        if (e != hipSuccess) {
            if (pc) (void)cache_free(pc, s);
            plan_release(&plan, s);
            return status_of(e);
        }
    }
    Timer kt(tm.on, s);
    st = run_numeric(&plan, A, B, (int32_t *)pc, (double *)pv, s, &kt);
    tm.mark();
    if (st == OPSP_OK && plan.check) st = check_errors(&plan, s);
    if (st != OPSP_OK) {
        if (pc) (void)cache_free(pc, s);
        if (pv) (void)cache_free(pv, s);
        plan_release(&plan, s);
        return st;
    }
    C->rows = A->rows;
    C->cols = B->cols;
    C->nnz = plan.nnzC;
    C->rpt = plan.crpt;
    C->col = (int32_t *)pc;
    C->val = (double *)pv;
    plan.crpt = nullptr;  // ownership moves to the caller
    if (stats) {
        *stats = plan.stats;
        if (tm.on) {
            (void)hipStreamSynchronize(s);
            // marks: 0 start, 1 setup kernel, 2 symbolic binning, 3 symbolic,
            // 4 numeric binning + scan + allocation, 5 numeric
            stats->ms_stage[0] = tm.between(0, 2);
            for (int k = 1; k < 4; ++k) stats->ms_stage[k] = tm.between(k + 1, k + 2);
            stats->ms_stage[4] = tm.between(0, 5);
            stats->ms_stage[5] = kt.between(0, 1);
            stats->ms_stage[6] = tm.between(0, 1);
        }
    }
    plan_release(&plan, s);
    return OPSP_OK;
}
}  // namespace

extern "C" {

opsp_status opsp_spgemm_ex(const opsp_csr *A, const opsp_csr *B, opsp_csr *C,
                           const opsp_config *config, opsp_stats *stats, void *stream) {
    return two_phase(A, B, C, config, stats, stream, false);
}

// The FP32 structs differ from opsp_csr only in the element type of val.
static_assert(sizeof(opsp_csr_f32) == sizeof(opsp_csr), "layouts");

opsp_status opsp_spgemm_f32(const opsp_csr_f32 *A, const opsp_csr_f32 *B, opsp_csr_f32 *C,
                            const opsp_config *config, opsp_stats *stats, void *stream) {
    if (!C) return OPSP_ERR_INVALID;
    opsp_csr a, b, c;
    memset(&c, 0, sizeof(c));
    const opsp_csr *pa = nullptr, *pb = nullptr;
    if (A) {
        a = opsp_csr{A->rows, A->cols, A->nnz, A->rpt, A->col, (double *)(void *)A->val};
        pa = &a;
    }
    if (B) {
        b = opsp_csr{B->rows, B->cols, B->nnz, B->rpt, B->col, (double *)(void *)B->val};
        pb = &b;
    }
    const opsp_status st = two_phase(pa, pb, &c, config, stats, stream, true);
    C->rows = c.rows;
    C->cols = c.cols;
    C->nnz = c.nnz;
    C->rpt = c.rpt;
    C->col = c.col;
    C->val = (float *)(void *)c.val;
    return st;
}

opsp_status opsp_csr_f32_free(opsp_csr_f32 *C, void *stream) {
    if (!C) return OPSP_ERR_INVALID;
    opsp_csr c{C->rows, C->cols, C->nnz, C->rpt, C->col, (double *)(void *)C->val};
    const opsp_status st = opsp_csr_free(&c, stream);
    memset(C, 0, sizeof(*C));
    return st;
}

opsp_status opsp_spgemm(const opsp_csr *A, const opsp_csr *B, opsp_csr *C, void *stream) {
    return opsp_spgemm_ex(A, B, C, nullptr, nullptr, stream);
}

opsp_status opsp_spgemm_symbolic(const opsp_csr *A, const opsp_csr *B, const opsp_config *config,
                                 opsp_plan **plan_out, int64_t *nnzC, void *stream) {
    if (!plan_out || !nnzC) return OPSP_ERR_INVALID;
    *plan_out = nullptr;
    *nnzC = 0;
    opsp_status st = check_inputs(A, B);
    if (st != OPSP_OK) return st;
    st = check_config(config);
    if (st != OPSP_OK) return st;
    opsp_plan *plan = new (std::nothrow) opsp_plan();
    if (!plan) return OPSP_ERR_ALLOC;
    hipStream_t s = (hipStream_t)stream;
    Timer tm(false, s);
    st = run_symbolic(A, B, config, s, plan, tm);
    if (st != OPSP_OK) {
        plan_release(plan, s);
        delete plan;
        return st;
    }
    *plan_out = plan;
    *nnzC = plan->nnzC;
    return OPSP_OK;
}

opsp_status opsp_spgemm_numeric(opsp_plan *plan, const opsp_csr *A, const opsp_csr *B,
                                opsp_csr *C, void *stream) {
    if (!plan || !C) return OPSP_ERR_INVALID;
    opsp_status st = check_inputs(A, B);
    if (st != OPSP_OK) return st;
    if (A->rows != plan->M || A->cols != plan->K || B->cols != plan->N) return OPSP_ERR_SHAPE;
    hipStream_t s = (hipStream_t)stream;
    plan->stream = s;
    const int64_t nnz = plan->nnzC;
    void *pr = C->rpt, *pc = C->col, *pv = C->val;
    const bool own_r = !pr, own_c = !pc && nnz > 0, own_v = !pv && nnz > 0;
    hipError_t e = hipSuccess;
    if (own_r) e = cache_alloc(&pr, sizeof(int64_t) * (size_t)(plan->M + 1), s);
    if (e == hipSuccess && own_c) e = cache_alloc(&pc, sizeof(int32_t) * (size_t)nnz, s);
    if (e == hipSuccess && own_v) e = cache_alloc(&pv, sizeof(double) * (size_t)nnz, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pr, plan->crpt, sizeof(int64_t) * (size_t)(plan->M + 1),
                           hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
        if (own_r && pr) (void)cache_free(pr, s);
        if (own_c && pc) (void)cache_free(pc, s);
        if (own_v && pv) (void)cache_free(pv, s);
        return status_of(e);
    }
    st = run_numeric(plan, A, B, (int32_t *)pc, (double *)pv, s);
    if (st == OPSP_OK && plan->check) st = check_errors(plan, s);
    if (st != OPSP_OK) {
        if (own_r) (void)cache_free(pr, s);
        if (own_c) (void)cache_free(pc, s);
        if (own_v) (void)cache_free(pv, s);
        return st;
    }
    C->rows = plan->M;
    C->cols = plan->N;
    C->nnz = nnz;
    C->rpt = (int64_t *)pr;
    C->col = (int32_t *)pc;
    C->val = (double *)pv;
    return OPSP_OK;
}

opsp_status opsp_spgemm_numeric_noalloc(opsp_plan *plan, const opsp_csr *A, const opsp_csr *B,
                                        opsp_csr *C, void *stream) {
    if (!plan || !C) return OPSP_ERR_INVALID;
    opsp_status st = check_inputs(A, B);
    if (st != OPSP_OK) return st;
    if (A->rows != plan->M || A->cols != plan->K || B->cols != plan->N) return OPSP_ERR_SHAPE;
    const int64_t nnz = plan->nnzC;
    if (!C->rpt || (nnz > 0 && (!C->col || !C->val))) return OPSP_ERR_INVALID;
    int dev = 0, cus = 256;
    st = init_device(&dev, &cus);
    if (st != OPSP_OK) return st;
    if (dev != plan->device) return OPSP_ERR_INVALID;
    void *base = nullptr;
    st = scratch_address(dev, &base);
    if (st != OPSP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    CHK(hipMemcpyAsync(C->rpt, plan->crpt, sizeof(int64_t) * (size_t)(plan->M + 1),
                       hipMemcpyDeviceToDevice, s));
    const ScratchBuf sb{(char *)base, (int64_t)OPSP_NOALLOC_SCRATCH_BYTES};
    st = run_numeric(plan, A, B, C->col, C->val, s, nullptr, &sb);
    if (st != OPSP_OK) return st;
    C->rows = plan->M;
    C->cols = plan->N;
    C->nnz = nnz;
    return OPSP_OK;
}

void opsp_plan_destroy(opsp_plan *plan) {
    if (!plan) return;
    plan_release(plan, plan->stream);
    delete plan;
}

opsp_status opsp_csr_free(opsp_csr *C, void *stream) {
    if (!C) return OPSP_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess, e2;
    if (C->rpt && (e2 = cache_free(C->rpt, s)) != hipSuccess) e = e2;
    if (C->col && (e2 = cache_free(C->col, s)) != hipSuccess) e = e2;
    if (C->val && (e2 = cache_free(C->val, s)) != hipSuccess) e = e2;
    memset(C, 0, sizeof(*C));
    return status_of(e);
}

opsp_status opsp_table_sizes(int32_t step, int64_t *out, int32_t n) {
    if (!out) return OPSP_ERR_INVALID;
    if (step == 0) {
        if (n < OPSP_SYM_BINS) return OPSP_ERR_INVALID;
        for (int j = 0; j < SYM_NLDS; ++j) out[j] = SYM_T[j];
        out[SYM_GLOBAL_BIN] = -1;
        return OPSP_OK;
    }
    if (step == 1) {
        if (n < OPSP_NUM_BINS) return OPSP_ERR_INVALID;
        for (int j = 0; j < NUM_NLDS; ++j) out[j] = NUM_T[j];
        out[NUM_GLOBAL_BIN] = -1;
        return OPSP_OK;
    }
    return OPSP_ERR_INVALID;
}

opsp_status opsp_bin_bounds(int32_t step, const int64_t *tsize, int32_t n, double ratio,
                            int64_t *out) {
    if (!tsize || !out || n < 1 || (step != 0 && step != 1) || !(ratio >= 1.0)) return OPSP_ERR_INVALID;
    for (int j = 0; j < n - 1; ++j) out[j] = bound_for(step, tsize[j], ratio);
    return OPSP_OK;
}

}  // extern "C"
