// Host-side helpers shared by the entry points of the library (internal).
#pragma once

#include <string.h>

#include "opsp.h"
#include "opsp_internal.h"

namespace opsp {
namespace host {

constexpr size_t PINNED_BYTES = 4096;   // per-thread pinned read-back buffer
constexpr int MAX_STREAMS = 4;           // calling stream + library side streams
// Bins on the calling stream only by default: spread over four streams the
// bin kernels measured slower on one MI355X (R-MAT 2^20 squared 411 -> 416
// ms, the 27-point stencil 3.98 -> 4.27 ms, the 64x64 Laplacian 0.11 -> 0.22
// ms): the persistent long-row kernels fill every CU and the side-stream
// kernels only delay their workgroups.
constexpr int DEFAULT_STREAMS = 1;

// The bin kernels of one step spread over the calling stream and up to
// MAX_STREAMS - 1 side streams: begin() makes the side streams wait for the
// work queued so far on the calling stream, end() makes the calling stream
// wait for the side streams.  Bin b runs on on(b): the longest-row bin on the
// calling stream, the others round-robin on the side streams.
struct Fork {
    hipStream_t s[MAX_STREAMS];
    int n;
    hipEvent_t *ev = nullptr;
    Fork(hipStream_t main, int want);
    hipError_t begin();
    hipError_t end();
    hipStream_t on(int bin, int longest) const {
        return (n <= 1 || bin >= longest) ? s[0] : s[1 + (longest - 1 - bin) % (n - 1)];
    }
};
// Streams a configuration asks for (1..MAX_STREAMS).
int streams_of(const opsp_config *c);

opsp_status status_of(hipError_t e);
// Current device and its compute-unit count; first use per device raises the
// release threshold of its default memory pool.
opsp_status init_device(int *dev_out, int *cus_out);
bool csr_ok(const opsp_csr *X);
opsp_status check_inputs(const opsp_csr *A, const opsp_csr *B);
DevCSR dev_of(const opsp_csr *X);
double sym_ratio(const opsp_config *c);
double num_ratio(const opsp_config *c);
int64_t bound_for(int step, int64_t t, double ratio);
// Bin bounds of step 0 (symbolic) or 1 (numeric) for a ratio (Section 5.7).
Bounds make_bounds(int step, double ratio, int force, int gv = 0);
// Bin 0 variant of a configuration (GROUP_GL / SYM_T0 / NUM_T0).
int gv_of(const opsp_config *c);
// Bin bounds of a step from a (checked) configuration: ratio rule, explicit
// per-bin bounds of version-2 configurations, forced bin.
Bounds config_bounds(int step, const opsp_config *c, int gv);
// Version, ratios, forced bins and explicit bounds of a configuration.
opsp_status check_config(const opsp_config *c);
// Device-to-host copy of a few bytes followed by a stream synchronisation.
hipError_t read_back(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t read_counters(Counters *dst, const Counters *src, size_t count, hipStream_t s);
RowSrc host_rows(const int32_t *bins, int64_t off, int64_t nrows);
// Validation mode: checks on the device that each of the `n` matrices is
// canonical CSR (monotone row pointer covering exactly nnz entries, column
// indices in range and strictly ascending per row) before anything gathers
// through them; OPSP_ERR_INVALID if one is not.  Blocks the host once.
opsp_status validate_csr(const opsp_csr *const *X, int n, hipStream_t s);
// Bytes the bucketed long-row kernel may take for staging.  Fixed, so that
// repeated products request the same block from the allocation cache (a
// budget following the free memory made the request size drift between
// calls and the cache free and re-map tens of GB each time).
constexpr int64_t STAGING_BUDGET = (int64_t)64 << 30;

// Stream-ordered allocations released on every exit path unless kept.
struct Arena {
    hipStream_t s;
    void *p[24];
    int n = 0;
    explicit Arena(hipStream_t st) : s(st) {}
    hipError_t alloc(void **out, size_t bytes) {
        *out = nullptr;
        if (bytes == 0) return hipSuccess;
        if (n >= 24) return hipErrorOutOfMemory;
        hipError_t e = cache_alloc(out, bytes, s);
        if (e == hipSuccess) p[n++] = *out;
        return e;
    }
    void keep(void *q) {
        for (int i = 0; i < n; ++i)
            if (p[i] == q) p[i] = nullptr;
    }
    ~Arena() {
        for (int i = 0; i < n; ++i)
            if (p[i]) (void)cache_free(p[i], s);
    }
};

// Events recorded between stages when enabled.
struct Timer {
    bool on;
    hipStream_t s;
    hipEvent_t ev[8];
    int n = 0;
    Timer(bool enable, hipStream_t st) : on(enable), s(st) {}
    void mark() {
        if (!on || n >= 8) return;
        if (hipEventCreate(&ev[n]) == hipSuccess) {
            (void)hipEventRecord(ev[n], s);
            ++n;
        }
    }
    float between(int a, int b) {
        float ms = 0.f;
        if (on && a < n && b < n) (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
        return ms;
    }
    ~Timer() {
        for (int i = 0; i < n; ++i) (void)hipEventDestroy(ev[i]);
    }
};

}  // namespace host
}  // namespace opsp

#define CHK(x)                                      \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return opsp::host::status_of(e_); \
    } while (0)
