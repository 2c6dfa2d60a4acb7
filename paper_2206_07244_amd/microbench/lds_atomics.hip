// Microbenchmark of the LDS atomics that the hash and dense accumulation
// kernels are built on (the second ceiling beside HBM bandwidth for the
// symbolic and numeric steps of Section 5.2): FP64 add without return
// (ds_add_f64; ds_add_f32 for the FP32 product), compare-and-swap with
// return (ds_cmpst_rtn_b32, the single-access probe of Alg. 4/5) and OR
// without return (ds_or_b32, the bitmaps), each with lanes on consecutive words (no bank conflict) and on
// pseudo-random words of a 64 KB table (the hash tables' access pattern).
// Not part of the library: built into libopsp_microbench.so and run by
// `bench.py --mode lds`.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int MB_T = 512;                 // threads per workgroup
constexpr int MB_WORDS = 16384;           // 64 KB of 32-bit words (8192 doubles)

// kind 0 = ds_add_f64, 1 = ds_cmpst_rtn_b32, 2 = ds_or_b32, 3 = ds_add_f32; pattern 0 =
// lane-consecutive, 1 = pseudo-random (a 32-bit LCG per lane, two VALU
// operations per step)
template <int KIND, int PATTERN>
__global__ __launch_bounds__(MB_T) void k_lds_atomics(int iters, unsigned int *sink) {
    __shared__ double tab[MB_WORDS / 2];
    unsigned int *w = reinterpret_cast<unsigned int *>(tab);
    const int t = threadIdx.x;
    for (int i = t; i < MB_WORDS; i += MB_T) w[i] = 0u;
    __syncthreads();
    uint32_t x = 2654435761u * (uint32_t)(t + 1) + (uint32_t)blockIdx.x;
    unsigned int acc = 0;
    for (int it = 0; it < iters; ++it) {
        uint32_t idx;
        if (PATTERN == 0) {
            idx = (uint32_t)(t + 64 * it);
        } else {
            x = x * 1664525u + 1013904223u;
            idx = x >> 8;
        }
        if (KIND == 0) {
            atomicAdd(&tab[idx & (MB_WORDS / 2 - 1)], 1.0);
        } else if (KIND == 1) {
            const uint32_t j = idx & (MB_WORDS - 1);
            acc += atomicCAS(&w[j], 0u, (unsigned int)t + 1u);
        } else if (KIND == 2) {
            atomicOr(&w[idx & (MB_WORDS - 1)], 1u << (t & 31));
        } else {
            atomicAdd(reinterpret_cast<float *>(&w[idx & (MB_WORDS - 1)]), 1.0f);
        }
    }
    __syncthreads();
    if (t == 0) acc += w[0];
    if (acc == 0xffffffffu) sink[blockIdx.x] = acc;   // keeps the loop; never true in practice
}

template <int KIND, int PATTERN>
hipError_t launch(int grid, int iters, unsigned int *sink, hipStream_t s) {
    hipLaunchKernelGGL((k_lds_atomics<KIND, PATTERN>), dim3((unsigned)grid), dim3(MB_T), 0, s, iters, sink);
    return hipGetLastError();
}

}  // namespace

extern "C" {

// Runs `reps` launches of `grid` workgroups of 512 threads, each thread
// issuing `iters` atomics of `kind` with `pattern`, and returns the mean time
// of one launch in *ms (HIP events).  0 on success, else a hipError_t.
int opsp_mb_lds_atomics(int kind, int pattern, int grid, int iters, int reps, float *ms) {
    if (kind < 0 || kind > 3 || pattern < 0 || pattern > 1 || grid <= 0 || iters <= 0 || reps <= 0 || !ms)
        return (int)hipErrorInvalidValue;
    unsigned int *sink = nullptr;
    hipError_t e = hipMalloc(&sink, sizeof(unsigned int) * (size_t)grid);
    if (e != hipSuccess) return (int)e;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    auto go = [&]() -> hipError_t {
        switch (kind * 2 + pattern) {
            case 0: return launch<0, 0>(grid, iters, sink, nullptr);
            case 1: return launch<0, 1>(grid, iters, sink, nullptr);
            case 2: return launch<1, 0>(grid, iters, sink, nullptr);
            case 3: return launch<1, 1>(grid, iters, sink, nullptr);
            case 4: return launch<2, 0>(grid, iters, sink, nullptr);
            case 5: return launch<2, 1>(grid, iters, sink, nullptr);
            case 6: return launch<3, 0>(grid, iters, sink, nullptr);
            default: return launch<3, 1>(grid, iters, sink, nullptr);
        }
    };
    e = go();   // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, nullptr);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = go();
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    *ms = t / (float)reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(sink);
    return (int)e;
}

}  // extern "C"
