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
    int32_t pad;
    int64_t ub[16];
};

__device__ __forceinline__ int bin_of(int64_t v, const Bounds &b) {
    int j = 0;
    while (j < b.nb - 1 && v > b.ub[j]) ++j;
    if (b.force >= 0 && (b.force >= b.nb - 1 || v <= b.ub[b.force])) j = b.force;
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
    unsigned long long pad[6];
};

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

}  // namespace opsp
