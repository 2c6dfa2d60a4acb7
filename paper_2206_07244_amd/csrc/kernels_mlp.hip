// Row-size predictor: a 3 -> 64 -> 64 -> 1 perceptron (ReLU) over the
// features x = log2(1 + (a_len, n_prod, b_max)) of a row of C = A*B,
// predicting log2(1 + nnz).  An extension on top of OpSparse: the paper's
// one-phase alternative (Section 2.2) stores rows into preallocated space;
// the predictor supplies a per-row capacity so that no symbolic pass runs.
//
// Parameters are bfloat16, packed W1[64][3], b1[64], W2[64][64], b2[64],
// W3[64], b3 (4481 values).  Arithmetic:
//   z1 = ((b1 + w0*x0) + w1*x1) + w2*x2 in float32, each step rounded (no
//        fused multiply-add), h1 = bf16(relu(z1)) (nearest, ties to even);
//   z2 = W2 h1 + b2 with float32 accumulation, h2 = relu(z2);
//   y  = W3 h2 + b3 in float32.
// Inference runs the 64x64 layer on the matrix cores: a wave takes 16 rows
// and issues 8 v_mfma_f32_16x16x32_bf16 (4 column tiles of 16 neurons, two
// K steps of 32); layer 1 and the output layer are VALU work in the lanes
// that hold the corresponding operand / result elements.
//
// Training (forward, backward, Adam) uses plain float32 VALU kernels: a
// workgroup takes 64 rows, keeps every per-row vector in LDS, and writes one
// partial gradient per workgroup; a second kernel sums the partials in a
// fixed order.  The bf16 rounding of h1 is passed straight through by the
// backward pass (derivative 1).
#include <math.h>

#include "opsp_internal.h"

namespace opsp {

namespace {

constexpr int H = 64;
constexpr int P_W1 = 0, P_B1 = 192, P_W2 = 256, P_B2 = 4352, P_W3 = 4416, P_B3 = 4480;
static_assert(P_B3 + 1 == MLP_NPARAM, "parameter layout");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// First-layer pre-activation with every product and sum rounded to float32
// in a fixed order: the bf16 rounding of the result is a decision that the
// reference evaluates the same way.
__device__ __forceinline__ float z1_of(float b, float w0, float w1, float w2, float x0, float x1,
                                       float x2) {
#pragma clang fp contract(off)
    float z = b + w0 * x0;
    z = z + w1 * x1;
    z = z + w2 * x2;
    return z;
}

__device__ __forceinline__ float feat(int64_t v) { return log2f(1.0f + (float)v); }

// Weights held by one lane of a wave for the 16-row tile product.  Lane l
// (r = l & 15, q = l >> 4) holds:
//  * layer 1 for the hidden units k = 32 s + 8 q + i (s < 2, i < 8): these
//    are the A-operand elements (row r, k) it feeds to the matrix cores;
//  * the B operand W2^T[k][n] for n = 16 t + r (t < 4), k = 32 s + 8 q + i:
//    eight consecutive bf16 of row n of W2;
//  * b2, W3 for its output columns n = 16 t + r.
struct MlpLane {
    float w1[16][3];
    float b1[16];
    bf16x8 w2[4][2];
    float b2[4], w3[4];
    float b3;
};

__device__ __forceinline__ void mlp_load(const uint16_t *__restrict__ P, MlpLane &w) {
    const int l = lane_id(), r = l & 15, q = l >> 4;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 32 * s + 8 * q + i;
            w.w1[8 * s + i][0] = bf2f(P[P_W1 + 3 * k]);
            w.w1[8 * s + i][1] = bf2f(P[P_W1 + 3 * k + 1]);
            w.w1[8 * s + i][2] = bf2f(P[P_W1 + 3 * k + 2]);
            w.b1[8 * s + i] = bf2f(P[P_B1 + k]);
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int n = 16 * t + r;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const s16x8 raw = *reinterpret_cast<const s16x8 *>(P + P_W2 + n * H + 32 * s + 8 * q);
            w.w2[t][s] = __builtin_bit_cast(bf16x8, raw);
        }
        w.b2[t] = bf2f(P[P_B2 + n]);
        w.w3[t] = bf2f(P[P_W3 + n]);
    }
    w.b3 = bf2f(P[P_B3]);
}

// Forward pass of a 16-row tile.  Lane l supplies the features of row l & 15
// (every group of 16 lanes loads the same 16 rows).  On return y[i] is the
// prediction of row 4 (l >> 4) + i, in every lane of that 16-lane group.
__device__ __forceinline__ void mlp_tile(const MlpLane &w, float x0, float x1, float x2, float y[4]) {
    bf16x8 a[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        s16x8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = 8 * s + i;
            const float z = z1_of(w.b1[j], w.w1[j][0], w.w1[j][1], w.w1[j][2], x0, x1, x2);
            v[i] = (short)f2bf(z > 0.0f ? z : 0.0f);
        }
        a[s] = __builtin_bit_cast(bf16x8, v);
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], w.w2[t][0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], w.w2[t][1], acc, 0, 0, 0);
        // acc[i] = z2 - b2 of row 4 (l >> 4) + i, unit 16 t + (l & 15)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = acc[i] + w.b2[t];
            part[i] += w.w3[t] * (z > 0.0f ? z : 0.0f);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) part[i] += __shfl_xor(part[i], o, 16);
        y[i] = part[i] + w.b3;
    }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_features(int64_t M, const int32_t *__restrict__ alen,
                                                      const int64_t *__restrict__ nprod,
                                                      const int32_t *__restrict__ bmax,
                                                      float *__restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M) return;
    X[3 * i] = feat(alen[i]);
    X[3 * i + 1] = feat(nprod[i]);
    X[3 * i + 2] = feat(bmax[i]);
}

// y[i] for n rows of given features; grid-stride over 16-row tiles.
__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t *__restrict__ P,
                                                     const float *__restrict__ X, int64_t n,
                                                     float *__restrict__ yout) {
    MlpLane w;
    mlp_load(P, w);
    const int l = lane_id(), r = l & 15, q = l >> 4;
    const int64_t tiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles;
         tile += (int64_t)gridDim.x * 4) {
        const int64_t row = tile * 16 + r;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if (row < n) {
            x0 = X[3 * row];
            x1 = X[3 * row + 1];
            x2 = X[3 * row + 2];
        }
        float y[4];
        mlp_tile(w, x0, x1, x2, y);
        if (r < 4) {
            const int64_t orow = tile * 16 + 4 * q + r;
            float v = y[0];
#pragma unroll
            for (int i = 1; i < 4; ++i) v = r == i ? y[i] : v;
            if (orow < n) yout[orow] = v;
        }
    }
}

// Capacity of one row (see launch_mlp_caps), computed in double precision;
// `cal` scales the network's estimate (sampled calibration, 1 = none).
__device__ __forceinline__ int64_t cap_of(const CapArgs &c, float pred, int64_t alen, int64_t np,
                                          int64_t bmax, double cal) {
    const int64_t hi = np < c.ncols ? np : c.ncols;
    int64_t cap;
    if (alen <= 1) {
        cap = np;
    } else if (c.kind == 1) {
        cap = hi;
    } else {
        const double est = c.kind == 0 ? (exp2((double)pred) - 1.0) * cal * (1.0 + c.margin)
                                       : (double)np / c.ratio * (1.0 + c.margin);
        const int64_t lo = bmax < hi ? bmax : hi;
        const double e = ceil(est);
        if (!(e == e) || e >= (double)hi) cap = hi;   // NaN or at / above the bound
        else if (e <= (double)lo) cap = lo;
        else cap = (int64_t)e;
    }
    if (c.scale != 1.0) cap = (int64_t)floor((double)cap * c.scale);
    return cap;
}

// Capacities of 256 rows per workgroup (a wave: 4 tiles of 16 rows), with
// the block's numeric-bin record (the first binning pass over capacities)
// and the n_prod total / maximum.
__global__ __launch_bounds__(256) void k_mlp_caps(int64_t M, CapArgs c,
                                                  const int32_t *__restrict__ alen,
                                                  const int64_t *__restrict__ nprod,
                                                  const int32_t *__restrict__ bmax,
                                                  int64_t *__restrict__ cap, Bounds bd,
                                                  BlockParts parts, LearnCtr *__restrict__ lc) {
    __shared__ unsigned int hist[BIN_SLOTS];
    __shared__ unsigned long long s_tot, s_max, s_np, s_npmax;
    if (threadIdx.x < BIN_SLOTS) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) { s_tot = 0; s_max = 0; s_np = 0; s_npmax = 0; }
    __syncthreads();
    const int l = lane_id(), r = l & 15, q = l >> 4, wv = threadIdx.x >> 6;
    const bool run_net = c.kind == 0 && !c.pred_in;
    // sampled calibration: exact / estimated sizes of the sampled rows of
    // each n_prod octave that has enough of them
    __shared__ double s_cal[CAL_OCT];
    if (threadIdx.x < CAL_OCT) {
        const int o = threadIdx.x;
        double v = 1.0;
        if (c.kind == 0 && c.calib && c.calmax && c.calib[2 * CAL_OCT + o] >= (double)CAL_MIN_ROWS)
            v = __longlong_as_double((long long)c.calmax[o]);
        s_cal[o] = v;
    }
    __syncthreads();
    MlpLane w;
    if (run_net) mlp_load(c.P, w);
    unsigned long long tot = 0, mx = 0, nps = 0, npm = 0;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
        const int64_t t0 = (int64_t)blockIdx.x * 256 + wv * 64 + j * 16;
        float y[4] = {0.f, 0.f, 0.f, 0.f};
        if (run_net) {
            const int64_t row = t0 + r;
            float x0 = 0.f, x1 = 0.f, x2 = 0.f;
            if (row < M) {
                x0 = feat(alen[row]);
                x1 = feat(nprod[row]);
                x2 = feat(bmax[row]);
            }
            mlp_tile(w, x0, x1, x2, y);
        }
        if (r < 4) {
            const int64_t row = t0 + 4 * q + r;
            float v = y[0];
#pragma unroll
            for (int i = 1; i < 4; ++i) v = r == i ? y[i] : v;
            if (row < M) {
                if (c.pred_in) v = c.pred_in[row];
                const int64_t np = nprod[row];
                const double cal = np >= 1 ? s_cal[63 - __clzll(np)] : 1.0;
                const int64_t cp = cap_of(c, v, alen[row], np, bmax[row], cal);
                cap[row] = cp;
                if (c.pred && !c.pred_in) c.pred[row] = v;
                atomicAdd(&hist[bin_of(cp, bd)], 1u);
                tot += (unsigned long long)cp;
                mx = (unsigned long long)cp > mx ? (unsigned long long)cp : mx;
                nps += (unsigned long long)np;
                npm = (unsigned long long)np > npm ? (unsigned long long)np : npm;
            }
        }
    }
    tot = wave_sum(tot);
    mx = wave_max(mx);
    nps = wave_sum(nps);
    npm = wave_max(npm);
    if (l == 0) {
        atomicAdd(&s_tot, tot);
        atomicMax(&s_max, mx);
        atomicAdd(&s_np, nps);
        atomicMax(&s_npmax, npm);
    }
    __syncthreads();
    if ((int)threadIdx.x < BIN_SLOTS)
        parts.hist[(int64_t)blockIdx.x * BIN_SLOTS + threadIdx.x] = hist[threadIdx.x];
    if (threadIdx.x == 0) {
        parts.tot[blockIdx.x] = s_tot;
        parts.mx[blockIdx.x] = s_max;
        atomicAdd(&lc->nprod_total, s_np);
        atomicMax(&lc->nprod_max, s_npmax);
    }
}

// Network outputs of every row (16-row tiles per wave) from the integer
// features; feeds the calibration sample and the capacity kernel.
__global__ __launch_bounds__(256) void k_mlp_pred(int64_t M, const uint16_t *__restrict__ P,
                                                  const int32_t *__restrict__ alen,
                                                  const int64_t *__restrict__ nprod,
                                                  const int32_t *__restrict__ bmax,
                                                  float *__restrict__ pred) {
    MlpLane w;
    mlp_load(P, w);
    const int l = lane_id(), r = l & 15, q = l >> 4;
    const int64_t tiles = (M + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles;
         tile += (int64_t)gridDim.x * 4) {
        const int64_t row = tile * 16 + r;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if (row < M) {
            x0 = feat(alen[row]);
            x1 = feat(nprod[row]);
            x2 = feat(bmax[row]);
        }
        float y[4];
        mlp_tile(w, x0, x1, x2, y);
        if (r < 4) {
            const int64_t orow = tile * 16 + 4 * q + r;
            float v = y[0];
#pragma unroll
            for (int i = 1; i < 4; ++i) v = r == i ? y[i] : v;
            if (orow < M) pred[orow] = v;
        }
    }
}

// Calibration sample (rule of launch_cal_hist / launch_cal_pick).
__device__ __forceinline__ bool cal_eligible(int32_t alen, int64_t np, int2 rg) {
    return alen >= 2 && np >= 1 && np < ((int64_t)2 << CAL_MAX_OCT) &&
           (int64_t)rg.y - rg.x + 1 <= CAL_SPAN_MAX;
}

// Rows per n_prod octave among the eligible rows.
__global__ __launch_bounds__(256) void k_cal_hist(int64_t M, const int32_t *__restrict__ alen,
                                                  const int64_t *__restrict__ nprod,
                                                  const int2 *__restrict__ rng,
                                                  unsigned long long *__restrict__ hist) {
    __shared__ unsigned int h[CAL_OCT];
    if (threadIdx.x < CAL_OCT) h[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256) {
        const int64_t np = nprod[i];
        if (cal_eligible(alen[i], np, rng[i])) atomicAdd(&h[63 - __clzll(np)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < CAL_OCT && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// Stride of every octave from its count c: ceil(c / K) with
// K = min(c, clamp(CAL_OCT_PRODUCTS >> o, CAL_MIN_ROWS, per_octave)).
__global__ void k_cal_quota(const unsigned long long *__restrict__ hist, int64_t per_octave,
                              unsigned long long *__restrict__ quota) {
    const int o = threadIdx.x;
    if (o >= CAL_OCT) return;
    const int64_t c = (int64_t)hist[o];
    int64_t k = o < 62 ? (CAL_OCT_PRODUCTS >> o) : 0;
    k = k < CAL_MIN_ROWS ? CAL_MIN_ROWS : (k > per_octave ? per_octave : k);
    k = k < c ? k : c;
    quota[o] = c > 0 ? (unsigned long long)k : 0ull;
}

// MurmurHash3's 64-bit finalizer (Appleby): every input bit affects every
// output bit, so the high half of the result is uniform over [0, 2^32)
// for any set of row indices, consecutive ones included.
__device__ __forceinline__ unsigned long long fmix64(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Eligible row i of an octave with c eligible rows and quota K is picked
// when u(i) * c < K * 2^32, u(i) the high half of fmix64(i): a Bernoulli
// draw of probability K / c, so an octave yields K rows on average and all
// of its rows when c <= K.  Picked rows are appended to `list` (which holds
// M entries, so it cannot overflow).
__global__ __launch_bounds__(256) void k_cal_pick(int64_t M, const int32_t *__restrict__ alen,
                                                  const int64_t *__restrict__ nprod,
                                                  const int2 *__restrict__ rng,
                                                  const unsigned long long *__restrict__ hist,
                                                  const unsigned long long *__restrict__ quota,
                                                  int32_t *__restrict__ list,
                                                  unsigned int *__restrict__ count) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256) {
        const int64_t np = nprod[i];
        if (!cal_eligible(alen[i], np, rng[i])) continue;
        const int o = 63 - __clzll(np);
        const unsigned long long u = fmix64((unsigned long long)i) >> 32;
        if (u * hist[o] < (quota[o] << 32)) list[atomicAdd(count, 1u)] = (int32_t)i;
    }
}

// Sums of the picked rows per octave (exact size, clamped estimate, 1) and
// the largest exact / estimate ratio.
__global__ __launch_bounds__(256) void k_cal_sum(const int32_t *__restrict__ list,
                                                 const unsigned int *__restrict__ count,
                                                 const int64_t *__restrict__ nprod,
                                                 const int32_t *__restrict__ bmax,
                                                 const float *__restrict__ pred,
                                                 const int64_t *__restrict__ exact, int64_t ncols,
                                                 double *__restrict__ calib,
                                                 unsigned long long *__restrict__ calmax) {
    const int64_t n = (int64_t)*count;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        const int64_t row = list[k];
        const int64_t np = nprod[row];
        const int64_t hi = np < ncols ? np : ncols;
        const int64_t bm = bmax[row];
        const double lo = (double)(bm < hi ? bm : hi);
        double e = exp2((double)pred[row]) - 1.0;
        e = e < lo ? lo : (e > (double)hi ? (double)hi : e);
        const int o = 63 - __clzll(np);
        unsafeAtomicAdd(&calib[o], (double)exact[row]);
        unsafeAtomicAdd(&calib[CAL_OCT + o], e);
        unsafeAtomicAdd(&calib[2 * CAL_OCT + o], 1.0);
        // largest ratio: positive doubles order like their bit patterns
        const double ratio = (double)exact[row] / e;
        atomicMax(&calmax[o], (unsigned long long)__double_as_longlong(ratio));
    }
}

// ---------------------------------------------------------------------------
// Training: gradient of the mean squared error (sum over rows of
// (y - t)^2 / n), or of the mean pinball loss of level tau, for GR rows per
// workgroup.
// ---------------------------------------------------------------------------
constexpr int GR = 64;
constexpr int LD = H + 1;   // padded LDS row stride

__global__ __launch_bounds__(256) void k_mlp_grad_part(const uint16_t *__restrict__ P,
                                                       const float *__restrict__ X,
                                                       const float *__restrict__ Tg, int64_t n,
                                                       float inv_n, float tau,
                                                       float *__restrict__ part) {
    __shared__ float sW1[H * 3], sb1[H], sW2[H * LD], sb2[H], sW3[H];
    __shared__ float sX[GR][3];
    __shared__ float sH1[GR][LD], sH2[GR][LD], sDZ2[GR][LD], sDZ1[GR][LD];
    __shared__ float sDY[GR], sL[GR];
    __shared__ float sb3;
    const int t = threadIdx.x;
    for (int i = t; i < H * 3; i += 256) sW1[i] = bf2f(P[P_W1 + i]);
    for (int i = t; i < H * H; i += 256) sW2[(i / H) * LD + (i % H)] = bf2f(P[P_W2 + i]);
    if (t < H) {
        sb1[t] = bf2f(P[P_B1 + t]);
        sb2[t] = bf2f(P[P_B2 + t]);
        sW3[t] = bf2f(P[P_W3 + t]);
    }
    if (t == 0) sb3 = bf2f(P[P_B3]);
    // phase A: four threads per row, thread q owns hidden units q, q+4, ...
    const int r = t >> 2, q = t & 3;
    const int64_t row = (int64_t)blockIdx.x * GR + r;
    const bool valid = row < n;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f;
    if (valid) {
        x0 = X[3 * row];
        x1 = X[3 * row + 1];
        x2 = X[3 * row + 2];
    }
    if (q == 0) {
        sX[r][0] = x0;
        sX[r][1] = x1;
        sX[r][2] = x2;
    }
    __syncthreads();
    float z1v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int k = q + 4 * m;
        const float z = z1_of(sb1[k], sW1[3 * k], sW1[3 * k + 1], sW1[3 * k + 2], x0, x1, x2);
        z1v[m] = z;
        sH1[r][k] = valid ? bf2f(f2bf(z > 0.f ? z : 0.f)) : 0.f;
    }
    __syncthreads();
    float z2v[16];
    float yp = 0.f;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int j = q + 4 * m;
        float acc = sb2[j];
#pragma unroll 8
        for (int k = 0; k < H; ++k) acc += sW2[j * LD + k] * sH1[r][k];
        z2v[m] = acc;
        const float h2 = acc > 0.f ? acc : 0.f;
        sH2[r][j] = valid ? h2 : 0.f;
        yp += sW3[j] * h2;
    }
    yp += __shfl_xor(yp, 1);
    yp += __shfl_xor(yp, 2);
    const float y = yp + sb3;
    const float diff = valid ? y - Tg[row] : 0.f;
    // squared error (tau == 0) or pinball loss of level tau on t - y
    float dy, lrow;
    if (tau > 0.f) {
        dy = valid ? (diff < 0.f ? -tau : 1.f - tau) * inv_n : 0.f;
        lrow = diff < 0.f ? -tau * diff : (1.f - tau) * diff;
    } else {
        dy = 2.f * diff * inv_n;
        lrow = diff * diff;
    }
    if (q == 0) {
        sDY[r] = dy;
        sL[r] = lrow;
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int j = q + 4 * m;
        sDZ2[r][j] = z2v[m] > 0.f ? dy * sW3[j] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int k = q + 4 * m;
        float acc = 0.f;
#pragma unroll 8
        for (int j = 0; j < H; ++j) acc += sDZ2[r][j] * sW2[j * LD + k];
        sDZ1[r][k] = z1v[m] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    // phase B: parameter partials, summed over the workgroup's rows
    float *out = part + (int64_t)blockIdx.x * (MLP_NPARAM + 1);
    {
        const int k = t & 63;
        for (int j = t >> 6; j < H; j += 4) {
            float acc = 0.f;
            for (int rr = 0; rr < GR; ++rr) acc += sDZ2[rr][j] * sH1[rr][k];
            out[P_W2 + j * H + k] = acc;
        }
    }
    if (t < 64) {
        const int k = t;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, ab = 0.f;
        for (int rr = 0; rr < GR; ++rr) {
            const float d = sDZ1[rr][k];
            a0 += d * sX[rr][0];
            a1 += d * sX[rr][1];
            a2 += d * sX[rr][2];
            ab += d;
        }
        out[P_W1 + 3 * k] = a0;
        out[P_W1 + 3 * k + 1] = a1;
        out[P_W1 + 3 * k + 2] = a2;
        out[P_B1 + k] = ab;
    } else if (t < 128) {
        const int j = t - 64;
        float ab = 0.f, aw = 0.f;
        for (int rr = 0; rr < GR; ++rr) {
            ab += sDZ2[rr][j];
            aw += sDY[rr] * sH2[rr][j];
        }
        out[P_B2 + j] = ab;
        out[P_W3 + j] = aw;
    } else if (t == 128) {
        float ab = 0.f, al = 0.f;
        for (int rr = 0; rr < GR; ++rr) {
            ab += sDY[rr];
            al += sL[rr];
        }
        out[P_B3] = ab;
        out[MLP_NPARAM] = al;
    }
}

// Sum of the per-workgroup partials in workgroup order (float64 running sum).
__global__ __launch_bounds__(256) void k_mlp_grad_reduce(const float *__restrict__ part, int64_t nblk,
                                                         float inv_n, float *__restrict__ grad,
                                                         float *__restrict__ loss) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > MLP_NPARAM) return;
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) acc += (double)part[b * (MLP_NPARAM + 1) + p];
    if (p < MLP_NPARAM) grad[p] = (float)acc;
    else if (loss) *loss = (float)(acc * (double)inv_n);
}

// Adam on float32 master weights; the bf16 copy is what the kernels read.
// c1 = 1 / (1 - beta1^step), c2 = 1 / (1 - beta2^step).
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ master, float *__restrict__ m,
                                                  float *__restrict__ v, const float *__restrict__ g,
                                                  float lr, float b1, float b2, float eps, float c1,
                                                  float c2, uint16_t *__restrict__ P) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float w = master[p] - lr * (mp * c1) / (sqrtf(vp * c2) + eps);
    master[p] = w;
    P[p] = f2bf(w);
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_mlp_features(int64_t M, const int32_t *alen, const int64_t *nprod,
                               const int32_t *bmax, float *X, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, M, alen,
                       nprod, bmax, X);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint16_t *P, const float *X, int64_t n, float *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + 15) / 16;
    int64_t grid = (tiles + 3) / 4;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)grid), dim3(256), 0, s, P, X, n, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const uint16_t *P, const float *X, const float *T, int64_t n, float tau,
                           float *part, float *grad, float *loss, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    const int64_t nblk = (n + GR - 1) / GR;
    hipLaunchKernelGGL(k_mlp_grad_part, dim3((unsigned)nblk), dim3(256), 0, s, P, X, T, n,
                       (float)(1.0 / (double)n), tau, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, s, part,
                       nblk, (float)(1.0 / (double)n), grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *master, float *m, float *v, const float *g, float lr, float b1,
                           float b2, float eps, float c1, float c2, uint16_t *P, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, master, m, v, g,
                       lr, b1, b2, eps, c1, c2, P);
    return hipGetLastError();
}

hipError_t launch_mlp_pred(int64_t M, const uint16_t *P, const int32_t *alen, const int64_t *nprod,
                           const int32_t *bmax, float *pred, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    const int64_t tiles = (M + 15) / 16;
    int64_t grid = (tiles + 3) / 4;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_mlp_pred, dim3((unsigned)grid), dim3(256), 0, s, M, P, alen, nprod, bmax, pred);
    return hipGetLastError();
}

hipError_t launch_cal_hist(int64_t M, const int32_t *alen, const int64_t *nprod, const int2 *rng,
                           unsigned long long *hist, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    const int64_t g = (M + 255) / 256 < 4096 ? (M + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_cal_hist, dim3((unsigned)g), dim3(256), 0, s, M, alen, nprod, rng, hist);
    return hipGetLastError();
}

hipError_t launch_cal_pick(int64_t M, const int32_t *alen, const int64_t *nprod, const int2 *rng,
                           const unsigned long long *hist, int64_t per_octave,
                           unsigned long long *quota, int32_t *list, unsigned int *count,
                           hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cal_quota, dim3(1), dim3(CAL_OCT), 0, s, hist, per_octave, quota);
    const int64_t g = (M + 255) / 256 < 4096 ? (M + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_cal_pick, dim3((unsigned)g), dim3(256), 0, s, M, alen, nprod, rng, hist, quota,
                       list, count);
    return hipGetLastError();
}

hipError_t launch_cal_sum(const int32_t *list, const unsigned int *count, const int64_t *nprod,
                          const int32_t *bmax, const float *pred, const int64_t *exact, int64_t ncols,
                          double *calib, unsigned long long *calmax, hipStream_t s) {
    hipLaunchKernelGGL(k_cal_sum, dim3(64), dim3(256), 0, s, list, count, nprod, bmax, pred, exact, ncols,
                       calib, calmax);
    return hipGetLastError();
}

hipError_t launch_mlp_caps(int64_t M, const CapArgs &ca, const int32_t *alen, const int64_t *nprod,
                           const int32_t *bmax, int64_t *cap, const Bounds &bd,
                           const BlockParts &parts, LearnCtr *lc, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_caps, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, M, ca, alen,
                       nprod, bmax, cap, bd, parts, lc);
    return hipGetLastError();
}

}  // namespace opsp
