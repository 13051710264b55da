// Device functions of the learned proposal: a normalizing flow of four
// piecewise-quadratic coupling layers over (0,1)^6 (the design of "Neural
// Importance Sampling", Müller et al. 2019): its dimensions and parameter
// layout, the one-blob encoding, the splines with their inverse and
// derivative (FP32), and a one-thread-per-sample form of a whole layer
// whose weights, the same for every lane, come through scalar loads (used
// by the FP32 flow-mapped iteration; the other FP32 kernels split the
// products over a workgroup, the BF16 ones run them on the matrix cores).
//
//   layer l keeps the coordinates A_l and maps every coordinate j of B_l
//   through the CDF of a piecewise-linear density on (0,1) with 16 bins;
//   the bin widths (softmax of 16 raw values) and the 17 vertex heights
//   (exp of 17 raw values, scaled so that the density integrates to 1) come
//   from a network of u_{A_l}: one-blob encoding (32 Gaussian bumps of width
//   1/32 per input), two hidden layers of 64 ReLU units, 3 x 33 linear
//   outputs.  A = {0,1,2}, {3,4,5}, {0,2,4}, {1,3,5}; B = the complement.
//   q(x) = product of the spline densities met on the way x -> z.
//
// Parameter layout of layer l (FP32, row-major, input index first), MCUBES_FLOW_PARAMS
// values in all: W1[96][64], b1[64], W2[64][64], b2[64], W3[64][99], b3[99].
#pragma once

#include "flow_internal.h"

namespace mcubes {
namespace flow {

constexpr int D = 6, L = 4, NA = 3, NB = 3, BLOBS = 32, IN = NA * BLOBS, HID = 64, BINS = 16;
constexpr int RAW = 2 * BINS + 1, OUT = NB * RAW;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + IN * HID, OFF_W2 = OFF_B1 + HID;
constexpr int OFF_B2 = OFF_W2 + HID * HID, OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * OUT;
constexpr int LP = OFF_B3 + OUT;  // parameters per layer
constexpr int PARAMS = L * LP;
static_assert(PARAMS == MCUBES_FLOW_PARAMS, "flow parameter count");

// Per-sample training scratch, one block of FS fields per layer, each field
// n floats (sample contiguous): the layer's input u (6), h1 and h2 (64
// each), the 99 spline parameters (replaced by their deltas in the backward
// pass) and the deltas after the second and the first ReLU.  The FP32
// training pass writes them all as FP32; the BF16 one writes u as FP32 and
// the rest as BF16 rows of n values in the upper half of the layer's block
// (bf16_rows in flow_bf16.hip).
constexpr int FS_U = 0, FS_H1 = FS_U + D, FS_H2 = FS_H1 + HID, FS_DOUT = FS_H2 + HID;
constexpr int FS_D2 = FS_DOUT + OUT, FS_D1 = FS_D2 + HID, FS = FS_D1 + HID;
// most sample slices the weight-gradient kernels cut a batch into (their
// partial sums follow the fields in the scratch buffer)
constexpr int kWgradSlices = 128;

// Gradient of parameter i: the slices' partial sums part[slice][i] added in
// slice order (sixteen loads in flight before their adds: with about one
// wave per SIMD the loads, not the adds, set the time).
__device__ __forceinline__ float slice_sum(const float *__restrict__ part, int slices, int i) {
    float a = 0.0f;
    int k = 0;
    for (; k + 16 <= slices; k += 16) {
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = part[(int64_t)(k + q) * PARAMS + i];
#pragma unroll
        for (int q = 0; q < 16; ++q) a += v[q];
    }
    for (; k < slices; ++k) a += part[(int64_t)k * PARAMS + i];
    return a;
}

// One Adam step of parameter i with gradient g on the FP32 master copy;
// c1 = 1 - beta1^t, c2 = 1 - beta2^t.  Returns the new parameter.
__device__ __forceinline__ float adam_update(float *__restrict__ theta, float *__restrict__ m,
                                             float *__restrict__ v, int i, float g, float lr,
                                             float beta1, float beta2, float eps, float c1,
                                             float c2) {
    const float mi = beta1 * m[i] + (1.0f - beta1) * g;
    const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float t = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = t;
    return t;
}

// Histogram of log2 of the flow-mapped weights (the tail diagnostic): bin
// floor(8 log2 w) + 2048, clamped to [0, 4095]; weights that are not
// positive (or not numbers) are not counted.  Kept per workgroup in LDS.
constexpr int WH_BINS = MCUBES_WTAIL_BINS, WH_PER_OCTAVE = 8, WH_ZERO = WH_BINS / 2;

__device__ __forceinline__ void wh_add(uint32_t *hist, double w) {
    if (!(w > 0.0)) return;
    double v = floor(log2(w) * (double)WH_PER_OCTAVE);
    v = fmin(fmax(v, -(double)WH_ZERO), (double)(WH_ZERO - 1));
    atomicAdd(&hist[(int)v + WH_ZERO], 1u);
}

__device__ __forceinline__ void wh_clear(uint32_t *hist) {
    for (int i = threadIdx.x; i < WH_BINS; i += blockDim.x) hist[i] = 0u;
}

// adds the workgroup's histogram to the global one (barrier first)
__device__ __forceinline__ void wh_flush(const uint32_t *hist, uint32_t *__restrict__ out) {
    __syncthreads();
    for (int i = threadIdx.x; i < WH_BINS; i += blockDim.x)
        if (hist[i]) atomicAdd(&out[i], hist[i]);
}

// coordinate t of A_l and of B_l
__device__ __forceinline__ int a_idx(int l, int t) {
    return l == 0 ? t : (l == 1 ? 3 + t : (l == 2 ? 2 * t : 2 * t + 1));
}
__device__ __forceinline__ int b_idx(int l, int t) {
    return l == 0 ? 3 + t : (l == 1 ? t : (l == 2 ? 2 * t + 1 : 2 * t));
}

// u[j] for a runtime j without indexing the register array
__device__ __forceinline__ float getu(const float u[D], int j) {
    float r = u[0];
#pragma unroll
    for (int k = 1; k < D; ++k) r = (j == k) ? u[k] : r;
    return r;
}
__device__ __forceinline__ void setu(float u[D], int j, float v) {
#pragma unroll
    for (int k = 0; k < D; ++k) u[k] = (j == k) ? v : u[k];
}

__device__ __forceinline__ float blob(float u, int k) {
    const float t = (u - ((float)k + 0.5f) * (1.0f / BLOBS)) * (float)BLOBS;
    return expf(-0.5f * t * t);
}

// Hidden layers of the conditioner of one layer (P = that layer's
// parameters): h1 = relu(W1^T e + b1), h2 = relu(W2^T h1 + b2).
__device__ __forceinline__ void hidden(const float *__restrict__ P, const float ua[NA],
                                       float h1[HID], float h2[HID]) {
#pragma unroll
    for (int o = 0; o < HID; ++o) h1[o] = 0.0f;
    for (int a = 0; a < NA; ++a) {
        const float ux = ua[a];
#pragma unroll 2
        for (int k = 0; k < BLOBS; ++k) {
            const float e = blob(ux, k);
            const float *row = P + OFF_W1 + (a * BLOBS + k) * HID;
#pragma unroll
            for (int o = 0; o < HID; ++o) h1[o] = __fmaf_rn(e, row[o], h1[o]);
        }
    }
#pragma unroll
    for (int o = 0; o < HID; ++o) h1[o] = fmaxf(h1[o] + P[OFF_B1 + o], 0.0f);
#pragma unroll
    for (int o = 0; o < HID; ++o) h2[o] = 0.0f;
#pragma unroll
    for (int i = 0; i < HID; ++i) {
        const float *row = P + OFF_W2 + i * HID;
#pragma unroll
        for (int o = 0; o < HID; ++o) h2[o] = __fmaf_rn(h1[i], row[o], h2[o]);
    }
#pragma unroll
    for (int o = 0; o < HID; ++o) h2[o] = fmaxf(h2[o] + P[OFF_B2 + o], 0.0f);
}

// Output values of transformed coordinate t: raw = W3[:, 33t .. 33t+32]^T h2 + b3.
__device__ __forceinline__ void out_chunk(const float *__restrict__ P, const float h2[HID], int t,
                                          float raw[RAW]) {
#pragma unroll
    for (int k = 0; k < RAW; ++k) raw[k] = 0.0f;
#pragma unroll
    for (int i = 0; i < HID; ++i) {
        const float *row = P + OFF_W3 + i * OUT + t * RAW;
#pragma unroll
        for (int k = 0; k < RAW; ++k) raw[k] = __fmaf_rn(h2[i], row[k], raw[k]);
    }
#pragma unroll
    for (int k = 0; k < RAW; ++k) raw[k] = raw[k] + P[OFF_B3 + t * RAW + k];
}

// Widths W (softmax), heights V = E / Z with E = exp(raw - max).
struct Spline {
    float W[BINS], V[BINS + 1], E[BINS + 1], Z;
};

// FAST: the hardware exponential (a few ulp instead of correctly rounded
// to 1 ulp), for the BF16 path whose spline inputs already carry the BF16
// products' ~1e-3 relative error.
template <bool FAST = false>
__device__ __forceinline__ float sexp(float x) {
    return FAST ? __expf(x) : expf(x);
}

template <bool FAST = false>
__device__ __forceinline__ void spline_setup(const float raw[RAW], Spline &s) {
    float mw = raw[0], mv = raw[BINS];
#pragma unroll
    for (int i = 1; i < BINS; ++i) mw = fmaxf(mw, raw[i]);
#pragma unroll
    for (int i = 1; i <= BINS; ++i) mv = fmaxf(mv, raw[BINS + i]);
    float sw = 0.0f;
#pragma unroll
    for (int i = 0; i < BINS; ++i) {
        s.W[i] = sexp<FAST>(raw[i] - mw);
        sw += s.W[i];
    }
    const float inv = 1.0f / sw;
#pragma unroll
    for (int i = 0; i < BINS; ++i) s.W[i] *= inv;
#pragma unroll
    for (int i = 0; i <= BINS; ++i) s.E[i] = sexp<FAST>(raw[BINS + i] - mv);
    float Z = 0.0f;
#pragma unroll
    for (int i = 0; i < BINS; ++i) Z += 0.5f * (s.E[i] + s.E[i + 1]) * s.W[i];
    s.Z = Z;
    const float iz = 1.0f / Z;
#pragma unroll
    for (int i = 0; i <= BINS; ++i) s.V[i] = s.E[i] * iz;
}

// The bin of u (by left edges, key = 0) or of y (by left CDF values, key = 1):
// the last k in 1..15 whose edge is <= the value, else 0.  Returns the bin's
// left edge X, left CDF value A, width, heights and its index.
struct Bin {
    float X, A, W, V0, V1;
    int k;
};

template <bool BY_CDF>
__device__ __forceinline__ Bin find_bin(const Spline &s, float v) {
    Bin b{0.0f, 0.0f, s.W[0], s.V[0], s.V[1], 0};
    float X = s.W[0], A = 0.5f * (s.V[0] + s.V[1]) * s.W[0];
#pragma unroll
    for (int k = 1; k < BINS; ++k) {
        const bool in = BY_CDF ? (A <= v) : (X <= v);
        if (in) {
            b.X = X;
            b.A = A;
            b.W = s.W[k];
            b.V0 = s.V[k];
            b.V1 = s.V[k + 1];
            b.k = k;
        }
        X += s.W[k];
        A += 0.5f * (s.V[k] + s.V[k + 1]) * s.W[k];
    }
    return b;
}

__device__ __forceinline__ void spline_forward(const Spline &s, float u, float &y, float &pdf) {
    const Bin b = find_bin<false>(s, u);
    const float a = fminf(fmaxf((u - b.X) / b.W, 0.0f), 1.0f);
    const float dV = b.V1 - b.V0;
    y = b.A + b.W * (a * b.V0 + 0.5f * a * a * dV);
    pdf = b.V0 + a * dV;
}

__device__ __forceinline__ void spline_inverse(const Spline &s, float y, float &u, float &pdf) {
    const Bin b = find_bin<true>(s, y);
    const float r = y - b.A;
    const float dV = b.V1 - b.V0;
    const float disc = fmaxf(b.V0 * b.V0 + 2.0f * dV * r / b.W, 0.0f);
    const float den = b.W * (b.V0 + sqrtf(disc));
    float a = den > 0.0f ? 2.0f * r / den : 0.0f;
    a = fminf(fmaxf(a, 0.0f), 1.0f);
    u = b.X + a * b.W;
    pdf = b.V0 + a * dV;
}

// Reverse-mode derivative of (y, pdf) at u: given gy = dL/dy and gp = dL/dpdf,
// graw = dL/draw (33 values) and gu = dL/du.
__device__ __forceinline__ void spline_backward(const Spline &s, float u, float gy, float gp,
                                                float graw[RAW], float &gu) {
    const Bin b = find_bin<false>(s, u);
    const float a = (u - b.X) / b.W;
    const float dV = b.V1 - b.V0;
    const float ga = gy * b.W * (b.V0 + a * dV) + gp * dV;
    const float gWb = gy * (a * b.V0 + 0.5f * a * a * dV) - ga * a / b.W;
    const float gV0 = gy * b.W * (a - 0.5f * a * a) + gp * (1.0f - a);
    const float gV1 = gy * b.W * 0.5f * a * a + gp * a;
    gu = ga / b.W;
    float gW[BINS], gV[BINS + 1];
#pragma unroll
    for (int k = 0; k <= BINS; ++k) gV[k] = 0.0f;
    // bins left of b: the CDF offset A_b and the edge X_b
#pragma unroll
    for (int k = 0; k < BINS; ++k) {
        const bool left = k < b.k;
        gW[k] = left ? 0.5f * gy * (s.V[k] + s.V[k + 1]) - ga / b.W : 0.0f;
        if (left) {
            gV[k] += 0.5f * gy * s.W[k];
            gV[k + 1] += 0.5f * gy * s.W[k];
        }
        if (k == b.k) {
            gW[k] += gWb;
            gV[k] += gV0;
            gV[k + 1] += gV1;
        }
    }
    // V = E / Z, Z = sum (E_i + E_{i+1}) W_i / 2
    float gZ = 0.0f;
    float gE[BINS + 1];
    const float iz = 1.0f / s.Z;
#pragma unroll
    for (int i = 0; i <= BINS; ++i) {
        gE[i] = gV[i] * iz;
        gZ -= gV[i] * s.V[i] * iz;
    }
#pragma unroll
    for (int i = 0; i < BINS; ++i) {
        gE[i] += gZ * 0.5f * s.W[i];
        gE[i + 1] += gZ * 0.5f * s.W[i];
        gW[i] += gZ * 0.5f * (s.E[i] + s.E[i + 1]);
    }
#pragma unroll
    for (int i = 0; i <= BINS; ++i) graw[BINS + i] = gE[i] * s.E[i];
    float dot = 0.0f;
#pragma unroll
    for (int k = 0; k < BINS; ++k) dot += gW[k] * s.W[k];
#pragma unroll
    for (int k = 0; k < BINS; ++k) graw[k] = s.W[k] * (gW[k] - dot);
}

// One coupling layer on one sample, P = that layer's parameters: density
// direction (u_B <- C(u_B)) or sampling direction (u_B <- C^-1(u_B));
// returns the log of the spline densities met.
template <bool INVERSE>
__device__ __forceinline__ float layer_step(const float *__restrict__ P, int l, float u[D]) {
    float ua[NA], h1[HID], h2[HID];
#pragma unroll
    for (int t = 0; t < NA; ++t) ua[t] = getu(u, a_idx(l, t));
    hidden(P, ua, h1, h2);
    float lq = 0.0f;
#pragma unroll 1
    for (int t = 0; t < NB; ++t) {
        float raw[RAW];
        out_chunk(P, h2, t, raw);
        Spline s;
        spline_setup(raw, s);
        const int j = b_idx(l, t);
        float v, pdf;
        if (INVERSE)
            spline_inverse(s, getu(u, j), v, pdf);
        else
            spline_forward(s, getu(u, j), v, pdf);
        setu(u, j, v);
        lq += logf(pdf);
    }
    return lq;
}

// Sampling direction through all layers with the weights read from theta
// (global memory, scalar loads), for a thread that runs whole samples.
__device__ __forceinline__ float sample(const float *__restrict__ theta, float u[D]) {
    float lq = 0.0f;
#pragma unroll 1
    for (int l = L - 1; l >= 0; --l) lq += layer_step<true>(theta + l * LP, l, u);
    return lq;
}

}  // namespace flow
}  // namespace mcubes
