// FP32 kernels of the learned proposal: density and sampling of the flow,
// the draw of training samples and the training pass (forward, then the
// backward pass into per-sample scratch fields), in a cooperative form with
// eight waves per 64 samples; the weight gradients as sums over the
// samples; Adam; the FP32 flow-mapped m-Cubes iteration (one thread per
// cube); and the export of one plain iteration's own samples and weights.
#include "flow_impl.h"
#include "vsample_impl.h"

namespace mcubes {

namespace {

using namespace flow;

// Cooperative form: a workgroup of CW waves takes CS = 64 samples (lane =
// sample).  Each matrix product is split over the waves by output feature,
// so the weights a wave reads are the same for all its lanes (scalar loads)
// and its inputs come from LDS, feature-major with one float per sample.
// The arithmetic, and its order, is that of one thread running one sample.
constexpr int CW = 8, CS = 64, CT = CW * CS;

// Transposed weights for the backward products, per layer:
// W1T[HID][IN], W2T[HID][HID], W3T[OUT][HID].
constexpr int T1 = 0, T2 = T1 + HID * IN, T3 = T2 + HID * HID, LPT = T3 + OUT * HID;

struct Coop {
    float X[OUT * CS], Y[OUT * CS];  // activations of the current product
    float U[L + 1][D * CS];          // input of each step, then the output
    float G[2][D * CS];              // dL/du (training)
    float LQ[L * NB * CS];           // log spline density per step and coordinate
};
static_assert(sizeof(Coop) <= 65536, "cooperative LDS");

// acc[j] = sum_i in[i] W[i ld + o0 + j], i ascending, fused: one sample's
// products for NO consecutive outputs; W is wave-uniform, in is LDS.
template <int NO, int NI>
__device__ __forceinline__ void gemm_rows(const float *__restrict__ W, int ld, int o0,
                                          const float *in, int lane, float acc[NO]) {
#pragma unroll
    for (int j = 0; j < NO; ++j) acc[j] = 0.0f;
#pragma unroll 4
    for (int i = 0; i < NI; ++i) {
        const float a = in[i * CS + lane];
        const float *w = W + i * ld + o0;
#pragma unroll
        for (int j = 0; j < NO; ++j) acc[j] = __fmaf_rn(a, w[j], acc[j]);
    }
}

// One coupling layer (P = its parameters) at step `step`: U[step] -> U[step+1].
// With SAVE the layer's input, hidden activations and spline parameters go
// to the sample's scratch fields sc (stride n).
template <bool INVERSE, bool SAVE>
__device__ __forceinline__ void coop_layer(const float *__restrict__ P, int l, int step, int q,
                                           int lane, Coop &S, float *__restrict__ sc, int64_t n,
                                           bool live) {
    const float *Uin = S.U[step];
    float *Uout = S.U[step + 1];
    // one-blob encoding of u_A, rows a BLOBS + k; 12 rows per wave
#pragma unroll
    for (int i = 0; i < IN / CW; ++i) {
        const int r = (IN / CW) * q + i;
        S.X[r * CS + lane] = blob(Uin[a_idx(l, r / BLOBS) * CS + lane], r % BLOBS);
    }
    if (q == CW - 1) {
#pragma unroll
        for (int j = 0; j < D; ++j)
            if (SAVE && live) sc[(FS_U + j) * n] = Uin[j * CS + lane];
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            const int a = a_idx(l, t);
            Uout[a * CS + lane] = Uin[a * CS + lane];
        }
    }
    __syncthreads();
    constexpr int NH = HID / CW, NO3 = (OUT + CW - 1) / CW;
    float acc[NO3];
    gemm_rows<NH, IN>(P + OFF_W1, HID, NH * q, S.X, lane, acc);
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int o = NH * q + j;
        const float h = fmaxf(acc[j] + P[OFF_B1 + o], 0.0f);
        S.Y[o * CS + lane] = h;
        if (SAVE && live) sc[(FS_H1 + o) * n] = h;
    }
    __syncthreads();
    gemm_rows<NH, HID>(P + OFF_W2, HID, NH * q, S.Y, lane, acc);
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int o = NH * q + j;
        const float h = fmaxf(acc[j] + P[OFF_B2 + o], 0.0f);
        S.X[o * CS + lane] = h;
        if (SAVE && live) sc[(FS_H2 + o) * n] = h;
    }
    __syncthreads();
    // (the last wave's columns run past OUT into the next row or b3: in the
    // layer's parameters, and not kept)
    gemm_rows<NO3, HID>(P + OFF_W3, OUT, NO3 * q, S.X, lane, acc);
#pragma unroll
    for (int j = 0; j < NO3; ++j) {
        const int k = NO3 * q + j;
        if (k < OUT) S.Y[k * CS + lane] = acc[j] + P[OFF_B3 + k];
    }
    __syncthreads();
    if (q < NB) {
        float raw[RAW];
#pragma unroll
        for (int k = 0; k < RAW; ++k) {
            raw[k] = S.Y[(q * RAW + k) * CS + lane];
            if (SAVE && live) sc[(FS_DOUT + q * RAW + k) * n] = raw[k];
        }
        Spline sp;
        spline_setup(raw, sp);
        const int j = b_idx(l, q);
        float v, pdf;
        if (INVERSE)
            spline_inverse(sp, Uin[j * CS + lane], v, pdf);
        else
            spline_forward(sp, Uin[j * CS + lane], v, pdf);
        Uout[j * CS + lane] = v;
        S.LQ[(step * NB + q) * CS + lane] = logf(pdf);
    }
    __syncthreads();
}

// Backward pass of layer l (PT = its transposed weights): dL/du at the
// layer's output G[gi] -> at its input G[gi ^ 1]; the deltas of the three
// products go to the scratch fields for the weight gradients.
__device__ __forceinline__ void coop_backward(const float *__restrict__ PT, int l, int q, int lane,
                                              Coop &S, float *__restrict__ sc, int64_t n,
                                              bool live, float c, int gi) {
    const float *Uin = S.U[l];
    const float *Gin = S.G[gi];
    float *Gout = S.G[gi ^ 1];
    if (q < NB) {
        float raw[RAW];
#pragma unroll
        for (int k = 0; k < RAW; ++k) raw[k] = live ? sc[(FS_DOUT + q * RAW + k) * n] : 0.0f;
        Spline sp;
        spline_setup(raw, sp);
        const int j = b_idx(l, q);
        const float ub = Uin[j * CS + lane];
        float y, pdf, gu, graw[RAW];
        spline_forward(sp, ub, y, pdf);
        spline_backward(sp, ub, Gin[j * CS + lane], c / pdf, graw, gu);
        Gout[j * CS + lane] = gu;
#pragma unroll
        for (int k = 0; k < RAW; ++k) {
            S.X[(q * RAW + k) * CS + lane] = graw[k];
            if (live) sc[(FS_DOUT + q * RAW + k) * n] = graw[k];
        }
    }
    __syncthreads();
    constexpr int NH = HID / CW, NR = IN / CW;
    float acc[NR];
    // through W3 and the second ReLU
    gemm_rows<NH, OUT>(PT + T3, HID, NH * q, S.X, lane, acc);
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int i = NH * q + j;
        const float h = live ? sc[(FS_H2 + i) * n] : 0.0f;
        const float d = h > 0.0f ? acc[j] : 0.0f;
        S.Y[i * CS + lane] = d;
        if (live) sc[(FS_D2 + i) * n] = d;
    }
    __syncthreads();
    // through W2 and the first ReLU
    gemm_rows<NH, HID>(PT + T2, HID, NH * q, S.Y, lane, acc);
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int i = NH * q + j;
        const float h = live ? sc[(FS_H1 + i) * n] : 0.0f;
        const float d = h > 0.0f ? acc[j] : 0.0f;
        S.X[i * CS + lane] = d;
        if (live) sc[(FS_D1 + i) * n] = d;
    }
    __syncthreads();
    // through W1 to the one-blob inputs
    gemm_rows<NR, HID>(PT + T1, IN, NR * q, S.X, lane, acc);
#pragma unroll
    for (int j = 0; j < NR; ++j) S.Y[(NR * q + j) * CS + lane] = acc[j];
    __syncthreads();
    // and through the encoding into the conditioning coordinates
    if (q < NA) {
        const int j = a_idx(l, q);
        const float ux = Uin[j * CS + lane];
        float a = 0.0f;
#pragma unroll 4
        for (int k = 0; k < BLOBS; ++k) {
            const float t = (ux - ((float)k + 0.5f) * (1.0f / BLOBS)) * (float)BLOBS;
            a = __fmaf_rn(S.Y[(q * BLOBS + k) * CS + lane], -expf(-0.5f * t * t) * t * (float)BLOBS,
                          a);
        }
        Gout[j * CS + lane] = Gin[j * CS + lane] + a;
    }
    __syncthreads();
}

// log q of the sample: the spline densities in the order they were met
__device__ __forceinline__ float coop_logq(const Coop &S, int lane) {
    float lq = 0.0f;
#pragma unroll
    for (int i = 0; i < L * NB; ++i) lq += S.LQ[i * CS + lane];
    return lq;
}

__device__ __forceinline__ int wave_index() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / CS));
}

// density (x -> z) or sampling (z -> x) of n samples
template <bool INVERSE>
__global__ __launch_bounds__(CT) void map_kernel(const float *__restrict__ theta,
                                                 const double *__restrict__ in, int64_t n,
                                                 double *__restrict__ out,
                                                 double *__restrict__ logq) {
    __shared__ Coop S;
    const int q = wave_index(), lane = threadIdx.x % CS;
    const int64_t s = (int64_t)blockIdx.x * CS + lane;
    const bool live = s < n;
    if (q == 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) S.U[0][j * CS + lane] = live ? (float)in[s * D + j] : 0.5f;
    }
    __syncthreads();
#pragma unroll 1
    for (int step = 0; step < L; ++step) {
        const int l = INVERSE ? L - 1 - step : step;
        coop_layer<INVERSE, false>(theta + l * LP, l, step, q, lane, S, nullptr, n, live);
    }
    if (q == 0 && live) {
#pragma unroll
        for (int j = 0; j < D; ++j) out[s * D + j] = (double)S.U[L][j * CS + lane];
        logq[s] = (double)coop_logq(S, lane);
    }
}

// transposed copies of the three weight matrices of every layer
__global__ void transpose_kernel(const float *__restrict__ theta, float *__restrict__ thetaT) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L * LPT) return;
    const float *P = theta + (i / LPT) * LP;
    int r = i % LPT;
    float v;
    if (r < T2) {
        v = P[OFF_W1 + (r % IN) * HID + r / IN];
    } else if (r < T3) {
        r -= T2;
        v = P[OFF_W2 + (r % HID) * HID + r / HID];
    } else {
        r -= T3;
        v = P[OFF_W3 + (r % HID) * OUT + r / HID];
    }
    thetaT[i] = v;
}

// sum of the n weights (one block of 1024 threads, fixed order)
__global__ __launch_bounds__(1024) void wsum_kernel(const double *__restrict__ w, int64_t n,
                                                    double *__restrict__ out) {
    __shared__ double red[1024];
    double a = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += 1024) a += w[s];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Forward and backward pass of the weighted negative log-likelihood: loss
// contribution c log q(x) of each sample, c = -w / sum w.  The weight
// gradients are formed afterwards from the scratch fields.
__global__ __launch_bounds__(CT, 4) void train_kernel(const float *__restrict__ theta,
                                                   const float *__restrict__ thetaT,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ w, int64_t n,
                                                   const double *__restrict__ wsum,
                                                   float *__restrict__ scratch,
                                                   double *__restrict__ loss) {
    __shared__ Coop S;
    const int q = wave_index(), lane = threadIdx.x % CS;
    const int64_t s = (int64_t)blockIdx.x * CS + lane;
    const bool live = s < n;
    const float c = live ? (float)(-w[s] / *wsum) : 0.0f;
    if (q == 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) S.U[0][j * CS + lane] = live ? (float)x[s * D + j] : 0.5f;
    }
    if (q == 1) {
#pragma unroll
        for (int j = 0; j < D; ++j) S.G[0][j * CS + lane] = 0.0f;
    }
    __syncthreads();
#pragma unroll 1
    for (int l = 0; l < L; ++l)
        coop_layer<false, true>(theta + l * LP, l, l, q, lane, S, scratch + (int64_t)l * FS * n + s,
                                n, live);
    int gi = 0;
#pragma unroll 1
    for (int l = L - 1; l >= 0; --l) {
        coop_backward(thetaT + l * LPT, l, q, lane, S, scratch + (int64_t)l * FS * n + s, n, live, c,
                      gi);
        gi ^= 1;
    }
    if (q == 0) {
        const double v = wave_sum(live ? (double)c * (double)coop_logq(S, lane) : 0.0);
        if (lane == 0) unsafeAtomicAdd(loss, v);
    }
}

// Weight gradients as sums over the batch of inputs x deltas: per layer
// W1 (96 x 64, inputs the one-blob encoding), W2 (64 x 64, inputs h1) and W3
// (64 x 99, inputs h2).  Output tiles of 64 x 64, 4 x 4 per thread, inputs
// and deltas staged in LDS sample-major 32 samples at a time; the batch is
// cut into slices of ks samples (blockIdx.y) whose partial sums land in
// part[slice][parameter] and are added in slice order afterwards, so the
// result does not depend on scheduling.  The tiles whose rows start at 0
// also sum their delta columns over the slice: the bias gradients.
constexpr int WT = 64, WKC = 32, WPAD = WT + 4;
constexpr int TILES_L = 5;  // W1 rows 0-63 | W1 rows 64-95 | W2 | W3 cols 0-63 | W3 cols 64-98
constexpr int kMaxSlices = 64;
static_assert(kMaxSlices <= kWgradSlices, "slice buffer");

__global__ __launch_bounds__(256) void wgrad_kernel(const float *__restrict__ scratch, int64_t n,
                                                    int64_t ks, float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) float As[WKC][WPAD];
    __shared__ __attribute__((aligned(16))) float Bs[WKC][WPAD];
    const int l = blockIdx.x / TILES_L, tile = blockIdx.x % TILES_L;
    const int64_t s_begin = (int64_t)blockIdx.y * ks;
    const int64_t s_end = s_begin + ks < n ? s_begin + ks : n;
    int mat, r0, rows, c0, cols;
    switch (tile) {
    case 0: mat = 0; r0 = 0; rows = 64; c0 = 0; cols = HID; break;
    case 1: mat = 0; r0 = 64; rows = IN - 64; c0 = 0; cols = HID; break;
    case 2: mat = 1; r0 = 0; rows = HID; c0 = 0; cols = HID; break;
    case 3: mat = 2; r0 = 0; rows = HID; c0 = 0; cols = 64; break;
    default: mat = 2; r0 = 0; rows = HID; c0 = 64; cols = OUT - 64; break;
    }
    const float *sc = scratch + (int64_t)l * FS * n;
    const int bfield = mat == 0 ? FS_D1 : (mat == 1 ? FS_D2 : FS_DOUT);
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
    const bool bias_tile = r0 == 0 && ty == 0;  // 16 threads, 4 columns each
    float acc[4][4], bsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
    for (int64_t s0 = s_begin; s0 < s_end; s0 += WKC) {
        // stage: thread -> (row, sample) pairs, samples contiguous in memory
#pragma unroll
        for (int i = 0; i < (WT * WKC) / 256; ++i) {
            const int idx = threadIdx.x + 256 * i;
            const int rr = idx / WKC, ss = idx % WKC;
            const int64_t s = s0 + ss;
            float av = 0.0f, bv = 0.0f;
            if (s < s_end) {
                if (rr < rows) {
                    const int R = r0 + rr;
                    if (mat == 0)
                        av = blob(sc[(FS_U + a_idx(l, R / BLOBS)) * n + s], R % BLOBS);
                    else
                        av = sc[((mat == 1 ? FS_H1 : FS_H2) + R) * n + s];
                }
                if (rr < cols) bv = sc[(bfield + c0 + rr) * n + s];
            }
            As[ss][rr] = av;
            Bs[ss][rr] = bv;
        }
        __syncthreads();
#pragma unroll 8
        for (int ss = 0; ss < WKC; ++ss) {
            const float4 a = *reinterpret_cast<const float4 *>(&As[ss][4 * ty]);
            const float4 b = *reinterpret_cast<const float4 *>(&Bs[ss][4 * tx]);
            const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __fmaf_rn(av[i], bv[j], acc[i][j]);
        }
        if (bias_tile) {
            for (int ss = 0; ss < WKC; ++ss) {
                const float4 b = *reinterpret_cast<const float4 *>(&Bs[ss][4 * tx]);
                bsum[0] += b.x;
                bsum[1] += b.y;
                bsum[2] += b.z;
                bsum[3] += b.w;
            }
        }
        __syncthreads();
    }
    float *G = part + (int64_t)blockIdx.y * PARAMS + l * LP;
    if (bias_tile) {
        const int boff = mat == 0 ? OFF_B1 : (mat == 1 ? OFF_B2 : OFF_B3);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (4 * tx + j < cols) G[boff + c0 + 4 * tx + j] = bsum[j];
    }
    const int off = mat == 0 ? OFF_W1 : (mat == 1 ? OFF_W2 : OFF_W3);
    const int ld = mat == 2 ? OUT : HID;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = 4 * ty + i;
        if (rr >= rows) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cc = 4 * tx + j;
            if (cc < cols) G[off + (r0 + rr) * ld + c0 + cc] = acc[i][j];
        }
    }
}

// grad[i] = sum over the slices, in slice order
__global__ void wgrad_sum_kernel(const float *__restrict__ part, int slices,
                                 float *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= PARAMS) return;
    grad[i] = slice_sum(part, slices, i);
}

// one workgroup per minibatch: the sum of its weights (fixed order)
__global__ __launch_bounds__(1024) void batch_wsum_kernel(const double *__restrict__ w, int64_t n,
                                                          int64_t batch, double *__restrict__ out) {
    __shared__ double red[1024];
    const int64_t b0 = (int64_t)blockIdx.x * batch;
    const int64_t b1 = b0 + batch < n ? b0 + batch : n;
    double a = 0.0;
    for (int64_t s = b0 + threadIdx.x; s < b1; s += 1024) a += w[s];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void zero_u32_kernel(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Records (I_t, var_t) of flow-mapped iteration t in the combined state and
// recombines iterations 0..t with equal weights: they all sample the same
// proposal with the same number of points, so the plain mean is unbiased
// (variance weights would favour the iterations that missed the rare large
// weights).  Ibar = sum I / T, sigma = sqrt(sum var) / T, chi2/dof over the
// iterations with var > 0.  Header layout as for the plain combination.
__global__ void flow_combine_kernel(const double *__restrict__ est, double *__restrict__ state,
                                    uint32_t t, double rel_tol, int min_iters) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double *hist = state + MCUBES_STATE_HEADER;
    const double It = est[0], Vt = est[1];
    hist[2 * t] = It;
    hist[2 * t + 1] = Vt;
    if (!isfinite(It) || !isfinite(Vt)) state[6] = 1.0;
    const int T = (int)t + 1;
    double si = 0.0, sv = 0.0;
    for (int q = 0; q < T; ++q) {
        si = si + hist[2 * q];
        sv = sv + hist[2 * q + 1];
    }
    const double Ibar = si / (double)T;
    double chi2 = 0.0, ss = 0.0;
    for (int q = 0; q < T; ++q) {
        const double dv = hist[2 * q] - Ibar;
        ss = ss + dv * dv;
        const double v = hist[2 * q + 1];
        if (v > 0.0) chi2 = chi2 + dv * dv / v;
    }
    // the standard deviation of the mean, from the iterations' own variances
    // and from the scatter of their estimates; the larger is reported
    const double s_w = sqrt(sv) / (double)T;
    const double s_b = T > 1 ? sqrt(ss / ((double)T * (double)(T - 1))) : 0.0;
    const double sigma = s_b > s_w ? s_b : s_w;
    state[0] = Ibar;
    state[1] = sigma;
    state[2] = T > 1 ? chi2 / (double)(T - 1) : 0.0;
    state[3] = (double)(T - 1);
    state[4] = (double)T;
    state[5] = (T >= min_iters && sigma <= rel_tol * fabs(Ibar)) ? 1.0 : 0.0;
}

// Row j of the output is row (a j) mod n of the input (x: 6 doubles per row,
// w: one); with a coprime to n this is a permutation.
__global__ void shuffle_rows_kernel(const double *__restrict__ x, const double *__restrict__ w,
                                    int64_t n, uint64_t a, double *__restrict__ xo,
                                    double *__restrict__ wo) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t src = (int64_t)(((uint64_t)j * a) % (uint64_t)n);
    const double *xi = x + src * flow::D;
    double *xj = xo + j * flow::D;
#pragma unroll
    for (int k = 0; k < flow::D; ++k) xj[k] = xi[k];
    wo[j] = w[src];
}

__global__ void widen_kernel(const float *__restrict__ in, int64_t n, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

__global__ void pow_kernel(double *__restrict__ w, int64_t n, double power) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = pow(w[i], power);
}

// One Adam step on the FP32 master parameters; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_kernel(float *__restrict__ theta, float *__restrict__ m,
                            float *__restrict__ v, const float *__restrict__ grad, int count,
                            float lr, float beta1, float beta2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    adam_update(theta, m, v, i, grad[i], lr, beta1, beta2, eps, c1, c2);
}

// The flow as the map of an m-Cubes iteration: cube c's sample k draws u
// from Philox as V-Sample does (stream word with the high bit set), z_j =
// (c_j + u_j) / g, x = flow sample of z (FP32), w = f(x) / q(x) in FP64.  A
// persistent grid walks the cubes; per-block partials (sum S_c, sum var_c).
template <int F>
__global__ __launch_bounds__(256) void flow_vsample_kernel(const float *__restrict__ theta,
                                                           const VsArgs A, uint32_t stream_word,
                                                           double *__restrict__ partials,
                                                           uint32_t *__restrict__ whist) {
    constexpr int NBLK = (D + 3) / 4;
    __shared__ uint32_t hist[WH_BINS];
    wh_clear(hist);
    __syncthreads();
    const uint32_t T = gridDim.x * blockDim.x;
    double tS = 0.0, tV = 0.0;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < A.m; c += T) {
        double dig[D];
        uint32_t rest = c;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            dig[j] = (double)(rest % A.g);
            rest /= A.g;
        }
        double S = 0.0, D1 = 0.0, D2 = 0.0, w0 = 0.0;
        for (uint32_t k = 0; k < A.p; ++k) {
            float u[D];
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                uint32_t r[4];
                philox10(c, stream_word, k * NBLK + b, A.iteration, A.key0, A.key1, r);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = 4 * b + q;
                    if (j < D) {
                        const double uu = __fma_rn((double)r[q], 0x1p-32, 0x1p-33);
                        u[j] = (float)((dig[j] + uu) / (double)A.g);
                    }
                }
            }
            const float lq = sample(theta, u);
            Acc acc = Family<F, D>::begin(A.phase);
#pragma unroll
            for (int j = 0; j < D; ++j) Family<F, D>::axis(acc, A.ca[j], A.cu[j], (double)u[j]);
            const double w = Family<F, D>::end(acc, A) / exp((double)lq);
            wh_add(hist, w);
            S = S + w;
            if (k == 0) w0 = w;
            const double dlt = w - w0;
            D1 = D1 + dlt;
            D2 = D2 + dlt * dlt;
        }
        tS += S;
        tV += (D2 - D1 * D1 * A.inv_p) * A.inv_pm1;
    }
    __shared__ double red[2][4];
    tS = wave_sum(tS);
    tV = wave_sum(tV);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = tS;
        red[1][threadIdx.x >> 6] = tV;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, v = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            s += red[0][q];
            v += red[1][q];
        }
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = v;
    }
    wh_flush(hist, whist);
}

// The FP32 flow-mapped iteration in the cooperative form, for p dividing
// 64: each pass of a workgroup takes 64 consecutive samples q (cube q / p,
// sample q % p), so the p samples of a cube sit in one wave; the same
// counters and map as flow_vsample_kernel, the flow run by the eight waves
// together, and the per-cube sums by butterfly shuffles in wave 0.
template <int F>
__global__ __launch_bounds__(CT) void flow_vsample_coop_kernel(const float *__restrict__ theta,
                                                               const VsArgs A,
                                                               uint32_t stream_word,
                                                               double *__restrict__ partials,
                                                               uint32_t *__restrict__ whist) {
    constexpr int NBLK = (D + 3) / 4;
    __shared__ Coop S;
    __shared__ uint32_t hist[WH_BINS];
    wh_clear(hist);
    const int q = wave_index(), lane = threadIdx.x % CS;
    const uint64_t N = (uint64_t)A.m * A.p;
    const int p = (int)A.p;
    double tS = 0.0, tV = 0.0;
    for (uint64_t base = (uint64_t)blockIdx.x * CS; base < N; base += (uint64_t)gridDim.x * CS) {
        const uint64_t qs = base + lane;
        const bool live = qs < N;  // N is a multiple of p: a cube is live or not as a whole
        if (q == 0) {
            const uint32_t c = live ? (uint32_t)(qs / p) : 0u;
            const uint32_t k = live ? (uint32_t)(qs % p) : 0u;
            uint32_t rest = c;
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                uint32_t r[4];
                philox10(c, stream_word, k * NBLK + b, A.iteration, A.key0, A.key1, r);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = 4 * b + i;
                    if (j < D) {
                        const double dig = (double)(rest % A.g);
                        rest /= A.g;
                        const double uu = __fma_rn((double)r[i], 0x1p-32, 0x1p-33);
                        S.U[0][j * CS + lane] = (float)((dig + uu) / (double)A.g);
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int step = 0; step < L; ++step)
            coop_layer<true, false>(theta + (L - 1 - step) * LP, L - 1 - step, step, q, lane, S,
                                    nullptr, 0, live);
        if (q == 0) {
            double w = 0.0;
            if (live) {
                Acc acc = Family<F, D>::begin(A.phase);
#pragma unroll
                for (int j = 0; j < D; ++j)
                    Family<F, D>::axis(acc, A.ca[j], A.cu[j], (double)S.U[L][j * CS + lane]);
                w = Family<F, D>::end(acc, A) / exp((double)coop_logq(S, lane));
                wh_add(hist, w);
            }
            // per-cube sums over the p lanes of the cube, shifted by its first sample
            const int first = lane - (lane % p);
            const double w0 = __shfl(w, first);
            const double dlt = w - w0;
            double Sc = w, D1 = dlt, D2 = dlt * dlt;
            for (int off = 1; off < p; off <<= 1) {
                Sc += __shfl_xor(Sc, off);
                D1 += __shfl_xor(D1, off);
                D2 += __shfl_xor(D2, off);
            }
            if (live && lane == first) {
                tS += Sc;
                tV += (D2 - D1 * D1 * A.inv_p) * A.inv_pm1;
            }
        }
        __syncthreads();  // S is reused by the next pass
    }
    if (q == 0) {
        tS = wave_sum(tS);
        tV = wave_sum(tV);
        if (lane == 0) {
            partials[2 * blockIdx.x] = tS;
            partials[2 * blockIdx.x + 1] = tV;
        }
    }
    wh_flush(hist, whist);
}

// The samples of work items [w0, w0 + count) of one plain iteration (cube
// (w mult) mod m, the order in which V-Sample's threads visit the cubes, so
// that a prefix of the work items is spread over the whole domain), with
// their weights w = f J: the same counters, bins and arithmetic as V-Sample,
// so these are samples that iteration draws.  x: (count p) x D, w: count p.
template <int F, int DIM>
__global__ __launch_bounds__(256) void dump_kernel(const VsArgs A, const double *__restrict__ grid,
                                                   uint32_t w0, uint32_t count,
                                                   double *__restrict__ xs,
                                                   double *__restrict__ ws) {
    constexpr int NBLK = (DIM + 3) / 4;
    const uint32_t q0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (q0 >= count) return;
    const uint32_t c = (uint32_t)(((uint64_t)(w0 + q0) * A.mult) % A.m);
    const int nb = (int)A.nb;
    double cb[DIM];
    uint32_t rest = c;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        cb[j] = __fma_rn((double)(rest % A.g), 0x1p32, 0.5);
        rest /= A.g;
    }
    for (uint32_t k = 0; k < A.p; ++k) {
        Acc acc = Family<F, DIM>::begin(A.phase);
        double prod = 1.0;
        const uint64_t row = (uint64_t)q0 * A.p + k;
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            uint32_t r[4];
            philox10(c, A.stream_id, k * NBLK + b, A.iteration, A.key0, A.key1, r);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = 4 * b + q;
                if (j < DIM) {
                    const double z = ((double)r[q] + cb[j]) * A.zscale;
                    int i = (int)z;
                    double phi;
                    if constexpr (DIM >= 2) {
                        phi = __builtin_amdgcn_fract(z);
                    } else {
                        i = i < nb - 1 ? i : nb - 1;
                        phi = z - (double)i;
                    }
                    const double *e = grid + j * (nb + 1) + i;
                    const double W = e[1] - e[0];
                    const double x = __fma_rn(W, phi, e[0]);
                    prod = prod * W;
                    Family<F, DIM>::axis(acc, A.ca[j], A.cu[j], x);
                    xs[row * DIM + j] = x;
                }
            }
        }
        ws[row] = Family<F, DIM>::end(acc, A) * (A.nbd * prod);
    }
}

// n plain (unstratified) samples of the flow with their weights w = f / q:
// sample i draws z from Philox counter (i, stream word, block, iteration).
template <int F>
__global__ __launch_bounds__(CT) void flow_draw_kernel(const float *__restrict__ theta,
                                                       const VsArgs A, uint32_t stream_word,
                                                       uint32_t n, double *__restrict__ xs,
                                                       double *__restrict__ ws) {
    constexpr int NBLK = (D + 3) / 4;
    __shared__ Coop S;
    const int q = wave_index(), lane = threadIdx.x % CS;
    const uint32_t i = blockIdx.x * CS + lane;
    const bool live = i < n;
    if (q == 0) {
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            uint32_t r[4];
            philox10(i, stream_word, b, A.iteration, A.key0, A.key1, r);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * b + t < D)
                    S.U[0][(4 * b + t) * CS + lane] = (float)__fma_rn((double)r[t], 0x1p-32, 0x1p-33);
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int step = 0; step < L; ++step)
        coop_layer<true, false>(theta + (L - 1 - step) * LP, L - 1 - step, step, q, lane, S,
                                nullptr, n, live);
    if (q != 0 || !live) return;
    Acc acc = Family<F, D>::begin(A.phase);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double u = (double)S.U[L][j * CS + lane];
        Family<F, D>::axis(acc, A.ca[j], A.cu[j], u);
        xs[(uint64_t)i * D + j] = u;
    }
    ws[i] = Family<F, D>::end(acc, A) / exp((double)coop_logq(S, lane));
}

template <int F>
hipError_t launch_flow_draw_f(const float *theta, const VsArgs &A, uint32_t stream_word,
                              uint32_t n, double *xs, double *ws, hipStream_t s) {
    hipLaunchKernelGGL((flow_draw_kernel<F>), dim3((n + CS - 1) / CS), dim3(CT), 0, s, theta, A,
                       stream_word, n, xs, ws);
    return hipGetLastError();
}

template <int F>
hipError_t launch_flow_vsample_f(const float *theta, const VsArgs &A, uint32_t stream_word,
                                 double *partials, uint32_t *whist, int blocks, hipStream_t s) {
    if (64 % A.p == 0)
        hipLaunchKernelGGL((flow_vsample_coop_kernel<F>), dim3(blocks), dim3(CT), 0, s, theta, A,
                           stream_word, partials, whist);
    else
        hipLaunchKernelGGL((flow_vsample_kernel<F>), dim3(blocks), dim3(256), 0, s, theta, A,
                           stream_word, partials, whist);
    return hipGetLastError();
}

template <int F>
hipError_t launch_dump_f(int dim, const VsArgs &A, const double *grid, uint32_t c0,
                         uint32_t count, double *xs, double *ws, hipStream_t s) {
    const dim3 grid_dim((count + 255) / 256);
#define DUMP_CASE(DD)                                                                            \
    case DD:                                                                                     \
        hipLaunchKernelGGL((dump_kernel<F, DD>), grid_dim, dim3(256), 0, s, A, grid, c0, count, \
                           xs, ws);                                                              \
        break;
    switch (dim) {
        DUMP_CASE(1) DUMP_CASE(2) DUMP_CASE(3) DUMP_CASE(4) DUMP_CASE(5)
        DUMP_CASE(6) DUMP_CASE(7) DUMP_CASE(8) DUMP_CASE(9) DUMP_CASE(10)
    default: return hipErrorInvalidValue;
    }
#undef DUMP_CASE
    return hipGetLastError();
}

}  // namespace

hipError_t launch_flow_density(const float *theta, const double *x, int64_t n, double *z,
                               double *logq, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(map_kernel<false>, dim3((unsigned)((n + CS - 1) / CS)), dim3(CT), 0, s,
                       theta, x, n, z, logq);
    return hipGetLastError();
}

hipError_t launch_flow_sample(const float *theta, const double *z, int64_t n, double *x,
                              double *logq, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(map_kernel<true>, dim3((unsigned)((n + CS - 1) / CS)), dim3(CT), 0, s,
                       theta, z, n, x, logq);
    return hipGetLastError();
}

// per-sample fields, the partial weight gradients of the slices, then the
// BF16 training pass's own per-sample state
int64_t flow_scratch_floats(int64_t n) {
    return (int64_t)L * FS * n + (int64_t)kWgradSlices * PARAMS + flow_bf16_train_extra_floats(n);
}

hipError_t launch_flow_wgrad_sum(const float *part, int slices, float *grad, hipStream_t s) {
    hipLaunchKernelGGL(wgrad_sum_kernel, dim3((PARAMS + 255) / 256), dim3(256), 0, s, part, slices,
                       grad);
    return hipGetLastError();
}

int64_t flow_transposed_floats() { return (int64_t)L * LPT; }

hipError_t launch_flow_wsum(const double *w, int64_t n, double *wsum, hipStream_t s) {
    hipLaunchKernelGGL(wsum_kernel, dim3(1), dim3(1024), 0, s, w, n, wsum);
    return hipGetLastError();
}

hipError_t launch_flow_train_fp32(const float *theta, float *thetaT, const double *x,
                                  const double *w, int64_t n, const double *wsum, float *scratch,
                                  double *loss, hipStream_t s) {
    hipLaunchKernelGGL(transpose_kernel, dim3((L * LPT + 255) / 256), dim3(256), 0, s, theta,
                       thetaT);
    hipLaunchKernelGGL(train_kernel, dim3((unsigned)((n + CS - 1) / CS)), dim3(CT), 0, s, theta,
                       thetaT, x, w, n, wsum, scratch, loss);
    return hipGetLastError();
}

hipError_t launch_flow_wgrad(const float *scratch_in, int64_t n, float *grad, hipStream_t s) {
    float *scratch = const_cast<float *>(scratch_in);
    // slices of at least 512 samples, at most kMaxSlices of them
    int64_t slices = (n + 511) / 512;
    if (slices > kMaxSlices) slices = kMaxSlices;
    int64_t ks = (n + slices - 1) / slices;
    ks = (ks + WKC - 1) / WKC * WKC;
    slices = (n + ks - 1) / ks;
    float *part = scratch + (int64_t)L * FS * n;
    hipLaunchKernelGGL(wgrad_kernel, dim3(L * TILES_L, (unsigned)slices), dim3(256), 0, s, scratch,
                       n, ks, part);
    hipLaunchKernelGGL(wgrad_sum_kernel, dim3((PARAMS + 255) / 256), dim3(256), 0, s, part,
                       (int)slices, grad);
    return hipGetLastError();
}

hipError_t launch_flow_batch_wsums(const double *w, int64_t n, int64_t batch, double *out,
                                   hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_wsum_kernel, dim3((unsigned)((n + batch - 1) / batch)), dim3(1024), 0,
                       s, w, n, batch, out);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_flow_combine(const double *est, double *state, uint32_t iteration,
                               double rel_tol, int min_iters, hipStream_t s) {
    hipLaunchKernelGGL(flow_combine_kernel, dim3(1), dim3(64), 0, s, est, state, iteration,
                       rel_tol, min_iters);
    return hipGetLastError();
}

hipError_t launch_flow_shuffle(const double *x, const double *w, int64_t n, uint64_t a,
                               double *xo, double *wo, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(shuffle_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x,
                       w, n, a, xo, wo);
    return hipGetLastError();
}

hipError_t launch_flow_widen(const float *in, int64_t n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_pow_weights(double *w, int64_t n, double power, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pow_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, n, power);
    return hipGetLastError();
}

hipError_t launch_flow_adam(float *theta, float *m, float *v, const float *grad, float lr,
                            float beta1, float beta2, float eps, float c1, float c2,
                            hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((PARAMS + 255) / 256), dim3(256), 0, s, theta, m, v,
                       grad, PARAMS, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_flow_vsample(int family, const float *theta, const VsArgs &A,
                               uint32_t stream_word, double *partials, uint32_t *whist,
                               int blocks, hipStream_t s) {
    switch (family) {
    case MCUBES_OSCILLATORY: return launch_flow_vsample_f<MCUBES_OSCILLATORY>(theta, A, stream_word, partials, whist, blocks, s);
    case MCUBES_PRODUCT_PEAK: return launch_flow_vsample_f<MCUBES_PRODUCT_PEAK>(theta, A, stream_word, partials, whist, blocks, s);
    case MCUBES_CORNER_PEAK: return launch_flow_vsample_f<MCUBES_CORNER_PEAK>(theta, A, stream_word, partials, whist, blocks, s);
    case MCUBES_GAUSSIAN: return launch_flow_vsample_f<MCUBES_GAUSSIAN>(theta, A, stream_word, partials, whist, blocks, s);
    case MCUBES_C0: return launch_flow_vsample_f<MCUBES_C0>(theta, A, stream_word, partials, whist, blocks, s);
    case MCUBES_DISCONTINUOUS: return launch_flow_vsample_f<MCUBES_DISCONTINUOUS>(theta, A, stream_word, partials, whist, blocks, s);
    case MCUBES_ADDITION: return launch_flow_vsample_f<MCUBES_ADDITION>(theta, A, stream_word, partials, whist, blocks, s);
    case MCUBES_MIXTURE: return launch_flow_vsample_f<MCUBES_MIXTURE>(theta, A, stream_word, partials, whist, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_flow_draw(int family, const float *theta, const VsArgs &A,
                            uint32_t stream_word, uint32_t n, double *xs, double *ws,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    switch (family) {
    case MCUBES_OSCILLATORY: return launch_flow_draw_f<MCUBES_OSCILLATORY>(theta, A, stream_word, n, xs, ws, s);
    case MCUBES_PRODUCT_PEAK: return launch_flow_draw_f<MCUBES_PRODUCT_PEAK>(theta, A, stream_word, n, xs, ws, s);
    case MCUBES_CORNER_PEAK: return launch_flow_draw_f<MCUBES_CORNER_PEAK>(theta, A, stream_word, n, xs, ws, s);
    case MCUBES_GAUSSIAN: return launch_flow_draw_f<MCUBES_GAUSSIAN>(theta, A, stream_word, n, xs, ws, s);
    case MCUBES_C0: return launch_flow_draw_f<MCUBES_C0>(theta, A, stream_word, n, xs, ws, s);
    case MCUBES_DISCONTINUOUS: return launch_flow_draw_f<MCUBES_DISCONTINUOUS>(theta, A, stream_word, n, xs, ws, s);
    case MCUBES_ADDITION: return launch_flow_draw_f<MCUBES_ADDITION>(theta, A, stream_word, n, xs, ws, s);
    case MCUBES_MIXTURE: return launch_flow_draw_f<MCUBES_MIXTURE>(theta, A, stream_word, n, xs, ws, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vsample_dump(int family, int dim, const VsArgs &A, const double *grid,
                               uint32_t c0, uint32_t count, double *xs, double *ws,
                               hipStream_t s) {
    if (count == 0) return hipSuccess;
    switch (family) {
    case MCUBES_OSCILLATORY: return launch_dump_f<MCUBES_OSCILLATORY>(dim, A, grid, c0, count, xs, ws, s);
    case MCUBES_PRODUCT_PEAK: return launch_dump_f<MCUBES_PRODUCT_PEAK>(dim, A, grid, c0, count, xs, ws, s);
    case MCUBES_CORNER_PEAK: return launch_dump_f<MCUBES_CORNER_PEAK>(dim, A, grid, c0, count, xs, ws, s);
    case MCUBES_GAUSSIAN: return launch_dump_f<MCUBES_GAUSSIAN>(dim, A, grid, c0, count, xs, ws, s);
    case MCUBES_C0: return launch_dump_f<MCUBES_C0>(dim, A, grid, c0, count, xs, ws, s);
    case MCUBES_DISCONTINUOUS: return launch_dump_f<MCUBES_DISCONTINUOUS>(dim, A, grid, c0, count, xs, ws, s);
    case MCUBES_ADDITION: return launch_dump_f<MCUBES_ADDITION>(dim, A, grid, c0, count, xs, ws, s);
    case MCUBES_MIXTURE: return launch_dump_f<MCUBES_MIXTURE>(dim, A, grid, c0, count, xs, ws, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mcubes
