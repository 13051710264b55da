// The flow on the BF16 matrix cores (gfx950 v_mfma_f32_32x32x16_bf16, FP32
// accumulation): sampling, the flow-mapped iteration (the proposal's hot
// loop) and the forward and backward pass of training.
//
// A wave carries 64 samples, one per lane for the per-sample work (Philox,
// spline inversion, integrand), and runs each conditioner as three chained
// matrix products in transposed form, out^T = W^T in^T: features are the
// matrix rows (M), the 64 samples two blocks of 32 columns (N).  With that
// orientation the accumulator of one product (lane l holds column l % 32 and
// rows 8 (r/4) + 4 (l/32) + r%4 of a 32-row tile, r = 0..15) is, after bias,
// ReLU and rounding to BF16, already the B operand of the next product (lane
// l holds K values 8 (l/32) .. +7 of column l % 32) provided the K order of a
// step is the one the accumulator registers hold: the weight fragments are
// packed with that order, so activations never leave the registers.  The
// one-blob inputs of the first product are computed directly in operand
// order.  At the end, one v_permlane32_swap per accumulator register gives
// every lane all 99 outputs of its own sample.
//
// Rounding: weights and the inputs of every product are BF16 (round to
// nearest even), biases and accumulation FP32, the splines FP32, the
// integrand and weights FP64.
#include "flow_impl.h"
#include "vsample_impl.h"

namespace mcubes {

namespace {

using namespace flow;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// fragments per layer: first product 2 row tiles x 6 K steps, second 2 x 4,
// third 4 x 4 (99 outputs padded to 128)
constexpr int G1T = 2, G1K = 6, G2T = 2, G2K = 4, G3T = 4, G3K = 4;
constexpr int OFF_G1 = 0, OFF_G2 = OFF_G1 + G1T * G1K, OFF_G3 = OFF_G2 + G2T * G2K;
constexpr int FRAGS = OFF_G3 + G3T * G3K;  // 36
// biases per layer in accumulator order: [tile][lane half][register]
constexpr int BOFF_1 = 0, BOFF_2 = BOFF_1 + G1T * 32, BOFF_3 = BOFF_2 + G2T * 32;
constexpr int BIAS = BOFF_3 + G3T * 32;  // 256

// feature held by accumulator register r of lane half h in row tile t
__host__ __device__ constexpr int acc_feature(int t, int r, int h) {
    return 32 * t + 8 * (r / 4) + 4 * h + (r % 4);
}

__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t b = __float_as_uint(f);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Eight consecutive biases (16-byte aligned: every run starts at a multiple
// of 8 floats) as two 16-byte loads.
__device__ __forceinline__ void load_bias8(const float *__restrict__ p, float b[8]) {
    const float4 x = *reinterpret_cast<const float4 *>(p);
    const float4 y = *reinterpret_cast<const float4 *>(p + 4);
    b[0] = x.x; b[1] = x.y; b[2] = x.z; b[3] = x.w;
    b[4] = y.x; b[5] = y.y; b[6] = y.z; b[7] = y.w;
}

__device__ __forceinline__ bf16x8 pack8(const float v[8]) {
    bf16x8 r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = __builtin_bit_cast(__bf16, bf16_bits(v[i]));
    return r;
}

// Eight consecutive bumps of the one-blob encoding, k = k0 .. k0 + 7:
// e_k = exp(-(t - k)^2 / 2) with t = 32 u - 1/2.  The first directly, the
// rest by the ratio e_{k+1} / e_k = exp(t - k - 1/2), which itself shrinks
// by the constant exp(-1) per step: 2 exponentials and 14 multiplications
// instead of 8 exponentials.  Relative error below 1e-6 (seven rounded
// products), far under the BF16 rounding these inputs receive.  Starting
// at k0 keeps the first term representable whenever any of the eight
// matters: |t - k0| <= 13 if some |t - k| <= 6 (exp(-84.5) > FLT_MIN).
__device__ __forceinline__ void blob8(float u, int k0, float e[8]) {
    const float d = u * (float)BLOBS - 0.5f - (float)k0;
    e[0] = expf(-0.5f * d * d);
    float r = expf(d - 0.5f);
#pragma unroll
    for (int i = 1; i < 8; ++i) {
        e[i] = e[i - 1] * r;
        r *= 0.36787944117144233f;
    }
}

// Where the parameters sit in the packed forms (indices into theta over all
// layers; -1 for padding).  Bias entry gid (< L BIAS) of the accumulator-
// order bias array:
__device__ __forceinline__ int bias_param(int gid) {
    const int l = gid / BIAS, q = gid % BIAS;
    int off, n, t;
    if (q < BOFF_2) {
        off = OFF_B1; n = HID; t = q / 32;
    } else if (q < BOFF_3) {
        off = OFF_B2; n = HID; t = (q - BOFF_2) / 32;
    } else {
        off = OFF_B3; n = OUT; t = (q - BOFF_3) / 32;
    }
    const int w = q % 32, h = w / 16, r = w % 16;
    const int f = acc_feature(t, r, h);
    return f < n ? l * LP + off + f : -1;
}

// element e of forward fragment slot gid = (layer, fragment, lane): the 8
// BF16 weights lane `lane` feeds to the matrix core
__device__ __forceinline__ int fwd_param(int gid, int e) {
    const int lane = gid % 64, fr = (gid / 64) % FRAGS, l = gid / (64 * FRAGS);
    const int row = lane % 32, h = lane / 32;
    if (fr < OFF_G2) {  // first product: natural K order over the 96 one-blob inputs
        const int t = fr / G1K, ks = fr % G1K;
        return l * LP + OFF_W1 + (16 * ks + 8 * h + e) * HID + 32 * t + row;
    }
    // second and third: K order of the previous accumulator registers
    const bool third = fr >= OFF_G3;
    const int q = fr - (third ? OFF_G3 : OFF_G2);
    const int t = q / 4, ks = q % 4;
    const int o = 32 * t + row;
    const int k = acc_feature(ks / 2, 8 * (ks % 2) + e, h);
    if (third) return o < OUT ? l * LP + OFF_W3 + k * OUT + o : -1;
    return l * LP + OFF_W2 + k * HID + o;
}

// One thread per (layer, fragment, lane): its 8 BF16 weights, and the biases
// in accumulator order.
__device__ __forceinline__ void pack_fwd(int gid, const float *__restrict__ theta,
                                         bf16x8 *__restrict__ frags, float *__restrict__ bias) {
    if (gid < L * BIAS) {
        const int p = bias_param(gid);
        bias[gid] = p >= 0 ? theta[p] : 0.0f;
    }
    if (gid >= L * FRAGS * 64) return;
    float v[8];
    for (int e = 0; e < 8; ++e) {
        const int p = fwd_param(gid, e);
        v[e] = p >= 0 ? theta[p] : 0.0f;
    }
    frags[gid] = pack8(v);
}

__global__ void pack_kernel(const float *__restrict__ theta, bf16x8 *__restrict__ frags,
                            float *__restrict__ bias) {
    pack_fwd(blockIdx.x * blockDim.x + threadIdx.x, theta, frags, bias);
}

// 64 samples through the inverse flow: lane s holds sample s in u[] and
// returns log q.  All 64 lanes must be active.
__device__ __forceinline__ float sample_wave(const bf16x8 *__restrict__ frags,
                                             const float *__restrict__ bias, float u[D]) {
    const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
    float lq = 0.0f;
#pragma unroll 1
    for (int l = L - 1; l >= 0; --l) {
        const bf16x8 *F = frags + (size_t)l * FRAGS * 64 + lane;
        const float *Bs = bias + l * BIAS + h * 16;
        f32x16 out[2][G3T];  // [sample block][row tile]
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) {
            // conditioning inputs of this lane's column sample
            float ua[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) ua[a] = __shfl(getu(u, a_idx(l, a)), 32 * sb + col);
            // first product: one-blob inputs computed in operand order
            f32x16 acc1[G1T];
#pragma unroll
            for (int t = 0; t < G1T; ++t) acc1[t] = f32x16{};
#pragma unroll
            for (int ks = 0; ks < G1K; ++ks) {
                float e[8];
                blob8(ua[ks >> 1], 16 * (ks & 1) + 8 * h, e);
                const bf16x8 bop = pack8(e);
#pragma unroll
                for (int t = 0; t < G1T; ++t)
                    acc1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F[(OFF_G1 + t * G1K + ks) * 64],
                                                                      bop, acc1[t], 0, 0, 0);
            }
            // h1 = relu(acc + b1) as the next operand
            bf16x8 h1[G2K];
#pragma unroll
            for (int ks = 0; ks < G2K; ++ks) {
                float v[8], bb[8];
                load_bias8(Bs + BOFF_1 + (ks / 2) * 32 + 8 * (ks % 2), bb);
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = fmaxf(acc1[ks / 2][8 * (ks % 2) + i] + bb[i], 0.0f);
                h1[ks] = pack8(v);
            }
            f32x16 acc2[G2T];
#pragma unroll
            for (int t = 0; t < G2T; ++t) acc2[t] = f32x16{};
#pragma unroll
            for (int ks = 0; ks < G2K; ++ks)
#pragma unroll
                for (int t = 0; t < G2T; ++t)
                    acc2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F[(OFF_G2 + t * G2K + ks) * 64],
                                                                      h1[ks], acc2[t], 0, 0, 0);
            bf16x8 h2[G3K];
#pragma unroll
            for (int ks = 0; ks < G3K; ++ks) {
                float v[8], bb[8];
                load_bias8(Bs + BOFF_2 + (ks / 2) * 32 + 8 * (ks % 2), bb);
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = fmaxf(acc2[ks / 2][8 * (ks % 2) + i] + bb[i], 0.0f);
                h2[ks] = pack8(v);
            }
#pragma unroll
            for (int t = 0; t < G3T; ++t) out[sb][t] = f32x16{};
#pragma unroll
            for (int ks = 0; ks < G3K; ++ks)
#pragma unroll
                for (int t = 0; t < G3T; ++t)
                    out[sb][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        F[(OFF_G3 + t * G3K + ks) * 64], h2[ks], out[sb][t], 0, 0, 0);
        }
        // hand every lane its own sample: lanes 32..63 of block 0 <-> lanes
        // 0..31 of block 1; then (in place) lane s holds the features of lane
        // half 0 in out[0] and of lane half 1 in out[1]
#pragma unroll
        for (int t = 0; t < G3T; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const auto sw = __builtin_amdgcn_permlane32_swap(
                    __float_as_uint(out[0][t][r]), __float_as_uint(out[1][t][r]), false, false);
                out[0][t][r] = __uint_as_float(sw[0]) + bias[l * BIAS + BOFF_3 + t * 32 + r];
                out[1][t][r] = __uint_as_float(sw[1]) + bias[l * BIAS + BOFF_3 + t * 32 + 16 + r];
            }
        f32x16(&own)[2][G3T] = out;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            float raw[RAW];
#pragma unroll
            for (int k = 0; k < RAW; ++k) {
                const int f = b * RAW + k, t = f / 32, w = f % 32;
                const int hh = (w / 4) % 2, r = 4 * (w / 8) + w % 4;
                raw[k] = own[hh][t][r];
            }
            Spline s;
            spline_setup<true>(raw, s);
            const int j = b_idx(l, b);
            float v, pdf;
            spline_inverse(s, getu(u, j), v, pdf);
            setu(u, j, v);
            lq += __logf(pdf);
        }
    }
    return lq;
}

// z (n x 6) -> x, log q, 64 samples per wave; lanes past n work on a copy of
// the last sample and store nothing.
__global__ __launch_bounds__(256) void sample_bf16_kernel(const bf16x8 *__restrict__ frags,
                                                          const float *__restrict__ bias,
                                                          const double *__restrict__ z, int64_t n,
                                                          double *__restrict__ x,
                                                          double *__restrict__ logq) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int64_t base = wid * 64; base < n; base += waves * 64) {
        const int64_t s = base + lane < n ? base + lane : n - 1;
        float u[D];
#pragma unroll
        for (int j = 0; j < D; ++j) u[j] = (float)z[s * D + j];
        const float lq = sample_wave(frags, bias, u);
        if (base + lane < n) {
#pragma unroll
            for (int j = 0; j < D; ++j) x[s * D + j] = (double)u[j];
            logq[s] = (double)lq;
        }
    }
}

// The flow-mapped iteration on the matrix cores: 64 consecutive samples per
// wave, sample q = cube q / p, index q % p (p divides 64, so a cube's
// samples share a wave); per-cube statistics by butterfly sums over the p
// lanes of a cube.
template <int F>
__global__ __launch_bounds__(256) void flow_vsample_bf16_kernel(const bf16x8 *__restrict__ frags,
                                                                const float *__restrict__ bias,
                                                                const VsArgs A,
                                                                uint32_t stream_word,
                                                                double *__restrict__ partials,
                                                                uint32_t *__restrict__ whist) {
    constexpr int NBLK = (D + 3) / 4;
    __shared__ uint32_t hist[WH_BINS];
    wh_clear(hist);
    __syncthreads();
    const uint64_t N = (uint64_t)A.m * A.p;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wid = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int p = (int)A.p;
    double tS = 0.0, tV = 0.0;
    for (uint64_t base = wid * 64; base < N; base += waves * 64) {
        const uint64_t q = base + lane;
        const bool live = q < N;
        const uint32_t c = live ? (uint32_t)(q / p) : 0u;
        const uint32_t k = live ? (uint32_t)(q % p) : 0u;
        float u[D];
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
                    u[j] = (float)((dig + uu) / (double)A.g);
                }
            }
        }
        const float lq = sample_wave(frags, bias, u);
        Acc acc = Family<F, D>::begin(A.phase);
#pragma unroll
        for (int j = 0; j < D; ++j) Family<F, D>::axis(acc, A.ca[j], A.cu[j], (double)u[j]);
        const double w = Family<F, D>::end(acc, A) / exp((double)lq);
        if (live) wh_add(hist, w);
        // per-cube sums over the p lanes of the cube, shifted by its first sample
        const int first = lane - (lane % p);
        const double w0 = __shfl(w, first);
        const double dlt = w - w0;
        double S = w, D1 = dlt, D2 = dlt * dlt;
        for (int off = 1; off < p; off <<= 1) {
            S += __shfl_xor(S, off);
            D1 += __shfl_xor(D1, off);
            D2 += __shfl_xor(D2, off);
        }
        if (live && lane == first) {
            tS += S;
            tV += (D2 - D1 * D1 * A.inv_p) * A.inv_pm1;
        }
    }
    __shared__ double red[2][4];
    tS = wave_sum(tS);
    tV = wave_sum(tV);
    if (lane == 0) {
        red[0][threadIdx.x >> 6] = tS;
        red[1][threadIdx.x >> 6] = tV;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            s += red[0][w];
            v += red[1][w];
        }
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = v;
    }
    wh_flush(hist, whist);
}

// n plain (unstratified) samples of the flow on the matrix cores with their
// weights w = f / q: sample i draws z from Philox counter (i, stream word,
// block, iteration), as the FP32 draw does; 64 samples per wave, lanes past
// n work on a copy of the last sample and store nothing.
template <int F>
__global__ __launch_bounds__(256) void flow_draw_bf16_kernel(const bf16x8 *__restrict__ frags,
                                                             const float *__restrict__ bias,
                                                             const VsArgs A, uint32_t stream_word,
                                                             uint32_t n, double *__restrict__ xs,
                                                             double *__restrict__ ws) {
    constexpr int NBLK = (D + 3) / 4;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wid = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (uint64_t base = wid * 64; base < n; base += waves * 64) {
        const bool live = base + lane < n;
        const uint32_t i = live ? (uint32_t)(base + lane) : n - 1;
        float u[D];
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            uint32_t r[4];
            philox10(i, stream_word, b, A.iteration, A.key0, A.key1, r);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * b + t < D) u[4 * b + t] = (float)__fma_rn((double)r[t], 0x1p-32, 0x1p-33);
        }
        const float lq = sample_wave(frags, bias, u);
        if (!live) continue;
        Acc acc = Family<F, D>::begin(A.phase);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            Family<F, D>::axis(acc, A.ca[j], A.cu[j], (double)u[j]);
            xs[(uint64_t)i * D + j] = (double)u[j];
        }
        ws[i] = Family<F, D>::end(acc, A) / exp((double)lq);
    }
}

// ---------------------------------------------------------------------
// Training on the matrix cores.  The backward pass runs the three products
// through the transposed weights in the same orientation (features = rows,
// samples = columns): dh2 = W3 draw, dh1 = W2 d2, de = W1 d1.  Their weight
// fragments: through W3, 2 row tiles (hidden units) x 7 K steps over the 99
// spline parameters (natural order, padded to 112); through W2, 2 x 4; and
// through W1, 3 row tiles (one-blob inputs) x 4; the last two in the K order
// of the accumulator registers, like the forward products.
constexpr int B3T = 2, B3K = 7, B2T = 2, B2K = 4, B1T = 3, B1K = 4;
constexpr int OFF_B3F = 0, OFF_B2F = OFF_B3F + B3T * B3K, OFF_B1F = OFF_B2F + B2T * B2K;
constexpr int BFRAGS = OFF_B1F + B1T * B1K;  // 34

// element e of backward fragment slot gid = (layer, fragment, lane)
__device__ __forceinline__ int bwd_param(int gid, int e) {
    const int lane = gid % 64, fr = (gid / 64) % BFRAGS, l = gid / (64 * BFRAGS);
    const int row = lane % 32, h = lane / 32;
    if (fr < OFF_B2F) {
        const int t = fr / B3K, ks = fr % B3K, i = 32 * t + row;
        const int k = 16 * ks + 8 * h + e;
        return k < OUT ? l * LP + OFF_W3 + i * OUT + k : -1;
    }
    if (fr < OFF_B1F) {
        const int q = fr - OFF_B2F, t = q / B2K, ks = q % B2K, i = 32 * t + row;
        return l * LP + OFF_W2 + i * HID + acc_feature(ks / 2, 8 * (ks % 2) + e, h);
    }
    const int q = fr - OFF_B1F, t = q / B1K, ks = q % B1K, r = 32 * t + row;
    return l * LP + OFF_W1 + r * HID + acc_feature(ks / 2, 8 * (ks % 2) + e, h);
}

__device__ __forceinline__ void pack_bwd(int gid, const float *__restrict__ theta,
                                         bf16x8 *__restrict__ frags) {
    if (gid >= L * BFRAGS * 64) return;
    float v[8];
    for (int e = 0; e < 8; ++e) {
        const int p = bwd_param(gid, e);
        v[e] = p >= 0 ? theta[p] : 0.0f;
    }
    frags[gid] = pack8(v);
}

// The inverse of the three maps: inv[3 p], inv[3 p + 1], inv[3 p + 2] = the
// BF16 element of the forward fragments, of the backward fragments and the
// bias entry that hold parameter p (-1 where none; the caller fills inv with
// -1 first).  Every weight sits in exactly one forward and one backward
// element, every bias in one bias entry, so the three are well defined.
__global__ void inverse_map_kernel(int *__restrict__ inv) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = L * FRAGS * 64, nb = L * BFRAGS * 64;
    if (gid < nf) {
        for (int e = 0; e < 8; ++e) {
            const int p = fwd_param(gid, e);
            if (p >= 0) inv[3 * p] = 8 * gid + e;
        }
    } else if (gid < nf + nb) {
        const int g = gid - nf;
        for (int e = 0; e < 8; ++e) {
            const int p = bwd_param(g, e);
            if (p >= 0) inv[3 * p + 1] = 8 * g + e;
        }
    }
    if (gid < L * BIAS) {
        const int p = bias_param(gid);
        if (p >= 0) inv[3 * p + 2] = gid;
    }
}

// The end of a BF16 training step in one launch: the gradient's slice sum
// (as wgrad_sum_kernel), the Adam step (as adam_kernel), and the new
// parameter written through the inverse map into both fragment sets and the
// bias array, the values pack_train_kernel would write from the new theta.
// The next step's training pass then starts without repacking.
__global__ void sum_adam_pack_kernel(const float *__restrict__ part, int slices,
                                     float *__restrict__ theta, float *__restrict__ m,
                                     float *__restrict__ v, float *__restrict__ grad, float lr,
                                     float beta1, float beta2, float eps, float c1, float c2,
                                     const int *__restrict__ inv, uint16_t *__restrict__ frags,
                                     uint16_t *__restrict__ bfrags, float *__restrict__ bias) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= PARAMS) return;
    const float g = slice_sum(part, slices, i);
    grad[i] = g;
    const float t = adam_update(theta, m, v, i, g, lr, beta1, beta2, eps, c1, c2);
    const int pf = inv[3 * i], pb = inv[3 * i + 1], pz = inv[3 * i + 2];
    const uint16_t bits = bf16_bits(t);
    if (pf >= 0) frags[pf] = bits;
    if (pb >= 0) bfrags[pb] = bits;
    if (pz >= 0) bias[pz] = t;
}

// forward and backward fragments (and biases) in one launch: threads
// [0, nf) pack the forward ones, the rest the backward ones
__global__ void pack_train_kernel(const float *__restrict__ theta, bf16x8 *__restrict__ frags,
                                  float *__restrict__ bias, bf16x8 *__restrict__ bfrags, int nf) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < nf)
        pack_fwd(gid, theta, frags, bias);
    else
        pack_bwd(gid - nf, theta, bfrags);
}

// lane < 32 gets (a of lane, a of lane + 32), lane >= 32 (b of lane - 32,
// b of lane), per 32-bit word
__device__ __forceinline__ void swap_halves(const bf16x8 &a, const bf16x8 &b, bf16x8 &lo,
                                            bf16x8 &hi) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 ua = __builtin_bit_cast(u32x4, a), ub = __builtin_bit_cast(u32x4, b);
    u32x4 r0, r1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto sw = __builtin_amdgcn_permlane32_swap(ua[i], ub[i], false, false);
        r0[i] = sw[0];
        r1[i] = sw[1];
    }
    lo = __builtin_bit_cast(bf16x8, r0);
    hi = __builtin_bit_cast(bf16x8, r1);
}

// The third product of layer l for one sample block from its BF16 operands;
// F3 points at the layer's 16 third-product fragments (this lane's entry).
__device__ __forceinline__ void third_product(const bf16x8 *__restrict__ F3,
                                              const bf16x8 (&h2)[G3K], f32x16 (&out)[G3T]) {
#pragma unroll
    for (int t = 0; t < G3T; ++t) out[t] = f32x16{};
#pragma unroll
    for (int ks = 0; ks < G3K; ++ks)
#pragma unroll
        for (int t = 0; t < G3T; ++t)
            out[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F3[(t * G3K + ks) * 64], h2[ks],
                                                             out[t], 0, 0, 0);
}

// Bias added, and every lane handed its own sample's 99 outputs: afterwards
// out[hh][t][r] holds feature acc_feature(t, r, hh) of the lane's sample.
__device__ __forceinline__ void own_outputs(const float *__restrict__ bias, int l,
                                            f32x16 (&out)[2][G3T]) {
#pragma unroll
    for (int t = 0; t < G3T; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const auto sw = __builtin_amdgcn_permlane32_swap(
                __float_as_uint(out[0][t][r]), __float_as_uint(out[1][t][r]), false, false);
            out[0][t][r] = __uint_as_float(sw[0]) + bias[l * BIAS + BOFF_3 + t * 32 + r];
            out[1][t][r] = __uint_as_float(sw[1]) + bias[l * BIAS + BOFF_3 + t * 32 + 16 + r];
        }
}

__device__ __forceinline__ void raw_of(const f32x16 (&own)[2][G3T], int b, float raw[RAW]) {
#pragma unroll
    for (int k = 0; k < RAW; ++k) {
        const int f = b * RAW + k, t = f / 32, ww = f % 32;
        raw[k] = own[(ww / 4) % 2][t][4 * (ww / 8) + ww % 4];
    }
}

// The training pass keeps u in FP32 fields (the backward pass and the first
// weight gradient recompute from it) and stores h1, h2 and the three deltas
// as the BF16 values the matrix cores take: row F of a layer's fields lies at
// uint16 index F n + s past the first half of the layer's FP32 region, above
// the u rows.
__device__ __forceinline__ uint16_t *bf16_rows(float *layer_fields, int64_t n) {
    return reinterpret_cast<uint16_t *>(layer_fields) + (int64_t)FS * n;
}
__device__ __forceinline__ const uint16_t *bf16_rows(const float *layer_fields, int64_t n) {
    return reinterpret_cast<const uint16_t *>(layer_fields) + (int64_t)FS * n;
}

// Per-wave training state beyond the FP32 fields, per layer and group of 64
// samples: the second hidden layer as the BF16 operands of the third product
// ([block][K step][lane], 8 KB), from which the backward pass recomputes the
// spline parameters, and the ReLU masks of h1 and h2 as bits ([block][h1,
// h2][lane], one word per lane: bit 16 t + r for accumulator register r of
// row tile t).
constexpr int BF_EXTRA = 36;  // floats per sample and layer

__device__ __forceinline__ bf16x8 *h2_ops(float *ext_l, int64_t group, int sb) {
    return reinterpret_cast<bf16x8 *>(ext_l) + (group * 2 + sb) * G3K * 64;
}
__device__ __forceinline__ uint32_t *relu_bits(float *ext_l, int64_t n64, int64_t group, int sb,
                                               int which) {
    return reinterpret_cast<uint32_t *>(ext_l + 32 * n64) + ((group * 2 + sb) * 2 + which) * 64;
}

// Forward and backward pass of the weighted negative log-likelihood, 64
// samples per wave (lane = sample for the per-sample work), the nine
// products per layer on the matrix cores.  Writes the scratch fields the
// weight-gradient kernel reads (u in FP32; h1, h2 and the deltas, taken from
// the FP32 accumulators, rounded to BF16 as the products take them); loss +=
// sum c log q with c = -w / sum w.  Lanes past n work on a copy of the last
// sample with c = 0 and store nothing.
// The weight fragments of the current layer are staged in LDS for the
// workgroup's TR_WAVES waves (one per SIMD): forward, the layer's FRAGS
// fragments; backward, its third-product fragments followed by its backward
// fragments.  Read from LDS, the matrix-core operands wait a fraction of an
// L2 round trip.
constexpr int TR_WAVES = 4;
constexpr int TR_SLOT = G3T * G3K + BFRAGS;  // 50 fragments >= FRAGS

// Copies FR fragments (FR x 64 lanes of 16 bytes) from src to dst, the
// workgroup's threads striding over them.  Every load is issued before the
// first LDS write, so the copy waits one memory round trip, not one per
// stride.
template <int FR>
__device__ __forceinline__ void stage_frags(bf16x8 *dst, const bf16x8 *__restrict__ src) {
    constexpr int N = FR * 64, T = TR_WAVES * 64, PER = (N + T - 1) / T;
    bf16x8 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < N) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < N) dst[i] = v[k];
    }
}

// The BF16 fields leave the pass through a per-wave LDS tile T[f][c] (nf
// features of NC consecutive samples, bf16 bits): a lane holds one sample's
// features, but a row of the field-major scratch wants samples side by side,
// so the tile turns the lane's one-element stores (one per feature) into
// 16-byte stores of 8 samples of one feature, eight times fewer.  (On this
// chip stores and loads share the vector-memory counter, so fewer stores in
// flight also shorten every later wait for a load.)  Rows start 16-byte
// aligned when n is a multiple of 8 (s0 is); otherwise, and for an octet
// reaching past n, element stores.  Tile writes and reads of one wave are
// executed in order by the LDS.
constexpr int TILE = NB * RAW * 64;  // the largest block: 99 spline deltas of 64 samples

template <int NC>
__device__ __forceinline__ void flush_tile(const uint16_t *T, int nf, uint16_t *__restrict__ b16,
                                           int F0, int64_t n, int64_t s0, int lane) {
    constexpr int OCT = NC / 8;
    const bool aligned = (n & 7) == 0;
    for (int q = lane; q < nf * OCT; q += 64) {
        const int f = q / OCT, k = q - f * OCT;
        const int64_t s = s0 + 8 * k;
        if (s >= n) continue;
        uint16_t *dst = b16 + (int64_t)(F0 + f) * n + s;
        const uint16_t *src = T + f * NC + 8 * k;
        if (aligned && s + 8 <= n) {
            *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
        } else {
            for (int e = 0; e < 8 && s + e < n; ++e) dst[e] = src[e];
        }
    }
}

__global__ __launch_bounds__(TR_WAVES * 64) void train_bf16_kernel(
    const bf16x8 *__restrict__ frags, const bf16x8 *__restrict__ bfrags,
    const float *__restrict__ bias, const double *__restrict__ x, const double *__restrict__ w,
    int64_t n, const double *__restrict__ wsum, float *__restrict__ scratch, float *__restrict__ ext,
    double *__restrict__ loss) {
    __shared__ bf16x8 slot[TR_SLOT * 64];
    __shared__ __align__(16) uint16_t tiles[TR_WAVES][TILE];
    const int wave = threadIdx.x >> 6;
    uint16_t *tile = tiles[wave];
    const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
    const int64_t n64 = (n + 63) / 64 * 64;
    double lsum = 0.0;
    // the workgroup takes TR_WAVES groups of 64 samples per pass, all its
    // waves in step (they share the staged fragments); a wave past n runs on
    // copies of the last sample and stores nothing
    for (int64_t gbase = (int64_t)blockIdx.x * TR_WAVES * 64; gbase < n;
         gbase += (int64_t)gridDim.x * TR_WAVES * 64) {
        const int64_t base = gbase + 64 * wave;
        const bool wlive = base < n;
        const int64_t group = (wlive ? base : n64 - 64) / 64;
        const bool live = base + lane < n;
        const int64_t s = live ? base + lane : n - 1;
        // the sample of column col in block sb, and whether it is real
        int64_t cs[2];
        bool clive[2];
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) {
            clive[sb] = base + 32 * sb + col < n;
            cs[sb] = clive[sb] ? base + 32 * sb + col : n - 1;
        }
        float u[D];
#pragma unroll
        for (int j = 0; j < D; ++j) u[j] = (float)x[s * D + j];
        const float c = live ? (float)(-w[s] / *wsum) : 0.0f;
        float lq = 0.0f;
        // ---- forward, x -> z
#pragma unroll 1
        for (int l = 0; l < L; ++l) {
            float *sc = scratch + (int64_t)l * FS * n;
            uint16_t *b16 = bf16_rows(sc, n);
            float *ext_l = ext + (int64_t)l * BF_EXTRA * n64;
            if (live) {
#pragma unroll
                for (int j = 0; j < D; ++j) sc[(FS_U + j) * n + s] = u[j];
            }
            __syncthreads();  // every wave is done with the previous fragments
            stage_frags<FRAGS>(slot, frags + (size_t)l * FRAGS * 64);
            __syncthreads();
            const bf16x8 *Fr = slot + lane;
            const float *Bs = bias + l * BIAS + h * 16;
            f32x16 own[2][G3T];
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                float ua[NA];
#pragma unroll
                for (int a = 0; a < NA; ++a) ua[a] = __shfl(getu(u, a_idx(l, a)), 32 * sb + col);
                f32x16 acc1[G1T];
#pragma unroll
                for (int t = 0; t < G1T; ++t) acc1[t] = f32x16{};
#pragma unroll
                for (int ks = 0; ks < G1K; ++ks) {
                    float e[8];
                    blob8(ua[ks >> 1], 16 * (ks & 1) + 8 * h, e);
                    const bf16x8 bop = pack8(e);
#pragma unroll
                    for (int t = 0; t < G1T; ++t)
                        acc1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            Fr[(OFF_G1 + t * G1K + ks) * 64], bop, acc1[t], 0, 0, 0);
                }
                bf16x8 h1[G2K];
                uint32_t m1 = 0u;
#pragma unroll
                for (int ks = 0; ks < G2K; ++ks) {
                    float v[8], bb[8];
                    load_bias8(Bs + BOFF_1 + (ks / 2) * 32 + 8 * (ks % 2), bb);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int r = 8 * (ks % 2) + i;
                        v[i] = fmaxf(acc1[ks / 2][r] + bb[i], 0.0f);
                        m1 |= (v[i] > 0.0f ? 1u : 0u) << (8 * ks + i);
                        tile[acc_feature(ks / 2, r, h) * 32 + col] = bf16_bits(v[i]);
                    }
                    h1[ks] = pack8(v);
                }
                flush_tile<32>(tile, HID, b16, FS_H1, n, base + 32 * sb, lane);
                if (wlive) relu_bits(ext_l, n64, group, sb, 0)[lane] = m1;
                f32x16 acc2[G2T];
#pragma unroll
                for (int t = 0; t < G2T; ++t) acc2[t] = f32x16{};
#pragma unroll
                for (int ks = 0; ks < G2K; ++ks)
#pragma unroll
                    for (int t = 0; t < G2T; ++t)
                        acc2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            Fr[(OFF_G2 + t * G2K + ks) * 64], h1[ks], acc2[t], 0, 0, 0);
                uint32_t m2 = 0u;
                bf16x8 *ops = h2_ops(ext_l, group, sb);
                bf16x8 h2[G3K];
#pragma unroll
                for (int ks = 0; ks < G3K; ++ks) {
                    float v[8], bb[8];
                    load_bias8(Bs + BOFF_2 + (ks / 2) * 32 + 8 * (ks % 2), bb);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int r = 8 * (ks % 2) + i;
                        v[i] = fmaxf(acc2[ks / 2][r] + bb[i], 0.0f);
                        m2 |= (v[i] > 0.0f ? 1u : 0u) << (8 * ks + i);
                        tile[acc_feature(ks / 2, r, h) * 32 + col] = bf16_bits(v[i]);
                    }
                    h2[ks] = pack8(v);
                    if (wlive) ops[ks * 64 + lane] = h2[ks];
                }
                flush_tile<32>(tile, HID, b16, FS_H2, n, base + 32 * sb, lane);
                if (wlive) relu_bits(ext_l, n64, group, sb, 1)[lane] = m2;
                third_product(Fr + OFF_G3 * 64, h2, own[sb]);
            }
            own_outputs(bias, l, own);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                float raw[RAW];
                raw_of(own, b, raw);
                Spline sp;
                spline_setup<true>(raw, sp);
                const int j = b_idx(l, b);
                float v, pdf;
                spline_forward(sp, getu(u, j), v, pdf);
                setu(u, j, v);
                lq += __logf(pdf);
            }
        }
        lsum += live ? (double)c * (double)lq : 0.0;
        // ---- backward; g = dL/du at the output of the current layer
        float g[D];
#pragma unroll
        for (int j = 0; j < D; ++j) g[j] = 0.0f;
#pragma unroll 1
        for (int l = L - 1; l >= 0; --l) {
            float *sc = scratch + (int64_t)l * FS * n;
            uint16_t *b16 = bf16_rows(sc, n);
            float *ext_l = ext + (int64_t)l * BF_EXTRA * n64;
            float uin[D], gprev[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                uin[j] = sc[(FS_U + j) * n + s];
                gprev[j] = g[j];
            }
            __syncthreads();  // every wave is done with the previous fragments
            stage_frags<G3T * G3K>(slot, frags + ((size_t)l * FRAGS + OFF_G3) * 64);
            stage_frags<BFRAGS>(slot + G3T * G3K * 64, bfrags + (size_t)l * BFRAGS * 64);
            __syncthreads();
            // the spline parameters again, from the stored operands
            f32x16 own[2][G3T];
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                const bf16x8 *ops = h2_ops(ext_l, group, sb);
                bf16x8 h2[G3K];
#pragma unroll
                for (int ks = 0; ks < G3K; ++ks) h2[ks] = ops[ks * 64 + lane];
                third_product(slot + lane, h2, own[sb]);
            }
            own_outputs(bias, l, own);
            // spline deltas of the own sample, natural order padded to 112,
            // packed to BF16 eight at a time as soon as each octet is complete
            float gr[16 * B3K];
            bf16x8 oct[2 * B3K];
#pragma unroll
            for (int k = NB * RAW; k < 16 * B3K; ++k) gr[k] = 0.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                float raw[RAW];
                raw_of(own, b, raw);
                Spline sp;
                spline_setup<true>(raw, sp);
                const int j = b_idx(l, b);
                const float ub = getu(uin, j);
                float y, pdf, gu, graw[RAW];
                spline_forward(sp, ub, y, pdf);
                spline_backward(sp, ub, getu(g, j), c / pdf, graw, gu);
                setu(gprev, j, gu);
#pragma unroll
                for (int k = 0; k < RAW; ++k) {
                    gr[b * RAW + k] = graw[k];
                    tile[(b * RAW + k) * 64 + lane] = bf16_bits(graw[k]);
                }
                const int from = (b * RAW) / 8, to = b == NB - 1 ? 2 * B3K : ((b + 1) * RAW) / 8;
#pragma unroll
                for (int o = 0; o < 2 * B3K; ++o)
                    if (o >= from && o < to) oct[o] = pack8(&gr[8 * o]);
            }
            flush_tile<64>(tile, NB * RAW, b16, FS_DOUT, n, base, lane);
            // operands of the two sample blocks
            bf16x8 X[2][B3K];
#pragma unroll
            for (int ks = 0; ks < B3K; ++ks) swap_halves(oct[2 * ks], oct[2 * ks + 1], X[0][ks], X[1][ks]);
            const bf16x8 *Br = slot + G3T * G3K * 64 + lane;
            float tot[NA];
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                const uint32_t m1 = relu_bits(ext_l, n64, group, sb, 0)[lane];
                const uint32_t m2 = relu_bits(ext_l, n64, group, sb, 1)[lane];
                // through W3 and the second ReLU
                f32x16 a3[B3T];
#pragma unroll
                for (int t = 0; t < B3T; ++t) a3[t] = f32x16{};
#pragma unroll
                for (int ks = 0; ks < B3K; ++ks)
#pragma unroll
                    for (int t = 0; t < B3T; ++t)
                        a3[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            Br[(OFF_B3F + t * B3K + ks) * 64], X[sb][ks], a3[t], 0, 0, 0);
                bf16x8 Y[B2K];
#pragma unroll
                for (int ks = 0; ks < B2K; ++ks) {
                    float v[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int r = 8 * (ks % 2) + i, f = acc_feature(ks / 2, r, h);
                        v[i] = ((m2 >> (8 * ks + i)) & 1u) ? a3[ks / 2][r] : 0.0f;
                        tile[f * 32 + col] = bf16_bits(v[i]);
                    }
                    Y[ks] = pack8(v);
                }
                flush_tile<32>(tile, HID, b16, FS_D2, n, base + 32 * sb, lane);
                // through W2 and the first ReLU
                f32x16 a2[B2T];
#pragma unroll
                for (int t = 0; t < B2T; ++t) a2[t] = f32x16{};
#pragma unroll
                for (int ks = 0; ks < B2K; ++ks)
#pragma unroll
                    for (int t = 0; t < B2T; ++t)
                        a2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            Br[(OFF_B2F + t * B2K + ks) * 64], Y[ks], a2[t], 0, 0, 0);
                bf16x8 Z[B1K];
#pragma unroll
                for (int ks = 0; ks < B1K; ++ks) {
                    float v[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int r = 8 * (ks % 2) + i, f = acc_feature(ks / 2, r, h);
                        v[i] = ((m1 >> (8 * ks + i)) & 1u) ? a2[ks / 2][r] : 0.0f;
                        tile[f * 32 + col] = bf16_bits(v[i]);
                    }
                    Z[ks] = pack8(v);
                }
                flush_tile<32>(tile, HID, b16, FS_D1, n, base + 32 * sb, lane);
                // through W1 to the one-blob inputs, then through the encoding:
                // row tile t holds the 32 bumps of conditioning coordinate t
#pragma unroll
                for (int t = 0; t < B1T; ++t) {
                    f32x16 a1 = f32x16{};
#pragma unroll
                    for (int ks = 0; ks < B1K; ++ks)
                        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            Br[(OFF_B1F + t * B1K + ks) * 64], Z[ks], a1, 0, 0, 0);
                    const float ux = __shfl(getu(uin, a_idx(l, t)), 32 * sb + col);
                    float part = 0.0f;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int k = acc_feature(0, r, h);
                        const float tt = (ux - ((float)k + 0.5f) * (1.0f / BLOBS)) * (float)BLOBS;
                        part = __fmaf_rn(a1[r], -expf(-0.5f * tt * tt) * tt * (float)BLOBS, part);
                    }
                    part += __shfl_xor(part, 32);
                    if (sb == h) tot[t] = part;
                }
            }
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int j = a_idx(l, a);
                setu(gprev, j, getu(gprev, j) + tot[a]);
            }
#pragma unroll
            for (int j = 0; j < D; ++j) g[j] = gprev[j];
        }
    }
    const double v = wave_sum(lsum);
    if (lane == 0) unsafeAtomicAdd(loss, v);
}

// Weight gradients of the BF16 form on the matrix cores: per layer the
// products inputs^T deltas over the batch as C[row][col] = sum_s A[row][s]
// B[s][col], K = samples: lane l of an operand holds feature l % 32 for the
// 8 consecutive samples 8 (l / 32) .. +7 of a 16-sample step, read straight
// from the field-major scratch: the BF16 rows of h1, h2 and the deltas as
// they are, the one-blob inputs encoded from the FP32 u rows (FP32
// accumulation).  One wave owns up to 2 x 2 output tiles of 32 x 32: W1 rows
// 0-63 | W1 rows 64-95 | W2 | W3 columns 0-63 | W3 columns 64-98 (padded to
// 128), over a slice of ks samples (blockIdx.y); the tiles whose rows start
// at 0 also sum their delta columns (the bias gradients, FP32 sums of the
// BF16 deltas).  Partial sums go to part[slice][parameter], added in slice
// order afterwards.
constexpr int WB_TILES = 5;
constexpr int WG_STEPS = 2;

// v[e] = row[sb + e] for the samples below s_end (zero past it, and all zero
// unless `use`); `whole`: all 8 are below s_end and 16-byte aligned.
__device__ __forceinline__ void load8(const float *__restrict__ row, int64_t sb, int64_t s_end,
                                      bool whole, bool use, float v[8]) {
    if (use && whole) {
        const float4 x = *reinterpret_cast<const float4 *>(row + sb);
        const float4 y = *reinterpret_cast<const float4 *>(row + sb + 4);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (use && sb + e < s_end) ? row[sb + e] : 0.0f;
    }
}

// The same for a BF16 row, as operand bits (zero past s_end); `whole`: all 8
// are below s_end and 16-byte aligned.
__device__ __forceinline__ bf16x8 load8_bf16(const uint16_t *__restrict__ row, int64_t sb,
                                             int64_t s_end, bool whole, bool use) {
    typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
    u16x8 v;
    if (use && whole) {
        v = *reinterpret_cast<const u16x8 *>(row + sb);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (use && sb + e < s_end) ? row[sb + e] : (uint16_t)0;
    }
    return __builtin_bit_cast(bf16x8, v);
}

// Four waves per SIMD (at most 128 VGPRs, the accumulators included): a
// 65,536-sample batch gives 2.5 waves per SIMD, all resident at once.
// Measured against one step per pass at three waves per SIMD: 93.4 against
// 100.0 us per 65,536 samples, bit-identical.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void wgrad_bf16_kernel(
    const float *__restrict__ scratch, int64_t n, int64_t ks, float *__restrict__ part) {
    const int l = blockIdx.x / WB_TILES, tile = blockIdx.x % WB_TILES;
    const int64_t s_begin = (int64_t)blockIdx.y * ks;
    const int64_t s_end = s_begin + ks < n ? s_begin + ks : n;
    int mat, r0, nrt, c0, cols;
    switch (tile) {
    case 0: mat = 0; r0 = 0; nrt = 2; c0 = 0; cols = HID; break;
    case 1: mat = 0; r0 = 64; nrt = 1; c0 = 0; cols = HID; break;
    case 2: mat = 1; r0 = 0; nrt = 2; c0 = 0; cols = HID; break;
    case 3: mat = 2; r0 = 0; nrt = 2; c0 = 0; cols = 64; break;
    default: mat = 2; r0 = 0; nrt = 2; c0 = 64; cols = OUT - 64; break;
    }
    const int lane = threadIdx.x, h = lane >> 5, idx = lane & 31;
    const float *sc = scratch + (int64_t)l * FS * n;
    const uint16_t *b16 = bf16_rows(sc, n);
    const int bfield = mat == 0 ? FS_D1 : (mat == 1 ? FS_D2 : FS_DOUT);
    const bool bias_tile = r0 == 0;
    f32x16 acc[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = f32x16{};
    float bsum[2] = {0.0f, 0.0f};
    // the 8 samples of a lane are two float4 of an FP32 row when n is a
    // multiple of 4, one 16-byte load of a BF16 row when n is a multiple of
    // 8 (slices are multiples of 16)
    const bool aligned32 = (n & 3) == 0, aligned16 = (n & 7) == 0;
    // WG_STEPS 16-sample steps per pass: their loads are issued together
    // (the lanes of a row read half of its 128-byte line at once instead of
    // a quarter), then the products follow in step order, so the sums are
    // those of one step at a time
    for (int64_t s0 = s_begin; s0 < s_end; s0 += 16 * WG_STEPS) {
        bf16x8 A[WG_STEPS][2], B[WG_STEPS][2];
#pragma unroll
        for (int k = 0; k < WG_STEPS; ++k) {
            const int64_t sb = s0 + 16 * k + 8 * h;
            const bool inside = sb + 8 <= s_end;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int R = r0 + 32 * rt + idx;
                if (mat == 0) {
                    float v[8];
                    load8(sc + (int64_t)(FS_U + a_idx(l, R / BLOBS)) * n, sb, s_end,
                          aligned32 && inside, rt < nrt, v);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        v[e] = (rt < nrt && sb + e < s_end) ? blob(v[e], R % BLOBS) : 0.0f;
                    A[k][rt] = pack8(v);
                } else {
                    A[k][rt] = load8_bf16(b16 + (int64_t)((mat == 1 ? FS_H1 : FS_H2) + R) * n, sb,
                                          s_end, aligned16 && inside, rt < nrt);
                }
            }
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int C = 32 * ct + idx;
                B[k][ct] = load8_bf16(b16 + (int64_t)(bfield + c0 + (C < cols ? C : 0)) * n, sb,
                                      s_end, aligned16 && inside, C < cols);
            }
        }
#pragma unroll
        for (int k = 0; k < WG_STEPS; ++k) {
            if (s0 + 16 * k >= s_end) break;
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int e = 0; e < 8; ++e) bsum[ct] += (float)B[k][ct][e];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
                    if (rt < nrt)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            A[k][rt], B[k][ct], acc[rt][ct], 0, 0, 0);
        }
    }
    float *G = part + (int64_t)blockIdx.y * PARAMS + l * LP;
    const int off = mat == 0 ? OFF_W1 : (mat == 1 ? OFF_W2 : OFF_W3);
    const int ld = mat == 2 ? OUT : HID;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        if (rt >= nrt) continue;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int C = 32 * ct + idx;
            if (C >= cols) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                G[off + (r0 + 32 * rt + acc_feature(0, r, h)) * ld + c0 + C] = acc[rt][ct][r];
        }
    }
    if (bias_tile) {
        const int boff = mat == 0 ? OFF_B1 : (mat == 1 ? OFF_B2 : OFF_B3);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const float tot = bsum[ct] + __shfl_xor(bsum[ct], 32);
            const int C = 32 * ct + idx;
            if (h == 0 && C < cols) G[boff + c0 + C] = tot;
        }
    }
}

template <int F>
hipError_t launch_bf16_f(const void *frags, const float *bias, const VsArgs &A,
                         uint32_t stream_word, double *partials, uint32_t *whist, int blocks,
                         hipStream_t s) {
    hipLaunchKernelGGL((flow_vsample_bf16_kernel<F>), dim3(blocks), dim3(256), 0, s,
                       (const bf16x8 *)frags, bias, A, stream_word, partials, whist);
    return hipGetLastError();
}

}  // namespace

int64_t flow_bf16_frag_bytes() { return (int64_t)L * FRAGS * 64 * sizeof(bf16x8); }
int64_t flow_bf16_bias_floats() { return (int64_t)L * BIAS; }

hipError_t launch_flow_pack_bf16(const float *theta, void *frags, float *bias, hipStream_t s) {
    const int n = L * FRAGS * 64;
    hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, theta,
                       (bf16x8 *)frags, bias);
    return hipGetLastError();
}

int64_t flow_bf16_bwd_frag_bytes() { return (int64_t)L * BFRAGS * 64 * sizeof(bf16x8); }
int64_t flow_bf16_train_extra_floats(int64_t n) { return (int64_t)L * BF_EXTRA * ((n + 63) / 64 * 64); }

hipError_t launch_flow_train_bf16(const float *theta, void *frags, void *bfrags, float *bias,
                                  const double *x, const double *w, int64_t n, const double *wsum,
                                  float *scratch, double *loss, int cus, bool pack,
                                  hipStream_t s) {
    if (pack) {
        // the forward part covers the bias entries too (L BIAS < L FRAGS 64)
        const int nf = L * FRAGS * 64, nb = L * BFRAGS * 64;
        hipLaunchKernelGGL(pack_train_kernel, dim3((nf + nb + 255) / 256), dim3(256), 0, s, theta,
                           (bf16x8 *)frags, bias, (bf16x8 *)bfrags, nf);
    }
    // one workgroup of TR_WAVES waves per TR_WAVES x 64 samples, at most one
    // per CU (a wave fills a SIMD's registers)
    int64_t blocks = (n + TR_WAVES * 64 - 1) / (TR_WAVES * 64);
    const int64_t cap = cus > 0 ? cus : 256;
    if (blocks > cap) blocks = cap;
    float *ext = scratch + (int64_t)L * FS * n + (int64_t)kWgradSlices * PARAMS;
    hipLaunchKernelGGL(train_bf16_kernel, dim3((unsigned)blocks), dim3(TR_WAVES * 64), 0, s,
                       (const bf16x8 *)frags, (const bf16x8 *)bfrags, bias, x, w, n, wsum, scratch,
                       ext, loss);
    return hipGetLastError();
}

namespace {

// slices of at least 512 samples (a multiple of 16), at most kWgradSlices;
// returns their number and their length in *ks
int wgrad_bf16_slices(int64_t n, int64_t *ks) {
    int64_t slices = (n + 511) / 512;
    if (slices > kWgradSlices) slices = kWgradSlices;
    int64_t k = (n + slices - 1) / slices;
    k = (k + 15) / 16 * 16;
    *ks = k;
    return (int)((n + k - 1) / k);
}

// the per-slice partial sums only; returns the slice count in *slices
hipError_t launch_wgrad_bf16_parts(const float *scratch_in, int64_t n, int *slices,
                                   hipStream_t s) {
    float *scratch = const_cast<float *>(scratch_in);
    int64_t ks = 0;
    *slices = wgrad_bf16_slices(n, &ks);
    float *part = scratch + (int64_t)L * FS * n;
    hipLaunchKernelGGL(wgrad_bf16_kernel, dim3(L * WB_TILES, (unsigned)*slices), dim3(64), 0, s,
                       scratch, n, ks, part);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_flow_wgrad_bf16(const float *scratch, int64_t n, float *grad,
                                  hipStream_t s) {
    int slices = 0;
    const hipError_t e = launch_wgrad_bf16_parts(scratch, n, &slices, s);
    if (e != hipSuccess) return e;
    return launch_flow_wgrad_sum(scratch + (int64_t)L * FS * n, slices, grad, s);
}

int64_t flow_bf16_inverse_map_ints() { return 3 * (int64_t)PARAMS; }

hipError_t launch_flow_inverse_map(int *inv, hipStream_t s) {
    const int threads = L * (FRAGS + BFRAGS) * 64;
    hipLaunchKernelGGL(inverse_map_kernel, dim3((threads + 255) / 256), dim3(256), 0, s, inv);
    return hipGetLastError();
}

hipError_t launch_flow_wgrad_adam_bf16(const float *scratch, int64_t n, float *theta, float *m,
                                       float *v, float *grad, float lr, float beta1, float beta2,
                                       float eps, float c1, float c2, const int *inv,
                                       void *frags, void *bfrags, float *bias, hipStream_t s) {
    int slices = 0;
    const hipError_t e = launch_wgrad_bf16_parts(scratch, n, &slices, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_adam_pack_kernel, dim3((PARAMS + 255) / 256), dim3(256), 0, s,
                       scratch + (int64_t)L * FS * n, slices, theta, m, v, grad, lr, beta1, beta2,
                       eps, c1, c2, inv, (uint16_t *)frags, (uint16_t *)bfrags, bias);
    return hipGetLastError();
}

template <int F>
hipError_t launch_draw_bf16_f(const void *frags, const float *bias, const VsArgs &A,
                              uint32_t stream_word, uint32_t n, double *xs, double *ws,
                              hipStream_t s) {
    int64_t blocks = ((int64_t)n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((flow_draw_bf16_kernel<F>), dim3((unsigned)blocks), dim3(256), 0, s,
                       (const bf16x8 *)frags, bias, A, stream_word, n, xs, ws);
    return hipGetLastError();
}

hipError_t launch_flow_draw_bf16(int family, const void *frags, const float *bias,
                                 const VsArgs &A, uint32_t stream_word, uint32_t n, double *xs,
                                 double *ws, hipStream_t s) {
    if (n == 0) return hipSuccess;
    switch (family) {
    case MCUBES_OSCILLATORY: return launch_draw_bf16_f<MCUBES_OSCILLATORY>(frags, bias, A, stream_word, n, xs, ws, s);
    case MCUBES_PRODUCT_PEAK: return launch_draw_bf16_f<MCUBES_PRODUCT_PEAK>(frags, bias, A, stream_word, n, xs, ws, s);
    case MCUBES_CORNER_PEAK: return launch_draw_bf16_f<MCUBES_CORNER_PEAK>(frags, bias, A, stream_word, n, xs, ws, s);
    case MCUBES_GAUSSIAN: return launch_draw_bf16_f<MCUBES_GAUSSIAN>(frags, bias, A, stream_word, n, xs, ws, s);
    case MCUBES_C0: return launch_draw_bf16_f<MCUBES_C0>(frags, bias, A, stream_word, n, xs, ws, s);
    case MCUBES_DISCONTINUOUS: return launch_draw_bf16_f<MCUBES_DISCONTINUOUS>(frags, bias, A, stream_word, n, xs, ws, s);
    case MCUBES_ADDITION: return launch_draw_bf16_f<MCUBES_ADDITION>(frags, bias, A, stream_word, n, xs, ws, s);
    case MCUBES_MIXTURE: return launch_draw_bf16_f<MCUBES_MIXTURE>(frags, bias, A, stream_word, n, xs, ws, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_flow_sample_bf16(const void *frags, const float *bias, const double *z,
                                   int64_t n, double *x, double *logq, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(sample_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const bf16x8 *)frags, bias, z, n, x, logq);
    return hipGetLastError();
}

hipError_t launch_flow_vsample_bf16(int family, const void *frags, const float *bias,
                                    const VsArgs &A, uint32_t stream_word, double *partials,
                                    uint32_t *whist, int blocks, hipStream_t s) {
    switch (family) {
    case MCUBES_OSCILLATORY: return launch_bf16_f<MCUBES_OSCILLATORY>(frags, bias, A, stream_word, partials, whist, blocks, s);
    case MCUBES_PRODUCT_PEAK: return launch_bf16_f<MCUBES_PRODUCT_PEAK>(frags, bias, A, stream_word, partials, whist, blocks, s);
    case MCUBES_CORNER_PEAK: return launch_bf16_f<MCUBES_CORNER_PEAK>(frags, bias, A, stream_word, partials, whist, blocks, s);
    case MCUBES_GAUSSIAN: return launch_bf16_f<MCUBES_GAUSSIAN>(frags, bias, A, stream_word, partials, whist, blocks, s);
    case MCUBES_C0: return launch_bf16_f<MCUBES_C0>(frags, bias, A, stream_word, partials, whist, blocks, s);
    case MCUBES_DISCONTINUOUS: return launch_bf16_f<MCUBES_DISCONTINUOUS>(frags, bias, A, stream_word, partials, whist, blocks, s);
    case MCUBES_ADDITION: return launch_bf16_f<MCUBES_ADDITION>(frags, bias, A, stream_word, partials, whist, blocks, s);
    case MCUBES_MIXTURE: return launch_bf16_f<MCUBES_MIXTURE>(frags, bias, A, stream_word, partials, whist, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mcubes
