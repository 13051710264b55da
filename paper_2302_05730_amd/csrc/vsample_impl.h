// V-Sample: the per-iteration sampling kernel of m-Cubes (Alg. 2, §3.2),
// written for CDNA4 (gfx950, wave64).
//
// Work decomposition.  The grid is persistent: enough blocks to fill every
// compute unit, each thread walking a strided sequence of work items
// w = tid, tid + T, tid + 2T, ... (T = threads in the grid).  Work item w is
// the cube c = (w * mult) mod m, with mult coprime to m: the 64 lanes of a
// wave then sit in unrelated cubes on every axis, so their bin indices spread
// over the whole histogram instead of piling onto the few bins of one slab
// (which serialises LDS atomics).  Each thread keeps both the linear cube id
// (a Philox counter word) and its base-g digits (the stratum on every axis)
// and advances them by a constant step with a digit-wise add-with-carry,
// which needs no division in the loop.  The results depend only on the cube
// id, never on the launch geometry.
//
// A sample reads the bin's left edge and width on every axis, from tables
// split between LDS (staged once per block) and the global grid row through
// the vector L1 cache (see VsLds and table_from_l1), and adds its bin
// contributions to an LDS-private FP64 histogram (ds_add_f64), flushed at
// the end with one global FP64 atomic per non-empty bin.  Per-thread sums of the cube sums and
// cube variances are reduced across the wave with shuffles, across the
// block in LDS, and written as one partial per block; a separate kernel adds
// the partials in a fixed order.
//
// Floating-point operation order matches the definition used throughout
// (multiply-adds are explicit fma; the library is built without contraction),
// so for integrands without libm calls each sample's weight is bit-identical
// to the plain definition.
#pragma once

#include "cos_reduced.h"
#include "mcubes_internal.h"

namespace mcubes {

// Philox4x32-10 (Salmon et al., SC'11).  The key is uniform across the
// wave, so the round keys are scalar adds; each output word's two xors are
// one gfx950 three-input bitwise op (truth table 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), x1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), x3, k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

// Integrand families, evaluated axis by axis in axis order (the same
// operation order as the plain definitions, without keeping x[] alive):
// begin() -> axis(j, x_j) for j = 0..D-1 -> end().  ca, cu are the folded
// coefficients (see VsArgs).
struct Acc {
    double s;
    bool inside;
    double s2, t1, t2;  // further sums (mixture family; unused fields cost nothing)
};

template <int F, int D>
struct Family;

template <int D>
struct Family<MCUBES_OSCILLATORY, D> {  // cos(2 pi u_0 + sum a_i x_i)
    static __device__ __forceinline__ Acc begin(double phase) { return {phase, true}; }
    static __device__ __forceinline__ void axis(Acc &a, double ca, double, double x) {
        a.s = __fma_rn(ca, x, a.s);
    }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &) {
        return cos_reduced(a.s);
    }
};

template <int D>
struct Family<MCUBES_PRODUCT_PEAK, D> {  // prod (a_i^-2 + (x_i - u_i)^2)^-1
    static __device__ __forceinline__ Acc begin(double) { return {1.0, true}; }
    static __device__ __forceinline__ void axis(Acc &a, double ca, double cu, double x) {
        const double t = x - cu;
        a.s = a.s * __fma_rn(t, t, ca);
    }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &) { return 1.0 / a.s; }
};

template <int D>
struct Family<MCUBES_CORNER_PEAK, D> {  // (1 + sum a_i x_i)^-(d+1)
    static __device__ __forceinline__ Acc begin(double) { return {1.0, true}; }
    static __device__ __forceinline__ void axis(Acc &a, double ca, double, double x) {
        a.s = __fma_rn(ca, x, a.s);
    }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &) {
        double pw = a.s;
#pragma unroll
        for (int k = 0; k < D; ++k) pw = pw * a.s;
        return 1.0 / pw;
    }
};

template <int D>
struct Family<MCUBES_GAUSSIAN, D> {  // exp(-sum a_i^2 (x_i - u_i)^2)
    static __device__ __forceinline__ Acc begin(double) { return {0.0, true}; }
    static __device__ __forceinline__ void axis(Acc &a, double ca, double cu, double x) {
        const double t = x - cu;
        a.s = __fma_rn(ca, t * t, a.s);
    }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &) { return exp(-a.s); }
};

template <int D>
struct Family<MCUBES_C0, D> {  // exp(-sum a_i |x_i - u_i|)
    static __device__ __forceinline__ Acc begin(double) { return {0.0, true}; }
    static __device__ __forceinline__ void axis(Acc &a, double ca, double cu, double x) {
        a.s = __fma_rn(ca, fabs(x - cu), a.s);
    }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &) { return exp(-a.s); }
};

template <int D>
struct Family<MCUBES_DISCONTINUOUS, D> {  // exp(sum a_i x_i) if x_i < u_i for all i
    static __device__ __forceinline__ Acc begin(double) { return {0.0, true}; }
    static __device__ __forceinline__ void axis(Acc &a, double ca, double cu, double x) {
        a.inside = a.inside && (x < cu);
        a.s = __fma_rn(ca, x, a.s);
    }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &) { return a.inside ? exp(a.s) : 0.0; }
};

template <int D>
struct Family<MCUBES_ADDITION, D> {  // sum x_i
    static __device__ __forceinline__ Acc begin(double) { return {0.0, true}; }
    static __device__ __forceinline__ void axis(Acc &a, double, double, double x) { a.s = a.s + x; }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &) { return a.s; }
};

// Equal mixture of two equicorrelated Gaussians centred at m_1 1 and m_2 1
// (ca = m_1, cu = m_2 on every axis): with S1_k = sum (x - m_k) and
// S2_k = sum (x - m_k)^2, f = norm (exp(-c2 (S2_1 - c1 S1_1^2)) +
// exp(-c2 (S2_2 - c1 S1_2^2))), c1 = r / (1 - r + d r), c2 = 1 / (2 s^2 (1 - r)).
template <int D>
struct Family<MCUBES_MIXTURE, D> {
    static __device__ __forceinline__ Acc begin(double) { return {0.0, true, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ void axis(Acc &a, double ca, double cu, double x) {
        const double t1 = x - ca, t2 = x - cu;
        a.s = a.s + t1;
        a.s2 = __fma_rn(t1, t1, a.s2);
        a.t1 = a.t1 + t2;
        a.t2 = __fma_rn(t2, t2, a.t2);
    }
    static __device__ __forceinline__ double end(const Acc &a, const VsArgs &A) {
        const double q1 = A.mix_c2 * (a.s2 - A.mix_c1 * a.s * a.s);
        const double q2 = A.mix_c2 * (a.t2 - A.mix_c1 * a.t1 * a.t1);
        return A.mix_norm * (exp(-q1) + exp(-q2));
    }
};

// FP32 forms of the families (precision option): same operations in the
// same axis order, on float values.
struct Acc32 {
    float s;
    bool inside;
    float s2, t1, t2;
};

template <int F, int D>
struct Family32;

template <int D>
struct Family32<MCUBES_OSCILLATORY, D> {
    static __device__ __forceinline__ Acc32 begin(float phase) { return {phase, true}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float ca, float, float x) {
        a.s = __fmaf_rn(ca, x, a.s);
    }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &) { return cosf(a.s); }
};

template <int D>
struct Family32<MCUBES_PRODUCT_PEAK, D> {
    static __device__ __forceinline__ Acc32 begin(float) { return {1.0f, true}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float ca, float cu, float x) {
        const float t = x - cu;
        a.s = a.s * __fmaf_rn(t, t, ca);
    }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &) { return 1.0f / a.s; }
};

template <int D>
struct Family32<MCUBES_CORNER_PEAK, D> {
    static __device__ __forceinline__ Acc32 begin(float) { return {1.0f, true}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float ca, float, float x) {
        a.s = __fmaf_rn(ca, x, a.s);
    }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &) {
        float pw = a.s;
#pragma unroll
        for (int k = 0; k < D; ++k) pw = pw * a.s;
        return 1.0f / pw;
    }
};

template <int D>
struct Family32<MCUBES_GAUSSIAN, D> {
    static __device__ __forceinline__ Acc32 begin(float) { return {0.0f, true}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float ca, float cu, float x) {
        const float t = x - cu;
        a.s = __fmaf_rn(ca, t * t, a.s);
    }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &) { return expf(-a.s); }
};

template <int D>
struct Family32<MCUBES_C0, D> {
    static __device__ __forceinline__ Acc32 begin(float) { return {0.0f, true}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float ca, float cu, float x) {
        a.s = __fmaf_rn(ca, fabsf(x - cu), a.s);
    }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &) { return expf(-a.s); }
};

template <int D>
struct Family32<MCUBES_DISCONTINUOUS, D> {
    static __device__ __forceinline__ Acc32 begin(float) { return {0.0f, true}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float ca, float cu, float x) {
        a.inside = a.inside && (x < cu);
        a.s = __fmaf_rn(ca, x, a.s);
    }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &) {
        return a.inside ? expf(a.s) : 0.0f;
    }
};

template <int D>
struct Family32<MCUBES_MIXTURE, D> {
    static __device__ __forceinline__ Acc32 begin(float) { return {0.0f, true, 0.0f, 0.0f, 0.0f}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float ca, float cu, float x) {
        const float t1 = x - ca, t2 = x - cu;
        a.s = a.s + t1;
        a.s2 = __fmaf_rn(t1, t1, a.s2);
        a.t1 = a.t1 + t2;
        a.t2 = __fmaf_rn(t2, t2, a.t2);
    }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &A) {
        const float c1 = (float)A.mix_c1, c2 = (float)A.mix_c2;
        const float q1 = c2 * (a.s2 - c1 * a.s * a.s);
        const float q2 = c2 * (a.t2 - c1 * a.t1 * a.t1);
        return (float)A.mix_norm * (expf(-q1) + expf(-q2));
    }
};

template <int D>
struct Family32<MCUBES_ADDITION, D> {
    static __device__ __forceinline__ Acc32 begin(float) { return {0.0f, true}; }
    static __device__ __forceinline__ void axis(Acc32 &a, float, float, float x) { a.s = a.s + x; }
    static __device__ __forceinline__ float end(const Acc32 &a, const VsArgs &) { return a.s; }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// LDS of one V-Sample block.  Every table holds one row of kMaxBins entries
// of 8 bytes per axis, so the offset of each row is a constant of the
// instantiation: one value, the bin index times 8, then addresses the bin in
// every table of its axis (the row offsets fold into the immediate offsets of
// the LDS instructions), and the same value is the byte offset of the bin's
// left edge in the axis's row of the global grid.
//   FP64 form: bin sums of every axis, and the edges E_i and widths W_i of the
//   staged axes (with bin sums, axes 0, 4, 8, the others reading (E_i, E_i+1)
//   from the global grid through the vector L1 cache; without bin sums, and
//   for d = 1, every axis).  With bin sums (d >= 2) a staged axis keeps
//   (E_i, W_i) side by side in a row of twice the width, read as one 16-byte
//   pair at twice the bin offset (the E and W regions together hold these
//   rows); otherwise E and W are separate rows.
//   FP32 form: bin sums, and (E_i, W_i) as a pair of floats for every axis.
template <int D, bool BINS, bool F32>
struct VsLds {
    static constexpr int kRow = kMaxBins * 8;
    static constexpr int kStaged = F32 ? D : (D >= 2 && BINS ? (D + 3) / 4 : D);
    static constexpr int kH = 0;                                   // FP64 sums, axis j
    static constexpr int kE = kH + (BINS ? D : 0) * kRow;         // FP64 E_i, staged axis l
    static constexpr int kW = kE + (F32 ? 0 : kStaged) * kRow;     // FP64 W_i, staged axis l
    static constexpr int kEW32 = kW + (F32 ? 0 : kStaged) * kRow;  // FP32 (E_i, W_i), axis j
    static constexpr int kBytes = kEW32 + (F32 ? D : 0) * kRow;
};

// Grid-table reads are split between the vector L1 cache (two adjacent edges
// of the global grid row, 4 KB per axis at 500 bins) and LDS, so that the two
// memory paths share the random reads.  With bin sums the LDS also takes d
// FP64 atomics per sample and is the busier path: three axes in four read
// through L1 (measured 6% faster over the three 8-D integrands than every
// other axis, and than all through L1).  Without bin sums the LDS is free
// and every axis reads it (3% faster than every other axis).
template <int D, bool BINS>
constexpr bool table_from_l1(int j) {
    return BINS && D >= 2 && (j & 3) != 0;
}

// Staged-table index of axis j (FP64 form).
template <int D, bool BINS>
constexpr int staged_axis(int j) {
    return BINS && D >= 2 ? j / 4 : j;
}

// The bin coordinate of axis j: z = (c_j + u) fl(nb/g) with u = (r + 1/2) 2^-32,
// evaluated as (c_j 2^32 + r + 1/2) (fl(nb/g) 2^-32).  The double whose high
// word is 0x43300000 + c_j and low word is r equals 2^52 + c_j 2^32 + r
// (c_j < 2^20); subtracting 2^52 - 1/2 leaves c_j 2^32 + r + 1/2 exactly (below
// 2^52 with one fractional bit), so the one rounding is that of the product,
// as in the plain definition.  hb = 0x43300000 + c_j is formed once per cube.
constexpr uint32_t kStratumHi = 0x43300000u;

__device__ __forceinline__ double bin_coordinate(uint32_t hb, uint32_t r, double zscale) {
    const double v = __hiloint2double((int)hb, (int)r);
    return (v - 0x1.fffffffffffffp+51) * zscale;
}

// One sample k of cube c: Philox words -> bin coordinates -> x through the
// grid tables -> weight w = f(x) J.  o8[j] receives 8 times the bin index on
// axis j (the byte offset of the bin in every table of the axis).
template <int F, int D, bool BINS>
__device__ __forceinline__ double draw(const VsArgs &A, uint32_t iteration, const double *ca,
                                       const double *cu, uint32_t c, uint32_t k, const uint32_t *hb,
                                       const unsigned char *lds, const char *const *row, int nb,
                                       uint32_t *o8) {
    using L = VsLds<D, BINS, false>;
    constexpr int NBLK = (D + 3) / 4;  // Philox blocks (4 words each) per sample
    // Axes in groups of four, one Philox block per group: the group's bin
    // indices and in-bin fractions first, then its table reads back to back,
    // then their uses, so that the reads are in flight together instead of
    // each one stalling the wave for a full round trip.
    Acc acc = Family<F, D>::begin(A.phase);
    double prod = 1.0;
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
        uint32_t r[4];
        philox10(c, A.stream_id, k * NBLK + b, iteration, A.key0, A.key1, r);
        double phi[4], e0[4], e1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < D) {
                const double z = bin_coordinate(hb[j], r[q], A.zscale);
                int i = (int)z;
                if constexpr (D >= 2) {
                    // g < 2^16 here, so z < nb and the bin clamp never fires:
                    // fract(z) = z - floor(z) = z - i exactly.
                    phi[q] = __builtin_amdgcn_fract(z);
                } else {
                    i = i < nb - 1 ? i : nb - 1;
                    phi[q] = z - (double)i;
                }
                o8[j] = (uint32_t)i << 3;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < D) {
                if (table_from_l1<D, BINS>(j)) {
                    // (E_i, E_i+1) of the global row; the width is formed below
                    // exactly as the staging loop forms the staged widths
                    const double2 e = *reinterpret_cast<const double2 *>(row[j] + o8[j]);
                    e0[q] = e.x;
                    e1[q] = e.y;
                } else if constexpr (BINS && D >= 2) {
                    // (E_i, W_i) side by side: one 16-byte LDS read at twice the
                    // bin offset
                    const int l = staged_axis<D, BINS>(j);
                    const double2 ew = *reinterpret_cast<const double2 *>(
                        lds + L::kE + 2 * l * L::kRow + (o8[j] << 1));
                    e0[q] = ew.x;
                    e1[q] = ew.y;
                } else {
                    const int l = staged_axis<D, BINS>(j);
                    e0[q] = *reinterpret_cast<const double *>(lds + L::kE + l * L::kRow + o8[j]);
                    e1[q] = *reinterpret_cast<const double *>(lds + L::kW + l * L::kRow + o8[j]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < D) {
                const double W = table_from_l1<D, BINS>(j) ? e1[q] - e0[q] : e1[q];
                const double x = __fma_rn(W, phi[q], e0[q]);
                prod = prod * W;
                Family<F, D>::axis(acc, ca[j], cu[j], x);
            }
        }
    }
    const double J = A.nbd * prod;
    return Family<F, D>::end(acc, A) * J;
}

// FP32 form of one sample: the bin coordinates, bin indices and in-bin
// fractions are formed in FP64 exactly as in draw() (same samples, same
// bins); the fraction is rounded to FP32 and the map and the integrand run in
// FP32 on an FP32 (edge, width) table.  The Jacobian fl(nb^d) prod W is formed
// in FP64 from the same FP32 widths the map uses, and the weight is returned
// in FP64.
template <int F, int D, bool BINS>
__device__ __forceinline__ double draw32(const VsArgs &A, uint32_t iteration, const float *ca,
                                         const float *cu, float phase, uint32_t c, uint32_t k,
                                         const uint32_t *hb, const unsigned char *lds, int nb,
                                         uint32_t *o8) {
    using L = VsLds<D, BINS, true>;
    constexpr int NBLK = (D + 3) / 4;
    Acc32 acc = Family32<F, D>::begin(phase);
    double prod = 1.0;
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
        uint32_t r[4];
        philox10(c, A.stream_id, k * NBLK + b, iteration, A.key0, A.key1, r);
        float phi[4];
        float2 ew[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < D) {
                const double z = bin_coordinate(hb[j], r[q], A.zscale);
                int i = (int)z;
                double ph;
                if constexpr (D >= 2) {
                    ph = __builtin_amdgcn_fract(z);
                } else {
                    i = i < nb - 1 ? i : nb - 1;
                    ph = z - (double)i;
                }
                phi[q] = (float)ph;
                o8[j] = (uint32_t)i << 3;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < D)
                ew[q] = *reinterpret_cast<const float2 *>(lds + L::kEW32 + j * L::kRow + o8[j]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < D) {
                const float x = __fmaf_rn(ew[q].y, phi[q], ew[q].x);
                prod = prod * (double)ew[q].y;
                Family32<F, D>::axis(acc, ca[j], cu[j], x);
            }
        }
    }
    return (double)Family32<F, D>::end(acc, A) * (A.nbd * prod);
}

// Adds w^2 to the bin of the sample on every axis (LDS FP64 atomics).
template <int D, bool F32>
__device__ __forceinline__ void add_bins(unsigned char *lds, const uint32_t *o8, double w2) {
    using L = VsLds<D, true, F32>;
#pragma unroll
    for (int j = 0; j < D; ++j)
        atomicAdd(reinterpret_cast<double *>(lds + L::kH + j * L::kRow + o8[j]), w2);
}

// Largest block of a V-Sample instantiation.  The LDS tables allow one block
// per CU at 8-D, so the block size sets the waves per SIMD and the register
// budget: 1024 threads -> 4 waves, 128 VGPRs; 768 -> 3 waves, 168 VGPRs for
// the instantiations whose live state does not fit 128 registers.
template <int F, int D>
constexpr int vs_max_block() {
    return (D >= 9 || (F == MCUBES_DISCONTINUOUS && D >= 8)) ? 768 : 1024;
}

// Shared memory of a V-Sample kernel: the grid tables and bin sums, the
// per-wave partial sums and the integrand coefficients.
template <int D, bool BINS, bool F32>
struct VsShared {
    alignas(16) unsigned char tables[VsLds<D, BINS, F32>::kBytes];
    double red[2][kMaxBlock / 64];
    double coef[2 * kMaxDim];
};

// The work of one block on a set of work items of one integrand: thread t
// handles `count` work items w0, w0 + stride, ... (cube (w * mult) mod m each;
// `step` = (stride * mult) mod m and its base-g digits advance the cube).
// Stages the grid into LDS, samples, reduces the block's (sum S_c, sum var_c)
// into partial[0..1] and flushes the block's bin sums into `bins`.  Callable
// repeatedly by a block (it synchronises before restaging).
template <int F, int D, bool P2, bool BINS, bool F32>
__device__ __forceinline__ void vs_block(const VsArgs &A, const double *__restrict__ grid,
                                         double *__restrict__ bins, double *__restrict__ partial,
                                         uint32_t w0, uint32_t stride, uint32_t count,
                                         uint32_t step, const uint32_t *step_digit,
                                         uint32_t iteration, VsShared<D, BINS, F32> &sh) {
    using L = VsLds<D, BINS, F32>;
    __syncthreads();  // a previous call may still read the LDS tables
    const int nb = (int)A.nb;
    const int nh = D * nb;
    unsigned char *lds = sh.tables;
    if (threadIdx.x < D) {
        sh.coef[threadIdx.x] = A.ca[threadIdx.x];
        sh.coef[kMaxDim + threadIdx.x] = A.cu[threadIdx.x];
    }
    for (int q = threadIdx.x; q < nh; q += blockDim.x) {
        const int j = q / nb, i = q - j * nb;
        const double e0 = grid[j * (nb + 1) + i];
        const double e1 = grid[j * (nb + 1) + i + 1];
        if constexpr (F32) {
            *reinterpret_cast<float2 *>(lds + L::kEW32 + j * L::kRow + 8 * i) =
                make_float2((float)e0, (float)(e1 - e0));
        } else if (!table_from_l1<D, BINS>(j)) {
            const int l = staged_axis<D, BINS>(j);
            if constexpr (BINS && D >= 2) {
                *reinterpret_cast<double2 *>(lds + L::kE + 2 * l * L::kRow + 16 * i) =
                    make_double2(e0, e1 - e0);
            } else {
                *reinterpret_cast<double *>(lds + L::kE + l * L::kRow + 8 * i) = e0;
                *reinterpret_cast<double *>(lds + L::kW + l * L::kRow + 8 * i) = e1 - e0;
            }
        }
        if constexpr (BINS) *reinterpret_cast<double *>(lds + L::kH + j * L::kRow + 8 * i) = 0.0;
    }
    __syncthreads();

    // The integrand coefficients are read back from LDS into per-lane
    // registers: used by every sample, they would otherwise crowd the scalar
    // register file (and spill) at high dimension.
    double ca[D], cu[D];
    float ca32[D], cu32[D];
    const char *row[D];  // global grid row of every axis (uniform)
#pragma unroll
    for (int j = 0; j < D; ++j) {
        ca[j] = sh.coef[j];
        cu[j] = sh.coef[kMaxDim + j];
        ca32[j] = (float)ca[j];
        cu32[j] = (float)cu[j];
        row[j] = reinterpret_cast<const char *>(grid + j * (nb + 1));
    }
    const float phase32 = (float)A.phase;

    double tS = 0.0, tV = 0.0;

    if (count > 0) {
        uint32_t c = (uint32_t)(((uint64_t)w0 * (uint64_t)A.mult) % (uint64_t)A.m);
        uint32_t dig[D];
        {
            uint32_t rest = c;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                dig[j] = rest % A.g;
                rest = rest / A.g;
            }
        }
        // add-with-carry constants: 2^32 - g detects a digit's wrap in the
        // carry of t + (2^32 - g); 2^32 - m does the same for the cube id
        const uint32_t neg_g = 0u - A.g;
        const uint32_t step_wrap = step - A.m;
        for (uint32_t n = 0; n < count; ++n) {
            uint32_t hb[D];
#pragma unroll
            for (int j = 0; j < D; ++j) hb[j] = kStratumHi + dig[j];
            uint32_t o8[D];
            if constexpr (P2) {
                // p = 2: both samples in straight-line code (independent chains
                // for the scheduler).  With w0 = wa the shifted sums are D1 = dlt,
                // D2 = dlt^2, and var_c = D2 - D1^2/2 = dlt^2 / 2.
                const double wa =
                    F32 ? draw32<F, D, BINS>(A, iteration, ca32, cu32, phase32, c, 0, hb, lds, nb, o8)
                        : draw<F, D, BINS>(A, iteration, ca, cu, c, 0, hb, lds, row, nb, o8);
                if constexpr (BINS) add_bins<D, F32>(lds, o8, wa * wa);
                // keep the two samples' register live ranges apart (128 VGPRs at
                // 1024 threads per block)
                __builtin_amdgcn_sched_barrier(0);
                const double wb =
                    F32 ? draw32<F, D, BINS>(A, iteration, ca32, cu32, phase32, c, 1, hb, lds, nb, o8)
                        : draw<F, D, BINS>(A, iteration, ca, cu, c, 1, hb, lds, row, nb, o8);
                if constexpr (BINS) add_bins<D, F32>(lds, o8, wb * wb);
                const double dlt = wb - wa;
                const double d2 = dlt * dlt;
                tS += wa + wb;
                tV += d2 - d2 * 0.5;
            } else {
                double S = 0.0, D1 = 0.0, D2 = 0.0, ws = 0.0;
                for (uint32_t k = 0; k < A.p; ++k) {
                    const double w =
                        F32 ? draw32<F, D, BINS>(A, iteration, ca32, cu32, phase32, c, k, hb, lds, nb, o8)
                            : draw<F, D, BINS>(A, iteration, ca, cu, c, k, hb, lds, row, nb, o8);
                    S = S + w;
                    if (k == 0) ws = w;
                    const double dlt = w - ws;
                    D1 = D1 + dlt;
                    D2 = D2 + dlt * dlt;
                    if constexpr (BINS) add_bins<D, F32>(lds, o8, w * w);
                }
                tS += S;
                tV += (D2 - D1 * D1 * A.inv_p) * A.inv_pm1;
            }

            // advance to the next work item: the cube id by `step` modulo m, and
            // its digits by the digits of `step` with carries (t = digit +
            // step digit + carry < 2g; t wraps exactly when t + (2^32 - g)
            // carries out, and then t - g is the smaller of the two)
            {
                uint32_t wrap;
                const uint32_t cw = __builtin_addc(c, step_wrap, 0u, &wrap);
                c = wrap ? cw : c + step;
            }
            uint32_t carry = 0u;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                uint32_t ignored;
                const uint32_t t = __builtin_addc(dig[j], step_digit[j], carry, &ignored);
                const uint32_t u = __builtin_addc(t, neg_g, 0u, &carry);
                dig[j] = u < t ? u : t;
            }
        }
    }

    // block reduction of (tS, tV) -> partials[blockIdx.x]
    tS = wave_sum(tS);
    tV = wave_sum(tV);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
        sh.red[0][wave] = tS;
        sh.red[1][wave] = tV;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0, v = 0.0;
        for (int q = 0; q < nw; ++q) {
            s += sh.red[0][q];
            v += sh.red[1][q];
        }
        partial[0] = s;
        partial[1] = v;
    }
    // flush the block's histogram: one global atomic per non-empty bin
    if constexpr (BINS) {
        for (int q = threadIdx.x; q < nh; q += blockDim.x) {
            const int j = q / nb, i = q - j * nb;
            const double v = *reinterpret_cast<const double *>(lds + L::kH + j * L::kRow + 8 * i);
            if (v != 0.0) unsafeAtomicAdd(bins + q, v);
        }
    }
}

template <int F, int D, bool P2, bool BINS, bool F32>
__global__ __launch_bounds__((vs_max_block<F, D>())) void vsample_kernel(const VsArgs A,
                                                           const double *__restrict__ grid,
                                                           double *__restrict__ bins,
                                                           double *__restrict__ partials) {
    __shared__ VsShared<D, BINS, F32> sh;
    // persistent grid: thread tid walks work items tid, tid + T, ... < m
    const uint32_t T = gridDim.x * blockDim.x;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t count = tid < A.m ? (A.m - 1u - tid) / T + 1u : 0u;
    vs_block<F, D, P2, BINS, F32>(A, grid, bins, partials + 2 * blockIdx.x, tid, T, count, A.step,
                                  A.step_digit, A.iteration, sh);
}

// Batched form: one launch per (family, dim, p = 2?) class of a batch, one
// workgroup per tile of the class's tile list (a tile is a range of work
// items of one integrand; the hardware dispatcher hands out the tiles as
// workgroups finish).  Tiles of integrands marked done exit at once.  The
// iteration number is read from device memory so that one captured graph
// serves every iteration.  F32 selects the FP32 map and integrand, as in
// the single form.
template <int F, int D, bool P2, bool BINS, bool F32>
__global__ __launch_bounds__((vs_max_block<F, D>())) void vsample_tiles_kernel(
    const BatchItem *__restrict__ items, const BatchTile *__restrict__ tiles,
    const double *__restrict__ grids, double *__restrict__ bins, double *__restrict__ partials,
    const uint32_t *__restrict__ iter, const uint32_t *__restrict__ done) {
    __shared__ VsShared<D, BINS, F32> sh;
    const BatchTile tile = tiles[blockIdx.x];
    if (done[tile.item] != 0u) return;
    const BatchItem &B = items[tile.item];
    const uint32_t w0 = tile.w_begin + threadIdx.x;
    const uint32_t count = w0 < tile.w_end ? (tile.w_end - 1u - w0) / blockDim.x + 1u : 0u;
    vs_block<F, D, P2, BINS, F32>(B.args, grids + B.grid_off, bins + B.bins_off,
                                    partials + 2 * (size_t)tile.partial, w0, blockDim.x, count,
                                    B.step_block, B.step_digit_block, *iter, sh);
}

template <int F, int D, bool P2, bool BINS, bool F32>
hipError_t launch_vsample_tiles(const BatchItem *items, const BatchTile *tiles, int ntiles,
                                const double *grids, double *bins, double *partials,
                                const uint32_t *iter, const uint32_t *done, int block,
                                hipStream_t stream) {
    hipLaunchKernelGGL((vsample_tiles_kernel<F, D, P2, BINS, F32>), dim3(ntiles), dim3(block), 0,
                       stream, items, tiles, grids, bins, partials, iter, done);
    return hipGetLastError();
}

template <int F, int D, bool P2, bool BINS, bool F32>
hipError_t launch_vsample(const VsArgs &args, const double *grid, double *bins, double *partials,
                          int blocks, int block, hipStream_t stream) {
    hipLaunchKernelGGL((vsample_kernel<F, D, P2, BINS, F32>), dim3(blocks), dim3(block), 0,
                       stream, args, grid, bins, partials);
    return hipGetLastError();
}

#define MCUBES_VS_FN(F, D, P2, BINS, F32) &launch_vsample<F, D, P2, BINS, F32>
#define MCUBES_VS_SYM(F, D, P2, BINS, F32) \
    reinterpret_cast<const void *>(&vsample_kernel<F, D, P2, BINS, F32>)
#define MCUBES_VS_SET(M, F, D, F32)                                            \
    {                                                                          \
        {M(F, D, false, true, F32), M(F, D, true, true, F32)},                 \
        {M(F, D, false, false, F32), M(F, D, true, false, F32)}                \
    }
#define MCUBES_VS_TFN(F, D, P2, BINS, F32) &launch_vsample_tiles<F, D, P2, BINS, F32>
#define MCUBES_VS_TSYM(F, D, P2, BINS, F32) \
    reinterpret_cast<const void *>(&vsample_tiles_kernel<F, D, P2, BINS, F32>)
#define MCUBES_VS_ENTRY(F, D)                                                              \
    VsKernel {                                                                             \
        {MCUBES_VS_SET(MCUBES_VS_FN, F, D, false), MCUBES_VS_SET(MCUBES_VS_FN, F, D, true)},   \
        {MCUBES_VS_SET(MCUBES_VS_SYM, F, D, false), MCUBES_VS_SET(MCUBES_VS_SYM, F, D, true)}, \
        {MCUBES_VS_SET(MCUBES_VS_TFN, F, D, false), MCUBES_VS_SET(MCUBES_VS_TFN, F, D, true)}, \
        {MCUBES_VS_SET(MCUBES_VS_TSYM, F, D, false), MCUBES_VS_SET(MCUBES_VS_TSYM, F, D, true)} \
    }

// A host function returning the table of one family (a namespace-scope const
// array would be promoted to device memory by the HIP compiler).
#define MCUBES_VS_TABLE(NAME, F)                                                             \
    const VsKernel *NAME() {                                                                 \
        static const VsKernel table[kMaxDim + 1] = {                                         \
            VsKernel{},                                                                      \
            MCUBES_VS_ENTRY(F, 1), MCUBES_VS_ENTRY(F, 2), MCUBES_VS_ENTRY(F, 3),             \
            MCUBES_VS_ENTRY(F, 4), MCUBES_VS_ENTRY(F, 5), MCUBES_VS_ENTRY(F, 6),             \
            MCUBES_VS_ENTRY(F, 7), MCUBES_VS_ENTRY(F, 8), MCUBES_VS_ENTRY(F, 9),             \
            MCUBES_VS_ENTRY(F, 10)};                                                         \
        return table;                                                                        \
    }

}  // namespace mcubes
