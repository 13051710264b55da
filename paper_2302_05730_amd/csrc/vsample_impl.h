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
// Per block, the grid of all axes is staged once into LDS as (edge, width)
// pairs (one 16-byte LDS read per axis and sample), and the bin contributions go into an
// LDS-private FP64 histogram (ds_add_f64), flushed at the end with one
// global FP64 atomic per non-empty bin.  Per-thread sums of the cube sums and
// cube variances are reduced across the wave with shuffles, across the
// block in LDS, and written as one partial per block; a separate kernel adds
// the partials in a fixed order.
//
// Floating-point operation order matches the definition used throughout
// (multiply-adds are explicit fma; the library is built without contraction),
// so for integrands without libm calls each sample's weight is bit-identical
// to the plain definition.
#pragma once

#include "mcubes_internal.h"

namespace mcubes {

// Philox4x32-10 (Salmon et al., SC'11).  The key is uniform across the
// wave, so the round keys are scalar adds.
__device__ __forceinline__ void philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
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

template <int F, int D>
struct Family;

template <int D>
struct Family<MCUBES_OSCILLATORY, D> {
    static __device__ __forceinline__ double eval(const VsArgs &A, const double *x) {
        double arg = A.phase;
#pragma unroll
        for (int i = 0; i < D; ++i) arg = __fma_rn(A.ca[i], x[i], arg);
        return cos(arg);
    }
};

template <int D>
struct Family<MCUBES_PRODUCT_PEAK, D> {
    static __device__ __forceinline__ double eval(const VsArgs &A, const double *x) {
        double den = 1.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double t = x[i] - A.cu[i];
            den = den * __fma_rn(t, t, A.ca[i]);
        }
        return 1.0 / den;
    }
};

template <int D>
struct Family<MCUBES_CORNER_PEAK, D> {
    static __device__ __forceinline__ double eval(const VsArgs &A, const double *x) {
        double s = 1.0;
#pragma unroll
        for (int i = 0; i < D; ++i) s = __fma_rn(A.ca[i], x[i], s);
        double pw = s;
#pragma unroll
        for (int k = 0; k < D; ++k) pw = pw * s;
        return 1.0 / pw;
    }
};

template <int D>
struct Family<MCUBES_GAUSSIAN, D> {
    static __device__ __forceinline__ double eval(const VsArgs &A, const double *x) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double t = x[i] - A.cu[i];
            s = __fma_rn(A.ca[i], t * t, s);
        }
        return exp(-s);
    }
};

template <int D>
struct Family<MCUBES_C0, D> {
    static __device__ __forceinline__ double eval(const VsArgs &A, const double *x) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) s = __fma_rn(A.ca[i], fabs(x[i] - A.cu[i]), s);
        return exp(-s);
    }
};

template <int D>
struct Family<MCUBES_DISCONTINUOUS, D> {
    static __device__ __forceinline__ double eval(const VsArgs &A, const double *x) {
        double s = 0.0;
        bool inside = true;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            inside = inside && (x[i] < A.cu[i]);
            s = __fma_rn(A.ca[i], x[i], s);
        }
        return inside ? exp(s) : 0.0;
    }
};

template <int D>
struct Family<MCUBES_ADDITION, D> {
    static __device__ __forceinline__ double eval(const VsArgs &, const double *x) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) s = s + x[i];
        return s;
    }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int F, int D>
__global__ __launch_bounds__(kMaxBlock) void vsample_kernel(const VsArgs A,
                                                           const double *__restrict__ grid,
                                                           double *__restrict__ bins,
                                                           double *__restrict__ partials) {
    constexpr int NBLK = (D + 3) / 4;  // Philox blocks (4 words each) per sample
    extern __shared__ double smem[];
    __shared__ double red[2][kMaxBlock / 64];

    const int nb = (int)A.nb;
    const int nh = D * nb;
    // LDS: (edge, width) pairs of every axis, 16-byte aligned, then the bin sums.
    double2 *sEW = reinterpret_cast<double2 *>(smem);  // axis j at [j*nb, (j+1)*nb)
    double *sH = smem + 2 * nh;                          // axis j at [j*nb, (j+1)*nb)

    for (int q = threadIdx.x; q < nh; q += blockDim.x) {
        const int j = q / nb, i = q - j * nb;
        const double e0 = grid[j * (nb + 1) + i];
        const double e1 = grid[j * (nb + 1) + i + 1];
        sEW[q] = make_double2(e0, e1 - e0);
        sH[q] = 0.0;
    }
    __syncthreads();

    const uint32_t T = gridDim.x * blockDim.x;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    double tS = 0.0, tV = 0.0;

    if (tid < A.m) {
        const uint32_t count = (A.m - 1u - tid) / T + 1u;
        uint32_t c = (uint32_t)(((uint64_t)tid * (uint64_t)A.mult) % (uint64_t)A.m);
        uint32_t dig[D];
        {
            uint32_t rest = c;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                dig[j] = rest % A.g;
                rest = rest / A.g;
            }
        }
        for (uint32_t n = 0; n < count; ++n) {
            // c_j + u_j = (c_j 2^32 + r + 1/2) 2^-32 with u_j = (r + 1/2) 2^-32; the
            // integer-plus-half c_j 2^32 + r + 1/2 is exact in FP64 (< 2^53), and
            // scaling fl(nb/g) by 2^-32 is exact, so z below rounds exactly once,
            // like (c_j + u_j) * fl(nb/g).
            double cb[D];
#pragma unroll
            for (int j = 0; j < D; ++j) cb[j] = __fma_rn((double)dig[j], 0x1p32, 0.5);

            double S = 0.0, D1 = 0.0, D2 = 0.0, w0 = 0.0;
            for (uint32_t k = 0; k < A.p; ++k) {
                uint32_t r[4 * NBLK];
#pragma unroll
                for (int b = 0; b < NBLK; ++b)
                    philox10(c, A.stream_id, k * NBLK + b, A.iteration, A.key0, A.key1, r + 4 * b);

                double x[D];
                int bin[D];
                double prod = 1.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double z = ((double)r[j] + cb[j]) * A.zscale;
                    int i = (int)z;
                    double phi;
                    if constexpr (D >= 2) {
                        // g < 2^16 here, so z < nb and the clamp below never fires:
                        // fract(z) = z - floor(z) = z - i exactly.
                        phi = __builtin_amdgcn_fract(z);
                    } else {
                        i = i < nb - 1 ? i : nb - 1;
                        phi = z - (double)i;
                    }
                    const double2 ew = sEW[j * nb + i];
                    x[j] = __fma_rn(ew.y, phi, ew.x);
                    prod = prod * ew.y;
                    bin[j] = i;
                }
                const double J = A.nbd * prod;
                const double f = Family<F, D>::eval(A, x);
                const double w = f * J;
                S = S + w;
                if (k == 0) w0 = w;
                const double dlt = w - w0;
                D1 = D1 + dlt;
                D2 = D2 + dlt * dlt;
                const double w2 = w * w;
#pragma unroll
                for (int j = 0; j < D; ++j) atomicAdd(sH + j * nb + bin[j], w2);
            }
            tS += S;
            tV += (D2 - D1 * D1 * A.inv_p) * A.inv_pm1;

            // advance to the next work item: linear id and digits by `step`
            uint32_t cn = c + A.step;
            if (cn < c || cn >= A.m) cn -= A.m;
            c = cn;
            uint32_t carry = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const uint32_t t = dig[j] + A.step_digit[j] + carry;
                carry = t >= A.g ? 1u : 0u;
                dig[j] = carry ? t - A.g : t;
            }
        }
    }

    // block reduction of (tS, tV) -> partials[blockIdx.x]
    tS = wave_sum(tS);
    tV = wave_sum(tV);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
        red[0][wave] = tS;
        red[1][wave] = tV;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0, v = 0.0;
        for (int q = 0; q < nw; ++q) {
            s += red[0][q];
            v += red[1][q];
        }
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = v;
    }
    // flush the block's histogram: one global atomic per non-empty bin
    for (int i = threadIdx.x; i < nh; i += blockDim.x) {
        const double v = sH[i];
        if (v != 0.0) unsafeAtomicAdd(bins + i, v);
    }
}

template <int F, int D>
hipError_t launch_vsample(const VsArgs &args, const double *grid, double *bins, double *partials,
                          int blocks, int block, size_t lds, hipStream_t stream) {
    hipLaunchKernelGGL((vsample_kernel<F, D>), dim3(blocks), dim3(block), lds, stream, args, grid,
                       bins, partials);
    return hipGetLastError();
}

#define MCUBES_VS_ENTRY(F, D) \
    VsKernel { &launch_vsample<F, D>, reinterpret_cast<const void *>(&vsample_kernel<F, D>) }

// A host function returning the table of one family (a namespace-scope const
// array would be promoted to device memory by the HIP compiler).
#define MCUBES_VS_TABLE(NAME, F)                                                             \
    const VsKernel *NAME() {                                                                 \
        static const VsKernel table[kMaxDim + 1] = {                                         \
            VsKernel{nullptr, nullptr}, MCUBES_VS_ENTRY(F, 1), MCUBES_VS_ENTRY(F, 2),        \
            MCUBES_VS_ENTRY(F, 3),      MCUBES_VS_ENTRY(F, 4), MCUBES_VS_ENTRY(F, 5),        \
            MCUBES_VS_ENTRY(F, 6),      MCUBES_VS_ENTRY(F, 7), MCUBES_VS_ENTRY(F, 8),        \
            MCUBES_VS_ENTRY(F, 9),      MCUBES_VS_ENTRY(F, 10)};                             \
        return table;                                                                        \
    }

}  // namespace mcubes
