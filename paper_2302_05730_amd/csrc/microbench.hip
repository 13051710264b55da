// Microbenchmarks that attribute V-Sample's time to its parts (the analogue
// of the integrand-invocation experiment of §5.1 of the paper, where every
// thread evaluates the integrand serially on points prepared on the host).
//
//   MCUBES_MB_INTEGRAND  f(x) of a family on points read from a device table
//   MCUBES_MB_PHILOX     the ceil(d/4) Philox4x32-10 blocks of one sample
//   MCUBES_MB_EXP64 ...  one libm call per step (FP64 and FP32 exp, cos, pow)
//
// Every thread accumulates its results and writes one value, so nothing is
// optimised away.
#include "vsample_impl.h"

namespace mcubes {

namespace {

template <int F, int D>
__global__ __launch_bounds__(256) void mb_integrand_kernel(VsArgs A, const double *__restrict__ pts,
                                                           int64_t npts, int64_t calls,
                                                           double *__restrict__ out) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double ca[D], cu[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        ca[j] = A.ca[j];
        cu[j] = A.cu[j];
    }
    double sum = 0.0;
    int64_t q = (tid * 7919) % npts;
    for (int64_t k = 0; k < calls; ++k) {
        const double *x = pts + q * D;
        Acc acc = Family<F, D>::begin(A.phase);
#pragma unroll
        for (int j = 0; j < D; ++j) Family<F, D>::axis(acc, ca[j], cu[j], x[j]);
        sum += Family<F, D>::end(acc, A);
        q = (q + 1 == npts) ? 0 : q + 1;
    }
    out[tid] = sum;
}

template <int D>
__global__ __launch_bounds__(256) void mb_philox_kernel(VsArgs A, int64_t calls,
                                                        double *__restrict__ out) {
    constexpr int NBLK = (D + 3) / 4;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int64_t k = 0; k < calls; ++k) {
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            uint32_t r[4];
            philox10(tid, A.stream_id, (uint32_t)k * NBLK + b, A.iteration, A.key0, A.key1, r);
            acc ^= r[0] ^ r[1] ^ r[2] ^ r[3];
        }
    }
    out[tid] = (double)acc;
}

__global__ __launch_bounds__(256) void mb_math_kernel(int kind, int64_t calls,
                                                      double *__restrict__ out) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x = 0.25 + 1e-9 * (double)(tid & 1023);
    float xf = (float)x;
    double acc = 0.0;
    float accf = 0.0f;
    for (int64_t k = 0; k < calls; ++k) {
        switch (kind) {
        case MCUBES_MB_EXP64: acc += exp(-x); x += 1e-7; break;
        case MCUBES_MB_COS64: acc += cos(x); x += 1e-3; break;
        case MCUBES_MB_POW64: acc += pow(x, 1.5); x += 1e-7; break;
        case MCUBES_MB_EXP32: accf += expf(-xf); xf += 1e-5f; break;
        case MCUBES_MB_COS32: accf += cosf(xf); xf += 1e-3f; break;
        default: accf += powf(xf, 1.5f); xf += 1e-5f; break;
        }
    }
    out[tid] = acc + (double)accf;
}

template <int F>
hipError_t launch_integrand_f(int dim, const VsArgs &A, const double *pts, int64_t npts,
                              int64_t calls, int blocks, int block, double *out,
                              hipStream_t s) {
#define MB_CASE(D)                                                                          \
    case D:                                                                                 \
        hipLaunchKernelGGL((mb_integrand_kernel<F, D>), dim3(blocks), dim3(block), 0, s, A, \
                           pts, npts, calls, out);                                          \
        break;
    switch (dim) {
        MB_CASE(1) MB_CASE(2) MB_CASE(3) MB_CASE(4) MB_CASE(5)
        MB_CASE(6) MB_CASE(7) MB_CASE(8) MB_CASE(9) MB_CASE(10)
    default: return hipErrorInvalidValue;
    }
#undef MB_CASE
    return hipGetLastError();
}

}  // namespace

hipError_t launch_microbench(int kind, int family, int dim, const VsArgs &A, const double *pts,
                             int64_t npts, int64_t calls, int blocks, int block, double *out,
                             hipStream_t s) {
    if (kind == MCUBES_MB_INTEGRAND) {
        switch (family) {
        case MCUBES_OSCILLATORY:
            return launch_integrand_f<MCUBES_OSCILLATORY>(dim, A, pts, npts, calls, blocks, block, out, s);
        case MCUBES_PRODUCT_PEAK:
            return launch_integrand_f<MCUBES_PRODUCT_PEAK>(dim, A, pts, npts, calls, blocks, block, out, s);
        case MCUBES_CORNER_PEAK:
            return launch_integrand_f<MCUBES_CORNER_PEAK>(dim, A, pts, npts, calls, blocks, block, out, s);
        case MCUBES_GAUSSIAN:
            return launch_integrand_f<MCUBES_GAUSSIAN>(dim, A, pts, npts, calls, blocks, block, out, s);
        case MCUBES_C0:
            return launch_integrand_f<MCUBES_C0>(dim, A, pts, npts, calls, blocks, block, out, s);
        case MCUBES_DISCONTINUOUS:
            return launch_integrand_f<MCUBES_DISCONTINUOUS>(dim, A, pts, npts, calls, blocks, block, out, s);
        case MCUBES_ADDITION:
            return launch_integrand_f<MCUBES_ADDITION>(dim, A, pts, npts, calls, blocks, block, out, s);
        case MCUBES_MIXTURE:
            return launch_integrand_f<MCUBES_MIXTURE>(dim, A, pts, npts, calls, blocks, block, out, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (kind == MCUBES_MB_PHILOX) {
#define MB_PCASE(D)                                                                            \
    case D:                                                                                    \
        hipLaunchKernelGGL((mb_philox_kernel<D>), dim3(blocks), dim3(block), 0, s, A, calls, \
                           out);                                                               \
        break;
        switch (dim) {
            MB_PCASE(1) MB_PCASE(2) MB_PCASE(3) MB_PCASE(4) MB_PCASE(5)
            MB_PCASE(6) MB_PCASE(7) MB_PCASE(8) MB_PCASE(9) MB_PCASE(10)
        default: return hipErrorInvalidValue;
        }
#undef MB_PCASE
        return hipGetLastError();
    }
    hipLaunchKernelGGL(mb_math_kernel, dim3(blocks), dim3(block), 0, s, kind, calls, out);
    return hipGetLastError();
}

}  // namespace mcubes
