// Small kernels around V-Sample: fixed-order reduction of the block partials,
// the iteration combination, the VEGAS grid refinement, fills and copies.
#include <math.h>

#include "support_impl.h"

namespace mcubes {

namespace {

__global__ void fill_kernel(double *__restrict__ d, int64_t n, double value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = value;
}

__global__ void copy_kernel(const double *__restrict__ s, double *__restrict__ d, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = s[i];
}

// E_j[i] = i / nb on every axis.
__global__ void init_grid_kernel(double *__restrict__ grid, int dim, int nb) {
    const int n = dim * (nb + 1);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const int i = q % (nb + 1);
        grid[q] = (double)i / (double)nb;
    }
}

// One block of 256 threads: thread t adds partials t, t+256, ... in order,
// then a fixed binary tree in LDS.  Deterministic for a given partial count.
__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ partials, int nparts,
                                                     double n_samples, double var_denom,
                                                     double *__restrict__ est) {
    __shared__ double sS[256], sV[256];
    double s = 0.0, v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 256) {
        s += partials[2 * b];
        v += partials[2 * b + 1];
    }
    sS[threadIdx.x] = s;
    sV[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sS[threadIdx.x] += sS[threadIdx.x + h];
            sV[threadIdx.x] += sV[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        est[0] = sS[0] / n_samples;
        est[1] = sV[0] / var_denom;
    }
}

// Inverse-variance combination of the recorded iterations skip..t (one
// thread; at most MCUBES_MAX_ITERATIONS entries).
__global__ void combine_kernel(const double *__restrict__ est, double *__restrict__ state,
                               uint32_t t, int skip, double rel_tol) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    combine_state(est[0], est[1], state, t, skip, rel_tol);
}

// VEGAS rebinning, one block per axis.
__global__ __launch_bounds__(512) void refine_kernel(const double *__restrict__ grid,
                                                     const double *__restrict__ bins,
                                                     double *__restrict__ grid_out, int nb,
                                                     double alpha) {
    __shared__ RefineLds lds;
    const int j = blockIdx.x;
    refine_axis(grid + (size_t)j * (nb + 1), bins + (size_t)j * nb, grid_out + (size_t)j * (nb + 1),
                nb, alpha, lds);
}

}  // namespace

hipError_t launch_fill(double *d, int64_t n, double value, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, d, n, value);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_init_grid(double *grid, int dim, int nb, hipStream_t stream) {
    const int n = dim * (nb + 1);
    hipLaunchKernelGGL(init_grid_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, grid, dim, nb);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nparts, double n_samples, double var_denom,
                         double *est, hipStream_t stream) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, stream, partials, nparts, n_samples,
                       var_denom, est);
    return hipGetLastError();
}

hipError_t launch_combine(const double *est, double *state, uint32_t iteration, int skip,
                          double rel_tol, hipStream_t stream) {
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, stream, est, state, iteration, skip,
                       rel_tol);
    return hipGetLastError();
}

hipError_t launch_refine(const double *grid, const double *bins, double *grid_out, int dim, int nb,
                         double alpha, hipStream_t stream) {
    hipLaunchKernelGGL(refine_kernel, dim3(dim), dim3(512), 0, stream, grid, bins, grid_out, nb,
                       alpha);
    return hipGetLastError();
}

}  // namespace mcubes
