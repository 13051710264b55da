// Support kernels of the batched form: per-integrand reduction of the tile
// partials, combination, refinement and the iteration counter.  Every kernel
// reads the iteration number and the done flags from device memory, so one
// captured graph serves every iteration of a batch.
#include "support_impl.h"

namespace mcubes {

namespace {

// states[i] <- 0, done[i] <- 0, iter <- 0 (a kernel rather than a memset, so
// that it can sit in a captured graph).
__global__ void batch_reset_kernel(double *__restrict__ states, int64_t state_len,
                                   uint32_t *__restrict__ done, int n, uint32_t *__restrict__ iter) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t q = tid; q < state_len; q += stride) states[q] = 0.0;
    for (int64_t q = tid; q < n; q += stride) done[q] = 0u;
    if (tid == 0) *iter = 0u;
}

// One block of 256 threads per integrand: the fixed-order reduction of the
// single-integrand form over the integrand's tile partials.
__global__ __launch_bounds__(256) void batch_reduce_kernel(const BatchItem *__restrict__ items,
                                                           const double *__restrict__ partials,
                                                           const uint32_t *__restrict__ done,
                                                           double *__restrict__ est) {
    const int i = blockIdx.x;
    if (done[i] != 0u) return;
    const BatchItem &B = items[i];
    __shared__ double sS[256], sV[256];
    double s = 0.0, v = 0.0;
    for (uint32_t b = B.part_begin + threadIdx.x; b < B.part_end; b += 256) {
        s += partials[2 * (size_t)b];
        v += partials[2 * (size_t)b + 1];
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
        est[2 * i] = sS[0] / B.n_samples;
        est[2 * i + 1] = sV[0] / B.var_denom;
    }
}

// One thread per integrand: record and recombine, then mark the integrand done
// when it converged or produced a non-finite estimate.  *active receives the
// number of integrands still running (one block, so the count is exact).
__global__ __launch_bounds__(1024) void batch_combine_kernel(
    int n, const double *__restrict__ est, double *__restrict__ states, uint32_t *__restrict__ done,
    uint32_t *__restrict__ active, const uint32_t *__restrict__ iter, int skip, double rel_tol) {
    __shared__ uint32_t count;
    if (threadIdx.x == 0) count = 0u;
    __syncthreads();
    const uint32_t t = *iter;
    uint32_t mine = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (done[i] != 0u) continue;
        double *state = states + (size_t)i * MCUBES_STATE_LEN;
        combine_state(est[2 * i], est[2 * i + 1], state, t, skip, rel_tol);
        if (state[5] != 0.0 || state[6] != 0.0)
            done[i] = 1u;
        else
            ++mine;
    }
    if (mine) atomicAdd(&count, mine);
    __syncthreads();
    if (threadIdx.x == 0) *active = count;
}

// One block per (integrand, axis): in-place VEGAS rebinning of the axes of
// the integrands that recorded iteration t (including one that converged at
// t, as the single-integrand loop refines after its last iteration) and whose
// estimates are all finite; of every integrand when `all` is set.
__global__ __launch_bounds__(512) void batch_refine_kernel(const BatchItem *__restrict__ items,
                                                           const uint2 *__restrict__ axes,
                                                           double *__restrict__ grids,
                                                           const double *__restrict__ bins,
                                                           const double *__restrict__ states,
                                                           const uint32_t *__restrict__ iter,
                                                           double alpha, int all) {
    __shared__ RefineLds lds;
    const uint2 ax = axes[blockIdx.x];
    const double *state = states + (size_t)ax.x * MCUBES_STATE_LEN;
    if (!all && (state[4] != (double)(*iter + 1u) || state[6] != 0.0)) return;
    const BatchItem &B = items[ax.x];
    const int nb = B.nb;
    double *row = grids + B.grid_off + (size_t)ax.y * (nb + 1);
    refine_axis(row, bins + B.bins_off + (size_t)ax.y * nb, row, nb, alpha, lds);
}

// One block per (integrand, axis): E_j[k] = k / nb.
__global__ __launch_bounds__(256) void batch_init_grids_kernel(const BatchItem *__restrict__ items,
                                                               const uint2 *__restrict__ axes,
                                                               double *__restrict__ grids) {
    const uint2 ax = axes[blockIdx.x];
    const BatchItem &B = items[ax.x];
    const int nb = B.nb;
    double *row = grids + B.grid_off + (size_t)ax.y * (nb + 1);
    for (int k = threadIdx.x; k <= nb; k += blockDim.x) row[k] = (double)k / (double)nb;
}

__global__ void batch_advance_kernel(uint32_t *__restrict__ iter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *iter = *iter + 1u;
}

}  // namespace

hipError_t launch_batch_reset(double *states, int64_t state_len, uint32_t *done, int n,
                              uint32_t *iter, hipStream_t stream) {
    int64_t blocks = (state_len + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, states,
                       state_len, done, n, iter);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchItem *items, int n, const double *partials,
                               const uint32_t *done, double *est, hipStream_t stream) {
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(n), dim3(256), 0, stream, items, partials, done,
                       est);
    return hipGetLastError();
}

hipError_t launch_batch_combine(int n, const double *est, double *states, uint32_t *done,
                                uint32_t *active, const uint32_t *iter, int skip, double rel_tol,
                                hipStream_t stream) {
    const int block = n < 64 ? 64 : (n > 1024 ? 1024 : (n + 63) / 64 * 64);
    hipLaunchKernelGGL(batch_combine_kernel, dim3(1), dim3(block), 0, stream, n, est, states, done,
                       active, iter, skip, rel_tol);
    return hipGetLastError();
}

hipError_t launch_batch_refine(const BatchItem *items, const uint2 *axes, int naxes,
                               double *grids, const double *bins, const double *states,
                               const uint32_t *iter, double alpha, bool all, hipStream_t stream) {
    hipLaunchKernelGGL(batch_refine_kernel, dim3(naxes), dim3(512), 0, stream, items, axes, grids,
                       bins, states, iter, alpha, all ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_init_grids(const BatchItem *items, const uint2 *axes, int naxes,
                                   double *grids, hipStream_t stream) {
    hipLaunchKernelGGL(batch_init_grids_kernel, dim3(naxes), dim3(256), 0, stream, items, axes,
                       grids);
    return hipGetLastError();
}

hipError_t launch_batch_advance(uint32_t *iter, hipStream_t stream) {
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, stream, iter);
    return hipGetLastError();
}

}  // namespace mcubes
