// Small kernels around V-Sample: fixed-order reduction of the block partials,
// the iteration combination, the VEGAS grid refinement, fills and copies.
#include <math.h>

#include "mcubes_internal.h"

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
    double *hist = state + MCUBES_STATE_HEADER;
    const double It = est[0], Vt = est[1];
    hist[2 * t] = It;
    hist[2 * t + 1] = Vt;
    if (!isfinite(It) || !isfinite(Vt)) state[6] = 1.0;
    const int T = (int)t + 1;
    state[4] = (double)T;
    const int n = T - skip;
    double Ibar = 0.0, sigma = INFINITY, chi2dof = 0.0;
    int dof = 0;
    if (n >= 1) {
        double sw = 0.0, swi = 0.0;
        int exact = -1;
        for (int q = skip; q < T; ++q) {
            const double v = hist[2 * q + 1];
            if (v == 0.0) {
                exact = q;
            } else {
                sw = sw + 1.0 / v;
                swi = swi + hist[2 * q] / v;
            }
        }
        dof = n - 1;
        if (exact >= 0) {
            Ibar = hist[2 * exact];
            sigma = 0.0;
        } else {
            Ibar = swi / sw;
            double chi2 = 0.0;
            for (int q = skip; q < T; ++q) {
                const double dv = hist[2 * q] - Ibar;
                chi2 = chi2 + dv * dv / hist[2 * q + 1];
            }
            sigma = 1.0 / sqrt(sw);
            chi2dof = n > 1 ? chi2 / (double)(n - 1) : 0.0;
        }
    }
    state[0] = Ibar;
    state[1] = sigma;
    state[2] = chi2dof;
    state[3] = (double)dof;
    state[5] = (n >= 1 && sigma <= rel_tol * fabs(Ibar)) ? 1.0 : 0.0;
}

// VEGAS rebinning, one block per axis, one thread per bin.  The two running
// sums (total smoothed weight, cumulative damped weight) are taken in bin
// order by one thread so that they round exactly like a sequential loop; the
// damping (log, pow) and the placement of the new edges run in parallel.  New
// edge k lies in the first old bin i whose cumulative damped weight reaches
// k T, found by binary search.
__global__ __launch_bounds__(512) void refine_kernel(const double *__restrict__ grid,
                                                     const double *__restrict__ bins,
                                                     double *__restrict__ grid_out, int nb,
                                                     double alpha) {
    __shared__ double sE[kMaxBins + 1], sd[kMaxBins], ss[kMaxBins], sr[kMaxBins],
        sR[kMaxBins + 1];
    __shared__ double sTot;
    const int j = blockIdx.x;
    const int k = threadIdx.x;
    const double *E = grid + (size_t)j * (nb + 1);
    const double *dj = bins + (size_t)j * nb;
    double *En = grid_out + (size_t)j * (nb + 1);

    if (k <= nb) sE[k] = E[k];
    if (k < nb) sd[k] = dj[k];
    __syncthreads();
    if (k < nb) {
        double s;
        if (k == 0)
            s = (sd[0] + sd[1]) / 2.0;
        else if (k == nb - 1)
            s = (sd[nb - 2] + sd[nb - 1]) / 2.0;
        else
            s = (sd[k - 1] + sd[k] + sd[k + 1]) / 3.0;
        ss[k] = s;
    }
    __syncthreads();
    if (k == 0) {
        double S = 0.0;
        for (int i = 0; i < nb; ++i) S = S + ss[i];
        sTot = S;
    }
    __syncthreads();
    const double S = sTot;
    if (!(S > 0.0)) {  // no weight on this axis: keep it
        if (k <= nb) En[k] = sE[k];
        return;
    }
    if (k < nb) {
        const double s = ss[k];
        const double rho = s / S;
        double r;
        if (s == 0.0)
            r = 0.0;
        else if (rho == 1.0)
            r = 1.0;
        else
            r = pow((rho - 1.0) / log(rho), alpha);
        sr[k] = r;
    }
    __syncthreads();
    if (k == 0) {
        double R = 0.0;
        sR[0] = 0.0;
        for (int i = 0; i < nb; ++i) {
            R = R + sr[i];
            sR[i + 1] = R;
        }
    }
    __syncthreads();
    const double T = sR[nb] / (double)nb;
    if (k == 0) {
        En[0] = 0.0;
        En[nb] = 1.0;
    } else if (k < nb) {
        const double target = (double)k * T;
        // first q in [1, nb] with R[q] >= target (nb if none), bin i = q - 1
        int lo = 1, hi = nb;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sR[mid] >= target)
                hi = mid;
            else
                lo = mid + 1;
        }
        const int i = lo - 1;
        const double W = sE[i + 1] - sE[i];
        double frac = (target - sR[i]) / sr[i];
        if (frac > 1.0) frac = 1.0;
        const double e = sE[i] + frac * W;
        En[k] = e < sE[i + 1] ? e : sE[i + 1];
    }
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
