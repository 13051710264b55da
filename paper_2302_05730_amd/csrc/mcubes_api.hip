// Host runtime and C interface of libmcubes (declared in include/mcubes.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "mcubes_internal.h"

using namespace mcubes;

namespace {
thread_local std::string g_error;
}  // namespace

namespace mcubes {

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(MCUBES_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const VsKernel *family_table(int family) {
    switch (family) {
    case MCUBES_OSCILLATORY: return kVsOscillatory();
    case MCUBES_PRODUCT_PEAK: return kVsProductPeak();
    case MCUBES_CORNER_PEAK: return kVsCornerPeak();
    case MCUBES_GAUSSIAN: return kVsGaussian();
    case MCUBES_C0: return kVsC0();
    case MCUBES_DISCONTINUOUS: return kVsDiscontinuous();
    case MCUBES_ADDITION: return kVsAddition();
    case MCUBES_MIXTURE: return kVsMixture();
    default: return nullptr;
    }
}

int64_t pow_capped(int64_t b, int e, int64_t cap) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) {
        if (r > cap / b) return cap + 1;
        r *= b;
    }
    return r;
}

int plan_sizes(int dim, int64_t ncall, int64_t out[4]) {
    if (dim < 1 || dim > MCUBES_MAX_DIM)
        return fail(MCUBES_E_ARG, "dim must be in [1, %d], got %d", MCUBES_MAX_DIM, dim);
    if (ncall < 2) return fail(MCUBES_E_ARG, "ncall must be >= 2, got %lld", (long long)ncall);
    const int64_t half = ncall / 2;
    int64_t g = (int64_t)floor(pow((double)half, 1.0 / dim));
    if (g < 1) g = 1;
    while (g > 1 && pow_capped(g, dim, half) > half) --g;
    while (pow_capped(g + 1, dim, half) <= half) ++g;
    if (g > MCUBES_MAX_SIDE) g = MCUBES_MAX_SIDE;  // dim = 1 only: keeps c_j + u exact
    const int64_t m = pow_capped(g, dim, half);
    int64_t p = ncall / m;
    if (p < 2) p = 2;
    out[0] = g;
    out[1] = m;
    out[2] = p;
    out[3] = m * p;
    return MCUBES_OK;
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int validate_params(int family, const double *params, int dim) {
    if (family < 0 || family >= kFamilies)
        return fail(MCUBES_E_INTEGRAND, "unknown integrand family %d", family);
    if (family == MCUBES_ADDITION) return MCUBES_OK;
    if (!params) return fail(MCUBES_E_INTEGRAND, "family %d needs 2*dim parameters", family);
    for (int i = 0; i < 2 * dim; ++i)
        if (!isfinite(params[i])) return fail(MCUBES_E_INTEGRAND, "parameter %d is not finite", i);
    if (family == MCUBES_PRODUCT_PEAK)
        for (int i = 0; i < dim; ++i)
            if (params[i] == 0.0) return fail(MCUBES_E_INTEGRAND, "product peak needs a_%d != 0", i);
    if (family == MCUBES_MIXTURE) {
        if (dim < 2) return fail(MCUBES_E_INTEGRAND, "the mixture needs dim >= 2");
        if (!(params[0] > 0.0)) return fail(MCUBES_E_INTEGRAND, "mixture: a_0 = s must be > 0");
        if (!(params[1] >= 0.0 && params[1] < 1.0))
            return fail(MCUBES_E_INTEGRAND, "mixture: a_1 = r must be in [0, 1)");
    }
    return MCUBES_OK;
}

// Fold the integrand parameters into the kernel's coefficients.
void fold_params(int family, const double *params, int dim, VsArgs &A) {
    for (int i = 0; i < kMaxDim; ++i) A.ca[i] = A.cu[i] = 0.0;
    A.phase = 0.0;
    if (family == MCUBES_ADDITION) return;
    const double *a = params, *u = params + dim;
    if (family == MCUBES_MIXTURE) {
        const double sg = a[0], r = a[1];
        const double lam = 1.0 - r + (double)dim * r;
        A.mix_c1 = r / lam;
        A.mix_c2 = 1.0 / (2.0 * sg * sg * (1.0 - r));
        A.mix_norm = 0.5 / (pow(2.0 * M_PI, 0.5 * (double)dim) * pow(sg, (double)dim) *
                            pow(1.0 - r, 0.5 * (double)(dim - 1)) * sqrt(lam));
        for (int i = 0; i < dim; ++i) {
            A.ca[i] = u[0];
            A.cu[i] = u[1];
        }
        return;
    }
    for (int i = 0; i < dim; ++i) {
        switch (family) {
        case MCUBES_PRODUCT_PEAK: A.ca[i] = 1.0 / (a[i] * a[i]); break;
        case MCUBES_GAUSSIAN: A.ca[i] = a[i] * a[i]; break;
        default: A.ca[i] = a[i]; break;
        }
        A.cu[i] = u[i];
    }
    if (family == MCUBES_OSCILLATORY) A.phase = (2.0 * M_PI) * u[0];
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

void set_step(VsArgs &A, int dim, uint64_t threads) {
    const uint64_t step = (uint64_t)(((unsigned __int128)threads * A.mult) % A.m);
    A.step = (uint32_t)step;
    uint64_t rest = step;
    for (int j = 0; j < kMaxDim; ++j) {
        A.step_digit[j] = j < dim ? (uint32_t)(rest % A.g) : 0u;
        if (j < dim) rest /= A.g;
    }
}

void make_args(int family, const double *params, int dim, int64_t g, int64_t m, int64_t p, int nb,
               uint64_t seed, uint32_t stream_id, VsArgs &A) {
    memset(&A, 0, sizeof A);
    fold_params(family, params, dim, A);
    A.zscale = ((double)nb / (double)g) * 0x1p-32;
    double nbd = (double)nb;
    for (int j = 1; j < dim; ++j) nbd = nbd * (double)nb;
    A.nbd = nbd;
    A.inv_p = 1.0 / (double)p;
    A.inv_pm1 = 1.0 / (double)(p - 1);
    A.key0 = (uint32_t)(seed & 0xffffffffu);
    A.key1 = (uint32_t)(seed >> 32);
    A.stream_id = stream_id;
    A.iteration = 0;
    A.g = (uint32_t)g;
    A.m = (uint32_t)m;
    A.p = (uint32_t)p;
    A.nb = (uint32_t)nb;
    // cube permutation multiplier: near m (sqrt(5)-1)/2, coprime to g (hence to m = g^d)
    int64_t mult = (int64_t)floor((double)m * 0.6180339887498949);
    if (mult < 1) mult = 1;
    while (gcd64(mult, g) != 1) ++mult;
    mult %= m;
    if (m == 1) mult = 0;
    A.mult = (uint32_t)mult;
}

int check_sizes(int64_t m, int64_t p, int dim) {
    if (m > 0xFFFFFFFFll) return fail(MCUBES_E_ARG, "too many cubes (%lld >= 2^32)", (long long)m);
    if (p * ((dim + 3) / 4) > 0xFFFFFFFFll) return fail(MCUBES_E_ARG, "too many samples per cube");
    return MCUBES_OK;
}


int plan_init(int family, const double *params, int dim, int64_t ncall, uint64_t seed,
              const mcubes_options *opt_in, mcubes_plan *P) {
    mcubes_options opt;
    mcubes_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int64_t sz[4];
    int rc = plan_sizes(dim, ncall, sz);
    if (rc != MCUBES_OK) return rc;
    rc = validate_params(family, params, dim);
    if (rc != MCUBES_OK) return rc;
    if (opt.nbins < 2 || opt.nbins > MCUBES_MAX_BINS)
        return fail(MCUBES_E_ARG, "nbins must be in [2, %d], got %d", MCUBES_MAX_BINS, opt.nbins);
    if (!(opt.alpha >= 0.0) || !isfinite(opt.alpha))
        return fail(MCUBES_E_ARG, "alpha must be finite and >= 0");
    if (opt.skip < 0) return fail(MCUBES_E_ARG, "skip must be >= 0");
    if (opt.block_size != 0 &&
        (opt.block_size < 64 || opt.block_size > kMaxBlock || opt.block_size % 64 != 0))
        return fail(MCUBES_E_ARG, "block_size must be 0 or a multiple of 64 in [64, %d]", kMaxBlock);
    if (opt.blocks < 0) return fail(MCUBES_E_ARG, "blocks must be >= 0");
    if (opt.precision != MCUBES_FP64 && opt.precision != MCUBES_FP32)
        return fail(MCUBES_E_ARG, "precision must be MCUBES_FP64 or MCUBES_FP32");
    const int64_t g = sz[0], m = sz[1], p = sz[2];
    rc = check_sizes(m, p, dim);
    if (rc != MCUBES_OK) return rc;

    // device and launch geometry
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(CUs)");

    const int prec = opt.precision == MCUBES_FP32 ? 1 : 0;
    const VsKernel &kern_set = family_table(family)[dim];
    const int variant = (p == 2) ? 1 : 0;
    const void *kfunc = kern_set.func[prec][0][variant];
    const int nb = opt.nbins;
    // the kernel's LDS is static: its tables have room for kMaxBins bins per axis
    hipFuncAttributes fattr;
    e = hipFuncGetAttributes(&fattr, kfunc);
    if (e != hipSuccess) return hip_fail(e, "hipFuncGetAttributes");
    const size_t lds = fattr.sharedSizeBytes;
    const int max_block = fattr.maxThreadsPerBlock;
    if (opt.block_size > max_block)
        return fail(MCUBES_E_ARG, "block_size %d exceeds this kernel's limit %d", opt.block_size,
                    max_block);
    const int block = opt.block_size ? opt.block_size : max_block;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfunc, block, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) return fail(MCUBES_E_ARG, "V-Sample does not fit: block %d, LDS %zu", block, lds);
    int64_t blocks = opt.blocks ? opt.blocks : (int64_t)per_cu * cus;
    const int64_t needed = (m + block - 1) / block;
    if (!opt.blocks && blocks > needed) blocks = needed;
    if (blocks < 1) blocks = 1;
    if (blocks * block > 0x7FFFFFFFll) return fail(MCUBES_E_ARG, "too many threads");

    P->family = family;
    P->precision = opt.precision;
    P->dim = dim;
    P->nb = nb;
    P->block = block;
    P->blocks = (int)blocks;
    P->lds = lds;
    P->adapt_iters = opt.adapt_iters;
    P->skip = opt.skip;
    P->alpha = opt.alpha;
    P->g = g;
    P->m = m;
    P->p = p;
    P->n = sz[3];
    P->launch[0] = kern_set.launch[prec][1][variant];
    P->launch[1] = kern_set.launch[prec][0][variant];
    P->func = kfunc;
    P->stream = opt.stream;
    P->ws = nullptr;
    P->ws_len = 0;

    make_args(family, params, dim, g, m, p, nb, seed, opt.stream_id, P->args);
    set_step(P->args, dim, (uint64_t)blocks * (uint64_t)block);
    return MCUBES_OK;
}


// Device buffers of integrate_run, in doubles: two grids, the bins, the
// block partials, the iteration estimate and the combined state.
int64_t integrate_buffer_len(const mcubes_plan &P) {
    const int64_t ng = (int64_t)P.dim * (P.nb + 1), nbn = (int64_t)P.dim * P.nb;
    return 2 * ng + nbn + 2 * (int64_t)P.blocks + 2 + MCUBES_STATE_LEN;
}

int integrate_run(const mcubes_plan &Pr, double *buf, int itmax, double rel_tol, bool timed,
                  mcubes_result *out, double *grid_out, double *trace) {
    const mcubes_plan *P = &Pr;
    hipStream_t s = as_stream(P->stream);
    const int64_t ng = (int64_t)P->dim * (P->nb + 1), nbn = (int64_t)P->dim * P->nb;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double head[MCUBES_STATE_HEADER];
    double kernel_ms = 0.0;
    int done = 0, rc = MCUBES_OK;
    hipError_t e = hipSuccess;
    double *grid[2] = {buf, buf + ng};
    double *bins = buf + 2 * ng;
    double *partials = bins + nbn;
    double *est = partials + 2 * (int64_t)P->blocks;
    double *state = est + 2;
    memset(head, 0, sizeof head);

#define MC_CHECK(expr, what)                 \
    do {                                     \
        e = (expr);                          \
        if (e != hipSuccess) {               \
            rc = hip_fail(e, what);          \
            goto cleanup;                    \
        }                                    \
    } while (0)
#define MC_CALL(expr)                        \
    do {                                     \
        rc = (expr);                         \
        if (rc != MCUBES_OK) goto cleanup;   \
    } while (0)

    if (timed) {
        MC_CHECK(hipEventCreate(&ev0), "hipEventCreate");
        MC_CHECK(hipEventCreate(&ev1), "hipEventCreate");
    }
    MC_CHECK(launch_init_grid(grid[0], P->dim, P->nb, s), "init_grid launch");
    MC_CHECK(launch_fill(state, MCUBES_STATE_LEN, 0.0, s), "fill launch");
    for (int t = 0; t < itmax; ++t) {
        double *g_in = grid[t & 1], *g_out = grid[(t + 1) & 1];
        const bool refine = P->adapt_iters < 0 || t < P->adapt_iters;
        if (refine) MC_CHECK(launch_fill(bins, nbn, 0.0, s), "fill launch");
        if (timed) MC_CHECK(hipEventRecord(ev0, s), "hipEventRecord");
        MC_CALL(mcubes_vsample(P, (uint32_t)t, g_in, refine ? bins : nullptr, partials,
                               P->stream));
        if (timed) MC_CHECK(hipEventRecord(ev1, s), "hipEventRecord");
        MC_CALL(mcubes_reduce(P, partials, est, P->stream));
        MC_CALL(mcubes_combine(P, (uint32_t)t, est, state, rel_tol, P->stream));
        if (refine)
            MC_CALL(mcubes_refine(P, g_in, bins, g_out, P->stream));
        else
            MC_CHECK(launch_copy(g_in, g_out, ng, s), "copy launch");
        MC_CHECK(hipMemcpyAsync(head, state, sizeof head, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        MC_CHECK(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (timed) {
            float ms = 0.0f;
            MC_CHECK(hipEventElapsedTime(&ms, ev0, ev1), "hipEventElapsedTime");
            kernel_ms += ms;
        }
        done = t + 1;
        if (head[6] != 0.0) {
            rc = fail(MCUBES_E_NONFINITE, "iteration %d produced a non-finite estimate", t);
            goto cleanup;
        }
        if (head[5] != 0.0) break;
    }
    if (trace) {
        MC_CHECK(hipMemcpyAsync(trace, state + MCUBES_STATE_HEADER,
                                (size_t)(2 * done) * sizeof(double), hipMemcpyDeviceToHost, s),
                 "hipMemcpyAsync trace");
    }
    if (grid_out) {
        MC_CHECK(hipMemcpyAsync(grid_out, grid[done & 1], (size_t)ng * sizeof(double),
                                hipMemcpyDeviceToHost, s),
                 "hipMemcpyAsync grid");
    }
    MC_CHECK(hipStreamSynchronize(s), "hipStreamSynchronize");
    out->estimate = head[0];
    out->error = head[1];
    out->chi2_dof = head[2];
    out->dof = (int32_t)head[3];
    out->iterations = done;
    out->converged = head[5] != 0.0;
    out->cube_side = P->g;
    out->ncubes = P->m;
    out->samples_per_cube = P->p;
    out->samples_per_iter = P->n;
    out->kernel_ms = kernel_ms;
    rc = out->converged ? MCUBES_OK : MCUBES_NOT_CONVERGED;
    out->status = rc;

cleanup:
#undef MC_CHECK
#undef MC_CALL
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    return rc;
}

}  // namespace mcubes

// Scratch of mcubes_integrate_noalloc: grids, bins, block partials, estimate
// and combined state of one integration, in the layout of integrate_run.  Each
// GPU holds its own copy for the life of the process.  In host code the name
// is not a device address: kernels and copies get the pointer that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[MCUBES_NOALLOC_SCRATCH];

namespace {

constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The current device's copy of `scratch` (looked up once per device).
int noalloc_scratch(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MCUBES_E_DEVICE, "device %d is beyond the %d this library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return MCUBES_OK;
}

}  // namespace

extern "C" {

void mcubes_default_options(mcubes_options *opt) {
    if (!opt) return;
    opt->nbins = 500;
    opt->adapt_iters = -1;
    opt->skip = 0;
    opt->block_size = 0;
    opt->blocks = 0;
    opt->stream_id = 0;
    opt->precision = MCUBES_FP64;
    opt->alpha = 1.5;
    opt->stream = nullptr;
}

const char *mcubes_last_error(void) { return g_error.c_str(); }

int mcubes_plan_sizes(int dim, int64_t ncall, int64_t out[4]) {
    if (!out) return fail(MCUBES_E_ARG, "out is NULL");
    int64_t tmp[4];
    const int rc = plan_sizes(dim, ncall, tmp);
    if (rc != MCUBES_OK) return rc;
    memcpy(out, tmp, sizeof tmp);
    return MCUBES_OK;
}

int mcubes_plan_create(int family, const double *params, int dim, int64_t ncall, uint64_t seed,
                       const mcubes_options *opt_in, mcubes_plan **plan_out) {
    if (!plan_out) return fail(MCUBES_E_ARG, "plan is NULL");
    mcubes_plan *P = new (std::nothrow) mcubes_plan();
    if (!P) return fail(MCUBES_E_ALLOC, "out of host memory");
    const int rc = plan_init(family, params, dim, ncall, seed, opt_in, P);
    if (rc != MCUBES_OK) {
        delete P;
        return rc;
    }
    *plan_out = P;
    return MCUBES_OK;
}

int mcubes_plan_get_info(const mcubes_plan *P, mcubes_plan_info *info) {
    if (!P || !info) return fail(MCUBES_E_ARG, "NULL argument");
    info->family = P->family;
    info->dim = P->dim;
    info->nbins = P->nb;
    info->block_size = P->block;
    info->blocks = P->blocks;
    info->lds_bytes = (int32_t)P->lds;
    info->precision = P->precision;
    info->cube_side = P->g;
    info->ncubes = P->m;
    info->samples_per_cube = P->p;
    info->samples_per_iter = P->n;
    info->grid_len = (int64_t)P->dim * (P->nb + 1);
    info->bins_len = (int64_t)P->dim * P->nb;
    info->partials_len = 2 * (int64_t)P->blocks;
    info->state_len = MCUBES_STATE_LEN;
    return MCUBES_OK;
}

void mcubes_plan_destroy(mcubes_plan *P) {
    if (!P) return;
    if (P->ws) (void)hipFree(P->ws);
    delete P;
}

int mcubes_init_grid(const mcubes_plan *P, double *d_grid, void *stream) {
    if (!P || !d_grid) return fail(MCUBES_E_ARG, "NULL argument");
    const hipError_t e = launch_init_grid(d_grid, P->dim, P->nb, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "init_grid launch");
}

int mcubes_fill(double *d, int64_t n, double value, void *stream) {
    if (n < 0 || (n > 0 && !d)) return fail(MCUBES_E_ARG, "bad buffer");
    const hipError_t e = launch_fill(d, n, value, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "fill launch");
}

int mcubes_vsample(const mcubes_plan *P, uint32_t iteration, const double *d_grid, double *d_bins,
                   double *d_partials, void *stream) {
    if (!P || !d_grid || !d_partials) return fail(MCUBES_E_ARG, "NULL argument");
    VsArgs A = P->args;
    A.iteration = iteration;
    const hipError_t e = P->launch[d_bins ? 1 : 0](A, d_grid, d_bins, d_partials, P->blocks,
                                                   P->block, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "V-Sample launch");
}

int mcubes_reduce(const mcubes_plan *P, const double *d_partials, double *d_est, void *stream) {
    if (!P || !d_partials || !d_est) return fail(MCUBES_E_ARG, "NULL argument");
    const double n = (double)P->m * (double)P->p;
    const double denom = (double)P->p * (double)P->m * (double)P->m;
    const hipError_t e = launch_reduce(d_partials, P->blocks, n, denom, d_est, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "reduce launch");
}

int mcubes_combine(const mcubes_plan *P, uint32_t iteration, const double *d_est, double *d_state,
                   double rel_tol, void *stream) {
    if (!P || !d_est || !d_state) return fail(MCUBES_E_ARG, "NULL argument");
    if (iteration >= MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "iteration %u >= %d", iteration, MCUBES_MAX_ITERATIONS);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(MCUBES_E_ARG, "rel_tol must be finite and >= 0");
    const hipError_t e = launch_combine(d_est, d_state, iteration, P->skip, rel_tol, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "combine launch");
}

int mcubes_refine(const mcubes_plan *P, const double *d_grid, const double *d_bins,
                  double *d_grid_out, void *stream) {
    if (!P || !d_grid || !d_bins || !d_grid_out) return fail(MCUBES_E_ARG, "NULL argument");
    if (d_grid == d_grid_out) return fail(MCUBES_E_ARG, "d_grid_out must not alias d_grid");
    const hipError_t e =
        launch_refine(d_grid, d_bins, d_grid_out, P->dim, P->nb, P->alpha, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "refine launch");
}

int mcubes_iteration(const mcubes_plan *P, uint32_t iteration, const double *d_grid,
                     double *d_grid_out, double *d_bins, double *d_partials, double *d_est,
                     double *d_state, double rel_tol, void *stream) {
    if (!P || !d_grid || !d_grid_out || !d_bins || !d_partials || !d_est || !d_state)
        return fail(MCUBES_E_ARG, "NULL argument");
    if (d_grid == d_grid_out) return fail(MCUBES_E_ARG, "d_grid_out must not alias d_grid");
    if (iteration >= MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "iteration %u >= %d", iteration, MCUBES_MAX_ITERATIONS);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(MCUBES_E_ARG, "rel_tol must be finite and >= 0");
    hipStream_t s = as_stream(stream);
    const bool refine = P->adapt_iters < 0 || (int64_t)iteration < P->adapt_iters;
    hipError_t e = hipSuccess;
    if (refine) {
        e = launch_fill(d_bins, (int64_t)P->dim * P->nb, 0.0, s);
        if (e != hipSuccess) return hip_fail(e, "fill launch");
    }
    int rc = mcubes_vsample(P, iteration, d_grid, refine ? d_bins : nullptr, d_partials, stream);
    if (rc != MCUBES_OK) return rc;
    rc = mcubes_reduce(P, d_partials, d_est, stream);
    if (rc != MCUBES_OK) return rc;
    rc = mcubes_combine(P, iteration, d_est, d_state, rel_tol, stream);
    if (rc != MCUBES_OK) return rc;
    if (refine) return mcubes_refine(P, d_grid, d_bins, d_grid_out, stream);
    e = launch_copy(d_grid, d_grid_out, (int64_t)P->dim * (P->nb + 1), s);
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "copy launch");
}

int mcubes_iterate(mcubes_plan *P, const double *grid_in, uint32_t iteration, double *I_t,
                   double *var_t, double *bins_out, double *grid_out) {
    if (!P || !grid_in || !I_t || !var_t) return fail(MCUBES_E_ARG, "NULL argument");
    const int nb = P->nb;
    for (int j = 0; j < P->dim; ++j) {
        const double *e = grid_in + (size_t)j * (nb + 1);
        if (e[0] != 0.0 || e[nb] != 1.0)
            return fail(MCUBES_E_ARG, "grid row %d does not run from 0 to 1", j);
        for (int i = 0; i < nb; ++i)
            if (!isfinite(e[i + 1]) || !(e[i + 1] >= e[i]))
                return fail(MCUBES_E_ARG, "grid row %d is not nondecreasing at edge %d", j, i + 1);
    }
    const int64_t ng = (int64_t)P->dim * (nb + 1), nbn = (int64_t)P->dim * nb;
    const int64_t need = 2 * ng + nbn + 2 * (int64_t)P->blocks + 2;
    hipError_t e = hipSuccess;
    if (!P->ws) {
        e = hipMalloc(&P->ws, (size_t)need * sizeof(double));
        if (e != hipSuccess) {
            P->ws = nullptr;
            return fail(MCUBES_E_ALLOC, "hipMalloc: %s", hipGetErrorString(e));
        }
        P->ws_len = need;
    }
    double *g_in = P->ws, *g_new = P->ws + ng, *bins = P->ws + 2 * ng;
    double *partials = bins + nbn, *est = partials + 2 * (int64_t)P->blocks;
    hipStream_t s = as_stream(P->stream);
    e = hipMemcpyAsync(g_in, grid_in, (size_t)ng * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync grid");
    e = launch_fill(bins, nbn, 0.0, s);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    int rc = mcubes_vsample(P, iteration, g_in, bins, partials, P->stream);
    if (rc != MCUBES_OK) return rc;
    rc = mcubes_reduce(P, partials, est, P->stream);
    if (rc != MCUBES_OK) return rc;
    if (grid_out) {
        rc = mcubes_refine(P, g_in, bins, g_new, P->stream);
        if (rc != MCUBES_OK) return rc;
    }
    double h_est[2];
    e = hipMemcpyAsync(h_est, est, sizeof h_est, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the estimate");
    if (!isfinite(h_est[0]) || !isfinite(h_est[1]))
        return fail(MCUBES_E_NONFINITE, "iteration %u produced a non-finite estimate", iteration);
    if (bins_out)
        e = hipMemcpyAsync(bins_out, bins, (size_t)nbn * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && grid_out)
        e = hipMemcpyAsync(grid_out, g_new, (size_t)ng * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the bins and grid");
    *I_t = h_est[0];
    *var_t = h_est[1];
    return MCUBES_OK;
}

int mcubes_microbench(int kind, int family, const double *params, int dim,
                      const double *d_points, int64_t npts, int64_t calls_per_thread, int blocks,
                      int block, double *d_out, void *stream) {
    if (kind < MCUBES_MB_INTEGRAND || kind > MCUBES_MB_POW32)
        return fail(MCUBES_E_ARG, "unknown microbenchmark kind %d", kind);
    if (calls_per_thread < 0) return fail(MCUBES_E_ARG, "calls_per_thread must be >= 0");
    if (blocks < 1 || block < 64 || block > 256 || block % 64 != 0)
        return fail(MCUBES_E_ARG, "blocks >= 1 and block in {64, 128, 192, 256} required");
    if (!d_out) return fail(MCUBES_E_ARG, "d_out is NULL");
    VsArgs A;
    memset(&A, 0, sizeof A);
    if (kind == MCUBES_MB_INTEGRAND || kind == MCUBES_MB_PHILOX) {
        if (dim < 1 || dim > MCUBES_MAX_DIM)
            return fail(MCUBES_E_ARG, "dim must be in [1, %d], got %d", MCUBES_MAX_DIM, dim);
    }
    if (kind == MCUBES_MB_INTEGRAND) {
        const int rc = validate_params(family, params, dim);
        if (rc != MCUBES_OK) return rc;
        if (!d_points || npts < 1) return fail(MCUBES_E_ARG, "d_points with npts >= 1 required");
        fold_params(family, params, dim, A);
    }
    const hipError_t e = launch_microbench(kind, family, dim, A, d_points, npts, calls_per_thread,
                                           blocks, block, d_out, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "microbenchmark launch");
}

int mcubes_integrate_noalloc(int family, const double *params, int dim, int64_t ncall,
                             int itmax, double rel_tol, uint64_t seed,
                             const mcubes_options *opt_in, mcubes_result *out, double *grid_out,
                             double *trace) {
    if (!out) return fail(MCUBES_E_ARG, "out is NULL");
    if (itmax < 1 || itmax > MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "itmax must be in [1, %d]", MCUBES_MAX_ITERATIONS);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(MCUBES_E_ARG, "rel_tol must be finite and >= 0");
    mcubes_plan P;  // built in place: no workspace, nothing to free
    int rc = plan_init(family, params, dim, ncall, seed, opt_in, &P);
    if (rc != MCUBES_OK) return rc;
    const int64_t need = integrate_buffer_len(P);
    if (need > MCUBES_NOALLOC_SCRATCH)
        return fail(MCUBES_E_ARG,
                    "this problem needs %lld doubles of scratch (dim %d, %d bins, %d blocks); "
                    "mcubes_integrate_noalloc holds %d",
                    (long long)need, P.dim, P.nb, P.blocks, MCUBES_NOALLOC_SCRATCH);
    double *buf = nullptr;
    rc = noalloc_scratch(&buf);
    if (rc != MCUBES_OK) return rc;
    return integrate_run(P, buf, itmax, rel_tol, false, out, grid_out, trace);
}

int mcubes_integrate(int family, const double *params, int dim, int64_t ncall, int itmax,
                     double rel_tol, uint64_t seed, const mcubes_options *opt_in,
                     mcubes_result *out, double *grid_out, double *trace) {
    if (!out) return fail(MCUBES_E_ARG, "out is NULL");
    if (itmax < 1 || itmax > MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "itmax must be in [1, %d]", MCUBES_MAX_ITERATIONS);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(MCUBES_E_ARG, "rel_tol must be finite and >= 0");
    mcubes_plan *P = nullptr;
    int rc = mcubes_plan_create(family, params, dim, ncall, seed, opt_in, &P);
    if (rc != MCUBES_OK) return rc;
    double *buf = nullptr;
    const hipError_t e = hipMalloc(&buf, (size_t)integrate_buffer_len(*P) * sizeof(double));
    if (e != hipSuccess) {
        mcubes_plan_destroy(P);
        return fail(MCUBES_E_ALLOC, "hipMalloc: %s", hipGetErrorString(e));
    }
    rc = integrate_run(*P, buf, itmax, rel_tol, true, out, grid_out, trace);
    (void)hipFree(buf);
    mcubes_plan_destroy(P);
    return rc;
}

}  // extern "C"
