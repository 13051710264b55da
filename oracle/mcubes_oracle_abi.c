/*
 * mcubes_oracle_abi.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * The boundary calls of the m-Cubes library, mirrored on the plain CPU
 * reference with the same argument lists, so that a test can call the HIP
 * library and the oracle through one signature table:
 *   mcubes_oracle_integrate      <-> mcubes_integrate      (§3.2: the
 *       iteration loop to a user threshold, the error from the standard
 *       deviation of the estimate)
 *   mcubes_oracle_plan_create / _plan_destroy / _iterate
 *                                <-> mcubes_plan_create / _destroy /
 *       mcubes_iterate (Alg. 2: one V-Sample over every sub-cube with a
 *       given grid -> the iteration estimate, its variance and the bin
 *       sums C; the refined grid from those bins)
 * The option and result records below are declared here, not shared with
 * the library: they follow the same field order and types, which is all a
 * C caller relies on.  Every result comes from the functions of
 * mcubes_oracle.c (plan, sample_range, estimates, refine, combine); this
 * file only validates arguments and moves numbers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mcubes_oracle.h"

enum { OK = 0, NOT_CONVERGED = 1, E_ARG = -1, E_INTEGRAND = -2, E_NONFINITE = -3, E_ALLOC = -5 };

static void default_options(mco_options *o)
{
    memset(o, 0, sizeof *o);
    o->nbins = 500;
    o->adapt_iters = -1;
    o->alpha = 1.5;
}

static int check_params(int family, const double *params, int dim)
{
    if (family < MCO_OSCILLATORY || family > MCO_MIXTURE) return E_INTEGRAND;
    if (family == MCO_ADDITION && !params) return OK;
    if (!params) return E_INTEGRAND;
    for (int i = 0; i < 2 * dim; ++i)
        if (!isfinite(params[i])) return E_INTEGRAND;
    if (family == MCO_PRODUCT_PEAK)
        for (int i = 0; i < dim; ++i)
            if (params[i] == 0.0) return E_INTEGRAND;
    if (family == MCO_MIXTURE &&
        (dim < 2 || !(params[0] > 0.0) || !(params[1] >= 0.0) || !(params[1] < 1.0)))
        return E_INTEGRAND;
    return OK;
}

static int check_options(const mco_options *o)
{
    if (o->nbins < 2 || o->nbins > MCO_MAX_BINS) return E_ARG;
    if (!(o->alpha >= 0.0) || !isfinite(o->alpha)) return E_ARG;
    if (o->skip < 0) return E_ARG;
    return OK;
}

/* every row from 0 to 1, finite and nondecreasing */
static int check_grid(int dim, int nb, const double *grid)
{
    for (int j = 0; j < dim; ++j) {
        const double *e = grid + (size_t)j * (nb + 1);
        if (e[0] != 0.0 || e[nb] != 1.0) return E_ARG;
        for (int i = 0; i < nb; ++i)
            if (!isfinite(e[i + 1]) || !(e[i + 1] >= e[i])) return E_ARG;
    }
    return OK;
}

int mcubes_oracle_integrate(int family, const double *params, int dim, int64_t ncall, int itmax,
                            double rel_tol, uint64_t seed, const mco_options *opt_in,
                            mco_result *out, double *grid_out, double *trace)
{
    mco_options opt;
    default_options(&opt);
    if (opt_in) opt = *opt_in;
    int64_t sz[4];
    if (!out || itmax < 1 || itmax > 1024 || !(rel_tol >= 0.0) || !isfinite(rel_tol)) return E_ARG;
    if (mco_plan(dim, ncall, sz) != 0 || check_options(&opt) != OK) return E_ARG;
    if (check_params(family, params, dim) != OK) return E_INTEGRAND;
    const int adapt = opt.adapt_iters < 0 ? itmax : opt.adapt_iters;
    double res[3];
    int64_t info[7];
    double *tI = (double *)malloc((size_t)itmax * sizeof(double));
    double *tV = (double *)malloc((size_t)itmax * sizeof(double));
    double *grid = (double *)malloc((size_t)dim * (size_t)(opt.nbins + 1) * sizeof(double));
    if (!tI || !tV || !grid) {
        free(tI); free(tV); free(grid);
        return E_ALLOC;
    }
    const int rc = mco_integrate(family, dim, params, ncall, itmax, rel_tol, seed, opt.stream_id,
                                 opt.nbins, opt.alpha, adapt, opt.skip, res, info, grid, tI, tV);
    if (rc != 0) {
        free(tI); free(tV); free(grid);
        return rc == -3 ? E_NONFINITE : (rc == -2 ? E_ALLOC : E_ARG);
    }
    const int done = (int)info[0];
    if (trace)
        for (int t = 0; t < done; ++t) {
            trace[2 * t] = tI[t];
            trace[2 * t + 1] = tV[t];
        }
    if (grid_out) memcpy(grid_out, grid, (size_t)dim * (size_t)(opt.nbins + 1) * sizeof(double));
    memset(out, 0, sizeof *out);
    out->estimate = res[0];
    out->error = res[1];
    out->chi2_dof = res[2];
    out->iterations = done;
    out->dof = (int32_t)info[1];
    out->converged = (int32_t)info[6];
    out->cube_side = info[2];
    out->ncubes = info[3];
    out->samples_per_cube = info[4];
    out->samples_per_iter = info[5];
    out->kernel_ms = 0.0;
    out->status = out->converged ? OK : NOT_CONVERGED;
    free(tI); free(tV); free(grid);
    return out->status;
}

struct mco_plan_s {
    int family, dim, nb;
    double alpha;
    uint64_t seed;
    uint32_t stream_id;
    int64_t g, m, p, n;
    double params[2 * MCO_MAX_DIM];
    int has_params;
};

int mcubes_oracle_plan_create(int family, const double *params, int dim, int64_t ncall,
                              uint64_t seed, const mco_options *opt_in, mco_plan_t **plan)
{
    mco_options opt;
    default_options(&opt);
    if (opt_in) opt = *opt_in;
    int64_t sz[4];
    if (!plan || mco_plan(dim, ncall, sz) != 0 || check_options(&opt) != OK) return E_ARG;
    if (check_params(family, params, dim) != OK) return E_INTEGRAND;
    mco_plan_t *P = (mco_plan_t *)calloc(1, sizeof *P);
    if (!P) return E_ALLOC;
    P->family = family;
    P->dim = dim;
    P->nb = opt.nbins;
    P->alpha = opt.alpha;
    P->seed = seed;
    P->stream_id = opt.stream_id;
    P->g = sz[0];
    P->m = sz[1];
    P->p = sz[2];
    P->n = sz[3];
    P->has_params = params != NULL;
    if (params) memcpy(P->params, params, (size_t)(2 * dim) * sizeof(double));
    *plan = P;
    return OK;
}

void mcubes_oracle_plan_destroy(mco_plan_t *plan) { free(plan); }

int mcubes_oracle_iterate(mco_plan_t *P, const double *grid_in, uint32_t iteration, double *I_t,
                          double *var_t, double *bins_out, double *grid_out)
{
    if (!P || !grid_in || !I_t || !var_t) return E_ARG;
    if (check_grid(P->dim, P->nb, grid_in) != OK) return E_ARG;
    const size_t nbn = (size_t)P->dim * (size_t)P->nb;
    double *bins = (double *)malloc(nbn * sizeof(double));
    if (!bins) return E_ALLOC;
    double sums[2], est[2];
    double zeros[2 * MCO_MAX_DIM] = {0};
    const int rc = mco_sample_range(P->family, P->dim, P->has_params ? P->params : zeros, P->nb,
                                    P->g, P->m, P->p, P->seed, P->stream_id, iteration, grid_in,
                                    0, P->m, sums, bins);
    if (rc != 0) {
        free(bins);
        return rc == -2 ? E_ALLOC : E_ARG;
    }
    mco_estimates(P->m, P->p, sums, est);
    if (!isfinite(est[0]) || !isfinite(est[1])) {
        free(bins);
        return E_NONFINITE;
    }
    *I_t = est[0];
    *var_t = est[1];
    if (bins_out) memcpy(bins_out, bins, nbn * sizeof(double));
    if (grid_out) mco_refine(P->dim, P->nb, P->alpha, grid_in, bins, grid_out);
    free(bins);
    return OK;
}
