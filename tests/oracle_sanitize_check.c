/* CPU driver of the oracle (test infrastructure), built by
 * tests/test_host_sanitizers.py together with the oracle's sources under
 * AddressSanitizer and UndefinedBehaviorSanitizer: every public function
 * runs at least once on small inputs, including the edge cases the tests use
 * (one cube, p > 2, 2 bins, 1-D and 10-D, a zero-weight axis, skip, the
 * mirrored boundary calls and the flow's training and sampling paths in both
 * precisions).  A sanitizer report aborts the run; otherwise it prints "ok"
 * and a checksum of the results. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "flow_oracle.h"
#include "mcubes_oracle.h"

static double checksum = 0.0;

static void add(double v) {
    if (isfinite(v)) checksum += v;
}

static void run_integrate(int family, int dim, int64_t ncall, int itmax, int nb, int adapt,
                          int skip) {
    double params[2 * MCO_MAX_DIM];
    for (int i = 0; i < dim; ++i) {
        params[i] = 2.0 + 0.5 * i;
        params[dim + i] = 0.3 + 0.04 * i;
    }
    double res[3];
    int64_t info[7];
    double *grid = calloc((size_t)dim * (nb + 1), sizeof(double));
    double *tI = calloc((size_t)itmax, sizeof(double)), *tV = calloc((size_t)itmax, sizeof(double));
    int rc = mco_integrate(family, dim, params, ncall, itmax, 1e-3, 7, 3, nb, 1.5, adapt, skip, res,
                           info, grid, tI, tV);
    if (rc < 0) {
        printf("mco_integrate rc %d\n", rc);
        exit(1);
    }
    add(res[0]);
    add(grid[dim * (nb + 1) / 2]);
    free(grid);
    free(tI);
    free(tV);
}

int main(void) {
    /* plans and single functions */
    int64_t sz[4];
    for (int d = 1; d <= MCO_MAX_DIM; ++d)
        for (int64_t n = 2; n < ((int64_t)1 << 40); n = n * 7 + 3)
            if (mco_plan(d, n, sz) == 0) add((double)sz[3]);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    mco_philox4x32_10(ctr, key, out);
    add(mco_uniform(out[0]));
    /* integrations: every family, edge sizes */
    for (int f = 0; f <= 6; ++f) run_integrate(f, 3, 2000, 4, 20, 4, 0);
    run_integrate(3, 1, 100, 3, 2, 3, 0);          /* 1-D, 2 bins */
    run_integrate(1, 10, 3000, 2, 500, 2, 1);      /* 10-D, 500 bins, skip */
    run_integrate(4, 2, 2, 3, 7, 1, 0);            /* one cube */
    run_integrate(2, 4, 50, 3, 9, 3, 0);           /* one cube, p > 2 */
    run_integrate(5, 5, 40000, 5, 50, 2, 2);       /* frozen grid after 2 */
    {   /* mixture */
        double mp[12] = {0.05, 0.9, 0, 0, 0, 0, 1.0 / 3, 2.0 / 3, 0, 0, 0, 0};
        double res[3], grid[6 * 31], tI[3], tV[3];
        int64_t info[7];
        mco_integrate(7, 6, mp, 5000, 3, 0.0, 1, 0, 30, 1.5, 3, 0, res, info, grid, tI, tV);
        add(res[0]);
    }
    /* refinement with a zero axis and a single non-empty bin */
    {
        double grid[2 * 6], bins[2 * 5] = {0}, o[2 * 6];
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i <= 5; ++i) grid[j * 6 + i] = i / 5.0;
        bins[5 + 2] = 3.0;
        mco_refine(2, 5, 1.5, grid, bins, o);
        add(o[8]);
        double I[3] = {1.0, 1.1, 0.9}, V[3] = {0.1, 0.2, 0.0}, c[3];
        mco_combine(3, I, V, 0, c);
        add(c[0]);
        mco_combine(3, I, V, 2, c);
        add(c[0]);
    }
    /* mirrored boundary calls */
    {
        mco_options opt;
        memset(&opt, 0, sizeof opt);
        opt.nbins = 40;
        opt.adapt_iters = -1;
        opt.alpha = 1.5;
        double params[6] = {5, 5, 5, 0.4, 0.5, 0.6}, grid[3 * 41], trace[2 * 4];
        mco_result r;
        mcubes_oracle_integrate(1, params, 3, 5000, 4, 0.0, 0, &opt, &r, grid, trace);
        add(r.estimate);
        mco_plan_t *P = NULL;
        if (mcubes_oracle_plan_create(1, params, 3, 5000, 0, &opt, &P) == 0) {
            double I, V, bins[3 * 40], g2[3 * 41];
            mcubes_oracle_iterate(P, grid, 1, &I, &V, bins, g2);
            add(I);
            mcubes_oracle_plan_destroy(P);
        }
    }
    /* the flow: density, sampling, loss gradient (both precisions), Adam,
     * flow-mapped iterations and the equal-weight combination */
    {
        const int np = mcf_param_count();
        double *theta = malloc((size_t)np * sizeof(double));
        double *grad = malloc((size_t)np * sizeof(double));
        double *gabs = malloc((size_t)np * sizeof(double));
        double *m = calloc((size_t)np, sizeof(double)), *v = calloc((size_t)np, sizeof(double));
        srand(3);
        for (int i = 0; i < np; ++i) theta[i] = 0.05 * ((double)rand() / RAND_MAX - 0.5);
        double xs[8 * MCF_D], ws[8];
        for (int s = 0; s < 8; ++s) {
            for (int j = 0; j < MCF_D; ++j) xs[s * MCF_D + j] = (s + 0.5 + 0.1 * j) / 9.0;
            ws[s] = 1.0 + s;
        }
        for (int bf = 0; bf < 2; ++bf) {
            double z[MCF_D], x[MCF_D], lq;
            mcf_density(theta, xs, bf, z, &lq);
            mcf_sample(theta, z, bf, x, &lq);
            add(x[0] + lq);
            add(mcf_loss_grad_ex(theta, 8, xs, ws, bf, grad, gabs));
            add(grad[np - 1]);
        }
        add(mcf_loss_grad(theta, 8, xs, ws, grad));
        mcf_adam(theta, m, v, grad, np, 1, 1e-3, 0.9, 0.999, 1e-8);
        double mp[12] = {0.05, 0.9, 0, 0, 0, 0, 1.0 / 3, 2.0 / 3, 0, 0, 0, 0}, sums[2];
        for (int bf = 0; bf < 2; ++bf) {
            mcf_proposal_range(theta, bf, 7, mp, 3, 729, 2, 5, 0x80000000u, 0, 0, 729, sums);
            add(sums[0]);
        }
        double I[4] = {1, 1.01, 0.99, 1.02}, V[4] = {1e-4, 2e-4, 1e-4, 3e-4}, c[3];
        mcf_combine_equal(4, I, V, c);
        add(c[0] + c[1]);
        double r[MCF_RAW], y, pdf, u;
        for (int k = 0; k < MCF_RAW; ++k) r[k] = 0.1 * k - 1.0;
        mcf_spline_forward(r, 0.3, &y, &pdf);
        mcf_spline_inverse(r, y, &u, &pdf);
        add(u);
        free(theta);
        free(grad);
        free(gabs);
        free(m);
        free(v);
    }
    printf("ok %.17g\n", checksum);
    return 0;
}
