/*
 * mcubes_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, single-threaded FP64 reference of the m-Cubes integrator:
 * the per-iteration sampling kernel of Alg. 2 ("mcubes-kernel", §3.2 of the
 * paper), the VEGAS grid refinement it feeds and the combination of the
 * iteration estimates.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * Everything is written for a reader holding the paper: loops run in the
 * order the method states them (cube, then sample, then axis), there is no
 * blocking or reordering, and every cross-cube sum is a Neumaier compensated
 * sum in cube order so that the reference is as close to the exact sum as
 * FP64 allows.
 *
 * Readings of points the paper leaves open (all of them are listed, with
 * reasons, in the design notes of the repository):
 *   - stratification: g = largest integer with g^d <= floor(ncall/2),
 *     m = g^d cubes, p = max(2, floor(ncall/m)) samples per cube (§3.2 says
 *     only that a 2-point MC runs in each cube and about ncall samples are
 *     drawn);
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     counter = (cube id, stream id, sample*ceil(d/4) + block, iteration),
 *     key = (low 32 bits of the seed, high 32 bits); word l of block b gives
 *     axis 4b+l as u = (r + 1/2) 2^-32 (the paper uses an unspecified
 *     "custom" generator, §4.2);
 *   - bin contribution of a sample on every axis = w^2 with w = f(x) J(y)
 *     (Alg. 2 adds the square of the sample estimate; the refinement is
 *     invariant to the constant factor 1/N);
 *   - per-cube variance = unbiased sample variance, from sums shifted by the
 *     first sample of the cube (Alg. 2 "UpdateVariance");
 *   - refinement and combination follow Lepage's VEGAS (cited by the paper
 *     but not described there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mcubes_oracle.h"

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of the Philox S-P network on a 128-bit counter  */
/* with a 64-bit key (Salmon et al., SC'11).  Each round multiplies words 0  */
/* and 2 by the two round multipliers, and builds the next counter from the  */
/* high/low halves of the products, xored with words 1 and 3 and the round   */
/* key.  The key is advanced by the two Weyl constants between rounds.       */
/* ------------------------------------------------------------------------ */
void mco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u; /* Weyl constant: golden ratio */
            k1 += 0xBB67AE85u; /* Weyl constant: sqrt(3) - 1 */
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* A 32-bit word r becomes the midpoint of the r-th of 2^32 equal cells of
 * (0,1): u = (r + 1/2) 2^-32, exact in FP64 and strictly inside (0,1). */
double mco_uniform(uint32_t r)
{
    return fma((double)r, 0x1p-32, 0x1p-33);
}

/* ------------------------------------------------------------------------ */
/* Stratification plan (§3.2: m sub-cubes, a 2-point MC in each, about     */
/* ncall samples in total).                                                  */
/* ------------------------------------------------------------------------ */

/* b^e, or cap+1 as soon as the power exceeds cap (no overflow). */
static int64_t pow_capped(int64_t b, int e, int64_t cap)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) {
        if (r > cap / b) return cap + 1;
        r *= b;
    }
    return r;
}

int mco_plan(int dim, int64_t ncall, int64_t out[4])
{
    if (dim < 1 || dim > MCO_MAX_DIM || ncall < 2) return -1;
    int64_t half = ncall / 2;
    int64_t g = (int64_t)floor(pow((double)half, 1.0 / (double)dim));
    if (g < 1) g = 1;
    while (g > 1 && pow_capped(g, dim, half) > half) --g;
    while (pow_capped(g + 1, dim, half) <= half) ++g;
    if (g > MCO_MAX_SIDE) g = MCO_MAX_SIDE;
    int64_t m = pow_capped(g, dim, half);
    int64_t p = ncall / m;
    if (p < 2) p = 2;
    out[0] = g;
    out[1] = m;
    out[2] = p;
    out[3] = m * p;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Integrand families (§5, eqs. 1-6 and the addition integrand of §5.3),     */
/* in the parameterised Genz form: params = [a_0..a_{d-1}, u_0..u_{d-1}].    */
/* ------------------------------------------------------------------------ */
double mco_integrand(int family, int dim, const double *params, const double *x)
{
    const double *a = params;
    const double *u = params + dim;
    switch (family) {
    case MCO_OSCILLATORY: { /* cos(2 pi u_0 + sum a_i x_i)           eq. 1 */
        double arg = (2.0 * M_PI) * u[0];
        for (int i = 0; i < dim; ++i) arg = fma(a[i], x[i], arg);
        return cos(arg);
    }
    case MCO_PRODUCT_PEAK: { /* prod (a_i^-2 + (x_i - u_i)^2)^-1      eq. 2 */
        double den = 1.0;
        for (int i = 0; i < dim; ++i) {
            double q = 1.0 / (a[i] * a[i]);
            double t = x[i] - u[i];
            den = den * fma(t, t, q);
        }
        return 1.0 / den;
    }
    case MCO_CORNER_PEAK: { /* (1 + sum a_i x_i)^-(d+1)               eq. 3 */
        double s = 1.0;
        for (int i = 0; i < dim; ++i) s = fma(a[i], x[i], s);
        double pw = s;
        for (int k = 0; k < dim; ++k) pw = pw * s;
        return 1.0 / pw;
    }
    case MCO_GAUSSIAN: { /* exp(-sum a_i^2 (x_i - u_i)^2)             eq. 4 */
        double s = 0.0;
        for (int i = 0; i < dim; ++i) {
            double t = x[i] - u[i];
            s = fma(a[i] * a[i], t * t, s);
        }
        return exp(-s);
    }
    case MCO_C0: { /* exp(-sum a_i |x_i - u_i|)                        eq. 5 */
        double s = 0.0;
        for (int i = 0; i < dim; ++i) s = fma(a[i], fabs(x[i] - u[i]), s);
        return exp(-s);
    }
    case MCO_DISCONTINUOUS: { /* exp(sum a_i x_i) if x_i < u_i for all i  eq. 6 */
        double s = 0.0;
        int inside = 1;
        for (int i = 0; i < dim; ++i) {
            if (!(x[i] < u[i])) inside = 0;
            s = fma(a[i], x[i], s);
        }
        return inside ? exp(s) : 0.0;
    }
    case MCO_ADDITION: { /* sum x_i                                     §5.3 */
        double s = 0.0;
        for (int i = 0; i < dim; ++i) s = s + x[i];
        return s;
    }
    case MCO_MIXTURE: {
        /* Equal mixture of two Gaussians N(m_k 1, S), k = 1, 2, with the
         * equicorrelated covariance S = s^2 [(1 - r) I + r 1 1^T]
         * (a_0 = s, a_1 = r, u_0 = m_1, u_1 = m_2; not one of the paper's
         * integrands).  S has eigenvalue s^2 (1 - r + d r) along 1 and
         * s^2 (1 - r) across it, so
         *   y^T S^-1 y = (|y|^2 - r/(1 - r + d r) (sum y)^2) / (s^2 (1 - r)),
         *   det S = s^(2d) (1 - r)^(d-1) (1 - r + d r). */
        const double s = a[0], r = a[1];
        const double lam = 1.0 - r + (double)dim * r;
        const double c1 = r / lam;
        const double c2 = 1.0 / (2.0 * s * s * (1.0 - r));
        const double norm = 0.5 / (pow(2.0 * M_PI, 0.5 * (double)dim) * pow(s, (double)dim) *
                                   pow(1.0 - r, 0.5 * (double)(dim - 1)) * sqrt(lam));
        double f = 0.0;
        for (int k = 0; k < 2; ++k) {
            double S1 = 0.0, S2 = 0.0;
            for (int i = 0; i < dim; ++i) {
                double t = x[i] - u[k];
                S1 = S1 + t;
                S2 = fma(t, t, S2);
            }
            f = f + exp(-(c2 * (S2 - c1 * S1 * S1)));
        }
        return norm * f;
    }
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* The separable importance map (§3.2: a step-wise density approximating the */
/* integrand).  Axis j has nb bins with edges E_j[0]=0 < ... < E_j[nb]=1;    */
/* each bin holds probability 1/nb.  A point is given by its position in    */
/* bin units z = y nb (y in (0,1)^d) and mapped bin-wise linearly:          */
/* i = floor(z) (clamped to nb-1), x = E_i + W_i (z - i), W_i = E_{i+1} -   */
/* E_i; the Jacobian is prod_j nb W_{i_j}, evaluated as fl(nb^d) * (W_{i_0} */
/* W_{i_1} ...), nb^d by repeated multiplication.                           */
/* ------------------------------------------------------------------------ */
double mco_map(int dim, int nb, const double *grid, const double *z, double *x, int *bin)
{
    double nbd = (double)nb;
    for (int j = 1; j < dim; ++j) nbd = nbd * (double)nb;
    double prod = 1.0;
    for (int j = 0; j < dim; ++j) {
        const double *E = grid + (size_t)j * (size_t)(nb + 1);
        int i = (int)z[j];
        if (i > nb - 1) i = nb - 1;
        double phi = z[j] - (double)i;
        double W = E[i + 1] - E[i];
        x[j] = fma(W, phi, E[i]);
        prod = prod * W;
        bin[j] = i;
    }
    return nbd * prod;
}

/* ------------------------------------------------------------------------ */
/* Neumaier compensated summation.                                           */
/* ------------------------------------------------------------------------ */
static void neumaier_add(double *sum, double *comp, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v))
        *comp += (*sum - t) + v;
    else
        *comp += (v - t) + *sum;
    *sum = t;
}

/* ------------------------------------------------------------------------ */
/* One iteration of Alg. 2 over the cube ids [c_begin, c_end).               */
/*   sums[0] = sum over those cubes of S_c = sum_k w_ck                      */
/*   sums[1] = sum over those cubes of the unbiased in-cube variance of w    */
/*   bins[j*nb + i] = sum of w^2 over the samples that used bin i on axis j  */
/* Cube c has base-g digits c_j = floor(c / g^j) mod g; sample k of cube c   */
/* draws y_j = (c_j + u_j) / g, i.e. z_j = y_j nb = (c_j + u_j) nb / g in     */
/* bin units, evaluated as (c_j + u_j) * fl(nb / g) (c_j + u_j is exact).    */
/* ------------------------------------------------------------------------ */
int mco_sample_range(int family, int dim, const double *params, int nb,
                     int64_t g, int64_t m, int64_t p, uint64_t seed, uint32_t stream,
                     uint32_t iteration, const double *grid,
                     int64_t c_begin, int64_t c_end, double sums[2], double *bins)
{
    if (dim < 1 || dim > MCO_MAX_DIM || nb < 2 || nb > MCO_MAX_BINS) return -1;
    if (c_begin < 0 || c_end > m || c_begin > c_end || p < 2) return -1;
    const int nblk = (dim + 3) / 4;
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    const double nb_over_g = (double)nb / (double)g;

    double *bin_comp = (double *)calloc((size_t)dim * (size_t)nb, sizeof(double));
    if (!bin_comp) return -2;
    for (int k = 0; k < dim * nb; ++k) bins[k] = 0.0;
    double s_sum = 0.0, s_comp = 0.0, v_sum = 0.0, v_comp = 0.0;

    for (int64_t c = c_begin; c < c_end; ++c) {
        int64_t digit[MCO_MAX_DIM];
        int64_t rest = c;
        for (int j = 0; j < dim; ++j) {
            digit[j] = rest % g;
            rest = rest / g;
        }
        double S = 0.0, D1 = 0.0, D2 = 0.0, w0 = 0.0;
        for (int64_t k = 0; k < p; ++k) {
            uint32_t r[4 * 3];
            for (int b = 0; b < nblk; ++b) {
                uint32_t ctr[4] = {(uint32_t)c, stream, (uint32_t)(k * nblk + b), iteration};
                mco_philox4x32_10(ctr, key, r + 4 * b);
            }
            double z[MCO_MAX_DIM], x[MCO_MAX_DIM];
            int bin[MCO_MAX_DIM];
            for (int j = 0; j < dim; ++j) z[j] = ((double)digit[j] + mco_uniform(r[j])) * nb_over_g;
            double J = mco_map(dim, nb, grid, z, x, bin);
            double f = mco_integrand(family, dim, params, x);
            double w = f * J;
            S = S + w;
            if (k == 0) w0 = w;
            double dlt = w - w0;
            D1 = D1 + dlt;
            D2 = D2 + dlt * dlt;
            double w2 = w * w;
            for (int j = 0; j < dim; ++j)
                neumaier_add(&bins[j * nb + bin[j]], &bin_comp[j * nb + bin[j]], w2);
        }
        double var = (D2 - D1 * D1 / (double)p) / (double)(p - 1);
        neumaier_add(&s_sum, &s_comp, S);
        neumaier_add(&v_sum, &v_comp, var);
    }
    sums[0] = s_sum + s_comp;
    sums[1] = v_sum + v_comp;
    for (int k = 0; k < dim * nb; ++k) bins[k] += bin_comp[k];
    free(bin_comp);
    return 0;
}

/* Iteration estimates from the cube sums: I_t = sum S / N and
 * var_t = sum var_c / (p m^2)  (each cube has volume 1/m in y-space and its
 * mean of p samples has variance var_c / p). */
void mco_estimates(int64_t m, int64_t p, const double sums[2], double est[2])
{
    double n = (double)m * (double)p;
    est[0] = sums[0] / n;
    est[1] = sums[1] / ((double)p * (double)m * (double)m);
}

int mco_iteration(int family, int dim, const double *params, int nb, int64_t ncall,
                  uint64_t seed, uint32_t stream, uint32_t iteration, const double *grid,
                  double est[2], double *bins)
{
    int64_t plan[4];
    if (mco_plan(dim, ncall, plan) != 0) return -1;
    double sums[2];
    int rc = mco_sample_range(family, dim, params, nb, plan[0], plan[1], plan[2], seed, stream,
                              iteration, grid, 0, plan[1], sums, bins);
    if (rc != 0) return rc;
    mco_estimates(plan[1], plan[2], sums, est);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Grid refinement (Lepage's VEGAS rebinning; the paper only says that the   */
/* step function is approximated progressively and that Alg. 2 outputs the  */
/* bin contributions).  Per axis:                                            */
/*   1. smooth the contributions d_i with their neighbours (1/2 at the ends, */
/*      1/3 inside);                                                          */
/*   2. if their sum S is 0 keep the axis unchanged;                          */
/*   3. damp: rho_i = s_i / S, r_i = ((rho_i - 1) / ln rho_i)^alpha, with    */
/*      r_i = 0 for s_i = 0 and r_i = 1 for rho_i = 1 (the limit);            */
/*   4. place the nb-1 inner edges so that every new bin holds the same      */
/*      share T = sum r / nb of the damped weight, the weight being spread   */
/*      uniformly inside each old bin.                                        */
/* ------------------------------------------------------------------------ */
int mco_refine(int dim, int nb, double alpha, const double *grid, const double *bins, double *out)
{
    if (dim < 1 || dim > MCO_MAX_DIM || nb < 2 || nb > MCO_MAX_BINS) return -1;
    double s[MCO_MAX_BINS], r[MCO_MAX_BINS], R[MCO_MAX_BINS + 1];
    for (int j = 0; j < dim; ++j) {
        const double *E = grid + (size_t)j * (size_t)(nb + 1);
        const double *dj = bins + (size_t)j * (size_t)nb;
        double *En = out + (size_t)j * (size_t)(nb + 1);

        s[0] = (dj[0] + dj[1]) / 2.0;
        for (int i = 1; i < nb - 1; ++i) s[i] = (dj[i - 1] + dj[i] + dj[i + 1]) / 3.0;
        s[nb - 1] = (dj[nb - 2] + dj[nb - 1]) / 2.0;

        double S = 0.0;
        for (int i = 0; i < nb; ++i) S = S + s[i];
        if (!(S > 0.0)) {
            for (int i = 0; i <= nb; ++i) En[i] = E[i];
            continue;
        }
        for (int i = 0; i < nb; ++i) {
            double rho = s[i] / S;
            if (s[i] == 0.0)
                r[i] = 0.0;
            else if (rho == 1.0)
                r[i] = 1.0;
            else
                r[i] = pow((rho - 1.0) / log(rho), alpha);
        }
        R[0] = 0.0;
        for (int i = 0; i < nb; ++i) R[i + 1] = R[i] + r[i];
        double T = R[nb] / (double)nb;

        En[0] = 0.0;
        En[nb] = 1.0;
        int i = 0;
        for (int k = 1; k < nb; ++k) {
            double target = (double)k * T;
            while (i < nb - 1 && R[i + 1] < target) ++i;
            double W = E[i + 1] - E[i];
            double frac = (target - R[i]) / r[i];
            if (frac > 1.0) frac = 1.0;
            double e = E[i] + frac * W;
            En[k] = (e < E[i + 1]) ? e : E[i + 1];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Combination of the iteration estimates t = skip..T-1 (Lepage: inverse-    */
/* variance weighting; the paper only says the error comes from the          */
/* standard deviation of the MC estimate, §3.2).                             */
/*   Ibar = sum(I_t / v_t) / sum(1 / v_t), sigma = (sum 1/v_t)^(-1/2),        */
/*   chi2/dof = sum (I_t - Ibar)^2 / v_t / (n - 1)   (0 when n = 1).         */
/* An iteration with v_t = 0 is exact: the latest one gives Ibar, sigma = 0. */
/* out = [Ibar, sigma, chi2/dof]; returns the degrees of freedom n - 1.      */
/* ------------------------------------------------------------------------ */
int mco_combine(int T, const double *I, const double *var, int skip, double out[3])
{
    int n = T - skip;
    if (n < 1) {
        out[0] = 0.0;
        out[1] = INFINITY;
        out[2] = 0.0;
        return 0;
    }
    double sw = 0.0, swi = 0.0;
    int exact = -1;
    for (int t = skip; t < T; ++t) {
        if (var[t] == 0.0) {
            exact = t;
        } else {
            sw = sw + 1.0 / var[t];
            swi = swi + I[t] / var[t];
        }
    }
    if (exact >= 0) {
        out[0] = I[exact];
        out[1] = 0.0;
        out[2] = 0.0;
        return n - 1;
    }
    double Ibar = swi / sw;
    double chi2 = 0.0;
    for (int t = skip; t < T; ++t) {
        double dv = I[t] - Ibar;
        chi2 = chi2 + dv * dv / var[t];
    }
    out[0] = Ibar;
    out[1] = 1.0 / sqrt(sw);
    out[2] = (n > 1) ? chi2 / (double)(n - 1) : 0.0;
    return n - 1;
}

/* ------------------------------------------------------------------------ */
/* The whole integrator: uniform start grid E_j[i] = i/nb; per iteration     */
/* t: sample with the grid, record (I_t, v_t), refine while t < adapt_iters, */
/* combine, stop once sigma <= rel_tol |Ibar|.                               */
/*   res  = [Ibar, sigma, chi2/dof]                                          */
/*   info = [iterations done, dof, g, m, p, N, converged]                    */
/*   grid_out (dim*(nb+1)) = grid after the last refinement; trace_I and     */
/*   trace_var (itmax entries, may be NULL) = the per-iteration estimates.   */
/* ------------------------------------------------------------------------ */
int mco_integrate(int family, int dim, const double *params, int64_t ncall, int itmax,
                  double rel_tol, uint64_t seed, uint32_t stream, int nb, double alpha,
                  int adapt_iters, int skip, double res[3], int64_t info[7], double *grid_out,
                  double *trace_I, double *trace_var)
{
    int64_t plan[4];
    if (mco_plan(dim, ncall, plan) != 0 || itmax < 1 || nb < 2 || nb > MCO_MAX_BINS) return -1;
    size_t ne = (size_t)dim * (size_t)(nb + 1);
    double *grid = (double *)malloc(ne * sizeof(double));
    double *next = (double *)malloc(ne * sizeof(double));
    double *bins = (double *)malloc((size_t)dim * (size_t)nb * sizeof(double));
    double *It = (double *)malloc((size_t)itmax * sizeof(double));
    double *Vt = (double *)malloc((size_t)itmax * sizeof(double));
    if (!grid || !next || !bins || !It || !Vt) {
        free(grid); free(next); free(bins); free(It); free(Vt);
        return -2;
    }
    for (int j = 0; j < dim; ++j)
        for (int i = 0; i <= nb; ++i) grid[j * (nb + 1) + i] = (double)i / (double)nb;

    int converged = 0, done = 0, dof = 0;
    double comb[3] = {0.0, INFINITY, 0.0};
    int rc = 0;
    for (int t = 0; t < itmax; ++t) {
        double sums[2], est[2];
        rc = mco_sample_range(family, dim, params, nb, plan[0], plan[1], plan[2], seed, stream,
                              (uint32_t)t, grid, 0, plan[1], sums, bins);
        if (rc != 0) break;
        mco_estimates(plan[1], plan[2], sums, est);
        It[t] = est[0];
        Vt[t] = est[1];
        if (trace_I) trace_I[t] = est[0];
        if (trace_var) trace_var[t] = est[1];
        done = t + 1;
        if (!isfinite(est[0]) || !isfinite(est[1])) {
            rc = -3;
            break;
        }
        if (t < adapt_iters) {
            mco_refine(dim, nb, alpha, grid, bins, next);
            double *tmp = grid;
            grid = next;
            next = tmp;
        }
        dof = mco_combine(done, It, Vt, skip, comb);
        if (done > skip && comb[1] <= rel_tol * fabs(comb[0])) {
            converged = 1;
            break;
        }
    }
    res[0] = comb[0];
    res[1] = comb[1];
    res[2] = comb[2];
    info[0] = done;
    info[1] = dof;
    info[2] = plan[0];
    info[3] = plan[1];
    info[4] = plan[2];
    info[5] = plan[3];
    info[6] = converged;
    if (grid_out) memcpy(grid_out, grid, ne * sizeof(double));
    free(grid); free(next); free(bins); free(It); free(Vt);
    return rc;
}
