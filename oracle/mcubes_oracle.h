/*
 * mcubes_oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 * Declarations of the plain CPU reference of the m-Cubes integrator
 * (Alg. 2, §3.2 of the paper).  See mcubes_oracle.c for the definitions.
 */
#ifndef MCUBES_ORACLE_H
#define MCUBES_ORACLE_H

#include <stdint.h>

#define MCO_MAX_DIM 10
#define MCO_MAX_BINS 500
/* At most 2^20 strata per axis: then digit + u (u with 32 random bits below
 * 2^-32 ... 2^-33) is exact in FP64.  Only a 1-D plan reaches it. */
#define MCO_MAX_SIDE 1048576

enum {
    MCO_OSCILLATORY = 0,
    MCO_PRODUCT_PEAK = 1,
    MCO_CORNER_PEAK = 2,
    MCO_GAUSSIAN = 3,
    MCO_C0 = 4,
    MCO_DISCONTINUOUS = 5,
    MCO_ADDITION = 6,
    MCO_MIXTURE = 7
};

void mco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double mco_uniform(uint32_t r);
int mco_plan(int dim, int64_t ncall, int64_t out[4]);
double mco_integrand(int family, int dim, const double *params, const double *x);
double mco_map(int dim, int nb, const double *grid, const double *z, double *x, int *bin);
int mco_sample_range(int family, int dim, const double *params, int nb,
                     int64_t g, int64_t m, int64_t p, uint64_t seed, uint32_t stream,
                     uint32_t iteration, const double *grid,
                     int64_t c_begin, int64_t c_end, double sums[2], double *bins);
void mco_estimates(int64_t m, int64_t p, const double sums[2], double est[2]);
int mco_iteration(int family, int dim, const double *params, int nb, int64_t ncall,
                  uint64_t seed, uint32_t stream, uint32_t iteration, const double *grid,
                  double est[2], double *bins);
int mco_refine(int dim, int nb, double alpha, const double *grid, const double *bins, double *out);
int mco_combine(int T, const double *I, const double *var, int skip, double out[3]);
int mco_integrate(int family, int dim, const double *params, int64_t ncall, int itmax,
                  double rel_tol, uint64_t seed, uint32_t stream, int nb, double alpha,
                  int adapt_iters, int skip, double res[3], int64_t info[7], double *grid_out,
                  double *trace_I, double *trace_var);

/* The library's boundary calls, mirrored (mcubes_oracle_abi.c).  The records
 * have the field order and types of the library's option and result
 * records. */
typedef struct {
    int32_t nbins, adapt_iters, skip, block_size, blocks;
    uint32_t stream_id;
    int32_t precision;
    double alpha;
    void *stream;
} mco_options;

typedef struct {
    double estimate, error, chi2_dof;
    int32_t iterations, dof, converged, status;
    int64_t cube_side, ncubes, samples_per_cube, samples_per_iter;
    double kernel_ms;
} mco_result;

typedef struct mco_plan_s mco_plan_t;

int mcubes_oracle_integrate(int family, const double *params, int dim, int64_t ncall, int itmax,
                            double rel_tol, uint64_t seed, const mco_options *opt,
                            mco_result *out, double *grid_out, double *trace);
int mcubes_oracle_plan_create(int family, const double *params, int dim, int64_t ncall,
                              uint64_t seed, const mco_options *opt, mco_plan_t **plan);
void mcubes_oracle_plan_destroy(mco_plan_t *plan);
int mcubes_oracle_iterate(mco_plan_t *plan, const double *grid_in, uint32_t iteration, double *I_t,
                          double *var_t, double *bins_out, double *grid_out);

#endif
