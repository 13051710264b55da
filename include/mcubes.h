/*
 * mcubes.h -- C interface of the MI355X (gfx950) m-Cubes integrator.
 *
 * m-Cubes (§3.2 of "Porting numerical integration codes from CUDA to oneAPI:
 * a case study", Sakiotis et al. 2023) is a VEGAS-style Monte Carlo
 * integrator over (0,1)^d.  Each iteration runs the sampling kernel of Alg. 2
 * ("V-Sample" here): the unit cube of y-space is split into m = g^d equal
 * sub-cubes, p samples are drawn in every sub-cube, each sample is mapped to
 * x through a separable step-function importance grid with nb bins per axis,
 * the integrand is evaluated, per-cube means and variances are reduced into
 * the iteration estimate (I_t, var_t), and every sample adds w^2 (w = f(x)
 * times the map's Jacobian) to the bin it used on each axis.  The bin sums
 * drive the refinement of the grid for the next iteration; the iteration
 * estimates are combined by inverse-variance weighting.
 *
 * Conventions shared by every entry point
 *   - Return value: an mcubes_status.  Negative values are errors; the
 *     outputs are then left untouched (for asynchronous entry points: no work
 *     was enqueued).  mcubes_last_error() gives a message for the calling
 *     thread's last error.
 *   - Integrand parameters: params = [a_0..a_{d-1}, u_0..u_{d-1}] (host
 *     memory, 2*dim doubles, copied at plan creation; may be NULL for
 *     MCUBES_ADDITION).  All must be finite; MCUBES_PRODUCT_PEAK needs a_i != 0.
 *   - Grid layout: dim rows of nbins+1 edges, row-major FP64;
 *     E_j[0] = 0 < ... < E_j[nbins] = 1.  Bin layout: dim rows of nbins FP64.
 *   - "d_" arguments are device pointers (HBM, e.g. torch tensors) owned by
 *     the caller; "stream" is a hipStream_t passed as void* (NULL = the null
 *     stream).  Device entry points only enqueue work and return.
 *   - Random numbers: Philox4x32-10 keyed by the 64-bit seed, with counter
 *     (cube id, stream id, sample * ceil(d/4) + block, iteration), so the
 *     samples, and therefore the results, do not depend on launch geometry.
 *   - Limits: 1 <= dim <= MCUBES_MAX_DIM, 2 <= nbins <= MCUBES_MAX_BINS,
 *     ncall >= 2, number of cubes m < 2^32, strata per axis g <=
 *     MCUBES_MAX_SIDE.
 *   - Threading: a plan may be used from one host thread / one stream at a
 *     time.  Calls on different plans are independent.
 */
#ifndef MCUBES_H
#define MCUBES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCUBES_MAX_DIM 10
#define MCUBES_MAX_BINS 500
/* Largest number of strata per axis, g (so that c_j + u, with c_j < g and u
 * carrying 32 random bits, is exact in FP64; matters only for dim = 1). */
#define MCUBES_MAX_SIDE 1048576
/* The learned proposal: dimension and number of parameters (see below). */
#define MCUBES_FLOW_DIM 6
#define MCUBES_FLOW_PARAMS 67212
/* Combined-state buffer: 8 scalars followed by (I_t, var_t) per iteration. */
#define MCUBES_STATE_HEADER 8
#define MCUBES_MAX_ITERATIONS 1024
#define MCUBES_STATE_LEN (MCUBES_STATE_HEADER + 2 * MCUBES_MAX_ITERATIONS)

typedef enum {
    MCUBES_OK = 0,
    MCUBES_NOT_CONVERGED = 1, /* valid result; error > rel_tol * |estimate| after itmax */
    MCUBES_E_ARG = -1,        /* invalid argument (message via mcubes_last_error) */
    MCUBES_E_INTEGRAND = -2,  /* unknown integrand family or invalid parameters */
    MCUBES_E_NONFINITE = -3,  /* an iteration estimate was NaN or infinite */
    MCUBES_E_DEVICE = -4,     /* no usable gfx950 device or a HIP runtime error */
    MCUBES_E_ALLOC = -5       /* host or device allocation failed */
} mcubes_status;

/* Integrand families (the paper's benchmark integrands of eqs. 1-6, §5, in
 * the parameterised form, plus the addition integrand of §5.3):
 *   OSCILLATORY    cos(2 pi u_0 + sum a_i x_i)                      eq. 1
 *   PRODUCT_PEAK   prod (a_i^-2 + (x_i - u_i)^2)^-1                 eq. 2
 *   CORNER_PEAK    (1 + sum a_i x_i)^-(d+1)                         eq. 3
 *   GAUSSIAN       exp(-sum a_i^2 (x_i - u_i)^2)                    eq. 4
 *   C0             exp(-sum a_i |x_i - u_i|)                        eq. 5
 *   DISCONTINUOUS  exp(sum a_i x_i) if x_i < u_i for all i, else 0  eq. 6
 *   ADDITION       sum x_i                                          §5.3
 *   MIXTURE        equal mixture of N(u_0 1, S) and N(u_1 1, S),
 *                  S = a_0^2 [(1 - a_1) I + a_1 1 1^T] (a_0 > 0,
 *                  0 <= a_1 < 1, dim >= 2; the other a_i, u_i unused):
 *                  a non-separable integrand (not in the paper) for the
 *                  learned proposal                                        */
typedef enum {
    MCUBES_OSCILLATORY = 0,
    MCUBES_PRODUCT_PEAK = 1,
    MCUBES_CORNER_PEAK = 2,
    MCUBES_GAUSSIAN = 3,
    MCUBES_C0 = 4,
    MCUBES_DISCONTINUOUS = 5,
    MCUBES_ADDITION = 6,
    MCUBES_MIXTURE = 7
} mcubes_family;

/* Arithmetic of the map and the integrand inside V-Sample.  MCUBES_FP32 draws
 * the same samples into the same bins (bin coordinates stay FP64) but maps
 * and evaluates the integrand in FP32 from an FP32 copy of the grid; the
 * Jacobian, weights, cube statistics, bin sums, reductions, refinement and
 * combination stay FP64. */
typedef enum { MCUBES_FP64 = 0, MCUBES_FP32 = 1, MCUBES_BF16 = 2 } mcubes_precision;

typedef struct {
    int32_t nbins;       /* bins per axis, 2..500; default 500 (Alg. 2 uses 500) */
    int32_t adapt_iters; /* refine the grid after iterations t < adapt_iters; <0 = always (default) */
    int32_t skip;        /* leading iterations left out of the combination; default 0 */
    int32_t block_size;  /* V-Sample threads per block (64..1024, multiple of 64); 0 = library choice */
    int32_t blocks;      /* V-Sample blocks; 0 = enough to fill every compute unit */
    uint32_t stream_id;  /* second Philox counter word; default 0 */
    int32_t precision;   /* mcubes_precision; default MCUBES_FP64 */
    double alpha;        /* refinement damping exponent; default 1.5 */
    void *stream;        /* hipStream_t for mcubes_integrate; NULL = null stream */
} mcubes_options;

typedef struct {
    double estimate;   /* combined integral estimate */
    double error;      /* its standard deviation */
    double chi2_dof;   /* chi^2 per degree of freedom of the combined iterations */
    int32_t iterations; /* iterations run */
    int32_t dof;       /* degrees of freedom (combined iterations - 1) */
    int32_t converged; /* 1 if error <= rel_tol * |estimate| */
    int32_t status;    /* same as the return value */
    int64_t cube_side; /* g: cubes per axis */
    int64_t ncubes;    /* m = g^dim */
    int64_t samples_per_cube; /* p */
    int64_t samples_per_iter; /* N = m p */
    double kernel_ms;  /* total V-Sample kernel time (HIP events) */
} mcubes_result;

typedef struct mcubes_plan mcubes_plan;

typedef struct {
    int32_t family, dim, nbins, block_size, blocks;
    int32_t lds_bytes;     /* LDS per V-Sample block (static) */
    int32_t precision;     /* mcubes_precision */
    int64_t cube_side, ncubes, samples_per_cube, samples_per_iter;
    int64_t grid_len;      /* dim * (nbins + 1) */
    int64_t bins_len;      /* dim * nbins */
    int64_t partials_len;  /* 2 * blocks: per-block (sum S_c, sum var_c) */
    int64_t state_len;     /* MCUBES_STATE_LEN */
} mcubes_plan_info;

/* Fill *opt with the defaults listed above (host only; no error).  Passage:
 * none -- the defaults are the readings of §3.2 and Alg. 2 (500 bins) and
 * of the VEGAS refinement §3.2 relies on (damping alpha = 1.5). */
void mcubes_default_options(mcubes_options *opt);

/* Message describing the calling thread's last error ("" if none).  The
 * string is owned by the library and valid until the thread's next call.
 * Passage: none (a convention of this interface). */
const char *mcubes_last_error(void);

/* Stratification.  Passage: §3.2 (m-Cubes splits the domain into m equal
 * sub-cubes and runs a 2-point Monte Carlo in each, about ncall samples in
 * all).  Reading: g = largest integer with g^dim <= floor(ncall/2), at
 * most MCUBES_MAX_SIDE, m = g^dim, p = max(2, floor(ncall/m)), N = m p.  out (host, 4 int64,
 * caller-owned) = [g, m, p, N].  Host only.  Errors: MCUBES_E_ARG (out NULL,
 * dim outside [1, MCUBES_MAX_DIM], ncall < 2, m >= 2^32); out untouched. */
int mcubes_plan_sizes(int dim, int64_t ncall, int64_t out[4]);

/* Whole integrator.  Passage: §3.2 (m-Cubes: iterations of stratified,
 * importance-sampled Monte Carlo whose separable grid is adapted after each
 * iteration, until the error estimate -- the standard deviation of the
 * estimate -- reaches a user-specified threshold) with Alg. 2 as the
 * iteration; the grid refinement and the combination are the VEGAS ones
 * (Lepage 1978) that §3.2 builds on.  Uniform start grid, then per
 * iteration t = 0..itmax-1 V-Sample -> estimate -> combine -> refine (while
 * t < adapt_iters), stopping after the first iteration whose combined
 * error <= rel_tol * |estimate|.  params and every output are host memory
 * owned by the caller; opt may be NULL (defaults).
 * out (host) receives the result.  grid_out (host, dim*(nbins+1), may be
 * NULL) receives the grid after the last refinement.  trace (host, 2*itmax
 * doubles, may be NULL) receives (I_t, var_t) per iteration run.
 * Allocates its device buffers itself and synchronises once per iteration.
 * Returns MCUBES_OK, MCUBES_NOT_CONVERGED or an error. */
int mcubes_integrate(int family, const double *params, int dim, int64_t ncall, int itmax,
                     double rel_tol, uint64_t seed, const mcubes_options *opt,
                     mcubes_result *out, double *grid_out, double *trace);

/* mcubes_integrate for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as mcubes_integrate
 * (kernel_ms is 0: no timing events), but every device buffer lives in one
 * library-owned array of MCUBES_NOALLOC_SCRATCH doubles per GPU, created with
 * the library and held until the process ends; no hipMalloc, hipFree or
 * allocating library call is made.  The scratch must hold 2 dim (nbins + 1)
 * + dim nbins + 2 blocks + 2 + MCUBES_STATE_LEN doubles; a larger problem
 * returns MCUBES_E_ARG before any device work.  All calls on one GPU share
 * its array, and every call initialises what it reads: calls that overlap
 * on one GPU (several host threads, or several streams) race and must be
 * serialised by the caller. */
#define MCUBES_NOALLOC_SCRATCH 32768
int mcubes_integrate_noalloc(int family, const double *params, int dim, int64_t ncall,
                             int itmax, double rel_tol, uint64_t seed, const mcubes_options *opt,
                             mcubes_result *out, double *grid_out, double *trace);

/* Plan: validated problem, stratification (§3.2, as mcubes_plan_sizes) and
 * V-Sample launch geometry for the entry points below.  params: host,
 * copied.  opt may be NULL (defaults).  *plan receives a plan owned by the
 * caller, freed with mcubes_plan_destroy (which also frees the workspace
 * mcubes_iterate allocates on its first call; the other entry points use
 * caller-owned device buffers, so a plan otherwise holds no device memory).
 * Errors: MCUBES_E_ARG (sizes, options), MCUBES_E_INTEGRAND (family or
 * parameters), MCUBES_E_DEVICE (no usable device); *plan untouched.
 * Passage: Alg. 2's inputs (f, d, the sub-cube count m, the samples per
 * sub-cube p, the grid B). */
int mcubes_plan_create(int family, const double *params, int dim, int64_t ncall, uint64_t seed,
                       const mcubes_options *opt, mcubes_plan **plan);
int mcubes_plan_get_info(const mcubes_plan *plan, mcubes_plan_info *info);
void mcubes_plan_destroy(mcubes_plan *plan);

/* d_grid (device, grid_len doubles, caller-owned) <- the uniform grid
 * E_j[i] = i/nbins, the importance grid of the first iteration (§3.2: the
 * step-function density starts flat).  Enqueued on `stream`. */
int mcubes_init_grid(const mcubes_plan *plan, double *d_grid, void *stream);

/* d[0..n) <- value: device buffer, caller-owned; a fill kernel (no memset
 * node, safe under graph capture).  Passage: none (a utility: the bins and
 * the combined state must start at zero).  MCUBES_E_ARG if n < 0 or d is
 * NULL with n > 0. */
int mcubes_fill(double *d, int64_t n, double value, void *stream);

/* V-Sample.  Passage: Alg. 2 (§3.2): per sub-cube, p samples drawn, mapped
 * through the grid (Get-Bin-ID), the integrand evaluated, the cube's mean
 * and variance accumulated (UpdateVariance), the squared sample estimates
 * added to the bins C they fell in, and the results reduced into the
 * iteration's integral and variance.  All pointers are caller-owned device
 * buffers; enqueued on `stream`.  For iteration `iteration` with grid
 * d_grid:
 *   d_bins[j*nbins + i] += sum of w^2 over the samples that used bin i on axis j;
 *   d_partials[2b], d_partials[2b+1] <- block b's sum of cube sums S_c = sum_k w_ck
 *   and of unbiased in-cube variances var_c.  Sizes from mcubes_plan_get_info.
 * d_bins may be NULL: the bin sums are then not formed (for iterations whose
 * grid is not refined afterwards); the partials are the same. */
int mcubes_vsample(const mcubes_plan *plan, uint32_t iteration, const double *d_grid,
                   double *d_bins, double *d_partials, void *stream);

/* Fixed-order reduction of the block partials (device, partials_len), the
 * Reduce step closing Alg. 2: d_est (device, 2 doubles) <- [I_t = sum S_c / N,
 * var_t = sum var_c / (p m^2)].  Enqueued on `stream`. */
int mcubes_reduce(const mcubes_plan *plan, const double *d_partials, double *d_est, void *stream);

/* Combination of iterations.  Passage: §3.2 (the error estimate is the
 * standard deviation of the combined estimate); the weighting is the
 * inverse-variance one of VEGAS (Lepage 1978), which §3.2 cites -- the
 * paper itself leaves it unstated.  Device buffers, caller-owned; enqueued
 * on `stream`.  Records (I_t, var_t) = d_est as iteration `iteration` in
 * d_state and recombines iterations skip..iteration:
 *   d_state[0] = estimate, [1] = error, [2] = chi2/dof, [3] = dof,
 *   [4] = iterations recorded, [5] = converged (error <= rel_tol |estimate|),
 *   [6] = 1 if any recorded estimate was not finite,
 *   [8 + 2t], [9 + 2t] = (I_t, var_t).
 * iteration must be < MCUBES_MAX_ITERATIONS; d_state must hold MCUBES_STATE_LEN
 * doubles and be zeroed before iteration 0. */
int mcubes_combine(const mcubes_plan *plan, uint32_t iteration, const double *d_est,
                   double *d_state, double rel_tol, void *stream);

/* Grid refinement.  Passage: §3.2 (the step-function importance density is
 * adapted between iterations from the bin contributions C of Alg. 2); the
 * rule is VEGAS's (Lepage 1978), which the paper does not spell out: per
 * axis, smooth the bin sums over neighbours, damp them as
 * ((r - 1)/ln r)^alpha, and re-divide into bins of equal damped weight.
 * Device buffers, caller-owned; d_grid_out may not alias d_grid
 * (MCUBES_E_ARG).  Enqueued on `stream`. */
int mcubes_refine(const mcubes_plan *plan, const double *d_grid, const double *d_bins,
                  double *d_grid_out, void *stream);

/* One whole iteration (Alg. 2 and the §3.2 loop body) on caller-owned
 * device buffers: zero d_bins, V-Sample, reduce, combine, then refine
 * d_grid into d_grid_out.  When iteration >= adapt_iters the grid is copied
 * unchanged and V-Sample runs without bin sums (d_bins is left untouched).
 * Enqueued on `stream`. */
int mcubes_iteration(const mcubes_plan *plan, uint32_t iteration, const double *d_grid,
                     double *d_grid_out, double *d_bins, double *d_partials, double *d_est,
                     double *d_state, double rel_tol, void *stream);

/* One iteration on host buffers: Alg. 2's inputs and outputs (§3.2) -- the
 * grid B in, the iteration estimate r = (I_t, var_t) and the bin sums C out
 * -- plus the refined grid.
 *   grid_in (host, grid_len doubles): the grid to sample with; every row
 *     must run from 0 to 1, finite and nondecreasing (MCUBES_E_ARG).
 *   *I_t, *var_t (host): the iteration estimate and its variance, as
 *     mcubes_reduce gives them.
 *   bins_out (host, bins_len doubles, may be NULL): the bin sums C.
 *   grid_out (host, grid_len doubles, may be NULL): the grid refined from
 *     those bins (as mcubes_refine), whatever adapt_iters says.
 * The samples are those of iteration `iteration` of mcubes_integrate with
 * the same plan.  Runs on the plan's options stream and returns when done.
 * The first call allocates a device workspace owned by the plan (freed by
 * mcubes_plan_destroy); later calls allocate nothing.  Errors leave every
 * output untouched: MCUBES_E_ARG, MCUBES_E_NONFINITE (I_t or var_t not
 * finite), MCUBES_E_ALLOC, MCUBES_E_DEVICE.  The plan is used from one host
 * thread at a time. */
int mcubes_iterate(mcubes_plan *plan, const double *grid_in, uint32_t iteration, double *I_t,
                   double *var_t, double *bins_out, double *grid_out);

/* Microbenchmarks that attribute V-Sample's time (the analogue of the
 * integrand-invocation experiment of §5.1 of the paper).  Each of the
 * blocks*block threads (block in {64, 128, 192, 256}) runs calls_per_thread
 * steps and writes one accumulated value to d_out[thread]:
 *   MCUBES_MB_INTEGRAND  f(x) of `family` with `params` (as for plans) on
 *                        points read cyclically from d_points (npts rows of
 *                        dim FP64 coordinates, device memory);
 *   MCUBES_MB_PHILOX     the ceil(dim/4) Philox4x32-10 blocks of one sample;
 *   MCUBES_MB_EXP64..POW32  one libm call (exp, cos, pow^1.5; FP64 / FP32).
 * d_out must hold blocks*block doubles. */
typedef enum {
    MCUBES_MB_INTEGRAND = 0,
    MCUBES_MB_PHILOX = 1,
    MCUBES_MB_EXP64 = 2,
    MCUBES_MB_COS64 = 3,
    MCUBES_MB_POW64 = 4,
    MCUBES_MB_EXP32 = 5,
    MCUBES_MB_COS32 = 6,
    MCUBES_MB_POW32 = 7
} mcubes_microbench_kind;

int mcubes_microbench(int kind, int family, const double *params, int dim,
                      const double *d_points, int64_t npts, int64_t calls_per_thread, int blocks,
                      int block, double *d_out, void *stream);

/* ------------------------------------------------------------------------
 * Batched form: many integrands of mixed family, dimension and sample budget
 * integrated together (the paper runs one integrand per launch; this form
 * keeps the whole GPU busy with small and mid-sized problems).
 *
 * Every integrand i runs m-Cubes exactly as mcubes_integrate would with the
 * same nbins, alpha, adapt_iters and skip and with Philox stream id
 * opt->stream_id + i: the samples are the same, so the results agree with
 * the single-integrand path up to the rounding of the sums.  Per iteration
 * the library launches one V-Sample kernel per (family, dim, p == 2) class,
 * whose samples are cut into equal contiguous shares and the shares at
 * integrand boundaries into tiles, one workgroup per tile, then
 * per-integrand reduction, combination, refinement (in place) and an
 * iteration counter, all reading the iteration number and the per-integrand
 * "done" flags from device memory; the sequence is captured once in a HIP
 * graph and replayed.  An integrand that converges (or produces a
 * non-finite estimate) is marked done on the device and no longer sampled
 * (its tiles return at once); the plan stays fixed for the whole call.
 *
 * The batch owns its device memory (grids, bins, states: about
 * 8 * (2 * sum dim_i * (nbins + 1) + n * MCUBES_STATE_LEN) bytes plus the
 * tile lists) and one internal HIP stream; mcubes_batch_integrate and
 * mcubes_batch_autotune order themselves after earlier work on opt->stream
 * and return when done.  opt->precision is MCUBES_FP64 or MCUBES_FP32 (the
 * FP32 map and integrand of mcubes_integrate, for every integrand of the
 * batch; its results then agree with the single-integrand FP32 path up to
 * the rounding of the sums).  opt->block_size, when not 0, fixes the block
 * size of every class; opt->blocks is ignored.
 * A batch may be used from one host thread at a time.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t family;  /* mcubes_family */
    int32_t dim;     /* 1..MCUBES_MAX_DIM */
    int64_t ncall;   /* sample budget per iteration (planned as in mcubes_plan_sizes) */
    double params[2 * MCUBES_MAX_DIM]; /* a_0..a_{dim-1}, u_0..u_{dim-1}; the rest unused */
} mcubes_batch_item;

typedef struct mcubes_batch mcubes_batch;

typedef struct {
    int32_t items;          /* integrands in the batch */
    int32_t classes;        /* (family, dim, p == 2) classes in the current plan */
    int32_t tiles;          /* work tiles in the current plan */
    int32_t launches;       /* kernel launches per iteration */
    int32_t nbins;
    int32_t tuned;          /* 1 after mcubes_batch_autotune */
    int32_t streams;        /* streams the class launches are spread over */
    int32_t precision;      /* mcubes_precision of every integrand's map and integrand */
    int64_t grids_len;      /* sum over i of dim_i * (nbins + 1): packed grids, item order */
    int64_t samples_per_iter; /* sum of N_i over the integrands still running */
    int64_t device_bytes;   /* device memory held by the batch */
    /* the last mcubes_batch_integrate call: */
    int32_t last_iterations;  /* iterations run (the most any integrand ran) */
    int32_t last_replans;     /* always 0: the work is not re-split during a call */
    int64_t last_samples;     /* samples evaluated, all integrands */
    double last_ms;           /* wall time of its iteration loop (HIP events) */
} mcubes_batch_info;

typedef struct {
    int32_t family, dim, p2; /* p2 = 1 when the class's integrands have p = 2 */
    int32_t items;           /* integrands of the class in the current plan */
    int32_t block_size;      /* V-Sample threads per workgroup */
    int32_t shares;          /* equal shares the class's samples are split into */
    int32_t tiles;           /* workgroups per launch: shares cut at integrand boundaries */
    int32_t lds_bytes;
    int64_t samples;         /* samples per iteration */
    double tuned_ms;         /* V-Sample time of the chosen geometry, measured by the
                                autotuner (0 if not tuned) */
    double default_ms;       /* ... and of the library's default geometry */
} mcubes_batch_class;

/* Validates every item (errors name the item), plans it, allocates the
 * batch's device memory and splits the work with the default geometry.
 * 1 <= n <= 65536.  Returns MCUBES_OK or an error. */
int mcubes_batch_create(const mcubes_batch_item *items, int n, uint64_t seed,
                        const mcubes_options *opt, mcubes_batch **batch);
void mcubes_batch_destroy(mcubes_batch *batch);
int mcubes_batch_get_info(const mcubes_batch *batch, mcubes_batch_info *info);
/* Class k (0 <= k < info.classes) of the current plan. */
int mcubes_batch_get_class(const mcubes_batch *batch, int k, mcubes_batch_class *out);

/* Sets the V-Sample geometry of class k: block_size a multiple of 64 up to
 * the kernel's limit, shares >= 1 (capped at the class's cube count and at
 * 2^20).  The samples do not depend on the geometry; only the order of the
 * partial sums does. */
int mcubes_batch_configure_class(mcubes_batch *batch, int k, int block_size, int shares);

/* Spreads the per-class V-Sample launches over `streams` (1..4) concurrent
 * HIP streams (branches of the captured graph), longest classes first onto
 * the least loaded stream, so that one class's tail overlaps the next
 * class's work.  Default 4. */
int mcubes_batch_set_streams(mcubes_batch *batch, int streams);

/* Autotuner: for every class times the V-Sample kernel on the batch's current
 * grids at the default geometry and over candidate block sizes (256, 512,
 * 768, 1024 within the kernel's limit) and share counts (2, 4, 8 or 16 times
 * the workgroups resident at once, or fewer shares with at least 4, 16 or 64
 * cubes per thread for small classes), and keeps the fastest.  The grids
 * and the results of later calls are unaffected (up to the order of the
 * partial sums); the combined states of the last mcubes_batch_integrate are
 * cleared.  Then times all classes together on 1 to 4 streams and keeps the
 * fastest (see mcubes_batch_set_streams).  Takes 3 launches per candidate. */
int mcubes_batch_autotune(mcubes_batch *batch);

/* One iteration of every integrand from caller-given grids, for lock-step
 * checking against a reference and for warm starts: V-Sample with Philox
 * iteration word `iteration`, the reduction, and the refinement of every
 * grid (as mcubes_iteration, without the combination).
 *   grids (host, grids_len doubles, packed in item order): in, the grids to
 *     sample with (each row monotone from 0 to 1, checked); out, the refined
 *     grids.
 *   est (host, 2 n doubles): out, (I_t, var_t) per integrand.
 * Afterwards the combined states of mcubes_batch_integrate are undefined
 * (the next mcubes_batch_integrate starts afresh). */
int mcubes_batch_step(mcubes_batch *batch, uint32_t iteration, double *grids, double *est);

/* Runs every integrand from a uniform grid: at most itmax iterations, each
 * integrand stopping after the first iteration whose combined error is
 * <= rel_tol * |estimate|.  use_graph = 1 replays the captured graph, 0
 * launches the same kernels one by one (same results).
 *   results (host, n entries): per-integrand result; status MCUBES_OK,
 *     MCUBES_NOT_CONVERGED or MCUBES_E_NONFINITE; kernel_ms is 0.
 *   grids_out (host, grids_len doubles, may be NULL): final grids, packed
 *     in item order.
 *   traces (host, n * 2 * itmax doubles, may be NULL): row i holds
 *     (I_t, var_t) of integrand i for the iterations it ran, zeros after.
 * Returns MCUBES_OK if every integrand converged, MCUBES_NOT_CONVERGED if
 * some did not, MCUBES_E_NONFINITE if some produced a non-finite estimate,
 * or an error (then results are not written). */
int mcubes_batch_integrate(mcubes_batch *batch, int itmax, double rel_tol, int use_graph,
                           mcubes_result *results, double *grids_out, double *traces);

/* ------------------------------------------------------------------------
 * Learned proposal (not part of the paper): a normalizing flow used in place
 * of the separable VEGAS map for non-separable integrands, after the design
 * of "Neural Importance Sampling" (Müller et al., 2019).  Over (0,1)^6 the
 * flow maps x to z through four coupling layers; layer l keeps coordinates
 * A_l = {0,1,2}, {3,4,5}, {0,2,4}, {1,3,5} and maps every other coordinate
 * through the CDF of a piecewise-linear density with 16 bins whose widths
 * (softmax) and 17 vertex heights (exp, scaled to integrate to 1) are the
 * 99 outputs of a network of u_{A_l}: one-blob encoding (32 Gaussian bumps
 * of width 1/32 per input), two hidden layers of 64 ReLU units.  q(x) is the
 * product of the spline densities met on the way x -> z; sampling draws z
 * and inverts the layers.  Parameters (MCUBES_FLOW_PARAMS values) per layer,
 * row-major with the input index first: W1[96][64], b1[64], W2[64][64],
 * b2[64], W3[64][99], b3[99].
 *
 * The flow keeps FP32 master parameters, Adam moments and a gradient on the
 * device.  Precision MCUBES_FP32 evaluates it in FP32, one thread per
 * sample; MCUBES_BF16 (sampling only) runs the network's matrix products on
 * the BF16 matrix cores with FP32 accumulation.
 * ---------------------------------------------------------------------- */
typedef struct mcubes_flow mcubes_flow;

/* theta: host, MCUBES_FLOW_PARAMS values (copied).  Adam state zeroed. */
int mcubes_flow_create(const double *theta, mcubes_flow **flow);
void mcubes_flow_destroy(mcubes_flow *flow);
/* theta (host) <- the current FP32 parameters. */
int mcubes_flow_get_params(const mcubes_flow *flow, double *theta);
/* Replaces the parameters and zeroes the Adam state. */
int mcubes_flow_set_params(mcubes_flow *flow, const double *theta);

/* d_x (n x 6, device) -> d_z (n x 6) and d_logq (n): the density direction. */
int mcubes_flow_density(mcubes_flow *flow, int precision, const double *d_x, int64_t n,
                        double *d_z, double *d_logq, void *stream);
/* d_z (n x 6, device, in (0,1)) -> d_x (n x 6) and d_logq = log q(x). */
int mcubes_flow_sample(mcubes_flow *flow, int precision, const double *d_z, int64_t n,
                       double *d_x, double *d_logq, void *stream);

/* Weighted negative log-likelihood of n samples (x_i, w_i >= 0, sum > 0):
 * *d_loss (device, 1 double) += -sum w_i log q(x_i) / sum w_i (zero it
 * first); the gradient with respect to the parameters is kept in the flow
 * (for mcubes_flow_adam_step) and copied to d_grad (device,
 * MCUBES_FLOW_PARAMS doubles) when that is not NULL.
 * precision: MCUBES_FP32 runs every product of the forward and backward
 * pass in FP32 on the vector units; MCUBES_BF16 runs the nine products per
 * layer on the matrix cores (BF16 weights and product inputs, FP32
 * accumulation; splines FP32), which makes the gradient approximate.  The
 * weight gradients (sums over the samples) are FP32 in both.  Enqueued on
 * `stream`; nothing is read back. */
int mcubes_flow_loss_grad(mcubes_flow *flow, int precision, const double *d_x, const double *d_w,
                          int64_t n, double *d_grad, double *d_loss, void *stream);
/* One Adam step (bias-corrected; the flow counts the steps) with the kept gradient. */
int mcubes_flow_adam_step(mcubes_flow *flow, double lr, double beta1, double beta2, double eps,
                          void *stream);
/* epochs passes of mini-batches of `batch` consecutive samples (the last one
 * shorter), one Adam step each (beta1 0.9, beta2 0.999, eps 1e-8).
 * losses (host, epochs doubles, may be NULL): mean batch loss per epoch.
 * precision as for mcubes_flow_loss_grad. */
int mcubes_flow_train(mcubes_flow *flow, int precision, const double *d_x, const double *d_w,
                      int64_t n, int epochs, int64_t batch, double lr, double *losses,
                      void *stream);

/* Shuffles n training rows (x: n x 6, w: n; device) into (d_x_out, d_w_out):
 * output row j is input row (a j) mod n, a = floor(n (sqrt(5) - 1)/2)
 * with its lowest bit set, stepped by 2 (mod n) until coprime to n.  A permutation whose
 * consecutive outputs lie about 0.618 n apart, so every mini-batch of
 * mcubes_flow_train (consecutive rows) draws evenly from the whole input,
 * e.g. from data gathered in blocks.  n in [0, 2^32); the outputs must not
 * overlap the inputs or each other (MCUBES_E_ARG).  Stream-ordered. */
int mcubes_flow_shuffle(const double *d_x, const double *d_w, int64_t n, double *d_x_out,
                        double *d_w_out, void *stream);

/* The samples and weights w = f J of work items [w_begin, w_begin + count)
 * of iteration `iteration` of the plain method on d_grid: work item w is
 * cube (w mult) mod m (V-Sample's visiting order, which spreads a prefix
 * over the whole domain; mult is coprime to the cube side), and its p
 * samples are exactly those V-Sample draws there.  d_x: count p x dim,
 * d_w: count p (device); rows in work-item order. */
int mcubes_vsample_dump(const mcubes_plan *plan, uint32_t iteration, const double *d_grid,
                        int64_t w_begin, int64_t count, double *d_x, double *d_w, void *stream);

/* n unstratified samples of the flow with weights w = f(x)/q(x) for the
 * plan's integrand (dim 6): sample i draws z from Philox counter
 * (i, stream_id | 0xC0000000, block, iteration) under the plan's seed and
 * maps it through the flow in `precision` (MCUBES_FP32, or MCUBES_BF16 on
 * the matrix cores).  d_x: n x 6, d_w: n (device).  Training data for
 * refining the flow on its own samples. */
int mcubes_flow_draw(mcubes_flow *flow, int precision, const mcubes_plan *plan,
                     uint32_t iteration, int64_t n, double *d_x, double *d_w, void *stream);

/* One m-Cubes iteration with the flow as the map (plan of dim 6, p >= 2):
 * cube c's sample k draws u from Philox with the plan's seed and stream word
 * stream_id | 0x80000000, z_j = (c_j + u_j)/g, x = flow sample of z and
 * w = f(x)/q(x).  d_est (device, 2 doubles) <- (I_t, var_t) as mcubes_reduce
 * gives them. */
int mcubes_flow_vsample(mcubes_flow *flow, int precision, const mcubes_plan *plan,
                        uint32_t iteration, double *d_est, void *stream);

/* Combination of flow-mapped iterations 0..iteration with the same flow and
 * plan (an extension: the paper combines only map-adapting iterations).
 * They are independent estimates of one distribution, so they are averaged
 * with equal weights, and the error is the standard deviation of that mean
 * (the error model of §3.2), estimated both from the iterations' own
 * variances and from the scatter of their estimates, the larger reported:
 *   Ibar = sum(I_t) / T,  T = iteration + 1,
 *   sigma = max(sqrt(sum var_t) / T, sqrt(sum (I_t - Ibar)^2 / (T (T - 1))))
 *     (the second term only for T >= 2),
 *   chi2/dof = sum over var_t > 0 of (I_t - Ibar)^2 / var_t, over T - 1,
 *   converged (d_state[5]) = T >= min_iters and sigma <= rel_tol |Ibar|.
 * (Inverse-variance weighting, mcubes_combine, is biased low here: with a
 * long-tailed weight distribution an iteration that caught a large weight
 * also has a large variance estimate and is weighted down; for the same
 * reason an iteration's own variance is usually too small, while an
 * iteration that caught a large weight stands out in the scatter.)  d_est
 * and d_state as for mcubes_combine, same header layout (device,
 * caller-owned); d_state must start zeroed.  Stream-ordered; errors:
 * MCUBES_E_ARG (NULL pointer, iteration >= MCUBES_MAX_ITERATIONS, rel_tol
 * not finite or < 0, min_iters outside [1, MCUBES_MAX_ITERATIONS]),
 * MCUBES_E_DEVICE. */
int mcubes_flow_combine(uint32_t iteration, const double *d_est, double *d_state, double rel_tol,
                        int min_iters, void *stream);

/* Tail diagnostic of importance weights.  Each mcubes_flow_vsample call
 * histograms log2 of its weights w = f/q: MCUBES_WTAIL_BINS bins, bin b
 * holding 2^((b - 2048)/8) <= w < 2^((b - 2047)/8) (the first and last bins
 * also take everything below and above; w <= 0 is not counted).  The shape
 * is the Hill estimate of the generalised Pareto shape of the upper tail,
 * xi = mean of ln(w / u) over the k = min(N/5, 3 sqrt N) largest weights, u
 * the lower edge of the bin where they start (the within-bin position is
 * taken at the bin's middle: at most 0.04 off).  Reading, for a Pareto
 * tail of shape xi (moments of order below 1/xi exist):
 *   xi < 0.25  the weights have a finite fourth moment, so the estimated
 *              variance is itself reliable: the error bar can be trusted;
 *   0.25-0.5   finite variance, but the variance estimate has none of its
 *              own: it is usually too small (rare large weights missing);
 *   xi >= 0.5  the variance is infinite: the error bar means nothing.
 * A bounded but strongly peaked weight distribution (a proposal much flatter
 * than f) reads high as well: there too a handful of weights decides the
 * estimate.  Host only: *shape = NaN when fewer than 100 weights were
 * counted; tail_count (may be NULL) receives k. */
#define MCUBES_WTAIL_BINS 4096
int mcubes_weight_tail_shape(const uint32_t *hist, double *shape, int64_t *tail_count);
/* The same for the weights of the last mcubes_flow_vsample call on `flow`
 * (synchronises with that call's stream). */
int mcubes_flow_weight_tail(mcubes_flow *flow, double *shape, int64_t *tail_count);

/* The whole learned-proposal pipeline for one integrand of dim 6:
 *   1. warmup_iters plain m-Cubes iterations (grid refined every time);
 *   2. the samples and weights of train_items work items, an equal share
 *      from each of them (mcubes_vsample_dump with that iteration's grid),
 *      shuffled (mcubes_flow_shuffle), train the flow for `epochs` epochs.
 *      The early iterations' broad grids keep every peak of f in the data:
 *      on a multimodal integrand a separable map can settle on one peak
 *      within a few iterations;
 *   3. `rounds` times: round_samples samples of the flow itself with weights
 *      f/q (mcubes_flow_draw, in train_precision), together with the
 *      warm-up samples in the first anchor_rounds (shuffled into them), train it
 *      for round_epochs epochs.  The flow never draws where it has lost a
 *      peak of f; the warm-up samples there pull it back; then
 *      tail_rounds more such rounds with the weights raised to tail_power
 *      (> 1 stresses the samples the flow under-weights: between the
 *      Kullback-Leibler objective, power 1, and the variance, power 2) at
 *      learning rate tail_lr;
 *   4. flow-mapped iterations (mcubes_flow_vsample, in `precision`) combined
 *      with equal weights (mcubes_flow_combine) until, after at least
 *      min_iters of them, error <= rel_tol |estimate| and the weight tail
 *      allows trusting that error (below), or itmax of them.
 * Plain m-Cubes stays the judge: if the first flow iteration's variance is
 * not below the last plain iteration's, the flow is dropped and the
 * remaining iterations run plain (report->used_flow = 0).  The weight
 * histograms of the flow iterations are pooled; report->tail_shape is the
 * weight-tail shape of the pooled histogram (see mcubes_weight_tail_shape).
 * A flow result is reported converged only if that shape is below 0.25,
 * or below 0.5 with the iterations agreeing within their stated errors
 * (chi2/dof below its 99% point): at 0.5 and above the variance is
 * infinite, and from 0.25 the variance estimates are themselves
 * unreliable.  `flow` is trained
 * in place (start from an identity flow for a fresh run).  out receives the
 * combined result of the iterations that decide it (flow, or plain on
 * fallback).  Synchronous; allocates its buffers.
 * The flow's weights have a long tail where it is thinner than f (regions
 * of f that training has barely sampled); the tail rounds exist to lighten
 * it.  On the 6-D correlated mixture the defaults gave, at 2^26 samples per
 * iteration, a median error of 1.7e-5 over 120 seeds, 107 of them within
 * two stated errors and 118 within three (of the other two, one at 3.3 and
 * one at 8.0 that came back not converged, its weight-tail shape 0.52); at
 * 2^22, 36 of 40 runs within two and all 40 within three. */
typedef struct {
    int32_t warmup_iters;  /* default 8 */
    int32_t precision;     /* proposal iterations: MCUBES_BF16 (default) or MCUBES_FP32 */
    int64_t train_items;   /* default 2^20 over all warm-up iterations (each gives p samples) */
    int32_t epochs;        /* default 10 */
    int32_t rounds;        /* default 4 */
    int64_t round_samples; /* default 2^25 */
    int32_t round_epochs;  /* default 2 */
    int32_t tail_rounds;   /* default 4 */
    int64_t batch;         /* default 65536 */
    double lr;             /* default 4e-3 */
    double round_lr;       /* default 2e-3 */
    double tail_power;     /* default 1.75 */
    double tail_lr;        /* default 8e-4 */
    int32_t train_precision; /* training products: MCUBES_BF16 (default) or MCUBES_FP32 */
    int32_t anchor_rounds; /* default 2: how many of the first `rounds` also train on
                              the warm-up samples */
    int32_t min_iters;     /* default 4: flow iterations before a result may count as
                              converged (1..itmax) */
} mcubes_flow_options;

typedef struct {
    double warmup_ms, train_ms, flow_ms, total_ms; /* wall time of the phases (HIP events) */
    double plain_estimate, plain_error, plain_chi2_dof; /* combined warm-up iterations */
    double last_plain_var, first_flow_var; /* the judge's comparison */
    double final_loss;     /* mean batch loss of the last training epoch */
    int32_t flow_iterations, used_flow;
    double tail_shape;     /* weight-tail shape of the flow iterations' pooled weights
                              (NaN if none) */
} mcubes_flow_report;

void mcubes_default_flow_options(mcubes_flow_options *opt);
int mcubes_flow_integrate(mcubes_flow *flow, int family, const double *params, int64_t ncall,
                          int itmax, double rel_tol, uint64_t seed, const mcubes_options *opt,
                          const mcubes_flow_options *fopt, mcubes_result *out,
                          mcubes_flow_report *report);

#ifdef __cplusplus
}
#endif

#endif /* MCUBES_H */
