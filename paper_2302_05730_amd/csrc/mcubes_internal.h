// Internal declarations shared by the HIP sources of libmcubes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_plan.h"
#include "mcubes.h"

namespace mcubes {

constexpr int kMaxDim = MCUBES_MAX_DIM;
constexpr int kMaxBins = MCUBES_MAX_BINS;
constexpr int kFamilies = 8;
constexpr int kMaxBlock = 1024;

// Uniform arguments of one V-Sample launch (kernel-argument segment, read
// through scalar loads).  Integrand coefficients are pre-folded per family:
//   oscillatory    ca = a,        phase = 2 pi u_0
//   product peak   ca = 1/(a a),  cu = u
//   corner peak    ca = a
//   Gaussian       ca = a a,      cu = u
//   C0             ca = a,        cu = u
//   discontinuous  ca = a,        cu = u
//   mixture        ca = m_1,      cu = m_2 (every axis), mix_* below
struct VsArgs {
    double ca[kMaxDim];
    double cu[kMaxDim];
    double phase;
    double mix_c1, mix_c2, mix_norm;  // mixture: r/(1-r+dr), 1/(2 s^2 (1-r)), normalisation / 2
    double zscale;      // fl(nb/g) * 2^-32: bin coordinate per unit of (c_j 2^32 + r + 1/2)
    double nbd;         // fl(nb^d) by repeated multiplication
    double inv_p;       // fl(1/p)
    double inv_pm1;     // fl(1/(p-1))
    uint32_t key0, key1;  // Philox key: low and high 32 bits of the seed
    uint32_t stream_id;
    uint32_t iteration;
    uint32_t g, m, p, nb;
    uint32_t mult;            // cube permutation: work item w -> cube (w * mult) mod m
    uint32_t step;            // (threads * mult) mod m
    uint32_t step_digit[kMaxDim];  // base-g digits of step
};

typedef hipError_t (*VsLaunchFn)(const VsArgs &args, const double *grid, double *bins,
                                 double *partials, int blocks, int block, hipStream_t stream);

// Batched form: one integrand of a batch (device-resident descriptor) and one
// tile of work (a range of permuted work items of one integrand).
struct BatchItem {
    VsArgs args;                         // folded problem (iteration is read elsewhere)
    uint32_t step_block;                 // (block * mult) mod m for the class kernel's block
    uint32_t step_digit_block[kMaxDim];  // its base-g digits
    int64_t grid_off, bins_off;          // offsets (doubles) into the packed grids / bins
    uint32_t part_begin, part_end;       // the item's partials (one per tile)
    int32_t dim, nb;
    double n_samples, var_denom;         // N = m p and p m^2
};


typedef hipError_t (*VsTilesLaunchFn)(const BatchItem *items, const BatchTile *tiles, int ntiles,
                                      const double *grids, double *bins, double *partials,
                                      const uint32_t *iter, const uint32_t *done, int block,
                                      hipStream_t stream);

// Eight variants per (family, dim): [fp32][nobins][p2] with fp32 = 1 for the
// FP32 map/integrand form, nobins = 1 when the bin sums are not wanted (no
// later refinement) and p2 = 1 for p = 2 (both samples of a cube in
// straight-line code).
struct VsKernel {
    VsLaunchFn launch[2][2][2];
    const void *func[2][2][2];  // kernel symbols, for occupancy queries and attributes
    VsTilesLaunchFn tiles_launch[2][2][2];  // batched form, [fp32][nobins][p2]
    const void *tiles_func[2][2][2];
};

// Per-family tables, index = dim (1..kMaxDim); defined in vsample_f<family>.hip.
const VsKernel *kVsOscillatory();
const VsKernel *kVsProductPeak();
const VsKernel *kVsCornerPeak();
const VsKernel *kVsGaussian();
const VsKernel *kVsC0();
const VsKernel *kVsDiscontinuous();
const VsKernel *kVsAddition();
const VsKernel *kVsMixture();

// Small kernels (support.hip).
hipError_t launch_fill(double *d, int64_t n, double value, hipStream_t stream);
hipError_t launch_init_grid(double *grid, int dim, int nb, hipStream_t stream);
hipError_t launch_reduce(const double *partials, int nparts, double n_samples, double var_denom,
                         double *est, hipStream_t stream);
hipError_t launch_combine(const double *est, double *state, uint32_t iteration, int skip,
                          double rel_tol, hipStream_t stream);
hipError_t launch_refine(const double *grid, const double *bins, double *grid_out, int dim, int nb,
                         double alpha, hipStream_t stream);
hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t stream);

// Batched support kernels (batch.hip).  done[i] != 0 marks integrand i as
// finished (converged or non-finite): it is no longer sampled or combined.
hipError_t launch_batch_reset(double *states, int64_t state_len, uint32_t *done, int n,
                              uint32_t *iter, hipStream_t stream);
hipError_t launch_batch_reduce(const BatchItem *items, int n, const double *partials,
                               const uint32_t *done, double *est, hipStream_t stream);
hipError_t launch_batch_combine(int n, const double *est, double *states, uint32_t *done,
                                uint32_t *active, const uint32_t *iter, int skip, double rel_tol,
                                hipStream_t stream);
hipError_t launch_batch_refine(const BatchItem *items, const uint2 *axes, int naxes,
                               double *grids, const double *bins, const double *states,
                               const uint32_t *iter, double alpha, bool all, hipStream_t stream);
hipError_t launch_batch_init_grids(const BatchItem *items, const uint2 *axes, int naxes,
                                   double *grids, hipStream_t stream);
hipError_t launch_batch_advance(uint32_t *iter, hipStream_t stream);

// Host helpers (mcubes_api.hip).  fail() records a message for
// mcubes_last_error() and returns `code`.
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
const VsKernel *family_table(int family);
int plan_sizes(int dim, int64_t ncall, int64_t out[4]);
int validate_params(int family, const double *params, int dim);
int check_sizes(int64_t m, int64_t p, int dim);
// Folded problem for V-Sample (step and step digits left zero).
void make_args(int family, const double *params, int dim, int64_t g, int64_t m, int64_t p, int nb,
               uint64_t seed, uint32_t stream_id, VsArgs &A);
// step = (threads * mult) mod m and its base-g digits: the advance of a work
// item when `threads` threads stride over the work items.
void set_step(VsArgs &A, int dim, uint64_t threads);
hipStream_t as_stream(void *s);

// A plan built in place (mcubes_plan_create allocates the object and calls
// this); the workspace of mcubes_iterate is left empty.
int plan_init(int family, const double *params, int dim, int64_t ncall, uint64_t seed,
              const mcubes_options *opt, mcubes_plan *P);
// The iteration loop of mcubes_integrate on a device buffer of
// integrate_buffer_len(P) doubles; `timed` records the V-Sample time with
// HIP events (kernel_ms, else 0).
int64_t integrate_buffer_len(const mcubes_plan &P);
int integrate_run(const mcubes_plan &P, double *buf, int itmax, double rel_tol,
                  bool timed, mcubes_result *out, double *grid_out, double *trace);

// Microbenchmarks (microbench.hip).
hipError_t launch_microbench(int kind, int family, int dim, const VsArgs &A, const double *pts,
                             int64_t npts, int64_t calls, int blocks, int block, double *out,
                             hipStream_t stream);

}  // namespace mcubes

// A validated problem with its stratification and V-Sample launch geometry.
struct mcubes_plan {
    int family, dim, nb, precision;
    int block, blocks;
    size_t lds;        // static LDS of the V-Sample kernel (bytes per block)
    int adapt_iters, skip;
    double alpha;
    int64_t g, m, p, n;
    mcubes::VsArgs args;
    mcubes::VsLaunchFn launch[2];  // [0] without bin sums, [1] with
    const void *func;
    void *stream;      // hipStream_t of the options (mcubes_iterate)
    double *ws;        // device workspace of mcubes_iterate (allocated on its first call)
    int64_t ws_len;    // doubles in ws
};
