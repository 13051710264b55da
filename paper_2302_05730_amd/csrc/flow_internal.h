// Internal declarations of the learned proposal's kernels (flow.hip,
// flow_bf16.hip), used by flow_api.hip.
#pragma once

#include "mcubes_internal.h"

namespace mcubes {

// Flow kernels (flow.hip).
hipError_t launch_flow_density(const float *theta, const double *x, int64_t n, double *z,
                               double *logq, hipStream_t s);
hipError_t launch_flow_sample(const float *theta, const double *z, int64_t n, double *x,
                              double *logq, hipStream_t s);
int64_t flow_scratch_floats(int64_t n);
int64_t flow_transposed_floats();
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);
// Records flow-mapped iteration `iteration`'s (I_t, var_t) from est in the
// combined state and recombines iterations 0..iteration with equal weights;
// converged only from min_iters iterations on.
hipError_t launch_flow_combine(const double *est, double *state, uint32_t iteration,
                               double rel_tol, int min_iters, hipStream_t s);
// Row j of (xo, wo) <- row (a j) mod n of (x, w); needs n < 2^32, a < 2^32
// and gcd(a, n) = 1.
hipError_t launch_flow_shuffle(const double *x, const double *w, int64_t n, uint64_t a,
                               double *xo, double *wo, hipStream_t s);
// out[i] <- (double)in[i]
hipError_t launch_flow_widen(const float *in, int64_t n, double *out, hipStream_t s);
// w[i] <- w[i]^power (training weights of the tail rounds)
hipError_t launch_pow_weights(double *w, int64_t n, double power, hipStream_t s);
// One training step's passes: wsum <- sum of the n weights; the forward and
// backward pass of the weighted NLL (loss += its value, per-sample fields in
// scratch; FP32 form: thetaT, flow_transposed_floats() floats, is rewritten
// from theta; BF16 form: the forward and backward fragments are repacked
// from theta when `pack`, else taken as they are); then the weight
// gradients from the scratch fields.
hipError_t launch_flow_wsum(const double *w, int64_t n, double *wsum, hipStream_t s);
hipError_t launch_flow_train_fp32(const float *theta, float *thetaT, const double *x,
                                  const double *w, int64_t n, const double *wsum, float *scratch,
                                  double *loss, hipStream_t s);
hipError_t launch_flow_train_bf16(const float *theta, void *frags, void *bfrags, float *bias,
                                  const double *x, const double *w, int64_t n, const double *wsum,
                                  float *scratch, double *loss, int cus, bool pack,
                                  hipStream_t s);
hipError_t launch_flow_wgrad(const float *scratch, int64_t n, float *grad, hipStream_t s);
// the same sums on the matrix cores (BF16 operands, FP32 accumulation)
hipError_t launch_flow_wgrad_bf16(const float *scratch, int64_t n, float *grad, hipStream_t s);
// grad[i] <- sum over the slices of part[slice][i], in slice order
hipError_t launch_flow_wgrad_sum(const float *part, int slices, float *grad, hipStream_t s);
// The BF16 weight gradients, then grad, the Adam step on theta (m, v) and the
// new parameters written into frags, bfrags and bias through inv (the
// inverse map, flow_bf16_inverse_map_ints() ints from launch_flow_inverse_map
// over a buffer filled with -1): bit for bit launch_flow_wgrad_bf16,
// launch_flow_adam and a repack, in two launches.
int64_t flow_bf16_inverse_map_ints();
hipError_t launch_flow_inverse_map(int *inv, hipStream_t s);
hipError_t launch_flow_wgrad_adam_bf16(const float *scratch, int64_t n, float *theta, float *m,
                                       float *v, float *grad, float lr, float beta1, float beta2,
                                       float eps, float c1, float c2, const int *inv,
                                       void *frags, void *bfrags, float *bias, hipStream_t s);
int64_t flow_bf16_bwd_frag_bytes();
int64_t flow_bf16_train_extra_floats(int64_t n);
hipError_t launch_flow_adam(float *theta, float *m, float *v, const float *grad, float lr,
                            float beta1, float beta2, float eps, float c1, float c2,
                            hipStream_t s);
// whist: MCUBES_WTAIL_BINS counters the log2 histogram of the weights is added to
hipError_t launch_flow_vsample(int family, const float *theta, const VsArgs &A,
                               uint32_t stream_word, double *partials, uint32_t *whist,
                               int blocks, hipStream_t s);
hipError_t launch_vsample_dump(int family, int dim, const VsArgs &A, const double *grid,
                               uint32_t w0, uint32_t count, double *xs, double *ws,
                               hipStream_t s);
hipError_t launch_flow_draw(int family, const float *theta, const VsArgs &A,
                            uint32_t stream_word, uint32_t n, double *xs, double *ws,
                            hipStream_t s);

// BF16 matrix-core flow sampling (flow_bf16.hip).
int64_t flow_bf16_frag_bytes();
int64_t flow_bf16_bias_floats();
hipError_t launch_flow_pack_bf16(const float *theta, void *frags, float *bias, hipStream_t s);
hipError_t launch_flow_sample_bf16(const void *frags, const float *bias, const double *z,
                                   int64_t n, double *x, double *logq, hipStream_t s);
hipError_t launch_flow_draw_bf16(int family, const void *frags, const float *bias,
                                 const VsArgs &A, uint32_t stream_word, uint32_t n, double *xs,
                                 double *ws, hipStream_t s);
// sums of the consecutive minibatches [k batch, (k + 1) batch) of w, one
// per entry of out (ceil(n / batch) of them)
hipError_t launch_flow_batch_wsums(const double *w, int64_t n, int64_t batch, double *out,
                                   hipStream_t s);
hipError_t launch_flow_vsample_bf16(int family, const void *frags, const float *bias,
                                    const VsArgs &A, uint32_t stream_word, double *partials,
                                    uint32_t *whist, int blocks, hipStream_t s);

}  // namespace mcubes
