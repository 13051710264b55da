// Host side of the learned proposal (declared in include/mcubes.h): the flow
// object (FP32 master parameters, BF16 copy, Adam moments, gradient,
// training scratch), training, and the flow-mapped iteration.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "flow_impl.h"

using namespace mcubes;

struct mcubes_flow {
    float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr;
    float *d_thetaT = nullptr;         // transposed weight matrices (backward pass)
    void *d_frags = nullptr;           // BF16 weight fragments for the matrix-core path
    void *d_bfrags = nullptr;          // BF16 fragments of the backward products
    float *d_fbias = nullptr;          // biases in accumulator order
    int *d_inv = nullptr;              // where each parameter sits in the three packed forms
    bool packed = false;               // fragments up to date with d_theta
    double *d_aux = nullptr;           // [0] sum of weights, [1] loss
    double *d_part = nullptr;          // per-block partials of the flow-mapped iteration
    uint32_t *d_whist = nullptr;       // log2 histogram of the last flow iteration's weights
    double *d_wsums = nullptr;         // weight sum of each minibatch of a training call
    int64_t wsums_cap = 0;
    hipStream_t last_stream = nullptr; // stream of the last flow iteration
    float *d_scratch = nullptr;
    int64_t scratch_n = 0;             // samples the scratch buffer holds
    int step = 0;                      // Adam steps taken
    int cus = 0;
};

namespace {

constexpr int64_t kMaxSamples = (int64_t)1 << 31;
constexpr int kVsBlocks = 2048;  // workgroups of the flow-mapped iteration (grid-stride)
constexpr double kTailLimit = 0.5;  // weight-tail shape from which the variance is infinite
// from this shape on the variance estimates have no finite variance of their
// own (no fourth moment): the error bar is trusted only when the iterations
// agree with each other
constexpr double kTailHeavy = 0.25;

// Upper 99% point of chi^2 with k degrees of freedom per degree of freedom
// (Wilson-Hilferty: chi^2_k / k is close to normal after a cube root).
double chi2_dof_99(int k) {
    if (k < 1) return INFINITY;
    const double a = 2.0 / (9.0 * k), z = 2.3263478740408408;
    const double c = 1.0 - a + z * sqrt(a);
    return c * c * c;
}

// Whether the error bar of flow iterations with pooled weight-tail shape xi
// and scatter chi2/dof (dof degrees of freedom) can be trusted: always
// below kTailHeavy, never from kTailLimit on, in between when the
// iterations agree within their stated errors (chi2/dof below its 99%
// point).  An undetermined shape (too few weights) is not trusted.
bool tail_trusted(double xi, double chi2_dof, int dof) {
    if (!(xi < kTailLimit)) return false;
    if (xi < kTailHeavy) return true;
    return dof >= 1 && chi2_dof <= chi2_dof_99(dof);
}

void release(mcubes_flow *F) {
    if (!F) return;
    (void)hipFree(F->d_theta);
    (void)hipFree(F->d_m);
    (void)hipFree(F->d_v);
    (void)hipFree(F->d_grad);
    (void)hipFree(F->d_thetaT);
    (void)hipFree(F->d_frags);
    (void)hipFree(F->d_bfrags);
    (void)hipFree(F->d_fbias);
    (void)hipFree(F->d_inv);
    (void)hipFree(F->d_aux);
    (void)hipFree(F->d_part);
    (void)hipFree(F->d_whist);
    (void)hipFree(F->d_wsums);
    (void)hipFree(F->d_scratch);
    delete F;
}

int upload(mcubes_flow *F, const double *theta) {
    std::vector<float> h(flow::PARAMS);
    for (int i = 0; i < flow::PARAMS; ++i) {
        if (!isfinite(theta[i])) return fail(MCUBES_E_ARG, "flow parameter %d is not finite", i);
        h[i] = (float)theta[i];
    }
    hipError_t e = hipMemcpy(F->d_theta, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(F->d_m, 0, h.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemset(F->d_v, 0, h.size() * sizeof(float));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "flow parameter upload");
    F->step = 0;
    F->packed = false;
    return MCUBES_OK;
}

// BF16 fragments of the current parameters (repacked after any change).
hipError_t ensure_packed(mcubes_flow *F, hipStream_t s) {
    if (F->packed) return hipSuccess;
    const hipError_t e = launch_flow_pack_bf16(F->d_theta, F->d_frags, F->d_fbias, s);
    if (e == hipSuccess) F->packed = true;
    return e;
}

int check_n(int64_t n) {
    if (n < 0 || n > kMaxSamples) return fail(MCUBES_E_ARG, "n must be in [0, 2^31]");
    return MCUBES_OK;
}

int ensure_scratch(mcubes_flow *F, int64_t n) {
    if (n <= F->scratch_n) return MCUBES_OK;
    (void)hipFree(F->d_scratch);
    F->d_scratch = nullptr;
    F->scratch_n = 0;
    const size_t bytes = (size_t)flow_scratch_floats(n) * sizeof(float);
    const hipError_t e = hipMalloc((void **)&F->d_scratch, bytes);
    if (e != hipSuccess) return fail(MCUBES_E_ALLOC, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    F->scratch_n = n;
    return MCUBES_OK;
}

// One step's forward/backward pass (loss += its value).  wsum: the sum of
// the n weights on the device, or NULL to form it first.  BF16: `pack`
// repacks the fragments from theta first; without it they must already hold
// theta (as the fused gradient and Adam launch leaves them).
hipError_t train_pass(mcubes_flow *F, int precision, const double *d_x, const double *d_w,
                      int64_t n, const double *wsum, double *d_loss, bool pack, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (!wsum) {
        e = launch_flow_wsum(d_w, n, F->d_aux, s);
        wsum = F->d_aux;
    }
    if (e != hipSuccess) return e;
    if (precision == MCUBES_BF16)
        return launch_flow_train_bf16(F->d_theta, F->d_frags, F->d_bfrags, F->d_fbias, d_x, d_w,
                                      n, wsum, F->d_scratch, d_loss, F->cus, pack, s);
    return launch_flow_train_fp32(F->d_theta, F->d_thetaT, d_x, d_w, n, wsum, F->d_scratch, d_loss,
                                  s);
}

// The pass and the weight gradients (in F->d_grad).
hipError_t train_step(mcubes_flow *F, int precision, const double *d_x, const double *d_w,
                      int64_t n, const double *wsum, double *d_loss, hipStream_t s) {
    const hipError_t e = train_pass(F, precision, d_x, d_w, n, wsum, d_loss, true, s);
    if (e != hipSuccess) return e;
    return precision == MCUBES_BF16 ? launch_flow_wgrad_bf16(F->d_scratch, n, F->d_grad, s)
                                    : launch_flow_wgrad(F->d_scratch, n, F->d_grad, s);
}

// A multiplier for the row shuffle: floor(n (sqrt(5)-1)/2) with its lowest bit
// set, stepped by 2 (mod n) until coprime to n, so that j -> a j mod n is a
// permutation whose consecutive outputs lie about 0.618 n apart: any run of
// rows draws evenly from the whole input.
uint64_t shuffle_multiplier(int64_t n) {
    if (n <= 2) return 1;
    const uint64_t un = (uint64_t)n;
    uint64_t a = ((uint64_t)((double)n * 0.6180339887498949) | 1u) % un;
    for (;;) {
        uint64_t x = a, y = un;
        while (y) {
            const uint64_t t = x % y;
            x = y;
            y = t;
        }
        if (x == 1) return a;
        a = (a + 2) % un;
    }
}

bool overlaps(const double *p, int64_t np, const double *q, int64_t nq) {
    return p < q + nq && q < p + np;
}

int check_train_precision(int precision) {
    if (precision != MCUBES_FP32 && precision != MCUBES_BF16)
        return fail(MCUBES_E_ARG, "precision must be MCUBES_FP32 or MCUBES_BF16");
    return MCUBES_OK;
}

}  // namespace

extern "C" {

int mcubes_flow_create(const double *theta, mcubes_flow **out) {
    if (!theta || !out) return fail(MCUBES_E_ARG, "NULL argument");
    for (int i = 0; i < flow::PARAMS; ++i)
        if (!isfinite(theta[i])) return fail(MCUBES_E_ARG, "flow parameter %d is not finite", i);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    mcubes_flow *F = new (std::nothrow) mcubes_flow();
    if (!F) return fail(MCUBES_E_ALLOC, "out of host memory");
    e = hipDeviceGetAttribute(&F->cus, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t pb = (size_t)flow::PARAMS * sizeof(float);
    if (e == hipSuccess) e = hipMalloc((void **)&F->d_theta, pb);
    if (e == hipSuccess) e = hipMalloc((void **)&F->d_m, pb);
    if (e == hipSuccess) e = hipMalloc((void **)&F->d_v, pb);
    if (e == hipSuccess) e = hipMalloc((void **)&F->d_grad, pb);
    if (e == hipSuccess)
        e = hipMalloc((void **)&F->d_thetaT, (size_t)flow_transposed_floats() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&F->d_frags, (size_t)flow_bf16_frag_bytes());
    if (e == hipSuccess) e = hipMalloc(&F->d_bfrags, (size_t)flow_bf16_bwd_frag_bytes());
    if (e == hipSuccess)
        e = hipMalloc((void **)&F->d_fbias, (size_t)flow_bf16_bias_floats() * sizeof(float));
    const size_t ib = (size_t)flow_bf16_inverse_map_ints() * sizeof(int);
    if (e == hipSuccess) e = hipMalloc((void **)&F->d_inv, ib);
    if (e == hipSuccess) e = hipMemset(F->d_inv, 0xff, ib);  // -1: no slot
    if (e == hipSuccess) e = launch_flow_inverse_map(F->d_inv, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = hipMalloc((void **)&F->d_aux, 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&F->d_part, 2 * kVsBlocks * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void **)&F->d_whist, (size_t)MCUBES_WTAIL_BINS * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(F->d_whist, 0, (size_t)MCUBES_WTAIL_BINS * sizeof(uint32_t));
    if (e != hipSuccess) {
        release(F);
        return fail(MCUBES_E_ALLOC, "flow allocation: %s", hipGetErrorString(e));
    }
    const int rc = upload(F, theta);
    if (rc != MCUBES_OK) {
        release(F);
        return rc;
    }
    *out = F;
    return MCUBES_OK;
}

void mcubes_flow_destroy(mcubes_flow *F) { release(F); }

int mcubes_flow_get_params(const mcubes_flow *F, double *theta) {
    if (!F || !theta) return fail(MCUBES_E_ARG, "NULL argument");
    std::vector<float> h(flow::PARAMS);
    const hipError_t e =
        hipMemcpy(h.data(), F->d_theta, h.size() * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "flow parameter download");
    for (int i = 0; i < flow::PARAMS; ++i) theta[i] = (double)h[i];
    return MCUBES_OK;
}

int mcubes_flow_set_params(mcubes_flow *F, const double *theta) {
    if (!F || !theta) return fail(MCUBES_E_ARG, "NULL argument");
    return upload(F, theta);
}

int mcubes_flow_density(mcubes_flow *F, int precision, const double *d_x, int64_t n, double *d_z,
                        double *d_logq, void *stream) {
    if (!F || (n > 0 && (!d_x || !d_z || !d_logq))) return fail(MCUBES_E_ARG, "NULL argument");
    int rc = check_n(n);
    if (rc != MCUBES_OK) return rc;
    if (precision != MCUBES_FP32)
        return fail(MCUBES_E_ARG, "the density direction is available in MCUBES_FP32 only");
    const hipError_t e = launch_flow_density(F->d_theta, d_x, n, d_z, d_logq, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "flow density launch");
}

int mcubes_flow_sample(mcubes_flow *F, int precision, const double *d_z, int64_t n, double *d_x,
                       double *d_logq, void *stream) {
    if (!F || (n > 0 && (!d_z || !d_x || !d_logq))) return fail(MCUBES_E_ARG, "NULL argument");
    int rc = check_n(n);
    if (rc != MCUBES_OK) return rc;
    if (precision != MCUBES_FP32 && precision != MCUBES_BF16)
        return fail(MCUBES_E_ARG, "precision must be MCUBES_FP32 or MCUBES_BF16");
    hipStream_t s = as_stream(stream);
    hipError_t e;
    if (precision == MCUBES_BF16) {
        e = ensure_packed(F, s);
        if (e == hipSuccess) e = launch_flow_sample_bf16(F->d_frags, F->d_fbias, d_z, n, d_x, d_logq, s);
    } else {
        e = launch_flow_sample(F->d_theta, d_z, n, d_x, d_logq, s);
    }
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "flow sample launch");
}

int mcubes_flow_loss_grad(mcubes_flow *F, int precision, const double *d_x, const double *d_w,
                          int64_t n, double *d_grad, double *d_loss, void *stream) {
    if (!F || !d_x || !d_w || !d_loss) return fail(MCUBES_E_ARG, "NULL argument");
    if (n < 1 || n > kMaxSamples) return fail(MCUBES_E_ARG, "n must be in [1, 2^31]");
    int rc = check_train_precision(precision);
    if (rc != MCUBES_OK) return rc;
    rc = ensure_scratch(F, n);
    if (rc != MCUBES_OK) return rc;
    hipStream_t s = as_stream(stream);
    hipError_t e = train_step(F, precision, d_x, d_w, n, nullptr, d_loss, s);
    // widen the kept FP32 gradient for the caller
    if (e == hipSuccess && d_grad) e = launch_flow_widen(F->d_grad, flow::PARAMS, d_grad, s);
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "flow gradient");
}

int mcubes_flow_adam_step(mcubes_flow *F, double lr, double beta1, double beta2, double eps,
                          void *stream) {
    if (!F) return fail(MCUBES_E_ARG, "NULL argument");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
        !(eps > 0.0))
        return fail(MCUBES_E_ARG, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
    F->step += 1;
    F->packed = false;
    const double c1 = 1.0 - pow(beta1, (double)F->step), c2 = 1.0 - pow(beta2, (double)F->step);
    const hipError_t e = launch_flow_adam(F->d_theta, F->d_m, F->d_v, F->d_grad, (float)lr,
                                          (float)beta1, (float)beta2, (float)eps, (float)c1,
                                          (float)c2, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "Adam launch");
}

int mcubes_flow_train(mcubes_flow *F, int precision, const double *d_x, const double *d_w,
                      int64_t n, int epochs, int64_t batch, double lr, double *losses,
                      void *stream) {
    if (!F || !d_x || !d_w) return fail(MCUBES_E_ARG, "NULL argument");
    if (n < 1 || n > kMaxSamples) return fail(MCUBES_E_ARG, "n must be in [1, 2^31]");
    if (epochs < 0 || batch < 1) return fail(MCUBES_E_ARG, "epochs >= 0 and batch >= 1 required");
    int rc = check_train_precision(precision);
    if (rc != MCUBES_OK) return rc;
    if (batch > n) batch = n;
    rc = ensure_scratch(F, batch);
    if (rc != MCUBES_OK) return rc;
    hipStream_t s = as_stream(stream);
    double *d_loss = F->d_aux + 1;
    F->packed = false;
    // the weights stay fixed: every minibatch's sum once, for all epochs
    const int64_t nb_total = (n + batch - 1) / batch;
    if (nb_total > F->wsums_cap) {
        (void)hipFree(F->d_wsums);
        F->d_wsums = nullptr;
        F->wsums_cap = 0;
        const hipError_t ea = hipMalloc((void **)&F->d_wsums, (size_t)nb_total * sizeof(double));
        if (ea != hipSuccess) return fail(MCUBES_E_ALLOC, "hipMalloc: %s", hipGetErrorString(ea));
        F->wsums_cap = nb_total;
    }
    hipError_t ew = launch_flow_batch_wsums(d_w, n, batch, F->d_wsums, s);
    if (ew != hipSuccess) return hip_fail(ew, "minibatch weight sums");
    bool first = true;
    for (int ep = 0; ep < epochs; ++ep) {
        hipError_t e = hipMemsetAsync(d_loss, 0, sizeof(double), s);
        int nbatch = 0;
        for (int64_t b0 = 0; b0 < n && e == hipSuccess; b0 += batch) {
            const int64_t nb = n - b0 < batch ? n - b0 : batch;
            // BF16: the step's last launch updates the fragments with theta,
            // so only the call's first pass packs them
            e = train_pass(F, precision, d_x + b0 * flow::D, d_w + b0, nb, F->d_wsums + b0 / batch,
                           d_loss, first, s);
            first = false;
            if (e != hipSuccess) break;
            F->step += 1;
            const double c1 = 1.0 - pow(0.9, (double)F->step);
            const double c2 = 1.0 - pow(0.999, (double)F->step);
            if (precision == MCUBES_BF16) {
                e = launch_flow_wgrad_adam_bf16(F->d_scratch, nb, F->d_theta, F->d_m, F->d_v,
                                                F->d_grad, (float)lr, 0.9f, 0.999f, 1e-8f,
                                                (float)c1, (float)c2, F->d_inv, F->d_frags,
                                                F->d_bfrags, F->d_fbias, s);
            } else {
                e = launch_flow_wgrad(F->d_scratch, nb, F->d_grad, s);
                if (e == hipSuccess)
                    e = launch_flow_adam(F->d_theta, F->d_m, F->d_v, F->d_grad, (float)lr, 0.9f,
                                         0.999f, 1e-8f, (float)c1, (float)c2, s);
            }
            ++nbatch;
        }
        if (e == hipSuccess && losses) {
            double h = 0.0;
            e = hipMemcpyAsync(&h, d_loss, sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            losses[ep] = h / (double)nbatch;
        }
        if (e != hipSuccess) return hip_fail(e, "flow training");
    }
    return MCUBES_OK;
}

int mcubes_vsample_dump(const mcubes_plan *P, uint32_t iteration, const double *d_grid,
                        int64_t w_begin, int64_t count, double *d_x, double *d_w, void *stream) {
    if (!P || !d_grid || (count > 0 && (!d_x || !d_w))) return fail(MCUBES_E_ARG, "NULL argument");
    if (w_begin < 0 || count < 0 || w_begin + count > P->m)
        return fail(MCUBES_E_ARG, "work items [%lld, %lld) outside [0, %lld)", (long long)w_begin,
                    (long long)(w_begin + count), (long long)P->m);
    VsArgs A = P->args;
    A.iteration = iteration;
    const hipError_t e = launch_vsample_dump(P->family, P->dim, A, d_grid, (uint32_t)w_begin,
                                             (uint32_t)count, d_x, d_w, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "sample export launch");
}

int mcubes_flow_draw(mcubes_flow *F, int precision, const mcubes_plan *P, uint32_t iteration,
                     int64_t n, double *d_x, double *d_w, void *stream) {
    if (!F || !P || (n > 0 && (!d_x || !d_w))) return fail(MCUBES_E_ARG, "NULL argument");
    if (P->dim != flow::D) return fail(MCUBES_E_ARG, "the flow needs a plan of dim %d", flow::D);
    if (n < 0 || n > 0xFFFFFFFFll) return fail(MCUBES_E_ARG, "n must be in [0, 2^32)");
    if (precision != MCUBES_FP32 && precision != MCUBES_BF16)
        return fail(MCUBES_E_ARG, "precision must be MCUBES_FP32 or MCUBES_BF16");
    VsArgs A = P->args;
    A.iteration = iteration;
    const uint32_t stream_word = A.stream_id | 0xC0000000u;
    hipStream_t s = as_stream(stream);
    hipError_t e;
    if (precision == MCUBES_BF16) {
        e = ensure_packed(F, s);
        if (e == hipSuccess)
            e = launch_flow_draw_bf16(P->family, F->d_frags, F->d_fbias, A, stream_word,
                                      (uint32_t)n, d_x, d_w, s);
    } else {
        e = launch_flow_draw(P->family, F->d_theta, A, stream_word, (uint32_t)n, d_x, d_w, s);
    }
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "flow draw launch");
}

int mcubes_flow_vsample(mcubes_flow *F, int precision, const mcubes_plan *P, uint32_t iteration,
                        double *d_est, void *stream) {
    if (!F || !P || !d_est) return fail(MCUBES_E_ARG, "NULL argument");
    if (P->dim != flow::D) return fail(MCUBES_E_ARG, "the flow needs a plan of dim %d", flow::D);
    if (precision != MCUBES_FP32 && precision != MCUBES_BF16)
        return fail(MCUBES_E_ARG, "precision must be MCUBES_FP32 or MCUBES_BF16");
    if (precision == MCUBES_BF16 && 64 % P->p != 0)
        return fail(MCUBES_E_ARG, "the BF16 flow iteration needs p dividing 64, got %lld",
                    (long long)P->p);
    VsArgs A = P->args;
    A.iteration = iteration;
    const uint32_t stream_word = A.stream_id | 0x80000000u;
    hipStream_t s = as_stream(stream);
    F->last_stream = s;
    hipError_t e = launch_zero_u32(F->d_whist, MCUBES_WTAIL_BINS, s);
    int blocks;
    if (precision == MCUBES_BF16) {
        // 256 samples per workgroup pass (four waves of 64)
        const int64_t groups = (P->m * P->p + 255) / 256;
        blocks = groups < kVsBlocks ? (int)groups : kVsBlocks;
        if (e == hipSuccess) e = ensure_packed(F, s);
        if (e == hipSuccess)
            e = launch_flow_vsample_bf16(P->family, F->d_frags, F->d_fbias, A, stream_word,
                                         F->d_part, F->d_whist, blocks, s);
    } else {
        // cooperative form for p dividing 64 (64 samples per workgroup pass),
        // else one cube per thread
        const int64_t groups = 64 % P->p == 0 ? (P->m * P->p + 63) / 64 : (P->m + 255) / 256;
        blocks = groups < kVsBlocks ? (int)groups : kVsBlocks;
        if (e == hipSuccess)
            e = launch_flow_vsample(P->family, F->d_theta, A, stream_word, F->d_part, F->d_whist,
                                    blocks, s);
    }
    const double n = (double)P->m * (double)P->p;
    const double denom = (double)P->p * (double)P->m * (double)P->m;
    if (e == hipSuccess) e = launch_reduce(F->d_part, blocks, n, denom, d_est, s);
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "flow V-Sample launch");
}

int mcubes_flow_shuffle(const double *d_x, const double *d_w, int64_t n, double *d_x_out,
                        double *d_w_out, void *stream) {
    if (n < 0 || n >= ((int64_t)1 << 32)) return fail(MCUBES_E_ARG, "n must be in [0, 2^32)");
    if (n == 0) return MCUBES_OK;
    if (!d_x || !d_w || !d_x_out || !d_w_out) return fail(MCUBES_E_ARG, "NULL argument");
    const int64_t nx = n * flow::D;
    if (overlaps(d_x, nx, d_x_out, nx) || overlaps(d_x, nx, d_w_out, n) ||
        overlaps(d_w, n, d_x_out, nx) || overlaps(d_w, n, d_w_out, n) ||
        overlaps(d_x_out, nx, d_w_out, n))
        return fail(MCUBES_E_ARG, "the shuffle's outputs must not overlap its inputs or each other");
    const hipError_t e = launch_flow_shuffle(d_x, d_w, n, shuffle_multiplier(n), d_x_out, d_w_out,
                                             as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "shuffle launch");
}

int mcubes_flow_combine(uint32_t iteration, const double *d_est, double *d_state, double rel_tol,
                        int min_iters, void *stream) {
    if (!d_est || !d_state) return fail(MCUBES_E_ARG, "NULL argument");
    if (iteration >= MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "iteration %u >= %d", iteration, MCUBES_MAX_ITERATIONS);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol))
        return fail(MCUBES_E_ARG, "rel_tol must be finite and >= 0");
    if (min_iters < 1 || min_iters > MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "min_iters must be in [1, %d]", MCUBES_MAX_ITERATIONS);
    const hipError_t e =
        launch_flow_combine(d_est, d_state, iteration, rel_tol, min_iters, as_stream(stream));
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "flow combine launch");
}

int mcubes_weight_tail_shape(const uint32_t *hist, double *shape, int64_t *tail_count) {
    if (!hist || !shape) return fail(MCUBES_E_ARG, "NULL argument");
    *shape = NAN;
    if (tail_count) *tail_count = 0;
    int64_t total = 0;
    for (int b = 0; b < MCUBES_WTAIL_BINS; ++b) total += hist[b];
    if (total < 100) return MCUBES_OK;
    const int64_t k = std::min<int64_t>(total / 5, (int64_t)floor(3.0 * sqrt((double)total)));
    // the bins holding the k largest weights, from the top down
    int b = MCUBES_WTAIL_BINS - 1;
    int64_t c = hist[b];
    while (c < k && b > 0) c += hist[--b];
    // Hill estimate over them, threshold the lower edge of bin b, each weight
    // at the middle of its bin (in log2, bins are 1/8 wide)
    double acc = 0.0;
    for (int q = b; q < MCUBES_WTAIL_BINS; ++q) acc += (double)hist[q] * ((double)(q - b) + 0.5);
    *shape = acc / (double)c * (log(2.0) / 8.0);
    if (tail_count) *tail_count = c;
    return MCUBES_OK;
}

int mcubes_flow_weight_tail(mcubes_flow *F, double *shape, int64_t *tail_count) {
    if (!F || !shape) return fail(MCUBES_E_ARG, "NULL argument");
    std::vector<uint32_t> h(MCUBES_WTAIL_BINS);
    hipError_t e = hipStreamSynchronize(F->last_stream);
    if (e == hipSuccess)
        e = hipMemcpy(h.data(), F->d_whist, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "weight histogram");
    return mcubes_weight_tail_shape(h.data(), shape, tail_count);
}

void mcubes_default_flow_options(mcubes_flow_options *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->warmup_iters = 8;
    o->precision = MCUBES_BF16;
    o->train_items = (int64_t)1 << 20;
    o->epochs = 10;
    o->rounds = 4;
    o->round_samples = (int64_t)1 << 25;
    o->round_epochs = 2;
    o->tail_rounds = 4;
    o->batch = 65536;
    o->lr = 4e-3;
    o->round_lr = 2e-3;
    o->tail_power = 1.75;
    o->tail_lr = 8e-4;
    o->train_precision = MCUBES_BF16;
    o->anchor_rounds = 2;
    o->min_iters = 4;
}

int mcubes_flow_integrate(mcubes_flow *F, int family, const double *params, int64_t ncall,
                          int itmax, double rel_tol, uint64_t seed, const mcubes_options *opt_in,
                          const mcubes_flow_options *fopt_in, mcubes_result *out,
                          mcubes_flow_report *rep) {
    if (!F || !out) return fail(MCUBES_E_ARG, "NULL argument");
    if (itmax < 1 || itmax > MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "itmax must be in [1, %d]", MCUBES_MAX_ITERATIONS);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(MCUBES_E_ARG, "rel_tol must be finite and >= 0");
    mcubes_flow_options fo;
    mcubes_default_flow_options(&fo);
    if (fopt_in) fo = *fopt_in;
    if (fo.warmup_iters < 1 || fo.warmup_iters + itmax > MCUBES_MAX_ITERATIONS || fo.epochs < 0 ||
        fo.rounds < 0 || fo.round_epochs < 0 || fo.tail_rounds < 0 || fo.batch < 1 ||
        fo.train_items < 1 || !(fo.tail_power >= 1.0 && fo.tail_power <= 4.0) ||
        !(fo.tail_lr > 0.0) ||
        (fo.train_precision != MCUBES_FP32 && fo.train_precision != MCUBES_BF16) ||
        fo.anchor_rounds < 0 || fo.min_iters < 1 || fo.min_iters > itmax ||
        fo.round_samples < 1 || fo.round_samples > ((int64_t)1 << 31) || !(fo.lr > 0.0) ||
        !(fo.round_lr > 0.0) || (fo.precision != MCUBES_FP32 && fo.precision != MCUBES_BF16))
        return fail(MCUBES_E_ARG, "invalid flow options");
    mcubes_options opt;
    mcubes_default_options(&opt);
    if (opt_in) opt = *opt_in;
    opt.precision = MCUBES_FP64;
    mcubes_plan *P = nullptr;
    int rc = mcubes_plan_create(family, params, flow::D, ncall, seed, &opt, &P);
    if (rc != MCUBES_OK) return rc;
    hipStream_t s = as_stream(opt.stream);
    const int64_t ng = (int64_t)P->dim * (P->nb + 1), nbn = (int64_t)P->dim * P->nb;
    const int64_t items = fo.train_items < P->m ? fo.train_items : P->m;
    // training rows: an equal share of the items from each warm-up iteration
    const int64_t per_it = items / fo.warmup_iters > 0 ? items / fo.warmup_iters : 1;
    const int64_t rows = per_it * P->p * fo.warmup_iters;
    int64_t trows = 0;
    // row buffers: [round draws | warm-up samples] and its shuffled copy
    const int64_t rs = fo.round_samples, urows = rs + rows;
    if (urows > kMaxSamples) {
        mcubes_plan_destroy(P);
        return fail(MCUBES_E_ARG, "round_samples plus the %lld warm-up rows exceed 2^31",
                    (long long)rows);
    }
    const int64_t total = 2 * ng + nbn + 2 * (int64_t)P->blocks + 2 + 2 * MCUBES_STATE_LEN +
                          14 * urows;
    double *buf = nullptr;
    hipEvent_t ev[4] = {};
    double head[MCUBES_STATE_HEADER];
    mcubes_flow_report R;
    memset(&R, 0, sizeof R);
    int done = 0, used = 1, plain_t = fo.warmup_iters;
    std::vector<uint32_t> hist(MCUBES_WTAIL_BINS), pooled(MCUBES_WTAIL_BINS, 0u);
    float ms = 0.0f;
    hipError_t e = hipMalloc(&buf, (size_t)total * sizeof(double));
    if (e != hipSuccess) {
        mcubes_plan_destroy(P);
        return fail(MCUBES_E_ALLOC, "hipMalloc: %s", hipGetErrorString(e));
    }
    double *grid[2] = {buf, buf + ng};
    double *bins = buf + 2 * ng;
    double *partials = bins + nbn;
    double *est = partials + 2 * (int64_t)P->blocks;
    double *st_plain = est + 2, *st_flow = st_plain + MCUBES_STATE_LEN;
    double *dx = st_flow + MCUBES_STATE_LEN, *dw = dx + 6 * urows;
    double *sx = dw + urows, *sw = sx + 6 * urows;
    double *wx = dx + 6 * rs, *ww = dw + rs;  // the warm-up samples
    double *state = st_flow;

#define FI_CHECK(expr, what)                 \
    do {                                     \
        e = (expr);                          \
        if (e != hipSuccess) {               \
            rc = hip_fail(e, what);          \
            goto cleanup;                    \
        }                                    \
    } while (0)
#define FI_CALL(expr)                        \
    do {                                     \
        rc = (expr);                         \
        if (rc != MCUBES_OK) goto cleanup;   \
    } while (0)

    for (auto &x : ev) FI_CHECK(hipEventCreate(&x), "hipEventCreate");
    FI_CHECK(hipEventRecord(ev[0], s), "hipEventRecord");
    // 1. plain warm-up iterations
    FI_CHECK(launch_init_grid(grid[0], P->dim, P->nb, s), "init_grid launch");
    FI_CHECK(launch_fill(st_plain, 2 * MCUBES_STATE_LEN, 0.0, s), "fill launch");
    // The training samples: an equal share of the work items from every
    // warm-up iteration, taken with that iteration's grid right after it
    // (the next iteration overwrites that grid).  Each share is an unbiased
    // weighted sample of f; the early, still broad grids reach every mode,
    // which the later ones may have given up (a separable map can settle on
    // one of several peaks).
    for (int t = 0; t < fo.warmup_iters; ++t) {
        FI_CALL(mcubes_iteration(P, (uint32_t)t, grid[t & 1], grid[(t + 1) & 1], bins, partials, est,
                                 st_plain, 0.0, opt.stream));
        FI_CALL(mcubes_vsample_dump(P, (uint32_t)t, grid[t & 1], 0, per_it, wx + trows * flow::D,
                                    ww + trows, opt.stream));
        trows += per_it * P->p;
    }
    FI_CHECK(hipMemcpyAsync(&R.last_plain_var, est + 1, sizeof(double), hipMemcpyDeviceToHost, s),
             "hipMemcpyAsync");
    FI_CHECK(hipMemcpyAsync(head, st_plain, sizeof head, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    FI_CHECK(hipEventRecord(ev[1], s), "hipEventRecord");
    // 2-3. training on the warm-up's samples, then on the flow's own.  The
    // mini-batches are runs of consecutive rows, so the rows are shuffled
    // first: the warm-up samples come in blocks, one per iteration.
    {
        double losses[1024];
        const int ep = fo.epochs < 1024 ? fo.epochs : 1024;
        if (ep > 0) {
            FI_CALL(mcubes_flow_shuffle(wx, ww, trows, sx, sw, opt.stream));
            FI_CALL(mcubes_flow_train(F, fo.train_precision, sx, sw, trows, ep, fo.batch, fo.lr,
                                      losses, opt.stream));
            R.final_loss = losses[ep - 1];
        }
        const int rep_ep = fo.round_epochs < 1024 ? fo.round_epochs : 1024;
        for (int r = 0; r < fo.rounds + fo.tail_rounds; ++r) {
            const bool tail = r >= fo.rounds;
            FI_CALL(mcubes_flow_draw(F, fo.train_precision, P, (uint32_t)(1000 + r), rs, dx, dw,
                                     opt.stream));
            if (tail && fo.tail_power != 1.0)
                FI_CHECK(launch_pow_weights(dw, rs, fo.tail_power, s), "weights launch");
            if (rep_ep <= 0) continue;
            // the anchored rounds also train on the warm-up samples (both
            // sets are weighted samples of f, on the same scale), which
            // keeps every peak of f in the data: a flow that has lost one
            // never draws there itself
            const bool anchored = r < fo.anchor_rounds && !tail;
            const int64_t n = anchored ? rs + trows : rs;
            if (anchored) FI_CALL(mcubes_flow_shuffle(dx, dw, n, sx, sw, opt.stream));
            FI_CALL(mcubes_flow_train(F, fo.train_precision, anchored ? sx : dx,
                                      anchored ? sw : dw, n, rep_ep, fo.batch,
                                      tail ? fo.tail_lr : fo.round_lr, losses, opt.stream));
            R.final_loss = losses[rep_ep - 1];
        }
    }
    FI_CHECK(hipEventRecord(ev[2], s), "hipEventRecord");
    R.tail_shape = NAN;
    R.plain_estimate = head[0];
    R.plain_error = head[1];
    R.plain_chi2_dof = head[2];
    // 4. flow-mapped iterations, judged against the plain method.  Their
    // weight histograms are pooled: the tail shape of all flow samples so far.
    for (int t = 0; t < itmax; ++t) {
        const uint32_t it = (uint32_t)(fo.warmup_iters + t);
        if (used) {
            FI_CALL(mcubes_flow_vsample(F, fo.precision, P, it, est, opt.stream));
            FI_CALL(mcubes_flow_combine((uint32_t)t, est, st_flow, rel_tol, fo.min_iters,
                                        opt.stream));
        } else {
            // plain iterations continue from the warm-up's grid and state
            FI_CALL(mcubes_iteration(P, (uint32_t)plain_t, grid[plain_t & 1],
                                     grid[(plain_t + 1) & 1], bins, partials, est, st_plain,
                                     rel_tol, opt.stream));
            ++plain_t;
        }
        FI_CHECK(hipMemcpyAsync(head, used ? st_flow : st_plain, sizeof head,
                                hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        double ev_var = 0.0;
        FI_CHECK(hipMemcpyAsync(&ev_var, est + 1, sizeof ev_var, hipMemcpyDeviceToHost, s),
                 "hipMemcpyAsync");
        if (used)
            FI_CHECK(hipMemcpyAsync(hist.data(), F->d_whist, hist.size() * sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        FI_CHECK(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (used) {
            for (size_t b = 0; b < hist.size(); ++b) pooled[b] += hist[b];
            FI_CALL(mcubes_weight_tail_shape(pooled.data(), &R.tail_shape, nullptr));
        }
        done = t + 1;
        if (used && t == 0) {
            R.first_flow_var = ev_var;
            if (!(ev_var < R.last_plain_var)) {
                used = 0;  // the flow lost: continue with plain iterations
                state = st_plain;
                R.tail_shape = NAN;
                continue;
            }
        }
        if (head[6] != 0.0) {
            rc = fail(MCUBES_E_NONFINITE, "iteration %d produced a non-finite estimate", t);
            goto cleanup;
        }
        if (head[5] != 0.0 && (!used || tail_trusted(R.tail_shape, head[2], (int)head[3]))) break;
    }
    FI_CHECK(hipEventRecord(ev[3], s), "hipEventRecord");
    FI_CHECK(hipEventSynchronize(ev[3]), "hipEventSynchronize");
    FI_CHECK(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
    R.warmup_ms = ms;
    FI_CHECK(hipEventElapsedTime(&ms, ev[1], ev[2]), "hipEventElapsedTime");
    R.train_ms = ms;
    FI_CHECK(hipEventElapsedTime(&ms, ev[2], ev[3]), "hipEventElapsedTime");
    R.flow_ms = ms;
    FI_CHECK(hipEventElapsedTime(&ms, ev[0], ev[3]), "hipEventElapsedTime");
    R.total_ms = ms;
    FI_CHECK(hipMemcpy(head, state, sizeof head, hipMemcpyDeviceToHost), "hipMemcpy");
    R.flow_iterations = used ? done : 1;
    R.used_flow = used;
    out->estimate = head[0];
    out->error = head[1];
    out->chi2_dof = head[2];
    out->dof = (int32_t)head[3];
    out->iterations = (int32_t)head[4];
    // the error bar of flow iterations whose weights have no finite
    // variance (tail shape >= 1/2) means nothing: never call that converged;
    // between 1/4 and 1/2 only when the iterations agree with each other
    out->converged = head[5] != 0.0 && (!used || tail_trusted(R.tail_shape, head[2], (int)head[3]));
    out->cube_side = P->g;
    out->ncubes = P->m;
    out->samples_per_cube = P->p;
    out->samples_per_iter = P->n;
    out->kernel_ms = R.flow_ms;
    rc = out->converged ? MCUBES_OK : MCUBES_NOT_CONVERGED;
    out->status = rc;
    if (rep) *rep = R;

cleanup:
#undef FI_CHECK
#undef FI_CALL
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(buf);
    mcubes_plan_destroy(P);
    return rc;
}

}  // extern "C"
