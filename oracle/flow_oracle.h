/*
 * flow_oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 * Plain FP64 reference of the learned proposal: a normalizing flow of
 * piecewise-quadratic coupling layers over (0,1)^6, its training loss and
 * gradient, one Adam step, an m-Cubes iteration that samples through it and
 * the equal-weight combination of such iterations.
 * See flow_oracle.c for the definitions.
 */
#ifndef FLOW_ORACLE_H
#define FLOW_ORACLE_H

#include <stdint.h>

#define MCF_D 6                     /* dimension */
#define MCF_LAYERS 4                /* coupling layers */
#define MCF_NA 3                    /* coordinates a layer conditions on */
#define MCF_NB 3                    /* coordinates a layer transforms */
#define MCF_BLOBS 32                /* one-blob encoding cells per input */
#define MCF_IN (MCF_NA * MCF_BLOBS) /* conditioner inputs */
#define MCF_HID 64                  /* hidden width (two hidden layers) */
#define MCF_BINS 16                 /* spline bins */
#define MCF_RAW (2 * MCF_BINS + 1)  /* raw spline parameters per coordinate */
#define MCF_OUT (MCF_NB * MCF_RAW)  /* conditioner outputs */
#define MCF_LAYER_PARAMS \
    (MCF_IN * MCF_HID + MCF_HID + MCF_HID * MCF_HID + MCF_HID + MCF_HID * MCF_OUT + MCF_OUT)
#define MCF_PARAMS (MCF_LAYERS * MCF_LAYER_PARAMS)

int mcf_param_count(void);
void mcf_masks(int layer, int a_idx[MCF_NA], int b_idx[MCF_NB]);
int mcf_spline_forward(const double raw[MCF_RAW], double u, double *y, double *pdf);
int mcf_spline_inverse(const double raw[MCF_RAW], double y, double *u, double *pdf);
void mcf_conditioner(const double *layer_params, const double ua[MCF_NA], int bf16,
                     double out[MCF_OUT]);
void mcf_density(const double *theta, const double x[MCF_D], int bf16, double z[MCF_D],
                 double *logq);
void mcf_sample(const double *theta, const double z[MCF_D], int bf16, double x[MCF_D],
                double *logq);
void mcf_bf16_array(const double *v, int64_t n, double *out);
double mcf_loss_grad(const double *theta, int64_t n, const double *xs, const double *ws,
                     double *grad);
double mcf_loss_grad_ex(const double *theta, int64_t n, const double *xs, const double *ws,
                        int bf16, double *grad, double *grad_abs);
void mcf_adam(double *theta, double *m, double *v, const double *grad, int64_t count, int step,
              double lr, double beta1, double beta2, double eps);
int mcf_proposal_range(const double *theta, int bf16, int family, const double *params, int64_t g,
                       int64_t m, int64_t p, uint64_t seed, uint32_t stream, uint32_t iteration,
                       int64_t c_begin, int64_t c_end, double sums[2]);
int mcf_combine_equal(int T, const double *I, const double *var, double out[3]);

#endif
