/*
 * flow_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain FP64 reference of the learned importance sampler used as an
 * alternative proposal for m-Cubes on non-separable integrands (not part of
 * the paper; its design follows "Neural Importance Sampling", Müller, McWilliams,
 * Rousselle, Gross, Novák, 2019: piecewise-quadratic coupling layers with a
 * one-blob encoded conditioner).  Only the test-suite, the smoke check and the
 * CPU baseline leg of the benchmark may load this library; it shares nothing
 * with the HIP library.
 *
 * The flow maps x in (0,1)^6 to z in (0,1)^6 through four coupling layers.
 * Layer l keeps the coordinates A_l and replaces every coordinate j of B_l
 * by C(u_j), the CDF of a piecewise-linear density on (0,1) whose 16 bin
 * widths and 17 vertex heights are computed from u_{A_l} by a small network:
 *   one-blob encoding: each of the 3 inputs becomes 32 values
 *     e_k = exp(-((u - (k + 1/2)/32) * 32)^2 / 2),
 *   two hidden layers of 64 ReLU units, a linear output of 3 x 33 values;
 *   widths W = softmax(first 16 raw values), heights V_i proportional to
 *   exp(raw_{16+i}), scaled so that sum_i (V_i + V_{i+1})/2 W_i = 1.
 * The density of the flow is q(x) = product over layers and transformed
 * coordinates of the spline densities, so sampling draws z uniformly and
 * inverts the layers in reverse order (each inverse CDF solves one
 * quadratic).  Training minimises the weighted negative log-likelihood
 * -sum w_i log q(x_i) / sum w_i of samples x_i with weights w_i
 * (for m-Cubes samples w = f J, so the minimiser approaches q ~ f).
 *
 * Parameter layout of layer l (row-major, input index first):
 *   W1[96][64], b1[64], W2[64][64], b2[64], W3[64][99], b3[99].
 * Masks: A = {0,1,2}, {3,4,5}, {0,2,4}, {1,3,5}; B = the other three, in
 * increasing order.
 *
 * bf16 = 1 evaluates the conditioner the way a BF16 matrix unit does: the
 * weights and the inputs of every matrix product rounded to bfloat16
 * (round to nearest even, through FP32), the biases to FP32, products
 * accumulated exactly (here in FP64).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "flow_oracle.h"
#include "mcubes_oracle.h"

static const int A_IDX[MCF_LAYERS][MCF_NA] = {{0, 1, 2}, {3, 4, 5}, {0, 2, 4}, {1, 3, 5}};
static const int B_IDX[MCF_LAYERS][MCF_NB] = {{3, 4, 5}, {0, 1, 2}, {1, 3, 5}, {0, 2, 4}};

/* offsets inside one layer's parameters */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MCF_IN * MCF_HID)
#define OFF_W2 (OFF_B1 + MCF_HID)
#define OFF_B2 (OFF_W2 + MCF_HID * MCF_HID)
#define OFF_W3 (OFF_B2 + MCF_HID)
#define OFF_B3 (OFF_W3 + MCF_HID * MCF_OUT)

int mcf_param_count(void) { return MCF_PARAMS; }

void mcf_masks(int layer, int a_idx[MCF_NA], int b_idx[MCF_NB])
{
    for (int t = 0; t < MCF_NA; ++t) a_idx[t] = A_IDX[layer][t];
    for (int t = 0; t < MCF_NB; ++t) b_idx[t] = B_IDX[layer][t];
}

/* Round to bfloat16, round to nearest with ties to even, through FP32 (the
 * network values the matrix units take are FP32).  Written from the
 * definition: the two bfloat16 values that bracket the FP32 value f are its
 * truncation toward zero (the top 16 bits of its encoding) and the next
 * bfloat16 away from zero; the nearer one wins, and on a tie the one whose
 * last kept mantissa bit is 0.  Past the largest finite bfloat16 the upper
 * neighbour is 2^128 (infinity), as for any IEEE overflow under rounding to
 * nearest.  The distances are exact in FP64.  Non-finite values pass. */
static float bits_to_float(uint32_t b)
{
    float f;
    memcpy(&f, &b, 4);
    return f;
}

static double bf16(double v)
{
    const float f = (float)v;
    if (!isfinite(f)) return (double)f;
    uint32_t b;
    memcpy(&b, &f, 4);
    const uint32_t lo_bits = b & 0xffff0000u;         /* toward zero */
    const uint32_t hi_bits = lo_bits + 0x00010000u;   /* away from zero */
    const double lo = (double)bits_to_float(lo_bits);
    const int hi_inf = (hi_bits & 0x7f800000u) == 0x7f800000u;
    const double hi = hi_inf ? copysign(ldexp(1.0, 128), (double)f)
                             : (double)bits_to_float(hi_bits);
    const double d_lo = fabs((double)f - lo), d_hi = fabs(hi - (double)f);
    int up;
    if (d_lo != d_hi)
        up = d_hi < d_lo;
    else
        up = (lo_bits & 0x00010000u) != 0; /* tie: keep the even neighbour */
    if (!up) return lo;
    return hi_inf ? copysign(INFINITY, (double)f) : hi;
}

void mcf_bf16_array(const double *v, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf16(v[i]);
}

/* ------------------------------------------------------------------------ */
/* The spline of one coordinate                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    double W[MCF_BINS];       /* bin widths, sum 1 */
    double V[MCF_BINS + 1];   /* vertex heights of the density */
    double E[MCF_BINS + 1];   /* exp(raw height - max), before scaling */
    double Z;                 /* scaling: V = E / Z */
    double X[MCF_BINS + 1];   /* left edges, X[K] = 1 */
    double Acum[MCF_BINS + 1];/* CDF at the left edges, Acum[K] = 1 */
} spline_t;

static void spline_setup(const double raw[MCF_RAW], spline_t *s)
{
    const double *wr = raw, *vr = raw + MCF_BINS;
    double mw = wr[0], mv = vr[0];
    for (int i = 1; i < MCF_BINS; ++i) mw = wr[i] > mw ? wr[i] : mw;
    for (int i = 1; i <= MCF_BINS; ++i) mv = vr[i] > mv ? vr[i] : mv;
    double sw = 0.0;
    for (int i = 0; i < MCF_BINS; ++i) {
        s->W[i] = exp(wr[i] - mw);
        sw += s->W[i];
    }
    for (int i = 0; i < MCF_BINS; ++i) s->W[i] /= sw;
    for (int i = 0; i <= MCF_BINS; ++i) s->E[i] = exp(vr[i] - mv);
    double Z = 0.0;
    for (int i = 0; i < MCF_BINS; ++i) Z += 0.5 * (s->E[i] + s->E[i + 1]) * s->W[i];
    s->Z = Z;
    for (int i = 0; i <= MCF_BINS; ++i) s->V[i] = s->E[i] / Z;
    s->X[0] = 0.0;
    s->Acum[0] = 0.0;
    for (int i = 0; i < MCF_BINS; ++i) {
        s->X[i + 1] = s->X[i] + s->W[i];
        s->Acum[i + 1] = s->Acum[i] + 0.5 * (s->V[i] + s->V[i + 1]) * s->W[i];
    }
}

static int bin_of(const double *edges, double t)
{
    int b = 0;
    for (int k = 1; k < MCF_BINS; ++k)
        if (edges[k] <= t) b = k;
    return b;
}

/* CDF and density at u: within bin b, with a = (u - X_b) / W_b,
 * y = A_b + W_b (a V_b + a^2 (V_{b+1} - V_b) / 2), pdf = V_b + a (V_{b+1} - V_b). */
int mcf_spline_forward(const double raw[MCF_RAW], double u, double *y, double *pdf)
{
    spline_t s;
    spline_setup(raw, &s);
    const int b = bin_of(s.X, u);
    double a = (u - s.X[b]) / s.W[b];
    if (a < 0.0) a = 0.0;
    if (a > 1.0) a = 1.0;
    const double dV = s.V[b + 1] - s.V[b];
    *y = s.Acum[b] + s.W[b] * (a * s.V[b] + 0.5 * a * a * dV);
    *pdf = s.V[b] + a * dV;
    return b;
}

/* Inverse CDF: the bin whose CDF range holds y, then the root in [0,1] of
 * W_b dV/2 a^2 + W_b V_b a - (y - A_b) = 0, written without cancellation. */
int mcf_spline_inverse(const double raw[MCF_RAW], double y, double *u, double *pdf)
{
    spline_t s;
    spline_setup(raw, &s);
    const int b = bin_of(s.Acum, y);
    const double r = y - s.Acum[b];
    const double dV = s.V[b + 1] - s.V[b];
    double disc = s.V[b] * s.V[b] + 2.0 * dV * r / s.W[b];
    if (disc < 0.0) disc = 0.0;
    const double den = s.W[b] * (s.V[b] + sqrt(disc));
    double a = den > 0.0 ? 2.0 * r / den : 0.0;
    if (a < 0.0) a = 0.0;
    if (a > 1.0) a = 1.0;
    *u = s.X[b] + a * s.W[b];
    *pdf = s.V[b] + a * dV;
    return b;
}

/* Reverse-mode derivative of (y, pdf) at u with respect to the raw spline
 * values and to u, given gy = dL/dy and gp = dL/dpdf. */
static void spline_backward(const double raw[MCF_RAW], double u, double gy, double gp,
                            double graw[MCF_RAW], double *gu)
{
    spline_t s;
    spline_setup(raw, &s);
    const int b = bin_of(s.X, u);
    const double a = (u - s.X[b]) / s.W[b];
    const double dV = s.V[b + 1] - s.V[b];
    double gW[MCF_BINS] = {0}, gV[MCF_BINS + 1] = {0};
    /* y = A_b + W_b (a V_b + a^2 dV / 2), pdf = V_b + a dV */
    const double ga = gy * s.W[b] * (s.V[b] + a * dV) + gp * dV;
    gV[b] += gy * s.W[b] * (a - 0.5 * a * a) + gp * (1.0 - a);
    gV[b + 1] += gy * s.W[b] * 0.5 * a * a + gp * a;
    gW[b] += gy * (a * s.V[b] + 0.5 * a * a * dV);
    /* A_b = sum_{k<b} (V_k + V_{k+1}) W_k / 2 */
    for (int k = 0; k < b; ++k) {
        gV[k] += 0.5 * gy * s.W[k];
        gV[k + 1] += 0.5 * gy * s.W[k];
        gW[k] += 0.5 * gy * (s.V[k] + s.V[k + 1]);
    }
    /* a = (u - X_b) / W_b, X_b = sum_{k<b} W_k */
    *gu = ga / s.W[b];
    gW[b] += -ga * a / s.W[b];
    for (int k = 0; k < b; ++k) gW[k] += -ga / s.W[b];
    /* V_i = E_i / Z, Z = sum_{i<K} (E_i + E_{i+1}) W_i / 2 */
    double gZ = 0.0;
    double gE[MCF_BINS + 1];
    for (int i = 0; i <= MCF_BINS; ++i) {
        gE[i] = gV[i] / s.Z;
        gZ += -gV[i] * s.V[i] / s.Z;
    }
    for (int i = 0; i < MCF_BINS; ++i) {
        gE[i] += gZ * 0.5 * s.W[i];
        gE[i + 1] += gZ * 0.5 * s.W[i];
        gW[i] += gZ * 0.5 * (s.E[i] + s.E[i + 1]);
    }
    /* E_i = exp(raw height_i - max): d/draw = E_i (the max cancels in V) */
    for (int i = 0; i <= MCF_BINS; ++i) graw[MCF_BINS + i] = gE[i] * s.E[i];
    /* W = softmax(raw widths) */
    double dot = 0.0;
    for (int k = 0; k < MCF_BINS; ++k) dot += gW[k] * s.W[k];
    for (int k = 0; k < MCF_BINS; ++k) graw[k] = s.W[k] * (gW[k] - dot);
}

/* ------------------------------------------------------------------------ */
/* The conditioner network                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double e[MCF_IN];
    double h1[MCF_HID], h2[MCF_HID]; /* after ReLU */
    double out[MCF_OUT];
} cond_cache_t;

static double blob_center(int k) { return ((double)k + 0.5) / (double)MCF_BLOBS; }

static void conditioner(const double *P, const double ua[MCF_NA], int use_bf16, cond_cache_t *c)
{
    const double *W1 = P + OFF_W1, *b1 = P + OFF_B1, *W2 = P + OFF_W2, *b2 = P + OFF_B2;
    const double *W3 = P + OFF_W3, *b3 = P + OFF_B3;
    for (int a = 0; a < MCF_NA; ++a)
        for (int k = 0; k < MCF_BLOBS; ++k) {
            const double t = (ua[a] - blob_center(k)) * (double)MCF_BLOBS;
            const double e = exp(-0.5 * t * t);
            c->e[a * MCF_BLOBS + k] = use_bf16 ? bf16(e) : e;
        }
    for (int o = 0; o < MCF_HID; ++o) {
        double s = 0.0;
        for (int i = 0; i < MCF_IN; ++i)
            s += c->e[i] * (use_bf16 ? bf16(W1[i * MCF_HID + o]) : W1[i * MCF_HID + o]);
        s += use_bf16 ? (double)(float)b1[o] : b1[o];
        const double h = s > 0.0 ? s : 0.0;
        c->h1[o] = use_bf16 ? bf16(h) : h;
    }
    for (int o = 0; o < MCF_HID; ++o) {
        double s = 0.0;
        for (int i = 0; i < MCF_HID; ++i)
            s += c->h1[i] * (use_bf16 ? bf16(W2[i * MCF_HID + o]) : W2[i * MCF_HID + o]);
        s += use_bf16 ? (double)(float)b2[o] : b2[o];
        const double h = s > 0.0 ? s : 0.0;
        c->h2[o] = use_bf16 ? bf16(h) : h;
    }
    for (int o = 0; o < MCF_OUT; ++o) {
        double s = 0.0;
        for (int i = 0; i < MCF_HID; ++i)
            s += c->h2[i] * (use_bf16 ? bf16(W3[i * MCF_OUT + o]) : W3[i * MCF_OUT + o]);
        s += use_bf16 ? (double)(float)b3[o] : b3[o];
        c->out[o] = s;
    }
}

void mcf_conditioner(const double *layer_params, const double ua[MCF_NA], int use_bf16,
                     double out[MCF_OUT])
{
    cond_cache_t c;
    conditioner(layer_params, ua, use_bf16, &c);
    memcpy(out, c.out, sizeof c.out);
}

/* ------------------------------------------------------------------------ */
/* Density (x -> z) and sampling (z -> x)                                    */
/* ------------------------------------------------------------------------ */
void mcf_density(const double *theta, const double x[MCF_D], int use_bf16, double z[MCF_D],
                 double *logq)
{
    double u[MCF_D];
    memcpy(u, x, sizeof u);
    double lq = 0.0;
    for (int l = 0; l < MCF_LAYERS; ++l) {
        double ua[MCF_NA];
        for (int t = 0; t < MCF_NA; ++t) ua[t] = u[A_IDX[l][t]];
        cond_cache_t c;
        conditioner(theta + (size_t)l * MCF_LAYER_PARAMS, ua, use_bf16, &c);
        for (int t = 0; t < MCF_NB; ++t) {
            const int j = B_IDX[l][t];
            double y, pdf;
            mcf_spline_forward(c.out + t * MCF_RAW, u[j], &y, &pdf);
            u[j] = y;
            lq += log(pdf);
        }
    }
    memcpy(z, u, sizeof u);
    *logq = lq;
}

void mcf_sample(const double *theta, const double z[MCF_D], int use_bf16, double x[MCF_D],
                double *logq)
{
    double u[MCF_D];
    memcpy(u, z, sizeof u);
    double lq = 0.0;
    for (int l = MCF_LAYERS - 1; l >= 0; --l) {
        double ua[MCF_NA];
        for (int t = 0; t < MCF_NA; ++t) ua[t] = u[A_IDX[l][t]];
        cond_cache_t c;
        conditioner(theta + (size_t)l * MCF_LAYER_PARAMS, ua, use_bf16, &c);
        for (int t = 0; t < MCF_NB; ++t) {
            const int j = B_IDX[l][t];
            double v, pdf;
            mcf_spline_inverse(c.out + t * MCF_RAW, u[j], &v, &pdf);
            u[j] = v;
            lq += log(pdf);
        }
    }
    memcpy(x, u, sizeof u);
    *logq = lq;
}

/* ------------------------------------------------------------------------ */
/* Training loss and its gradient                                           */
/*                                                                          */
/* loss = -sum_s w_s log q(x_s) / sum_s w_s, by reverse-mode                */
/* differentiation through the four coupling layers (the chain rule over    */
/* the spline CDFs, the output layer, the two ReLU layers and the one-blob  */
/* encoding).                                                               */
/*                                                                          */
/* use_bf16 = 0: FP64 throughout.  use_bf16 = 1: the same sums with the     */
/* operands of every matrix product rounded to bfloat16, as a matrix unit   */
/* with BF16 inputs and wide accumulation computes them: the forward        */
/* conditioner as in mcf_conditioner(bf16 = 1); in the backward pass the    */
/* spline-parameter deltas, and the deltas after each ReLU, are rounded     */
/* before they meet the (rounded) weights, and the weight gradients are     */
/* sums of products of rounded operands (inputs h1, h2 and the encoding as  */
/* the forward pass rounded them); bias gradients sum the rounded deltas.   */
/* The derivative of the encoding itself (de/du) is taken exactly.          */
/*                                                                          */
/* grad_abs (may be NULL) receives, per parameter, the sum over samples of  */
/* the absolute values of the terms that make up its gradient: the scale    */
/* against which rounding differences in those terms are measured.         */
/* ------------------------------------------------------------------------ */
static double loss_grad(const double *theta, int64_t n, const double *xs, const double *ws,
                        int use_bf16, double *grad, double *grad_abs)
{
#define RND(v) (use_bf16 ? bf16(v) : (v))
    double sw = 0.0;
    for (int64_t i = 0; i < n; ++i) sw += ws[i];
    memset(grad, 0, sizeof(double) * MCF_PARAMS);
    if (grad_abs) memset(grad_abs, 0, sizeof(double) * MCF_PARAMS);
    double loss = 0.0;
    cond_cache_t cache[MCF_LAYERS];
    double uin[MCF_LAYERS][MCF_D];
    for (int64_t s = 0; s < n; ++s) {
        const double c = -ws[s] / sw; /* loss = sum_s c_s log q(x_s) */
        double u[MCF_D];
        memcpy(u, xs + s * MCF_D, sizeof u);
        double lq = 0.0;
        for (int l = 0; l < MCF_LAYERS; ++l) {
            memcpy(uin[l], u, sizeof u);
            double ua[MCF_NA];
            for (int t = 0; t < MCF_NA; ++t) ua[t] = u[A_IDX[l][t]];
            conditioner(theta + (size_t)l * MCF_LAYER_PARAMS, ua, use_bf16, &cache[l]);
            for (int t = 0; t < MCF_NB; ++t) {
                const int j = B_IDX[l][t];
                double y, pdf;
                mcf_spline_forward(cache[l].out + t * MCF_RAW, u[j], &y, &pdf);
                u[j] = y;
                lq += log(pdf);
            }
        }
        loss += c * lq;
        /* backward: g = dL/du at the output of the current layer */
        double g[MCF_D] = {0};
        for (int l = MCF_LAYERS - 1; l >= 0; --l) {
            const double *P = theta + (size_t)l * MCF_LAYER_PARAMS;
            double *G = grad + (size_t)l * MCF_LAYER_PARAMS;
            double *GA = grad_abs ? grad_abs + (size_t)l * MCF_LAYER_PARAMS : NULL;
            const cond_cache_t *cc = &cache[l];
            double gout[MCF_OUT];
            double gprev[MCF_D];
            memcpy(gprev, g, sizeof g);
            for (int t = 0; t < MCF_NB; ++t) {
                const int j = B_IDX[l][t];
                double y, pdf;
                mcf_spline_forward(cc->out + t * MCF_RAW, uin[l][j], &y, &pdf);
                double gu;
                spline_backward(cc->out + t * MCF_RAW, uin[l][j], g[j], c / pdf,
                                gout + t * MCF_RAW, &gu);
                gprev[j] = gu;
            }
            for (int o = 0; o < MCF_OUT; ++o) gout[o] = RND(gout[o]);
            /* output layer */
            double gh2[MCF_HID] = {0};
            for (int o = 0; o < MCF_OUT; ++o) {
                G[OFF_B3 + o] += gout[o];
                if (GA) GA[OFF_B3 + o] += fabs(gout[o]);
                for (int i = 0; i < MCF_HID; ++i) {
                    G[OFF_W3 + i * MCF_OUT + o] += cc->h2[i] * gout[o];
                    if (GA) GA[OFF_W3 + i * MCF_OUT + o] += fabs(cc->h2[i] * gout[o]);
                    gh2[i] += RND(P[OFF_W3 + i * MCF_OUT + o]) * gout[o];
                }
            }
            /* second hidden layer (ReLU: zero where the output is zero) */
            double gh1[MCF_HID] = {0};
            for (int o = 0; o < MCF_HID; ++o) {
                const double d = RND(cc->h2[o] > 0.0 ? gh2[o] : 0.0);
                G[OFF_B2 + o] += d;
                if (GA) GA[OFF_B2 + o] += fabs(d);
                for (int i = 0; i < MCF_HID; ++i) {
                    G[OFF_W2 + i * MCF_HID + o] += cc->h1[i] * d;
                    if (GA) GA[OFF_W2 + i * MCF_HID + o] += fabs(cc->h1[i] * d);
                    gh1[i] += RND(P[OFF_W2 + i * MCF_HID + o]) * d;
                }
            }
            /* first hidden layer and the encoding */
            double ge[MCF_IN] = {0};
            for (int o = 0; o < MCF_HID; ++o) {
                const double d = RND(cc->h1[o] > 0.0 ? gh1[o] : 0.0);
                G[OFF_B1 + o] += d;
                if (GA) GA[OFF_B1 + o] += fabs(d);
                for (int i = 0; i < MCF_IN; ++i) {
                    G[OFF_W1 + i * MCF_HID + o] += cc->e[i] * d;
                    if (GA) GA[OFF_W1 + i * MCF_HID + o] += fabs(cc->e[i] * d);
                    ge[i] += RND(P[OFF_W1 + i * MCF_HID + o]) * d;
                }
            }
            for (int a = 0; a < MCF_NA; ++a) {
                const int j = A_IDX[l][a];
                for (int k = 0; k < MCF_BLOBS; ++k) {
                    const double t = (uin[l][j] - blob_center(k)) * (double)MCF_BLOBS;
                    /* de/du = -e t * 32, with e the unrounded bump */
                    const double e = exp(-0.5 * t * t);
                    gprev[j] += ge[a * MCF_BLOBS + k] * (-e * t * (double)MCF_BLOBS);
                }
            }
            memcpy(g, gprev, sizeof g);
        }
    }
    return loss;
#undef RND
}

double mcf_loss_grad(const double *theta, int64_t n, const double *xs, const double *ws,
                     double *grad)
{
    return loss_grad(theta, n, xs, ws, 0, grad, NULL);
}

double mcf_loss_grad_ex(const double *theta, int64_t n, const double *xs, const double *ws,
                        int use_bf16, double *grad, double *grad_abs)
{
    return loss_grad(theta, n, xs, ws, use_bf16 != 0, grad, grad_abs);
}

/* One Adam step (Kingma & Ba, 2015) with bias correction; step counts from 1. */
void mcf_adam(double *theta, double *m, double *v, const double *grad, int64_t count, int step,
              double lr, double beta1, double beta2, double eps)
{
    const double c1 = 1.0 - pow(beta1, (double)step);
    const double c2 = 1.0 - pow(beta2, (double)step);
    for (int64_t i = 0; i < count; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        const double mh = m[i] / c1, vh = v[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* One m-Cubes iteration with the flow as the map: cube c's sample k draws  */
/* u from Philox exactly as V-Sample does, sets z_j = (c_j + u_j) / g,       */
/* x = flow sample of z and weighs w = f(x) / q(x).  Cube sums and unbiased */
/* in-cube variances are accumulated as in mco_sample_range.                */
/* ------------------------------------------------------------------------ */
static void nadd(double *s, double *c, double v)
{
    const double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

int mcf_proposal_range(const double *theta, int use_bf16, int family, const double *params,
                       int64_t g, int64_t m, int64_t p, uint64_t seed, uint32_t stream,
                       uint32_t iteration, int64_t c_begin, int64_t c_end, double sums[2])
{
    const int nblk = (MCF_D + 3) / 4;
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    double ss = 0.0, sc = 0.0, vs = 0.0, vc = 0.0;
    if (c_begin < 0 || c_end > m || p < 2) return -1;
    for (int64_t c = c_begin; c < c_end; ++c) {
        int64_t digit[MCF_D], rest = c;
        for (int j = 0; j < MCF_D; ++j) {
            digit[j] = rest % g;
            rest /= g;
        }
        double S = 0.0, D1 = 0.0, D2 = 0.0, w0 = 0.0;
        for (int64_t k = 0; k < p; ++k) {
            double z[MCF_D];
            for (int b = 0; b < nblk; ++b) {
                const uint32_t ctr[4] = {(uint32_t)c, stream, (uint32_t)(k * nblk + b), iteration};
                uint32_t r[4];
                mco_philox4x32_10(ctr, key, r);
                for (int l = 0; l < 4 && 4 * b + l < MCF_D; ++l)
                    z[4 * b + l] = ((double)digit[4 * b + l] + mco_uniform(r[l])) / (double)g;
            }
            double x[MCF_D], lq;
            mcf_sample(theta, z, use_bf16, x, &lq);
            const double w = mco_integrand(family, MCF_D, params, x) / exp(lq);
            S = S + w;
            if (k == 0) w0 = w;
            const double dlt = w - w0;
            D1 = D1 + dlt;
            D2 = D2 + dlt * dlt;
        }
        nadd(&ss, &sc, S);
        nadd(&vs, &vc, (D2 - D1 * D1 / (double)p) / (double)(p - 1));
    }
    sums[0] = ss + sc;
    sums[1] = vs + vc;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Combination of flow-mapped iterations t = 0..T-1.  Every one of them     */
/* samples the same fixed proposal with the same number of points, so the   */
/* estimates are independent draws of one distribution and the plain mean   */
/* is the unbiased combination (weighting by the estimated variances, as    */
/* VEGAS does for iterations whose map changes, favours the iterations that */
/* missed the rare large weights):                                          */
/*   Ibar = sum(I_t) / T.                                                   */
/* Its error is the standard deviation of that mean (the error model of     */
/* m-Cubes), estimated two ways, the larger one reported:                   */
/*   from the iterations' own variances   s_w^2 = sum(v_t) / T^2,           */
/*   from the scatter of their estimates  s_b^2 = sum (I_t - Ibar)^2        */
/*                                               / (T (T - 1))  (T >= 2).   */
/* With importance weights of a long tail an iteration's own variance       */
/* misses the rare large weights it did not draw; an iteration that drew    */
/* one stands out from the others, which the scatter sees.                  */
/*   chi2/dof = sum over v_t > 0 of (I_t - Ibar)^2 / v_t, over (T - 1)        */
/*   (0 when T = 1).                                                         */
/* out = [Ibar, sigma, chi2/dof]; returns the degrees of freedom T - 1.      */
/* ------------------------------------------------------------------------ */
int mcf_combine_equal(int T, const double *I, const double *var, double out[3])
{
    if (T < 1) {
        out[0] = 0.0;
        out[1] = INFINITY;
        out[2] = 0.0;
        return 0;
    }
    double si = 0.0, sv = 0.0;
    for (int t = 0; t < T; ++t) {
        si = si + I[t];
        sv = sv + var[t];
    }
    const double Ibar = si / (double)T;
    double chi2 = 0.0, ss = 0.0;
    for (int t = 0; t < T; ++t) {
        const double dv = I[t] - Ibar;
        ss = ss + dv * dv;
        if (var[t] > 0.0) chi2 = chi2 + dv * dv / var[t];
    }
    const double s_w = sqrt(sv) / (double)T;
    const double s_b = T > 1 ? sqrt(ss / ((double)T * (double)(T - 1))) : 0.0;
    out[0] = Ibar;
    out[1] = s_b > s_w ? s_b : s_w;
    out[2] = (T > 1) ? chi2 / (double)(T - 1) : 0.0;
    return T - 1;
}
