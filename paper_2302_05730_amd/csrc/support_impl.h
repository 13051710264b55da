// Device bodies shared by the single-integrand and the batched support
// kernels: the inverse-variance combination of the iteration estimates and
// the VEGAS rebinning of one axis.
#pragma once

#include <math.h>

#include "mcubes_internal.h"

namespace mcubes {

// Records (It, Vt) as iteration t in `state` (layout of mcubes_combine) and
// recombines iterations skip..t.  One thread.  If no recorded iteration has
// zero variance the estimate is the inverse-variance weighted mean, its
// error (sum 1/var)^-1/2 and chi^2 the weighted squared deviations; an
// iteration with zero variance is exact and its estimate is taken as is.
__device__ __forceinline__ void combine_state(double It, double Vt, double *__restrict__ state,
                                              uint32_t t, int skip, double rel_tol) {
    double *hist = state + MCUBES_STATE_HEADER;
    hist[2 * t] = It;
    hist[2 * t + 1] = Vt;
    if (!isfinite(It) || !isfinite(Vt)) state[6] = 1.0;
    const int T = (int)t + 1;
    state[4] = (double)T;
    const int n = T - skip;
    double Ibar = 0.0, sigma = INFINITY, chi2dof = 0.0;
    int dof = 0;
    if (n >= 1) {
        double sw = 0.0, swi = 0.0;
        int exact = -1;
        for (int q = skip; q < T; ++q) {
            const double v = hist[2 * q + 1];
            if (v == 0.0) {
                exact = q;
            } else {
                sw = sw + 1.0 / v;
                swi = swi + hist[2 * q] / v;
            }
        }
        dof = n - 1;
        if (exact >= 0) {
            Ibar = hist[2 * exact];
            sigma = 0.0;
        } else {
            Ibar = swi / sw;
            double chi2 = 0.0;
            for (int q = skip; q < T; ++q) {
                const double dv = hist[2 * q] - Ibar;
                chi2 = chi2 + dv * dv / hist[2 * q + 1];
            }
            sigma = 1.0 / sqrt(sw);
            chi2dof = n > 1 ? chi2 / (double)(n - 1) : 0.0;
        }
    }
    state[0] = Ibar;
    state[1] = sigma;
    state[2] = chi2dof;
    state[3] = (double)dof;
    state[5] = (n >= 1 && sigma <= rel_tol * fabs(Ibar)) ? 1.0 : 0.0;
}

struct RefineLds {
    double E[kMaxBins + 1], d[kMaxBins], s[kMaxBins], r[kMaxBins], R[kMaxBins + 1];
    double tot;
};

// VEGAS rebinning of one axis by one block of at least nb + 1 threads, one
// thread per bin.  The two running sums (total smoothed weight, cumulative
// damped weight) are taken in bin order by one thread so that they round
// exactly like a sequential loop; the damping (log, pow) and the placement
// of the new edges run in parallel.  New edge k lies in the first old bin i
// whose cumulative damped weight reaches k T, found by binary search.  The
// old edges are read into LDS before any new edge is written, so En may be
// the same row as E.
__device__ __forceinline__ void refine_axis(const double *E, const double *__restrict__ dj,
                                            double *En, int nb, double alpha, RefineLds &L) {
    const int k = threadIdx.x;
    double *sE = L.E, *sd = L.d, *ss = L.s, *sr = L.r, *sR = L.R;

    if (k <= nb) sE[k] = E[k];
    if (k < nb) sd[k] = dj[k];
    __syncthreads();
    if (k < nb) {
        double s;
        if (k == 0)
            s = (sd[0] + sd[1]) / 2.0;
        else if (k == nb - 1)
            s = (sd[nb - 2] + sd[nb - 1]) / 2.0;
        else
            s = (sd[k - 1] + sd[k] + sd[k + 1]) / 3.0;
        ss[k] = s;
    }
    __syncthreads();
    if (k == 0) {
        double S = 0.0;
        for (int i = 0; i < nb; ++i) S = S + ss[i];
        L.tot = S;
    }
    __syncthreads();
    const double S = L.tot;
    if (!(S > 0.0)) {  // no weight on this axis: keep it
        if (k <= nb) En[k] = sE[k];
        return;
    }
    if (k < nb) {
        const double s = ss[k];
        const double rho = s / S;
        double r;
        if (s == 0.0)
            r = 0.0;
        else if (rho == 1.0)
            r = 1.0;
        else
            r = pow((rho - 1.0) / log(rho), alpha);
        sr[k] = r;
    }
    __syncthreads();
    if (k == 0) {
        double R = 0.0;
        sR[0] = 0.0;
        for (int i = 0; i < nb; ++i) {
            R = R + sr[i];
            sR[i + 1] = R;
        }
    }
    __syncthreads();
    const double T = sR[nb] / (double)nb;
    if (k == 0) {
        En[0] = 0.0;
        En[nb] = 1.0;
    } else if (k < nb) {
        const double target = (double)k * T;
        // first q in [1, nb] with R[q] >= target (nb if none), bin i = q - 1
        int lo = 1, hi = nb;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sR[mid] >= target)
                hi = mid;
            else
                lo = mid + 1;
        }
        const int i = lo - 1;
        const double W = sE[i + 1] - sE[i];
        double frac = (target - sR[i]) / sr[i];
        if (frac > 1.0) frac = 1.0;
        const double e = sE[i] + frac * W;
        En[k] = e < sE[i + 1] ? e : sE[i + 1];
    }
}

}  // namespace mcubes
