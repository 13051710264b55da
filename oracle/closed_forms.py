"""Exact integrals over the unit cube of the integrand families -- TEST INFRASTRUCTURE.

The paper's benchmark integrands (eqs. 1-6, §5) and the addition integrand
(§5.3) are special cases of the parameterised Genz families evaluated by the
oracle.  Each integral factorises (or, for the corner peak, telescopes) and is
derived here by calculus; every function is evaluated with mpmath at 50
significant digits, or exactly with rational arithmetic where the closed form
cancels badly in floating point.

Families take params = [a_0..a_{d-1}, u_0..u_{d-1}] as in the oracle.
"""
from fractions import Fraction
from itertools import combinations
from math import factorial

import mpmath as mp

mp.mp.dps = 50


def _split(params, dim):
    a = [mp.mpf(float(v)) for v in params[:dim]]
    u = [mp.mpf(float(v)) for v in params[dim:2 * dim]]
    return a, u


def oscillatory(params, dim):
    """int cos(2 pi u_0 + sum a_i x_i) dx = Re[e^{2 pi i u_0} prod (e^{i a_j} - 1)/(i a_j)]."""
    a, u = _split(params, dim)
    z = mp.exp(mp.mpc(0, 1) * 2 * mp.pi * u[0])
    for aj in a:
        if aj == 0:
            continue
        z *= (mp.exp(mp.mpc(0, 1) * aj) - 1) / (mp.mpc(0, 1) * aj)
    return mp.re(z)


def product_peak(params, dim):
    """int prod (a^-2 + (x-u)^2)^-1 dx = prod a [atan(a (1-u)) + atan(a u)]."""
    a, u = _split(params, dim)
    r = mp.mpf(1)
    for aj, uj in zip(a, u):
        r *= aj * (mp.atan(aj * (1 - uj)) + mp.atan(aj * uj))
    return r


def corner_peak_exact(params, dim):
    """int (1 + sum a x)^-(d+1) dx = (1/(d! prod a)) sum_{S} (-1)^|S| / (1 + sum_{i in S} a_i).

    Integrating one axis at a time lowers the exponent by one and turns every
    term into a difference; the result is exact as a Fraction of the FP64
    parameters.
    """
    a = [Fraction(float(v)) for v in params[:dim]]
    total = Fraction(0)
    for k in range(dim + 1):
        for sub in combinations(range(dim), k):
            total += Fraction((-1) ** k) / (1 + sum((a[i] for i in sub), Fraction(0)))
    pa = Fraction(1)
    for v in a:
        pa *= v
    return total / (factorial(dim) * pa)


def corner_peak(params, dim):
    f = corner_peak_exact(params, dim)
    return mp.mpf(f.numerator) / mp.mpf(f.denominator)


def gaussian(params, dim):
    """int exp(-sum a^2 (x-u)^2) dx = prod sqrt(pi)/(2a) [erf(a(1-u)) + erf(a u)]."""
    a, u = _split(params, dim)
    r = mp.mpf(1)
    for aj, uj in zip(a, u):
        if aj == 0:
            continue
        r *= mp.sqrt(mp.pi) / (2 * aj) * (mp.erf(aj * (1 - uj)) + mp.erf(aj * uj))
    return r


def c0(params, dim):
    """int exp(-sum a |x-u|) dx = prod (2 - e^{-a u} - e^{-a (1-u)}) / a."""
    a, u = _split(params, dim)
    r = mp.mpf(1)
    for aj, uj in zip(a, u):
        r *= (2 - mp.exp(-aj * uj) - mp.exp(-aj * (1 - uj))) / aj
    return r


def discontinuous(params, dim):
    """int exp(sum a x) [x_i < u_i for all i] dx = prod (e^{a min(u,1)} - 1) / a."""
    a, u = _split(params, dim)
    r = mp.mpf(1)
    for aj, uj in zip(a, u):
        c = min(max(uj, mp.mpf(0)), mp.mpf(1))
        r *= (mp.exp(aj * c) - 1) / aj if aj != 0 else c
    return r


def addition(params, dim):
    """int sum x_i dx = d/2."""
    return mp.mpf(dim) / 2


def mixture(params, dim):
    """Equal mixture of N(m_k 1, s^2 [(1 - r) I + r 1 1^T]), k = 1, 2, over the
    unit cube (a_0 = s, a_1 = r >= 0, u_0 = m_1, u_1 = m_2).  An equicorrelated
    Gaussian vector is m + s (sqrt(1 - r) e_j + sqrt(r) h) with independent
    standard normals e_j, h; given h the coordinates are independent, so
      P(box) = int phi(h) [Phi((1 - m - s sqrt(r) h) / (s sqrt(1 - r)))
                           - Phi((-m - s sqrt(r) h) / (s sqrt(1 - r)))]^d dh."""
    s, r = mp.mpf(float(params[0])), mp.mpf(float(params[1]))
    total = mp.mpf(0)
    for m in (mp.mpf(float(params[dim])), mp.mpf(float(params[dim + 1]))):
        sd = s * mp.sqrt(1 - r)

        def integrand(h, m=m, sd=sd):
            c = m + s * mp.sqrt(r) * h
            return mp.npdf(h) * (mp.ncdf((1 - c) / sd) - mp.ncdf(-c / sd)) ** dim
        total += mp.quad(integrand, [-mp.inf, -10, -5, 0, 5, 10, mp.inf])
    return total / 2


BY_FAMILY = [oscillatory, product_peak, corner_peak, gaussian, c0, discontinuous, addition,
             mixture]


def integral(family, params, dim):
    """Exact integral (mpmath mpf) of family `family` with the given parameters."""
    return BY_FAMILY[family](params, dim)


def paper_params(k, dim):
    """Parameters that turn the families into the paper's f_k (eqs. 1-6); the
    choice is recorded once, in workloads.paper_integrand."""
    import workloads
    return workloads.paper_integrand(k, dim)
