"""Pins of the integrand families (eqs. 1-6 and the addition integrand of §5.3)
and of their closed-form integrals.

* The oracle's FP64 integrand values are compared with a 50-digit mpmath
  evaluation of the printed formulas at random points.
* The closed forms are compared with adaptive quadrature (mpmath.quad) in 1-D
  and 2-D, and the corner peak's exact rational form with scipy's nquad in 3-D.
* The table of the paper's f1-f6 closed forms in tests/golden is a regression
  pin written by tests/golden/make_paper_closed_forms.py.
"""
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate as sint

import oracle
from oracle import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_closed_forms.txt")


def _mp_formula(family, params, x):
    """The printed formulas, evaluated in 50-digit arithmetic."""
    d = len(x)
    a = [mp.mpf(v) for v in params[:d]]
    u = [mp.mpf(v) for v in params[d:2 * d]]
    x = [mp.mpf(v) for v in x]
    if family == 0:
        return mp.cos(2 * mp.pi * u[0] + sum(ai * xi for ai, xi in zip(a, x)))
    if family == 1:
        r = mp.mpf(1)
        for ai, ui, xi in zip(a, u, x):
            r *= 1 / (ai**-2 + (xi - ui) ** 2)
        return r
    if family == 2:
        return (1 + sum(ai * xi for ai, xi in zip(a, x))) ** (-(d + 1))
    if family == 3:
        return mp.exp(-sum(ai**2 * (xi - ui) ** 2 for ai, ui, xi in zip(a, u, x)))
    if family == 4:
        return mp.exp(-sum(ai * abs(xi - ui) for ai, ui, xi in zip(a, u, x)))
    if family == 5:
        if all(xi < ui for xi, ui in zip(x, u)):
            return mp.exp(sum(ai * xi for ai, xi in zip(a, x)))
        return mp.mpf(0)
    if family == 6:
        return sum(x)
    raise ValueError


@pytest.mark.parametrize("family", range(7))
@pytest.mark.parametrize("dim", [1, 3, 8, 10])
def test_integrand_matches_formula(family, dim):
    rng = np.random.default_rng(100 * family + dim)
    for _ in range(40):
        a = rng.uniform(0.5, 12.0, dim)
        u = rng.uniform(0.05, 1.1, dim)
        x = rng.uniform(0, 1, dim)
        params = list(a) + list(u)
        got = oracle.integrand(family, params, x)
        ref = _mp_formula(family, params, x)
        if family == 0:
            # cos near a zero: compare absolutely against the argument's size
            arg = abs(2 * np.pi * u[0]) + float(np.dot(a, x))
            assert abs(got - float(ref)) <= 8 * arg * 2.0**-53
        elif ref == 0:
            assert got == 0.0
        else:
            # exp(+-s) turns the few-ulp rounding of s into a relative error ~|s| ulp
            cond = 1.0 + (abs(float(mp.log(abs(ref)))) if family in (3, 4, 5) else 0.0)
            assert abs(got - float(ref)) <= 8 * dim * cond * 2.0**-53 * abs(float(ref)) + 1e-300


@pytest.mark.parametrize("family", range(7))
def test_closed_form_1d_matches_quadrature(family):
    rng = np.random.default_rng(7 + family)
    for _ in range(3):
        a = float(rng.uniform(1.0, 12.0))
        u = float(rng.uniform(0.1, 0.9))
        params = [a, u]
        exact = cf.integral(family, params, 1)
        f = lambda x: _mp_formula(family, params, [x])  # noqa: E731
        pts = [0, u, 1] if family in (4, 5) else [0, 1]
        quad = mp.quad(f, pts)
        assert abs(exact - quad) <= mp.mpf(1e-20) * (1 + abs(quad))


@pytest.mark.parametrize("family", range(7))
def test_closed_form_2d_matches_quadrature(family):
    rng = np.random.default_rng(70 + family)
    a = list(rng.uniform(1.0, 8.0, 2))
    u = list(rng.uniform(0.2, 0.8, 2))
    params = a + u
    exact = cf.integral(family, params, 2)
    old = mp.mp.dps
    mp.mp.dps = 20
    try:
        f = lambda x, y: _mp_formula(family, params, [x, y])  # noqa: E731
        if family in (4, 5):
            quad = mp.quad(f, [0, u[0], 1], [0, u[1], 1])
        else:
            quad = mp.quad(f, [0, 1], [0, 1])
    finally:
        mp.mp.dps = old
    assert abs(float(exact) - float(quad)) <= 1e-12 * (1 + abs(float(quad)))


def test_corner_peak_exact_3d_nquad():
    params = [1.5, 2.5, 0.75, 0, 0, 0]
    exact = float(cf.corner_peak(params, 3))
    val, err = sint.nquad(lambda x, y, z: (1 + 1.5 * x + 2.5 * y + 0.75 * z) ** -4,
                          [[0, 1]] * 3, opts={"epsabs": 1e-14, "epsrel": 1e-12})
    assert abs(val - exact) <= 1e-10 * exact


def test_paper_closed_form_table():
    """Regression pin: f1-f6 at d = 2..8 (values generated from the closed forms)."""
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, d, v = line.split()
            rows[(int(k), int(d))] = float(v)
    assert len(rows) == 6 * 7
    for (k, d), v in rows.items():
        fam, params = cf.paper_params(k, d)
        got = float(cf.integral(fam, params, d))
        assert got == pytest.approx(v, rel=1e-14), (k, d)
    # the 2-D entries are also pinned by direct 2-D quadrature (scipy, breakpoints at
    # the peaks and at the cut of f6)
    for k in range(1, 7):
        fam, params = cf.paper_params(k, 2)
        f = lambda y, x: float(_mp_formula(fam, params, [x, y]))  # noqa: E731
        pts = [[0.5], [0.5]] if k in (2, 4, 5) else ([[params[2]], [params[3]]] if k == 6
                                                       else [None, None])
        opts = [dict({"epsabs": 0.0, "epsrel": 1e-12, "limit": 200},
                     **({"points": pts[i]} if pts[i] else {})) for i in (1, 0)]
        q, _ = sint.nquad(f, [[0, 1], [0, 1]], opts=opts)
        assert q == pytest.approx(rows[(k, 2)], rel=1e-9), k
