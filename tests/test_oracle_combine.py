"""Pins of the combination of iteration estimates (Lepage's inverse-variance
weighting; the paper takes the error from the MC standard deviation, §3.2),
and of the equal-weight combination of flow-mapped iterations."""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def test_hand_example():
    # I = (1, 2, 4), var = (1, 1, 4): weights 1, 1, 1/4
    #   Ibar = (1 + 2 + 1) / (9/4) = 16/9,   sigma = (9/4)^(-1/2) = 2/3
    #   chi2 = (1-16/9)^2 + (2-16/9)^2 + (4-16/9)^2/4 = 49/81 + 4/81 + 100/81 = 153/81
    #   chi2/dof = 153/162 = 17/18
    Ibar, sigma, chi2, dof = oracle.combine([1.0, 2.0, 4.0], [1.0, 1.0, 4.0])
    assert Ibar == pytest.approx(float(Fraction(16, 9)), rel=1e-15)
    assert sigma == pytest.approx(2.0 / 3.0, rel=1e-15)
    assert chi2 == pytest.approx(float(Fraction(17, 18)), rel=1e-14)
    assert dof == 2


def test_skip_and_single():
    Ibar, sigma, chi2, dof = oracle.combine([5.0, 1.0, 2.0, 4.0], [9.0, 1.0, 1.0, 4.0], skip=1)
    assert Ibar == pytest.approx(16 / 9, rel=1e-15) and dof == 2
    Ibar, sigma, chi2, dof = oracle.combine([3.25], [0.0625])
    assert (Ibar, sigma, chi2, dof) == (3.25, 0.25, 0.0, 0)


def test_identical_iterations_have_zero_chi2():
    Ibar, sigma, chi2, dof = oracle.combine([2.5] * 6, [0.5] * 6)
    assert Ibar == 2.5 and chi2 == 0.0 and dof == 5
    assert sigma == pytest.approx((6 / 0.5) ** -0.5, rel=1e-15)


def test_exact_iteration_dominates():
    Ibar, sigma, chi2, dof = oracle.combine([1.0, 7.0, 1.5], [1.0, 0.0, 2.0])
    assert Ibar == 7.0 and sigma == 0.0


# --- equal-weight combination of flow-mapped iterations ---------------------
# Every flow-mapped iteration samples one fixed proposal with the same number
# of points, so the estimates are independent draws of one distribution: the
# plain mean is unbiased.  Its standard deviation is estimated from the
# iterations' variances (sum(var_t) / T^2) and from the scatter of their
# estimates (the standard error of a mean of T draws), the larger reported.


def test_flow_combine_hand_example():
    # I = (1, 2, 4), var = (1, 1, 4): Ibar = 7/3; within: sqrt(6)/3;
    # scatter: sum (I - Ibar)^2 = 42/9, over T (T - 1) = 6 -> 7/9, sqrt(7)/3
    # (the larger); chi2 = (4/3)^2 + (1/3)^2 + (5/3)^2/4 = 31/12, /dof 31/24
    Ibar, sigma, chi2, dof = oracle.flow_combine([1.0, 2.0, 4.0], [1.0, 1.0, 4.0])
    assert Ibar == pytest.approx(float(Fraction(7, 3)), rel=1e-15)
    assert sigma == pytest.approx(7 ** 0.5 / 3, rel=1e-15)
    assert chi2 == pytest.approx(float(Fraction(31, 24)), rel=1e-14)
    assert dof == 2
    # the same estimates with larger own variances: the within part wins
    Ibar, sigma, chi2, dof = oracle.flow_combine([1.0, 2.0, 4.0], [4.0, 4.0, 4.0])
    assert sigma == pytest.approx(12 ** 0.5 / 3, rel=1e-15)


def test_flow_combine_scatter_is_the_standard_error_of_the_mean():
    rng = np.random.default_rng(3)
    for T in (2, 4, 7, 30):
        I = rng.normal(1.0, 0.1, T)
        v = np.full(T, 1e-8)  # own variances far below the scatter
        sigma = oracle.flow_combine(I, v)[1]
        assert sigma == pytest.approx(np.std(I, ddof=1) / np.sqrt(T), rel=1e-13)


def test_flow_combine_within_part_reduces_to_inverse_variance():
    """Equal variances and a small scatter: the estimate, its error and chi2
    are those of inverse-variance weighting."""
    I = [1.0, 1.1, 0.95, 1.05, 1.02]
    v = [0.04] * 5
    a = oracle.flow_combine(I, v)
    b = oracle.combine(I, v)
    assert a[3] == b[3]
    for x, y in zip(a[:3], b[:3]):
        assert x == pytest.approx(y, rel=1e-14)


def test_flow_combine_single_and_empty():
    assert oracle.flow_combine([3.25], [0.0625]) == (3.25, 0.25, 0.0, 0)
    Ibar, sigma, chi2, dof = oracle.flow_combine([], [])
    assert (Ibar, chi2, dof) == (0.0, 0.0, 0) and sigma == float("inf")
    # an exact iteration (var 0) adds nothing to chi2 or to the within part;
    # the scatter of (2, 4) is sqrt(2 / 2) = 1
    Ibar, sigma, chi2, dof = oracle.flow_combine([2.0, 4.0], [0.0, 1.0])
    assert (Ibar, sigma, dof) == (3.0, 1.0, 1) and chi2 == 1.0


def test_flow_combine_is_unbiased_on_heavy_tailed_iterations():
    """Iterations = means of 200 log-normal(0, 1.5) draws (mean e^1.125, a
    long right tail like importance weights).  Over 3000 repetitions of 8
    iterations the equal-weight mean is unbiased and sigma^2 does not fall
    short of the scatter of Ibar (the larger of two estimates of it), while
    the inverse-variance mean is far too low: an iteration that caught a
    large draw also has a large variance estimate and is weighted down."""
    import math

    rng = np.random.default_rng(5)
    mu = math.exp(1.5 ** 2 / 2)
    eq, ivw, s2 = [], [], []
    for _ in range(3000):
        x = rng.lognormal(0.0, 1.5, size=(8, 200))
        I = x.mean(1)
        v = x.var(1, ddof=1) / 200
        a = oracle.flow_combine(I, v)
        eq.append(a[0] - mu)
        s2.append(a[1] ** 2)
        ivw.append(oracle.combine(I, v)[0] - mu)
    eq, ivw = np.array(eq), np.array(ivw)
    se = eq.std() / len(eq) ** 0.5
    assert abs(eq.mean()) < 4 * se
    assert 1.0 <= np.mean(s2) / eq.var() <= 2.0
    assert ivw.mean() < -20 * se


def test_flow_combine_scatter_raises_coverage_on_pareto_weights():
    """Four iterations, each the mean of 2000 Pareto weights of tail shape
    0.4 (finite variance, no finite fourth moment: the own-variance
    estimate is usually too small).  Taking the larger of the two error
    estimates covers the true mean at 2 sigma more often than the
    within-iteration estimate alone."""
    rng = np.random.default_rng(17)
    xi = 0.4
    mu = 1.0 / (1.0 - xi)  # mean of the Pareto with x_min 1, shape 1/xi
    hit_max = hit_w = 0
    R = 2000
    for _ in range(R):
        x = (1.0 - rng.random((4, 2000))) ** (-xi)
        I = x.mean(1)
        v = x.var(1, ddof=1) / 2000
        Ibar, sigma = oracle.flow_combine(I, v)[:2]
        s_w = np.sqrt(v.sum()) / 4
        hit_max += abs(Ibar - mu) <= 2 * sigma
        hit_w += abs(Ibar - mu) <= 2 * s_w
    assert hit_max > hit_w
    assert hit_max / R >= 0.85
