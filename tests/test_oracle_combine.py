"""Pins of the combination of iteration estimates (Lepage's inverse-variance
weighting; the paper takes the error from the MC standard deviation, §3.2)."""
from fractions import Fraction

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
