"""Pins of the stratification plan (§3.2: m sub-cubes, a 2-point MC in each,
about ncall samples per iteration)."""
import pytest

import oracle


@pytest.mark.parametrize("dim", range(1, 11))
@pytest.mark.parametrize("ncall", [2, 3, 10, 1000, 10**5, 12345677, 2**26, 2**30, 3 * 10**9])
def test_plan_invariants(dim, ncall):
    g, m, p, n = oracle.plan(dim, ncall)
    half = ncall // 2
    assert g >= 1 and m == g**dim
    if g < 2**20:
        assert m <= half < (g + 1) ** dim      # g is the largest admissible cube side
    else:
        assert dim == 1 and g == 2**20 <= half  # at most 2^20 strata per axis
    assert p == max(2, ncall // m) and p >= 2
    assert n == m * p
    assert n <= ncall or m == 1 and n == 2 * 1  # never more samples than asked for (ncall >= 2)


def test_plan_known_sizes():
    # sizes worked out by hand from the rule
    assert oracle.plan(3, 100_000) == (36, 46656, 2, 93312)        # 36^3 <= 50000 < 37^3
    assert oracle.plan(8, 2**30) == (12, 429981696, 2, 859963392)  # 12^8 <= 2^29 < 13^8
    assert oracle.plan(10, 10**8) == (5, 9765625, 10, 97656250)
    assert oracle.plan(1, 2) == (1, 1, 2, 2)
    assert oracle.plan(2, 5) == (1, 1, 5, 5)
    # 1-D: at most 2^20 strata, so that digit + u (32 random bits) is exact
    assert oracle.plan(1, 2**21 + 1) == (2**20, 2**20, 2, 2**21)
    assert oracle.plan(1, 2**21 - 1) == (2**20 - 1, 2**20 - 1, 2, 2**21 - 2)
    assert oracle.plan(1, 3 * 10**9) == (2**20, 2**20, 2861, 2**20 * 2861)


def test_stratum_offset_is_exact_up_to_the_cap():
    # digit + (r + 1/2) 2^-32 is exact in FP64 for every digit below 2^20 (the
    # plan's cap), and first rounds at digit = 2^20
    import numpy as np
    rng = np.random.default_rng(5)
    from fractions import Fraction
    for digit in [0, 1, 2**19, 2**20 - 1] + list(rng.integers(0, 2**20, 50)):
        for r in [0, 1, 2**31, 2**32 - 1] + list(rng.integers(0, 2**32, 20)):
            exact = Fraction(int(digit)) + (Fraction(int(r)) + Fraction(1, 2)) / 2**32
            assert Fraction(float(digit) + oracle.uniform(int(r))) == exact
    exact = Fraction(2**20) + (Fraction(2**32 - 1) + Fraction(1, 2)) / 2**32
    assert Fraction(float(2**20) + oracle.uniform(2**32 - 1)) != exact


@pytest.mark.parametrize("dim,ncall", [(0, 100), (11, 100), (3, 1), (3, 0), (3, -5)])
def test_plan_rejects(dim, ncall):
    with pytest.raises(ValueError):
        oracle.plan(dim, ncall)
