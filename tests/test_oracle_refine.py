"""Pins of the grid refinement (Lepage's VEGAS rebinning: smooth, damp,
re-divide into bins of equal damped weight).

* invariants: first edge 0, last edge 1, nondecreasing, widths sum to 1;
* each new bin holds the same damped weight (measured from the output edges
  by integrating the piecewise-constant weight density);
* an independent construction of the new edges with numpy (convolution for
  the smoothing, np.interp on the cumulative weight for the re-division);
* scale invariance in the contributions and the uniform fixed point.
"""
import numpy as np
import pytest

import oracle


def random_grid(rng, dim, nb):
    g = np.zeros((dim, nb + 1))
    for j in range(dim):
        w = rng.gamma(1.0, size=nb)
        g[j, 1:] = np.cumsum(w) / w.sum()
        g[j, -1] = 1.0
    return g


def _damped(bins, alpha):
    """Smoothing by convolution (1/2 at the ends, 1/3 inside) and the damping."""
    s = np.convolve(bins, np.ones(3), mode="same")
    s[1:-1] /= 3.0
    s[0] /= 2.0
    s[-1] /= 2.0
    rho = s / s.sum()
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(s > 0, ((rho - 1) / np.log(rho)) ** alpha, 0.0)
    return r


def _weight_in(edges_old, r, lo, hi):
    """Damped weight of [lo, hi] when bin i carries r_i spread uniformly."""
    tot = 0.0
    for i in range(len(r)):
        a, b = max(lo, edges_old[i]), min(hi, edges_old[i + 1])
        if b > a:
            tot += r[i] * (b - a) / (edges_old[i + 1] - edges_old[i])
    return tot


@pytest.mark.parametrize("dim,nb", [(1, 2), (2, 3), (3, 50), (8, 500)])
def test_refine_invariants(dim, nb):
    rng = np.random.default_rng(dim + nb)
    grid = random_grid(rng, dim, nb)
    bins = rng.gamma(0.5, size=(dim, nb)) ** 2
    bins[:, rng.integers(0, nb, size=max(1, nb // 10))] = 0.0
    new = oracle.refine(grid, bins)
    assert np.all(new[:, 0] == 0.0) and np.all(new[:, -1] == 1.0)
    assert np.all(np.diff(new, axis=1) >= 0)
    assert np.all(np.abs(np.diff(new, axis=1).sum(axis=1) - 1.0) <= nb * 2.0**-53)


@pytest.mark.parametrize("nb", [5, 40, 500])
def test_refine_equal_weight_and_numpy_construction(nb):
    rng = np.random.default_rng(nb)
    grid = random_grid(rng, 1, nb)
    bins = rng.gamma(0.8, size=(1, nb)) + 1e-3
    new = oracle.refine(grid, bins)[0]
    r = _damped(bins[0], 1.5)
    T = r.sum() / nb
    # every new bin holds the same damped weight
    for k in range(nb):
        assert _weight_in(grid[0], r, new[k], new[k + 1]) == pytest.approx(T, rel=1e-10)
    # independent construction: invert the piecewise-linear cumulative weight
    R = np.concatenate([[0.0], np.cumsum(r)])
    ref = np.interp(np.arange(1, nb) * T, R, grid[0])
    assert np.allclose(new[1:-1], ref, rtol=0, atol=1e-13)


def test_refine_zero_weight_bins_get_no_edges():
    rng = np.random.default_rng(4)
    nb = 30
    grid = random_grid(rng, 1, nb)
    bins = np.ones((1, nb))
    bins[0, 10:20] = 0.0  # after smoothing bins 11..18 carry no weight
    new = oracle.refine(grid, bins)[0]
    lo, hi = grid[0, 11], grid[0, 19]
    assert not np.any((new > lo) & (new < hi))


def test_refine_scale_invariance_and_fixed_point():
    rng = np.random.default_rng(8)
    grid = random_grid(rng, 3, 64)
    bins = rng.gamma(1.0, size=(3, 64))
    a = oracle.refine(grid, bins)
    assert np.array_equal(a, oracle.refine(grid, 4.0 * bins))     # powers of 2: bitwise
    assert np.allclose(a, oracle.refine(grid, 3.7 * bins), rtol=0, atol=1e-15)
    uni = oracle.uniform_grid(2, 100)
    same = oracle.refine(uni, np.full((2, 100), 0.25))
    # the running sum of the 100 equal weights carries ~100 ulp of rounding
    assert np.allclose(same, uni, rtol=0, atol=100 * 2.0**-53)


def test_refine_zero_contributions_keep_grid():
    rng = np.random.default_rng(2)
    grid = random_grid(rng, 2, 17)
    bins = np.zeros((2, 17))
    bins[1, 3] = 1.0
    new = oracle.refine(grid, bins)
    assert np.array_equal(new[0], grid[0])
    assert not np.array_equal(new[1], grid[1])


def test_refine_concentrates_on_peak():
    nb = 100
    grid = oracle.uniform_grid(1, nb)
    centres = (np.arange(nb) + 0.5) / nb
    bins = np.exp(-((centres - 0.3) / 0.05) ** 2)[None, :]
    new = oracle.refine(grid, bins)[0]
    widths = np.diff(new)
    assert widths[int(0.3 * nb)] < widths[int(0.9 * nb)]
