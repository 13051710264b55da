"""Pins of the separable importance map (§3.2: a step-wise density mirroring
the integrand) and of its Jacobian.

For any monotone grid the change of variables must preserve the integral:
int_(0,1)^d f(x(y)) J(y) dy = int_(0,1)^d f(x) dx.  The left side is computed
with Gauss-Legendre rules on every bin of y-space (where the map is affine),
the right side is the closed form -- a wrong Jacobian factor, bin index or
edge interpolation breaks the identity.
"""
import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf


def random_grid(rng, dim, nb):
    g = np.zeros((dim, nb + 1))
    for j in range(dim):
        w = rng.gamma(0.7, size=nb)
        g[j, 1:] = np.cumsum(w) / w.sum()
        g[j, -1] = 1.0
    return g


@pytest.mark.parametrize("dim,nb", [(1, 2), (3, 10), (8, 500), (10, 137)])
def test_uniform_grid_is_identity(dim, nb):
    rng = np.random.default_rng(dim * nb)
    grid = oracle.uniform_grid(dim, nb)
    for _ in range(200):
        y = rng.uniform(0, 1, dim)
        x, J, bins = oracle.map_point(grid, y * nb)
        assert np.all(np.abs(x - y) <= 4 * 2.0**-53)
        # W = E[i+1] - E[i] cancels: its relative rounding error is up to ~nb ulp
        assert abs(J - 1.0) <= 2 * dim * (nb + 1) * 2.0**-53
        assert np.array_equal(bins, np.minimum(np.floor(y * nb), nb - 1).astype(np.int64))


def test_map_hits_edges_and_is_monotone():
    rng = np.random.default_rng(3)
    grid = random_grid(rng, 1, 9)
    for i in range(10):
        x, _, _ = oracle.map_point(grid, [float(i)])
        assert x[0] == pytest.approx(grid[0, i], abs=2e-16)
    ys = np.linspace(0, 1, 2001)
    xs = [oracle.map_point(grid, [9 * y])[0][0] for y in ys]
    assert np.all(np.diff(xs) >= 0)
    # y beyond the last cell is clamped into the last bin
    x, J, b = oracle.map_point(grid, [9.0])
    assert b[0] == 8 and x[0] == pytest.approx(1.0)


def _mapped_integral(family, params, grid, nodes=16):
    """int f(x(y)) J(y) dy over (0,1)^d by tensor Gauss-Legendre per y-bin."""
    dim, nbp1 = grid.shape
    nb = nbp1 - 1
    t, w = np.polynomial.legendre.leggauss(nodes)
    ys_1d = ((np.arange(nb)[:, None] + (t[None, :] + 1) / 2) / nb).ravel()
    ws_1d = np.tile(w / 2 / nb, nb)
    total = 0.0
    mesh = np.meshgrid(*([np.arange(len(ys_1d))] * dim), indexing="ij")
    idx = np.stack([m.ravel() for m in mesh], axis=1)
    for row in idx:
        y = ys_1d[row]
        x, J, _ = oracle.map_point(grid, y * nb)
        total += np.prod(ws_1d[row]) * oracle.integrand(family, params, x) * J
    return total


@pytest.mark.parametrize("family", [0, 1, 2, 3, 6])
def test_jacobian_identity_1d(family):
    rng = np.random.default_rng(11 + family)
    grid = random_grid(rng, 1, 7)
    params = [float(rng.uniform(1, 4)), float(rng.uniform(0.2, 0.8))]
    got = _mapped_integral(family, params, grid, nodes=40)
    exact = float(cf.integral(family, params, 1))
    assert got == pytest.approx(exact, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("family", [0, 1, 3])
def test_jacobian_identity_2d(family):
    rng = np.random.default_rng(21 + family)
    grid = random_grid(rng, 2, 4)
    params = list(rng.uniform(1, 3, 2)) + list(rng.uniform(0.3, 0.7, 2))
    got = _mapped_integral(family, params, grid, nodes=14)
    exact = float(cf.integral(family, params, 2))
    assert got == pytest.approx(exact, rel=1e-12, abs=1e-14)
