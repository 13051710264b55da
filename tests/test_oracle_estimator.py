"""Pins of the per-iteration estimator of Alg. 2 and of the whole integrator.

* a constant integrand on the uniform grid gives exactly 1 with zero variance;
* at a fixed non-uniform grid the iteration estimate is unbiased (mean over
  many Philox seeds vs the closed form) and its variance estimate is
  calibrated (spread over seeds vs the mean reported variance), for p = 2 and
  p > 2 samples per cube;
* every sample adds w^2 to exactly one bin per axis, so all axes carry the
  same total;
* sums over cube ranges add up to the full iteration;
* end to end the combined estimate covers the closed form at the stated
  error, including the paper's f1-f6.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import closed_forms as cf


def random_grid(rng, dim, nb):
    g = np.zeros((dim, nb + 1))
    for j in range(dim):
        w = rng.gamma(2.0, size=nb)
        g[j, 1:] = np.cumsum(w) / w.sum()
        g[j, -1] = 1.0
    return g


def test_constant_integrand_is_exact():
    # Gaussian with a = 0 is f = 1; on the uniform grid w = J = 1 up to rounding
    dim, nb = 4, 50
    I, var, bins = oracle.iteration(3, [0.0] * dim + [0.5] * dim, dim, nb, 5000, 0, 0,
                                    oracle.uniform_grid(dim, nb))
    assert abs(I - 1.0) < 1e-14
    assert var < 1e-28


@pytest.mark.parametrize("dim,ncall,p", [(2, 200, 2), (2, 17, 4), (3, 100, 3)])
def test_unbiased_and_calibrated(dim, ncall, p):
    rng = np.random.default_rng(dim * 1000 + ncall)
    nb = 12
    grid = random_grid(rng, dim, nb)
    params = list(rng.uniform(2, 5, dim)) + list(rng.uniform(0.3, 0.7, dim))
    exact = float(cf.integral(3, params, dim))
    assert oracle.plan(dim, ncall)[2] == p
    Is, Vs = [], []
    for seed in range(4000):
        I, v, _ = oracle.iteration(3, params, dim, nb, ncall, seed, 0, grid)
        Is.append(I)
        Vs.append(v)
    Is, Vs = np.array(Is), np.array(Vs)
    se = Is.std(ddof=1) / math.sqrt(len(Is))
    assert abs(Is.mean() - exact) < 4.5 * se
    ratio = Is.var(ddof=1) / Vs.mean()
    assert 0.88 < ratio < 1.12, ratio


def test_bins_are_consistent_across_axes():
    dim, nb = 5, 30
    rng = np.random.default_rng(1)
    grid = random_grid(rng, dim, nb)
    params = list(rng.uniform(2, 6, dim)) + list(rng.uniform(0.2, 0.8, dim))
    _, _, bins = oracle.iteration(1, params, dim, nb, 20000, 3, 2, grid)
    tot = bins.sum(axis=1)
    assert np.all(np.abs(tot - tot[0]) <= 1e-13 * tot[0])
    assert np.all(bins >= 0)


def test_bins_hold_squared_weights():
    """On the uniform grid J = 1, so bin i of axis j collects f^2 over the samples whose
    x_j falls in it: its expectation over N samples is N * int_{bin i} f_j^2 dx_j *
    prod_{k != j} int f_k^2 for the separable Gaussian f = prod_j exp(-a_j^2 (x_j-u_j)^2),
    and f^2 is again a Gaussian with a_j -> sqrt(2) a_j."""
    from scipy.special import erf
    dim, nb, ncall = 2, 8, 400_000
    a = np.array([3.0, 5.0])
    u = np.array([0.4, 0.7])
    _, _, bins = oracle.iteration(3, list(a) + list(u), dim, nb, ncall, 21, 0,
                                  oracle.uniform_grid(dim, nb))
    n = oracle.plan(dim, ncall)[3]
    b = np.sqrt(2.0) * a
    edges = np.arange(nb + 1) / nb
    for j in range(dim):
        cdf = erf(b[j] * (edges - u[j]))
        per_bin = np.sqrt(np.pi) / (2 * b[j]) * np.diff(cdf)
        other = [np.sqrt(np.pi) / (2 * b[k]) * (erf(b[k] * (1 - u[k])) + erf(b[k] * u[k]))
                 for k in range(dim) if k != j]
        expect = n * per_bin * np.prod(other)
        big = expect > 0.05 * expect.max()
        assert np.allclose(bins[j][big], expect[big], rtol=0.05), (j, bins[j], expect)


def test_ranges_add_up_and_counters_matter():
    dim, nb, ncall = 3, 40, 30000
    g, m, p, _ = oracle.plan(dim, ncall)
    rng = np.random.default_rng(6)
    grid = random_grid(rng, dim, nb)
    params = list(rng.uniform(2, 6, dim)) + list(rng.uniform(0.2, 0.8, dim))
    full = oracle.sample_range(3, params, dim, nb, g, m, p, 9, 4, grid, 0, m)
    cut = [0, 1, m // 3, m // 2 + 7, m - 1, m]
    parts = [oracle.sample_range(3, params, dim, nb, g, m, p, 9, 4, grid, a, b)
             for a, b in zip(cut[:-1], cut[1:])]
    assert math.fsum(x[0] for x in parts) == pytest.approx(full[0], rel=1e-15)
    assert math.fsum(x[1] for x in parts) == pytest.approx(full[1], rel=1e-15)
    assert np.allclose(sum(x[2] for x in parts), full[2], rtol=1e-14, atol=0)
    empty = oracle.sample_range(3, params, dim, nb, g, m, p, 9, 4, grid, 5, 5)
    assert empty[0] == 0.0 and empty[1] == 0.0 and not empty[2].any()
    other_it = oracle.sample_range(3, params, dim, nb, g, m, p, 9, 5, grid, 0, m)
    other_seed = oracle.sample_range(3, params, dim, nb, g, m, p, 10, 4, grid, 0, m)
    other_stream = oracle.sample_range(3, params, dim, nb, g, m, p, 9, 4, grid, 0, m, stream=1)
    for o in (other_it, other_seed, other_stream):
        assert o[0] != full[0]


def test_small_product_peak_covers_closed_form():
    pr = workloads.small_product_peak()
    r = oracle.integrate(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax, 0.0, pr.seed,
                         nb=pr.nbins)
    exact = float(cf.integral(pr.family, pr.params, pr.dim))
    assert r["iterations"] == 10 and r["rc"] == 0
    assert abs(r["estimate"] - exact) <= 3 * r["error"]
    assert 0.2 < r["chi2_dof"] < 3.0
    g = r["grid"]
    assert np.all(g[:, 0] == 0) and np.all(g[:, -1] == 1) and np.all(np.diff(g, axis=1) >= 0)


@pytest.mark.parametrize("k", range(1, 7))
def test_paper_integrands_5d(k):
    fam, params = cf.paper_params(k, 5)
    exact = float(cf.integral(fam, params, 5))
    r = oracle.integrate(fam, params, 5, 200_000, 8, 0.0, 11, nb=100)
    assert abs(r["estimate"] - exact) <= 4 * r["error"], (r["estimate"], exact, r["error"])


def test_coverage_over_seeds():
    """|Ibar - I| <= sigma in about 68% of runs and <= 2 sigma in about 95%."""
    params = [4.0, 7.0, 0.35, 0.6]
    exact = float(cf.integral(1, params, 2))
    within1 = within2 = 0
    n = 400
    for seed in range(n):
        r = oracle.integrate(1, params, 2, 4000, 5, 0.0, 1000 + seed, nb=50)
        z = abs(r["estimate"] - exact) / r["error"]
        within1 += z <= 1
        within2 += z <= 2
    assert 0.60 < within1 / n < 0.77, within1 / n
    assert 0.91 < within2 / n < 0.99, within2 / n


def test_stop_rule():
    params = [4.0, 7.0, 0.35, 0.6]
    r = oracle.integrate(1, params, 2, 20000, 50, 3e-5, 0, nb=50)
    assert r["converged"] and 3 <= r["iterations"] < 50
    assert r["error"] <= 3e-5 * abs(r["estimate"])
    r2 = oracle.integrate(1, params, 2, 20000, r["iterations"] - 1, 3e-5, 0, nb=50)
    assert not r2["converged"] and r2["iterations"] == r["iterations"] - 1
    assert r2["error"] > 3e-5 * abs(r2["estimate"])


def test_integrate_stream_is_the_second_counter_word():
    """integrate(stream=s) is the loop of iteration(stream=s), refine and
    combine (the stream word reaches every Philox counter), and differs from
    another stream's run only through the samples: both estimate the same
    integral within their errors."""
    params = [6.0, 3.0, 0.3, 0.7]
    r5 = oracle.integrate(3, params, 2, 6000, 3, 0.0, 4, nb=30, stream=5)
    grid = oracle.uniform_grid(2, 30)
    I, V = [], []
    for t in range(3):
        i_t, v_t, bins = oracle.iteration(3, params, 2, 30, 6000, 4, t, grid, stream=5)
        I.append(i_t)
        V.append(v_t)
        grid = oracle.refine(grid, bins)
    assert list(r5["trace_I"]) == I and list(r5["trace_var"]) == V
    assert np.array_equal(r5["grid"], grid)
    r0 = oracle.integrate(3, params, 2, 6000, 3, 0.0, 4, nb=30)
    assert r0["trace_I"][0] != r5["trace_I"][0]
    exact = float(cf.integral(3, params, 2))
    for r in (r0, r5):
        assert abs(r["estimate"] - exact) <= 4 * r["error"]
