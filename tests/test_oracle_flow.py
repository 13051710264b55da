"""Pins of the flow oracle (the learned proposal) and of the mixture
integrand: each check rests on mathematics independent of the formula it
tests (quadrature of the density against the CDF, the Jacobian determinant of
the map by finite differences against the product of spline densities,
finite-difference gradients, invariances, a library bivariate normal CDF)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import workloads
from oracle import closed_forms as cf


def _raws(seed, n, scale=1.5):
    rng = np.random.default_rng(seed)
    return [rng.normal(scale=scale, size=oracle.FLOW_RAW) for _ in range(n)]


# ---------------------------------------------------------------- spline
def test_spline_identity_for_zero_parameters():
    raw = np.zeros(oracle.FLOW_RAW)
    for u in np.linspace(0, 1, 41):
        y, pdf, _ = oracle.spline_forward(raw, u)
        assert y == pytest.approx(u, abs=1e-15) and pdf == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_spline_cdf_is_the_integral_of_its_density(seed):
    """C(u) = int_0^u pdf, C(0) = 0, C(1) = 1, C increasing: the CDF formula
    against quadrature of the density formula (exact per bin: the density is
    linear there)."""
    raw = _raws(seed, 1)[0]
    pdf = lambda t: oracle.spline_forward(raw, t)[1]  # noqa: E731
    edges = np.concatenate([[0.0], np.cumsum(np.exp(raw[:16] - raw[:16].max())
                                             / np.exp(raw[:16] - raw[:16].max()).sum())])
    assert oracle.spline_forward(raw, 0.0)[0] == pytest.approx(0.0, abs=1e-15)
    assert oracle.spline_forward(raw, 1.0)[0] == pytest.approx(1.0, abs=1e-14)
    prev = -1.0
    for u in np.linspace(0, 1, 37):
        y = oracle.spline_forward(raw, u)[0]
        pts = [e for e in edges if 0 < e < u]
        q, _ = integrate.quad(pdf, 0.0, u, points=pts or None, limit=200, epsabs=1e-14)
        assert y == pytest.approx(q, abs=1e-11)
        assert y >= prev
        prev = y


@pytest.mark.parametrize("seed", range(5))
def test_spline_inverse_round_trip(seed):
    raw = _raws(100 + seed, 1)[0]
    for u in np.random.default_rng(seed).uniform(0, 1, 50):
        y, p1, b1 = oracle.spline_forward(raw, u)
        v, p2, b2 = oracle.spline_inverse(raw, y)
        assert v == pytest.approx(u, abs=1e-13)
        assert p2 == pytest.approx(p1, rel=1e-11)


def test_spline_invariances():
    """Adding a constant to all width logits or to all height logits leaves
    the spline unchanged (softmax and the height scaling are shift-free)."""
    raw = _raws(7, 1)[0]
    shifted = raw.copy()
    shifted[:16] += 3.7
    shifted[16:] -= 11.0
    for u in (0.01, 0.3, 0.77, 0.999):
        a, b = oracle.spline_forward(raw, u), oracle.spline_forward(shifted, u)
        assert a[0] == pytest.approx(b[0], rel=1e-13) and a[1] == pytest.approx(b[1], rel=1e-13)


# ------------------------------------------------------------------ flow
def test_zero_output_layer_is_the_identity():
    theta = workloads.flow_init(3)
    for x in np.random.default_rng(0).uniform(0, 1, (20, 6)):
        z, lq = oracle.flow_density(theta, x)
        assert np.array_equal(z, x) and lq == 0.0
        xs, lq2 = oracle.flow_sample(theta, x)
        assert np.array_equal(xs, x) and lq2 == 0.0


@pytest.mark.parametrize("seed", range(3))
def test_sample_and_density_are_inverse(seed):
    theta = workloads.flow_random(seed, out_scale=0.3)
    for z in np.random.default_rng(seed).uniform(0, 1, (30, 6)):
        x, lq = oracle.flow_sample(theta, z)
        z2, lq2 = oracle.flow_density(theta, x)
        assert np.allclose(z2, z, atol=1e-12)
        assert lq2 == pytest.approx(lq, abs=1e-10)
        assert np.all((x >= 0) & (x <= 1))


@pytest.mark.parametrize("seed", range(3))
def test_log_density_is_the_log_jacobian_of_the_map(seed):
    """log q(x) = log |det dz/dx|, the determinant taken numerically (central
    differences of the whole 6-D map) -- independent of the spline density
    formula and of the triangular structure."""
    theta = workloads.flow_random(10 + seed, out_scale=0.3)
    rng = np.random.default_rng(seed)
    h = 1e-6
    for x in rng.uniform(0.05, 0.95, (8, 6)):
        J = np.zeros((6, 6))
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            J[:, k] = (oracle.flow_density(theta, x + e)[0] - oracle.flow_density(theta, x - e)[0]) \
                / (2 * h)
        _, lq = oracle.flow_density(theta, x)
        assert math.log(abs(np.linalg.det(J))) == pytest.approx(lq, abs=2e-6)


def test_density_integrates_to_one():
    """E_{x ~ U(0,1)^6} q(x) = 1: Monte Carlo over 40000 uniform points."""
    theta = workloads.flow_random(21, out_scale=0.3)
    xs = np.random.default_rng(5).uniform(0, 1, (40000, 6))
    q = np.array([math.exp(oracle.flow_density(theta, x)[1]) for x in xs])
    se = q.std() / math.sqrt(len(q))
    assert abs(q.mean() - 1.0) <= 4 * se, (q.mean(), se)
    assert q.std() > 0.05  # the flow is not the identity


def test_loss_gradient_matches_finite_differences():
    """The analytic gradient of -sum w log q / sum w against central
    differences on parameters drawn from every block of every layer."""
    theta = workloads.flow_random(4, out_scale=0.4)
    rng = np.random.default_rng(9)
    xs = rng.uniform(0.02, 0.98, (6, 6))
    ws = rng.uniform(0.5, 2.0, 6)
    loss, grad = oracle.flow_loss_grad(theta, xs, ws)
    lq = np.array([oracle.flow_density(theta, x)[1] for x in xs])
    assert loss == pytest.approx(-(ws * lq).sum() / ws.sum(), rel=1e-12)
    L = oracle.FLOW_LAYER_PARAMS
    blocks = [(0, 96 * 64), (96 * 64, 64), (96 * 64 + 64, 64 * 64), (96 * 64 + 64 + 4096, 64),
              (96 * 64 + 128 + 4096, 64 * 99), (L - 99, 99)]
    idx = []
    for layer in range(4):
        for off, n in blocks:
            idx += list(layer * L + off + rng.choice(n, 3, replace=False))
    h = 1e-6
    bad = []
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (oracle.flow_loss_grad(tp, xs, ws)[0] - oracle.flow_loss_grad(tm, xs, ws)[0]) / (2 * h)
        if abs(fd - grad[i]) > 1e-6 * max(1.0, abs(fd)) + 1e-8:
            bad.append((i, fd, grad[i]))
    assert not bad, bad[:5]
    assert np.count_nonzero(grad) > 0.5 * len(grad)


def test_adam_first_steps():
    """Bias-corrected Adam moves every parameter by lr (times the sign of a
    constant gradient) on every step while |g| >> eps, and by nothing where
    the gradient is zero."""
    rng = np.random.default_rng(3)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    g[::7] = 0.0
    m = np.zeros(50)
    v = np.zeros(50)
    t = theta.copy()
    for step in range(1, 4):
        t, m, v = oracle.flow_adam(t, m, v, g, step, lr=1e-2, eps=1e-12)
        expect = theta - step * 1e-2 * np.sign(g)
        # |g| / (|g| + eps) differs from 1 by eps / |g| per step
        # (plus the rounding of the updates, a few ulp of theta)
        tol = step * (1e-2 * 1e-12 / np.maximum(np.abs(g), 1e-300) + 1e-15 * (1 + np.abs(theta)))
        assert np.all(np.abs(t - expect) <= np.where(g == 0, 0.0, tol))


# --------------------------------------------------------------- mixture
def _mixture_numpy(params, x):
    d = len(x)
    s, r, m1, m2 = params[0], params[1], params[d], params[d + 1]
    S = s * s * ((1 - r) * np.eye(d) + r * np.ones((d, d)))
    Si = np.linalg.inv(S)
    norm = 1.0 / math.sqrt((2 * math.pi) ** d * np.linalg.det(S))
    out = 0.0
    for m in (m1, m2):
        y = np.asarray(x) - m
        out += 0.5 * norm * math.exp(-0.5 * y @ Si @ y)
    return out


@pytest.mark.parametrize("dim,s,r", [(6, 0.05, 0.9), (2, 0.2, 0.5), (4, 0.1, 0.0), (3, 0.3, 0.7)])
def test_mixture_integrand_against_matrix_formula(dim, s, r):
    params = [s, r] + [0.0] * (dim - 2) + [1 / 3, 2 / 3] + [0.0] * (dim - 2)
    for x in np.random.default_rng(dim).uniform(0.2, 0.8, (20, dim)):
        ref = _mixture_numpy(params, x)
        got = oracle.integrand(oracle.MIXTURE, params, x)
        assert got == pytest.approx(ref, rel=1e-10, abs=1e-300)


def test_mixture_box_integral_against_bivariate_cdf():
    """The one-dimensional representation of the box probability against
    scipy's bivariate normal CDF (d = 2)."""
    s, r = 0.2, 0.6
    params = [s, r, 0.4, 0.7]
    cov = s * s * np.array([[1, r], [r, 1]])
    ref = 0.0
    for m in (0.4, 0.7):
        mvn = stats.multivariate_normal(mean=[m, m], cov=cov)
        ref += 0.5 * (mvn.cdf([1, 1]) - mvn.cdf([0, 1]) - mvn.cdf([1, 0]) + mvn.cdf([0, 0]))
    assert float(cf.mixture(params, 2)) == pytest.approx(ref, abs=2e-7)


def test_mixture_6d_integral_is_one_within_the_tail_bound():
    pr = workloads.mixture_6d()
    val = float(cf.mixture(pr.params, 6))
    assert 1.0 - 12 * stats.norm.cdf(-20 / 3) <= val <= 1.0


# -------------------------------------------------------- proposal iteration
def test_identity_flow_iteration_is_plain_mcubes_on_the_uniform_grid():
    """With the identity flow the proposal draws the same points as plain
    m-Cubes on a uniform grid (same Philox counters when the stream words
    agree) and q = 1 = J."""
    pr = workloads.mixture_6d()
    theta = workloads.flow_init(1)
    g, m, p, n = oracle.plan(6, 20000)
    a = oracle.flow_proposal_range(theta, pr.family, pr.params, g, m, p, 5, 0, 2, 0, m)
    b = oracle.sample_range(pr.family, pr.params, 6, 20, g, m, p, 5, 2,
                            oracle.uniform_grid(6, 20), 0, m)
    assert a[0] == pytest.approx(b[0], rel=1e-12) and a[1] == pytest.approx(b[1], rel=1e-10)


def test_flow_iteration_is_unbiased():
    """With a random flow the proposal estimate of a Gaussian integral is
    unbiased: the mean over 40 seeds is within 4 standard errors of the closed
    form, and the per-iteration variance estimate matches the spread."""
    theta = workloads.flow_random(2, out_scale=0.5)
    params = [4.0] * 6 + [0.45, 0.5, 0.55, 0.5, 0.4, 0.6]
    exact = float(cf.integral(oracle.GAUSSIAN, params, 6))
    g, m, p, n = oracle.plan(6, 3000)
    est, var = [], []
    for seed in range(40):
        s, v = oracle.flow_proposal_range(theta, oracle.GAUSSIAN, params, g, m, p, seed,
                                          0x80000000, 0, 0, m)
        I, V = oracle.estimates(m, p, s, v)
        est.append(I)
        var.append(V)
    est, var = np.array(est), np.array(var)
    se = est.std(ddof=1) / math.sqrt(len(est))
    assert abs(est.mean() - exact) <= 4 * se
    assert 0.5 < est.var(ddof=1) / var.mean() < 2.0
