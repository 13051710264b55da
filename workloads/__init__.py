"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module only draws integrand parameters and names problem sizes; it holds
none of the integrator's arithmetic.  Parameters come from numpy's PCG64
``default_rng(seed)``, so they are identical on every machine.

Families (ids shared with the C interface): 0 oscillatory, 1 product peak,
2 corner peak, 3 Gaussian, 4 C0, 5 discontinuous, 6 addition.  The paper's
benchmark integrands (eqs. 1-6, §5) are members of the first six families.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS, ADDITION, MIXTURE = range(8)
FAMILY_NAMES = ["oscillatory", "product_peak", "corner_peak", "gaussian", "c0",
                "discontinuous", "addition", "mixture"]


@dataclass
class Problem:
    name: str
    family: int
    dim: int
    params: List[float]
    ncall: int
    nbins: int = 500
    itmax: int = 10
    rel_tol: float = 0.0
    seed: int = 0
    extra: dict = field(default_factory=dict)


def genz_params(rng, dim, a_lo, a_hi, u_lo, u_hi):
    a = rng.uniform(a_lo, a_hi, size=dim)
    u = rng.uniform(u_lo, u_hi, size=dim)
    return [float(v) for v in a] + [float(v) for v in u]


def small_product_peak():
    """3-D product peak, a_i = 5, u_i ~ U(0.2, 0.8) (parameter seed 0), 100 bins,
    1e5 samples per iteration, 10 iterations, Philox seed 0."""
    rng = np.random.default_rng(0)
    u = rng.uniform(0.2, 0.8, size=3)
    params = [5.0] * 3 + [float(v) for v in u]
    return Problem("product_peak_3d", PRODUCT_PEAK, 3, params, ncall=100_000, nbins=100,
                   itmax=10, rel_tol=0.0, seed=0)


# Parameter seeds of the three 8-D integrands of the large workload.
LARGE_SEEDS = {GAUSSIAN: 1, OSCILLATORY: 2, CORNER_PEAK: 3}


def large_8d(family, ncall=1 << 30, itmax=50, rel_tol=1e-4):
    """8-D Genz integrand with a_i ~ U(5, 15), u_i ~ U(0, 1), 500 bins, 2^30
    samples per iteration, up to 50 iterations, rel_tol 1e-4."""
    rng = np.random.default_rng(LARGE_SEEDS[family])
    params = genz_params(rng, 8, 5.0, 15.0, 0.0, 1.0)
    return Problem(f"{FAMILY_NAMES[family]}_8d", family, 8, params, ncall=ncall, nbins=500,
                   itmax=itmax, rel_tol=rel_tol, seed=0)


def large_8d_set(ncall=1 << 30, itmax=50, rel_tol=1e-4):
    return [large_8d(f, ncall, itmax, rel_tol) for f in (GAUSSIAN, OSCILLATORY, CORNER_PEAK)]


def paper_integrand(k, dim):
    """(family, params) of the paper's benchmark integrand f_k (eqs. 1-6, §5):
    f1 = cos(sum i x_i)                       oscillatory, a_i = i, u_0 = 0
    f2 = prod (1/50^2 + (x_i - 1/2)^2)^-1     product peak, a_i = 50, u_i = 1/2
    f3 = (1 + sum i x_i)^-(d+1)               corner peak, a_i = i
    f4 = exp(-625 sum (x_i - 1/2)^2)          Gaussian, a_i = 25, u_i = 1/2
    f5 = exp(-10 sum |x_i - 1/2|)             C0, a_i = 10, u_i = 1/2
    f6 = exp(sum (i+4) x_i) if x_i < (3+i)/10 discontinuous, a_i = i+4, u_i = (3+i)/10
    (i counts axes from 1); k = 7 is the addition integrand sum x_i of §5.3."""
    idx = range(1, dim + 1)
    if k == 1:
        return OSCILLATORY, [float(i) for i in idx] + [0.0] * dim
    if k == 2:
        return PRODUCT_PEAK, [50.0] * dim + [0.5] * dim
    if k == 3:
        return CORNER_PEAK, [float(i) for i in idx] + [0.0] * dim
    if k == 4:
        return GAUSSIAN, [25.0] * dim + [0.5] * dim
    if k == 5:
        return C0, [10.0] * dim + [0.5] * dim
    if k == 6:
        return DISCONTINUOUS, [float(i + 4) for i in idx] + [(3.0 + i) / 10.0 for i in idx]
    if k == 7:
        return ADDITION, [0.0] * (2 * dim)
    raise ValueError(k)


def random_problem(rng, family, dim, ncall, nbins):
    """A random member of a family with parameters in the ranges the paper's
    integrands span (a in [5, 15] scaled down for the peaked families at high
    dimension so that the integral stays representable)."""
    if family == ADDITION:
        params = [0.0] * (2 * dim)
    elif family == MIXTURE:
        s, r = rng.uniform(0.05, 0.3), rng.uniform(0.0, 0.95)
        m1, m2 = rng.uniform(0.2, 0.5), rng.uniform(0.5, 0.8)
        params = [float(s), float(r)] + [0.0] * (dim - 2) + [float(m1), float(m2)] + \
            [0.0] * (dim - 2)
    elif family == DISCONTINUOUS:
        params = genz_params(rng, dim, 1.0, 8.0, 0.3, 1.2)
    elif family == CORNER_PEAK:
        params = genz_params(rng, dim, 0.5, 5.0, 0.0, 1.0)
    else:
        params = genz_params(rng, dim, 2.0, 12.0, 0.0, 1.0)
    return Problem(f"{FAMILY_NAMES[family]}_{dim}d", family, dim, params, ncall=ncall,
                   nbins=nbins)


# Parameter seed of the batched workload.
BATCH_SEED = 4


def batch_problems(n=512, seed=BATCH_SEED, ncall_lo=1e6, ncall_hi=1e8, nbins=500,
                   families=(OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS),
                   dims=tuple(range(2, 11))):
    """n integrands for the batched form: family uniform over the six Genz
    families of the paper's benchmark, dimension uniform over 2..10, sample
    budget per iteration log-uniform in [ncall_lo, ncall_hi], parameters as in
    random_problem.  The default is the 512-integrand workload."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        fam = int(families[rng.integers(0, len(families))])
        dim = int(dims[rng.integers(0, len(dims))])
        ncall = int(round(float(np.exp(rng.uniform(np.log(ncall_lo), np.log(ncall_hi))))))
        pr = random_problem(rng, fam, dim, ncall, nbins)
        pr.name = f"batch{i}_{pr.name}"
        out.append(pr)
    return out


def mixture_6d(ncall=1 << 26, itmax=50, rel_tol=1e-3):
    """6-D equal mixture of two correlated Gaussians centred at 1/3 and 2/3 on
    the diagonal, standard deviation 0.05 and correlation 0.9 on every pair of
    axes; 2^26 samples per iteration.  Its integral over the unit cube is 1 to
    within 12 Phi(-20/3) ~ 1.6e-10 (the mass outside the cube)."""
    params = [0.05, 0.9] + [0.0] * 4 + [1.0 / 3.0, 2.0 / 3.0] + [0.0] * 4
    return Problem("mixture_6d", MIXTURE, 6, params, ncall=ncall, nbins=500, itmax=itmax,
                   rel_tol=rel_tol, seed=0)


def flow_init(seed=7, scale=1.0):
    """Initial flow parameters (67212 FP64 values in the layout of the flow):
    Glorot-uniform hidden weights (numpy PCG64, seeded) times `scale`, small
    hidden biases, and a zero output layer, so that the initial flow is the
    identity map with density 1."""
    return flow_random(seed, scale=scale, out_scale=0.0)


def flow_random(seed, scale=1.0, out_scale=0.1):
    """Random flow parameters for tests: Glorot-uniform weights times `scale`
    for the hidden layers and `out_scale` for the output layer, small random
    biases."""
    blobs, na, hid, bins, nb = 32, 3, 64, 16, 3
    n_in, n_out = na * blobs, nb * (2 * bins + 1)
    rng = np.random.default_rng(seed)
    parts = []
    for _ in range(4):
        lim1 = scale * np.sqrt(6.0 / (n_in + hid))
        lim2 = scale * np.sqrt(6.0 / (hid + hid))
        lim3 = out_scale * np.sqrt(6.0 / (hid + n_out))
        parts += [rng.uniform(-lim1, lim1, n_in * hid), rng.uniform(-0.05, 0.05, hid) * scale,
                  rng.uniform(-lim2, lim2, hid * hid), rng.uniform(-0.05, 0.05, hid) * scale,
                  rng.uniform(-lim3, lim3, hid * n_out),
                  rng.uniform(-1.0, 1.0, n_out) * out_scale]
    return np.concatenate(parts)
