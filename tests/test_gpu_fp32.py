"""GPU parity of the FP32 precision form against the FP64 oracle.

The FP32 form draws the same samples into the same bins as the FP64 path
(bin coordinates stay FP64) and rounds only the map and the integrand to
FP32.  Bound on the relative error of one sample weight, delta:
  * the mapped point x = E + W phi in FP32 (E, W, phi each rounded once, one
    fma) is within 4 ulp_32 = 4 * 2^-24 of the exact map on every axis
    (x in [0, 1]);
  * that moves ln f by at most L_j * 4 * 2^-24 per axis, with L_j the largest
    |d ln f / d x_j| of the family over the unit cube;
  * evaluating f in FP32 adds at most (3 d + 8) * 2^-24 (one rounding per
    operation, 2 ulp for expf);
  * the Jacobian is formed in FP64 from the rounded widths: 2 d * 2^-24.
Then |I32 - I64| <= delta * mean |w| (<= delta |I| for positive integrands),
every bin (a sum of w^2) moves by at most 2 delta relative, and
var_t = sum (w1 - w0)^2 / 2 by at most 2 delta sqrt(Q / (2 sum var_c)).
The oscillatory family is bounded through the absolute error of cos
(its argument is off by at most sum_j a_j * 4 * 2^-24 + its own rounding).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import closed_forms as cf
from parity_util import random_grid

pytestmark = pytest.mark.gpu
U32 = 2.0**-24


@pytest.fixture(scope="module")
def mc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_05730_amd as m
    m.lib()
    return m


def lipschitz_log(family, params, dim):
    a = np.abs(np.array(params[:dim]))
    if family == 1:   # d/dx ln (a^-2 + t^2)^-1 = -2t / (a^-2 + t^2) <= a
        return a
    if family == 2:   # (d+1) a_j / (1 + sum a x) <= (d+1) a_j
        return (dim + 1) * a
    if family == 3:   # 2 a^2 |x - u| <= 2 a^2 max(u, 1 - u)
        u = np.array(params[dim:2 * dim])
        return 2 * a * a * np.maximum(np.abs(u), np.abs(1 - u))
    if family in (4, 5):
        return a
    if family == 6:   # d/dx ln(sum x) = 1 / sum x: bounded via the absolute error instead
        return np.zeros(dim)
    raise ValueError(family)


def delta(family, params, dim):
    return (float(np.sum(lipschitz_log(family, params, dim))) * 4 * U32
            + (3 * dim + 8) * U32 + 2 * dim * U32)


def gpu32(mc, plan, it, grid):
    import torch
    info = plan.info
    d_grid = torch.from_numpy(np.ascontiguousarray(grid).ravel()).cuda()
    d_bins = torch.zeros(info["bins_len"], dtype=torch.float64, device="cuda")
    d_part = torch.empty(info["partials_len"], dtype=torch.float64, device="cuda")
    d_est = torch.empty(2, dtype=torch.float64, device="cuda")
    mc.mcubes_vsample(plan, it, d_grid, d_bins, d_part)
    mc.mcubes_reduce(plan, d_part, d_est)
    torch.cuda.synchronize()
    I, v = d_est.cpu().tolist()
    return I, v, d_bins.cpu().numpy().reshape(info["dim"], info["nbins"])


CASES = [(3, 8, 500, 1_000_000), (3, 3, 100, 200_000), (1, 5, 64, 300_000), (2, 8, 500, 500_000),
         (4, 6, 200, 300_000), (5, 4, 50, 200_000), (6, 8, 500, 400_000), (0, 8, 500, 600_000),
         (0, 2, 30, 50_000), (1, 1, 17, 10_001)]


@pytest.mark.parametrize("family,dim,nb,ncall", CASES)
def test_fp32_form_against_fp64_oracle(mc, family, dim, nb, ncall):
    rng = np.random.default_rng(500 + 10 * family + dim)
    pr = workloads.random_problem(rng, family, dim, ncall, nb)
    grid = random_grid(rng, dim, nb)
    g, m, p, n = oracle.plan(dim, ncall)
    plan = mc.mcubes_plan_create(family, pr.params, dim, ncall, 11,
                                 mc.mcubes_default_options(nbins=nb, precision=mc.MCUBES_FP32))
    assert plan.info["precision"] == mc.MCUBES_FP32
    I, v, bins = gpu32(mc, plan, 2, grid)
    rI, rv, rbins = oracle.iteration(family, pr.params, dim, nb, ncall, 11, 2, grid)
    Q = float(rbins[0].sum())
    rms = math.sqrt(Q / n)
    if family == 0:
        arg_err = (float(np.sum(np.abs(pr.params[:dim]))) * 4 + 8) * U32 * 4
        tol_I = arg_err * rms * 2
        tol_bins = None
    else:
        d = delta(family, pr.params, dim)
        tol_I = d * (abs(rI) if family != 6 else rms) * 2 + 1e-300
        tol_bins = 4 * d
        if family == 6:
            tol_bins = 4 * (dim * 8 + 16) * U32
    print(f"family={family} dim={dim}: |dI|/I={abs(I - rI) / max(abs(rI), 1e-300):.2e} "
          f"(tol {tol_I / max(abs(rI), 1e-300):.2e})", flush=True)
    assert abs(I - rI) <= tol_I
    if tol_bins is not None:
        assert np.all(np.abs(bins - rbins) <= tol_bins * np.abs(rbins) + 1e-300)
        if rv > 0:
            tol_v = 2 * (tol_bins / 4) * math.sqrt(Q / (2 * rv * p * m * m)) * 2
            assert abs(v - rv) <= max(tol_v, 1e-9) * rv


@pytest.mark.parametrize("family", [3, 2])
def test_fp32_form_8d_covers_closed_form(mc, family):
    pr = workloads.large_8d(family, ncall=1 << 26, itmax=30, rel_tol=1e-3)
    exact = float(cf.integral(family, pr.params, 8))
    r = mc.mcubes_integrate(family, pr.params, 8, pr.ncall, pr.itmax, pr.rel_tol, pr.seed,
                            mc.mcubes_default_options(nbins=500, precision=mc.MCUBES_FP32))
    r64 = mc.mcubes_integrate(family, pr.params, 8, pr.ncall, pr.itmax, pr.rel_tol, pr.seed,
                              mc.mcubes_default_options(nbins=500))
    print(f"8-D family={family}: fp32 {r['estimate']!r} +- {r['error']!r}, fp64 "
          f"{r64['estimate']!r}, exact {exact!r}", flush=True)
    assert r["converged"]
    assert abs(r["estimate"] - exact) <= 4 * r["error"]
    # same samples: the two forms agree far inside the statistical error
    assert abs(r["estimate"] - r64["estimate"]) <= 0.1 * r64["error"]
