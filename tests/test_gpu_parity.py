"""GPU parity: the HIP V-Sample path (through the C interface) against the CPU
oracle on the same seeded inputs.  Tolerances are described in parity_util."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import closed_forms as cf
from parity_util import (assert_iteration_close, gpu_iteration, gpu_refine,
                         oracle_iteration_parallel, random_grid)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_05730_amd as m
    m.lib()
    return m


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def test_small_product_peak_lockstep(mc):
    """3-D product peak, 100 bins, 1e5 samples/iteration, 10 iterations: the GPU
    iteration and the GPU refinement fed the oracle's grid of every iteration."""
    pr = workloads.small_product_peak()
    g, m, p, n = oracle.plan(pr.dim, pr.ncall)
    plan = mc.mcubes_plan_create(pr.family, pr.params, pr.dim, pr.ncall, pr.seed,
                                 mc.mcubes_default_options(nbins=pr.nbins))
    grid = oracle.uniform_grid(pr.dim, pr.nbins)
    for t in range(pr.itmax):
        _say(f"lockstep t={t}")
        ref = oracle.iteration(pr.family, pr.params, pr.dim, pr.nbins, pr.ncall, pr.seed, t, grid)
        got = gpu_iteration(plan, t, grid)
        assert_iteration_close(pr.family, got, ref, m, p, f"t={t}")
        new_ref = oracle.refine(grid, ref[2])
        new_gpu = gpu_refine(plan, grid, ref[2])
        assert np.allclose(new_gpu, new_ref, rtol=1e-12, atol=1e-15), t
        grid = new_ref


def test_small_product_peak_free_running(mc):
    """The whole integrator on the GPU vs the whole oracle, iteration by iteration."""
    pr = workloads.small_product_peak()
    ref = oracle.integrate(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax, 0.0, pr.seed,
                           nb=pr.nbins)
    got = mc.mcubes_integrate(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax, 0.0, pr.seed,
                              mc.mcubes_default_options(nbins=pr.nbins))
    assert got["iterations"] == ref["iterations"] == pr.itmax
    assert np.allclose(got["trace_I"], ref["trace_I"], rtol=1e-12, atol=0)
    assert np.allclose(got["trace_var"], ref["trace_var"], rtol=1e-12, atol=0)
    assert got["estimate"] == pytest.approx(ref["estimate"], rel=1e-12)
    assert got["error"] == pytest.approx(ref["error"], rel=1e-12)
    assert got["chi2_dof"] == pytest.approx(ref["chi2_dof"], rel=1e-9, abs=1e-12)
    assert np.allclose(np.array(got["grid"]), ref["grid"], rtol=1e-12, atol=1e-15)
    exact = float(cf.integral(pr.family, pr.params, pr.dim))
    assert abs(got["estimate"] - exact) <= 3 * got["error"]
    assert (got["cube_side"], got["ncubes"], got["samples_per_cube"], got["samples_per_iter"]) \
        == (36, 46656, 2, 93312)


CASES = [
    # family, dim, nbins, ncall -- m spans several tiles of the persistent grid and
    # is never a multiple of the block size (ragged tail)
    (0, 1, 500, 200_001), (0, 5, 37, 300_000), (0, 8, 500, 1_000_000),
    (1, 2, 2, 50_000), (1, 3, 100, 400_000), (1, 10, 500, 300_000),
    (2, 4, 64, 250_000), (2, 7, 500, 500_000), (2, 9, 211, 200_000),
    (3, 1, 17, 99_999), (3, 6, 500, 400_000), (3, 8, 500, 1_000_000),
    (4, 3, 300, 150_000), (4, 8, 120, 300_000),
    (5, 2, 500, 120_000), (5, 5, 50, 200_000), (5, 10, 10, 100_000),
    (6, 1, 3, 1000), (6, 5, 500, 300_000), (6, 8, 500, 600_000), (6, 10, 500, 400_000),
    (7, 2, 50, 100_001), (7, 6, 500, 500_000), (7, 10, 211, 300_000),
]


@pytest.mark.parametrize("family,dim,nb,ncall", CASES)
def test_families_and_dims(mc, family, dim, nb, ncall):
    rng = np.random.default_rng(1000 * family + 10 * dim + nb % 7)
    pr = workloads.random_problem(rng, family, dim, ncall, nb)
    grid = random_grid(rng, dim, nb)
    g, m, p, n = oracle.plan(dim, ncall)
    seed = int(rng.integers(0, 2**63))
    _say(f"case family={family} dim={dim} nb={nb} ncall={ncall} m={m} p={p}")
    plan = mc.mcubes_plan_create(family, pr.params, dim, ncall, seed,
                                 mc.mcubes_default_options(nbins=nb))
    for t in (0, 3):
        ref = oracle.iteration(family, pr.params, dim, nb, ncall, seed, t, grid)
        got = gpu_iteration(plan, t, grid)
        assert_iteration_close(family, got, ref, m, p, f"t={t}")
    new_ref = oracle.refine(grid, ref[2])
    assert np.allclose(gpu_refine(plan, grid, ref[2]), new_ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("dim,ncall,nb", [(1, 2, 2), (3, 15, 5), (5, 100, 8), (10, 2048, 500),
                                          (2, 17, 3), (4, 3, 500)])
def test_degenerate_sizes(mc, dim, ncall, nb):
    """One cube (m = 1, p = ncall), p > 2, tiny grids, 10-D with 500 bins."""
    g, m, p, n = oracle.plan(dim, ncall)
    rng = np.random.default_rng(dim * 31 + ncall)
    params = list(rng.uniform(1, 4, dim)) + list(rng.uniform(0.2, 0.8, dim))
    grid = random_grid(rng, dim, nb)
    for family in (1, 3):
        plan = mc.mcubes_plan_create(family, params, dim, ncall, 5,
                                     mc.mcubes_default_options(nbins=nb))
        assert plan.info["ncubes"] == m and plan.info["samples_per_cube"] == p
        ref = oracle.iteration(family, params, dim, nb, ncall, 5, 1, grid)
        got = gpu_iteration(plan, 1, grid)
        assert_iteration_close(family, got, ref, m, p, f"family={family}")


@pytest.mark.parametrize("block,blocks", [(64, 1), (64, 7), (256, 0), (1024, 0), (1024, 3)])
def test_launch_geometry_does_not_change_results(mc, block, blocks):
    family, dim, nb, ncall = 2, 6, 100, 700_001
    rng = np.random.default_rng(77)
    params = list(rng.uniform(0.5, 3, dim)) + [0.0] * dim
    grid = random_grid(rng, dim, nb)
    g, m, p, n = oracle.plan(dim, ncall)
    ref = oracle.iteration(family, params, dim, nb, ncall, 9, 2, grid)
    plan = mc.mcubes_plan_create(family, params, dim, ncall, 9,
                                 mc.mcubes_default_options(nbins=nb, block_size=block,
                                                           blocks=blocks))
    assert plan.info["block_size"] == block
    got = gpu_iteration(plan, 2, grid)
    assert_iteration_close(family, got, ref, m, p, f"block={block} blocks={blocks}")


@pytest.mark.parametrize("family", [0, 3, 5])
def test_many_samples_per_cube_on_one_workgroup(mc, family):
    """p > 2 (10-D, g = 3, p = 17) on a grid of one workgroup, so that every
    thread walks many cubes."""
    dim, nb, ncall = 10, 50, 1 << 20
    g, m, p, n = oracle.plan(dim, ncall)
    assert p > 2
    rng = np.random.default_rng(101 + family)
    params = list(rng.uniform(0.2, 1.0, dim)) + list(rng.uniform(0.2, 0.8, dim))
    grid = random_grid(rng, dim, nb)
    ref = oracle.iteration(family, params, dim, nb, ncall, 4, 1, grid)
    plan = mc.mcubes_plan_create(family, params, dim, ncall, 4,
                                 mc.mcubes_default_options(nbins=nb, block_size=256, blocks=1))
    got = gpu_iteration(plan, 1, grid)
    assert_iteration_close(family, got, ref, m, p, f"family={family}")


def test_repeatable(mc):
    family, dim, nb, ncall = 3, 5, 200, 500_000
    rng = np.random.default_rng(5)
    params = list(rng.uniform(2, 8, dim)) + list(rng.uniform(0.2, 0.8, dim))
    grid = random_grid(rng, dim, nb)
    plan = mc.mcubes_plan_create(family, params, dim, ncall, 1,
                                 mc.mcubes_default_options(nbins=nb))
    a = gpu_iteration(plan, 0, grid)
    b = gpu_iteration(plan, 0, grid)
    assert a[0] == b[0] and a[1] == b[1]  # fixed-order reductions
    assert np.allclose(a[2], b[2], rtol=1e-14, atol=0)  # bins: atomics, order varies


@pytest.mark.parametrize("family,dim,ncall", [(3, 8, 1_000_000), (2, 5, 300_001), (6, 3, 99_999),
                                               (1, 2, 17)])
def test_without_bins_same_estimates(mc, family, dim, ncall):
    """V-Sample without bin sums (iterations whose grid is not refined) gives the
    identical estimates: same samples, same arithmetic, same reduction order."""
    rng = np.random.default_rng(family * 7 + dim)
    pr = workloads.random_problem(rng, family, dim, ncall, 50)
    grid = random_grid(rng, dim, 50)
    plan = mc.mcubes_plan_create(family, pr.params, dim, ncall, 3,
                                 mc.mcubes_default_options(nbins=50))
    a = gpu_iteration(plan, 4, grid, with_bins=True)
    b = gpu_iteration(plan, 4, grid, with_bins=False)
    assert a[0] == b[0] and a[1] == b[1]
    assert b[2] is None


def test_adapt_iters_and_skip(mc):
    pr = workloads.small_product_peak()
    kw = dict(nb=pr.nbins, adapt_iters=3, skip=2)
    ref = oracle.integrate(pr.family, pr.params, pr.dim, pr.ncall, 7, 0.0, 4, **kw)
    got = mc.mcubes_integrate(pr.family, pr.params, pr.dim, pr.ncall, 7, 0.0, 4,
                              mc.mcubes_default_options(nbins=pr.nbins, adapt_iters=3, skip=2))
    assert np.allclose(got["trace_I"], ref["trace_I"], rtol=1e-12, atol=0)
    assert got["estimate"] == pytest.approx(ref["estimate"], rel=1e-12)
    assert got["dof"] == ref["dof"] == 4
    assert np.allclose(np.array(got["grid"]), ref["grid"], rtol=1e-12, atol=1e-15)


def test_stop_rule_matches_oracle(mc):
    params = [4.0, 7.0, 0.35, 0.6]
    ref = oracle.integrate(1, params, 2, 20000, 50, 3e-5, 0, nb=50)
    got = mc.mcubes_integrate(1, params, 2, 20000, 50, 3e-5, 0,
                              mc.mcubes_default_options(nbins=50))
    assert got["converged"] and ref["converged"]
    assert got["iterations"] == ref["iterations"] >= 3
    assert got["status"] == mc.MCUBES_OK
    capped = mc.mcubes_integrate(1, params, 2, 20000, ref["iterations"] - 1, 3e-5, 0,
                                 mc.mcubes_default_options(nbins=50))
    assert capped["status"] == mc.MCUBES_NOT_CONVERGED and not capped["converged"]


def test_constant_integrand_is_exact(mc):
    got = mc.mcubes_integrate(3, [0.0] * 4 + [0.5] * 4, 4, 50_000, 5, 1e-6, 0,
                              mc.mcubes_default_options(nbins=50))
    assert abs(got["estimate"] - 1.0) < 1e-13 and got["iterations"] == 1 and got["converged"]


def test_nonfinite_is_reported(mc):
    # exp(sum a x) with a = 1000 and no cut overflows to infinity
    with pytest.raises(mc.MCubesError) as ei:
        mc.mcubes_integrate(5, [1000.0] * 2 + [2.0] * 2, 2, 10_000, 3, 0.0, 0)
    assert ei.value.code == mc.MCUBES_E_NONFINITE


@pytest.mark.parametrize("family", [3, 2])
def test_8d_covers_closed_form(mc, family):
    """The 8-D Gaussian and corner peak (a ~ U(5, 15), u ~ U(0, 1), 500 bins) at
    2^26 samples per iteration integrate to 1e-3 relative error and cover the
    closed form within 4 standard deviations."""
    pr = workloads.large_8d(family, ncall=1 << 26, itmax=30, rel_tol=1e-3)
    exact = float(cf.integral(family, pr.params, 8))
    r = mc.mcubes_integrate(family, pr.params, 8, pr.ncall, pr.itmax, pr.rel_tol, pr.seed,
                            mc.mcubes_default_options(nbins=500))
    _say(f"8-D family={family}: {r['estimate']!r} +- {r['error']!r} vs {exact!r}, "
         f"{r['iterations']} iterations")
    assert r["converged"]
    assert abs(r["estimate"] - exact) <= 4 * r["error"]
    assert r["chi2_dof"] < 5


@pytest.mark.slow
@pytest.mark.parametrize("family", [3, 0, 2])
def test_full_size_8d_iteration(mc, family):
    """8-D Genz integrand at the full 2^30 samples/iteration and 500 bins, in the
    launch configuration the benchmark times: one whole iteration on an adapted
    grid, compared with the oracle run over all 859,963,392 samples."""
    pr = workloads.large_8d(family)
    warm = oracle.integrate(family, pr.params, 8, 1 << 20, 3, 0.0, 123, nb=500)
    grid = warm["grid"]
    g, m, p, n = oracle.plan(8, pr.ncall)
    _say(f"full-size family={family} m={m} oracle threads start")
    ref = oracle_iteration_parallel(family, pr.params, 8, 500, pr.ncall, pr.seed, 7, grid)
    plan = mc.mcubes_plan_create(family, pr.params, 8, pr.ncall, pr.seed,
                                 mc.mcubes_default_options(nbins=500))
    got = gpu_iteration(plan, 7, grid)
    _say(f"full-size family={family} I={got[0]!r} ref={ref[0]!r} var={got[1]!r} ref={ref[1]!r}")
    assert_iteration_close(family, got, ref, m, p, f"full-size family={family}")
    assert np.allclose(gpu_refine(plan, grid, ref[2]), oracle.refine(grid, ref[2]),
                       rtol=1e-12, atol=1e-15)


def test_boundary_calls_match_the_oracles_through_one_table(mc):
    """The two boundary calls §8's interface names, driven through one
    signature table on both libraries (mcubes_* and mcubes_oracle_*): one
    iteration of the 3-D product-peak workload from the same random grid
    with the host-pointer iterate call (I_t, var_t, bins, refined grid to
    the 1e-12 bar), a second iteration from the first's refined oracle grid,
    and the whole integrator (10 iterations, trace and result)."""
    import abi_mirror as am
    pr = workloads.small_product_peak()
    g, m, p, n = oracle.plan(pr.dim, pr.ncall)
    sides = {k: am.Side(path, am.PREFIX[k]) for k, path in
             (("gpu", mc.LIB_PATH), ("oracle", oracle.LIB_PATH))}
    opt = am.options(nbins=pr.nbins)
    plans = {}
    for k, side in sides.items():
        rc, h = side.plan(pr.family, pr.params, pr.dim, pr.ncall, pr.seed, opt)
        assert rc == 0, (k, rc)
        plans[k] = h
    try:
        grid = random_grid(np.random.default_rng(8), pr.dim, pr.nbins)
        for t in (0, 1):
            _say(f"iterate t={t}")
            out = {k: sides[k].iterate(plans[k], grid, t, pr.dim, pr.nbins) for k in sides}
            rc_g, I_g, v_g, b_g, new_g = out["gpu"]
            rc_o, I_o, v_o, b_o, new_o = out["oracle"]
            assert rc_g == rc_o == 0
            assert_iteration_close(pr.family, (I_g, v_g, b_g), (I_o, v_o, b_o), m, p, f"t={t}")
            assert np.allclose(new_g, new_o, rtol=1e-12, atol=1e-15)
            grid = new_o
        # the host-pointer call rejects what the oracle's rejects
        bad = grid.copy()
        bad[1, -1] = 0.999
        assert sides["gpu"].iterate(plans["gpu"], bad, 0, pr.dim, pr.nbins)[0] == -1
        assert sides["oracle"].iterate(plans["oracle"], bad, 0, pr.dim, pr.nbins)[0] == -1
    finally:
        for k, h in plans.items():
            sides[k].destroy(h)
    _say("integrate through both tables")
    res = {k: sides[k].integrate(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax, 0.0, pr.seed,
                                 opt) for k in sides}
    (rc_g, r_g, grid_g, tr_g), (rc_o, r_o, grid_o, tr_o) = res["gpu"], res["oracle"]
    assert rc_g == rc_o == 1 and r_g.iterations == r_o.iterations == pr.itmax
    assert np.allclose(tr_g, tr_o, rtol=1e-12, atol=0)
    assert r_g.estimate == pytest.approx(r_o.estimate, rel=1e-12)
    assert r_g.error == pytest.approx(r_o.error, rel=1e-12)
    assert np.allclose(grid_g, grid_o, rtol=1e-12, atol=1e-15)
    assert (r_g.cube_side, r_g.ncubes, r_g.samples_per_cube) == (g, m, p)
