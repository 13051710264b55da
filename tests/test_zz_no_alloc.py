"""mcubes_integrate_noalloc -- the whole integrator with every device buffer in
the library's static scratch array -- against mcubes_integrate, through the C
interface.  Both run the same kernels with the same launch geometry:
  * without grid refinement (adapt_iters = 0) every iteration samples the
    uniform grid and its estimate comes from fixed-order reductions, so the
    results are identical bit for bit;
  * with refinement, the first iteration is still identical; the bin sums
    are accumulated with FP64 atomics in an order that varies between runs,
    so the refined edges of two runs differ in their last bits, and later
    iterations drift apart by a few ulps of the estimate (3.6e-16 relative
    measured after six iterations of the 8-D Gaussian); asked: 1e-9 relative
    per iteration and 1e-9 on the edges, far below the statistical error
    (~1e-5 relative) and far above the drift.
Two problems in a row, the second smaller (the scratch keeps the first call's
contents, which the second must not read), and a problem too large for the
scratch is refused before any device work."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_05730_amd as m
    m.lib()
    return m


_SAME = ("iterations", "dof", "converged", "status", "cube_side", "ncubes", "samples_per_cube",
         "samples_per_iter")


def _close(got, ref, what, exact):
    for k in _SAME:
        assert got[k] == ref[k], (what, k, got[k], ref[k])
    gI, rI = np.array(got["trace_I"]), np.array(ref["trace_I"])
    gV, rV = np.array(got["trace_var"]), np.array(ref["trace_var"])
    assert gI[0] == rI[0] and gV[0] == rV[0], what  # the first iteration: uniform grid
    tol = 0.0 if exact else 1e-9
    assert np.all(np.abs(gI - rI) <= tol * np.abs(rI)), (what, gI - rI)
    assert np.all(np.abs(gV - rV) <= tol * np.abs(rV)), (what, gV - rV)
    for k in ("estimate", "error", "chi2_dof"):
        assert abs(got[k] - ref[k]) <= tol * abs(ref[k]), (what, k, got[k], ref[k])
    assert np.all(np.abs(np.array(got["grid"]) - np.array(ref["grid"])) <= tol), what


@pytest.mark.parametrize("adapt", [0, -1])
def test_noalloc_matches_integrate_twice_then_smaller(mc, adapt):
    big = workloads.large_8d(workloads.GAUSSIAN, ncall=1 << 22, itmax=6, rel_tol=1e-4)
    small = workloads.small_product_peak()
    for pr in (big, small):
        print(f"noalloc: {pr.name} dim {pr.dim} ncall {pr.ncall} bins {pr.nbins} adapt {adapt}",
              file=sys.stderr, flush=True)
        opts = mc.mcubes_default_options(nbins=pr.nbins, adapt_iters=adapt)
        ref = mc.mcubes_integrate(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax, pr.rel_tol,
                                  pr.seed, opts)
        got = mc.mcubes_integrate_noalloc(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax,
                                          pr.rel_tol, pr.seed, opts)
        _close(got, ref, f"{pr.name} adapt {adapt}", exact=adapt == 0)
        assert got["kernel_ms"] == 0.0


def test_noalloc_refuses_a_problem_beyond_its_scratch(mc):
    # 10-D, 500 bins and 8000 blocks: 2 * 10 * 501 + 10 * 500 + 2 * 8000 + 2 +
    # MCUBES_STATE_LEN = 33078 doubles > MCUBES_NOALLOC_SCRATCH = 32768
    opts = mc.mcubes_default_options(nbins=500, blocks=8000)
    with pytest.raises(mc.MCubesError) as ei:
        mc.mcubes_integrate_noalloc(3, [1.0] * 20, 10, 10**6, 2, 0.0, 0, opts)
    assert ei.value.code == mc.MCUBES_E_ARG
    assert "scratch" in mc.mcubes_last_error()
